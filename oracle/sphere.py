"""Oracle: closed-form potential of a current dipole in a multilayer sphere.

Test infrastructure only (see the package docstring).

Solves the governing equation of Sec. 2, div(sigma grad u) = div J^p, for a
point dipole J^p = q delta(r - r0) inside the innermost of K concentric
shells (outer radii r_1 < ... < r_K, conductivities sigma_1..sigma_K) with
no normal current through the outer surface (condition (I) of App. A.1 with
no electrodes).  In an unbounded medium of conductivity sigma the solution is
u = q.(r - r0) / (4 pi sigma |r - r0|^3).

Expanding 1/|r - r0| in Legendre polynomials, q . grad_{r0} turns the degree-n
term into rho^(n-1) Theta_n / r^(n+1) with rho = |r0|, cos g = rhat.r0hat and

    Theta_n = n P_n(cos g) (q.r0hat) + P_n'(cos g) (q.rhat - cos g q.r0hat),

a degree-n surface harmonic.  For each n the radial factor is a combination
of r^n and r^-(n+1) in every shell, with potential and sigma du/dr continuous
at each interface and du/dr = 0 at r_K.  Writing the shell-k factor as
c_k [(r/r_k)^n + t_k (r_k/r)^(n+1)] keeps every quantity bounded:

* outer shell: t_K = n/(n+1) (zero normal derivative at r_K);
* going inward across r_{k-1}, continuity of sigma u'/u fixes t_{k-1};
* in shell 1 the r^-(n+1) coefficient must be the source's 1/(4 pi sigma_1);
* continuity of u carries the amplitude back out to r_K.

One shell (K = 1) gives the textbook factor (2n+1) / (n R^(n+1)), and a
centred dipole gives 3 q.rhat / (4 pi sigma R^2).
"""
from __future__ import annotations

import math

import numpy as np


def _legendre(nmax, x):
    """P_n(x) and P_n'(x) for n = 0..nmax (arrays over x)."""
    x = np.asarray(x, dtype=np.float64)
    P = np.zeros((nmax + 1,) + x.shape)
    dP = np.zeros_like(P)
    P[0] = 1.0
    if nmax >= 1:
        P[1] = x
        dP[1] = 1.0
    for n in range(1, nmax):
        P[n + 1] = ((2 * n + 1) * x * P[n] - n * P[n - 1]) / (n + 1)
        dP[n + 1] = dP[n - 1] + (2 * n + 1) * P[n]
    return P, dP


def radial_factor(n, rho, radii, sigmas):
    """rho^(n-1) R_n(r_K) for degree n >= 1 (the factor multiplying Theta_n).

    R_n is the radial function of the degree-n term, normalised so that the
    singular part in shell 1 is r^-(n+1) / (4 pi sigma_1).
    """
    K = len(radii)
    t = [0.0] * K
    t[K - 1] = n / (n + 1.0)
    for k in range(K - 1, 0, -1):
        x = radii[k - 1] / radii[k]
        x2 = x ** (2 * n + 1)
        if x2 == 0.0:
            raise OverflowError("degree too high for the shell ratios")
        s, sk, tk = sigmas[k - 1], sigmas[k], t[k]
        # Matching sigma u'/u at r_{k-1}, written without cancellation:
        # shell k gives sigma_k (n x2 - (n+1) t_k) / (r_{k-1} (x2 + t_k)).
        t[k - 1] = ((n * x2 * (s - sk) + tk * (s * n + sk * (n + 1)))
                    / (x2 * (s * (n + 1) + sk * n) + (n + 1) * tk * (s - sk)))
    # amplitude: shell 1 factor c_1 = 1/(4 pi s1 t_1 r_1^(n+1)); the rho^(n-1)
    # is folded in as (rho/r_1)^(n-1) / r_1^2.
    amp = (rho / radii[0]) ** (n - 1) / (4.0 * math.pi * sigmas[0] * t[0] * radii[0] ** 2)
    for k in range(1, K):
        x = radii[k - 1] / radii[k]
        amp *= (1.0 + t[k - 1]) * x ** (n + 1) / (x ** (2 * n + 1) + t[k])
    amp *= 1.0 + t[K - 1]
    if not math.isfinite(amp):
        raise OverflowError("degree too high for the shell ratios")
    return amp


def potential(points, r0, q, radii, sigmas, rel_tol=1e-14, nmax=3000):
    """Potential at points on the outer surface |r| = r_K.

    points (P, 3), r0 (3,), q (3,).  The dipole must lie in shell 1; the
    series converges like (|r0|/r_1)^n, so keep |r0| <= 0.9 r_1.
    """
    points = np.atleast_2d(np.asarray(points, dtype=np.float64))
    r0 = np.asarray(r0, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    rho = float(np.linalg.norm(r0))
    if rho >= radii[0]:
        raise ValueError("dipole must lie inside the innermost shell")
    rhat = points / np.linalg.norm(points, axis=1, keepdims=True)
    if rho == 0.0:
        return radial_factor(1, 0.0, radii, sigmas) * (rhat @ q)
    r0hat = r0 / rho
    cg = np.clip(rhat @ r0hat, -1.0, 1.0)
    q_r0 = q @ r0hat
    q_r = rhat @ q
    total = np.zeros(points.shape[0])
    chunk = 64
    n0 = 1
    while n0 <= nmax:
        n1 = min(nmax, n0 + chunk - 1)
        P, dP = _legendre(n1, cg)
        done = False
        for n in range(n0, n1 + 1):
            theta = n * P[n] * q_r0 + dP[n] * (q_r - cg * q_r0)
            term = radial_factor(n, rho, radii, sigmas) * theta
            total += term
            scale = np.abs(total).max()
            if n > 3 and np.abs(term).max() <= rel_tol * max(scale, 1e-300) \
                    and radial_factor(n, rho, radii, sigmas) * (n * n + 1) <= \
                    rel_tol * max(scale, 1e-300):
                done = True
                break
        if done:
            return total
        n0 = n1 + 1
    raise RuntimeError("multilayer series did not converge")
