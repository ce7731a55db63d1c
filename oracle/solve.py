"""Oracle: the transfer matrix T = A^-1 B (App. A.4) and the PCG of Sec. 2.3.1.

Test infrastructure only (see the package docstring).

``transfer_direct`` computes T exactly up to round-off with a library
factorisation (dense Cholesky for small systems, sparse LU otherwise).
``pcg`` is the preconditioned conjugate gradient method with a diagonal
preconditioner, one right-hand side at a time, in its textbook form
(Golub & Van Loan): it is what the GPU path iterates, and is used to pin
iteration counts.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def factorize(A):
    """A solver object for the grounded SPD matrix A: x = f(b)."""
    n = A.shape[0]
    if n <= 12000:
        c = sla.cho_factor(A.toarray(), lower=True)
        return lambda b: sla.cho_solve(c, b)
    lu = spla.splu(sp.csc_matrix(A), permc_spec="COLAMD")
    return lambda b: lu.solve(np.asarray(b, dtype=np.float64))


def transfer_direct(A, B, solver=None):
    """T = A^-1 B, one column per electrode (App. A.4), n x L dense."""
    f = solver or factorize(A)
    Bd = B.toarray() if sp.issparse(B) else np.asarray(B)
    return np.asarray(f(Bd))


class NotConverged(RuntimeError):
    pass


def pcg(A, b, d, tol=1e-8, maxit=50000, x0=None):
    """Solve A x = b by PCG with the diagonal preconditioner D = diag(d).

    Steps: r = b - A x, z = D^-1 r, p = z, rho = r.z; then repeat
    q = A p, alpha = rho / p.q, x += alpha p, r -= alpha q; stop when
    ||r||_2 <= tol ||b||_2 (the count is the number of updates done);
    else z = D^-1 r, rho' = r.z, beta = rho'/rho, p = z + beta p.

    Returns (x, iterations, ||r||/||b|| of the recurrence).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0, 0.0
    r = b - A @ x
    if np.linalg.norm(r) <= tol * bnorm:
        return x, 0, np.linalg.norm(r) / bnorm
    z = r / d
    p = z.copy()
    rho = r @ z
    for k in range(1, maxit + 1):
        q = A @ p
        pq = p @ q
        if not pq > 0.0:
            raise NotConverged("p.Ap <= 0: the matrix is not positive definite")
        alpha = rho / pq
        x += alpha * p
        r -= alpha * q
        rn = np.linalg.norm(r)
        if rn <= tol * bnorm:
            return x, k, rn / bnorm
        z = r / d
        rho_new = r @ z
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    raise NotConverged(f"no convergence in {maxit} iterations")


def transfer_pcg(A, B, d, tol=1e-8, maxit=50000, columns=None):
    """T column by column with ``pcg``; returns (T, iterations, relres)."""
    Bd = B.toarray() if sp.issparse(B) else np.asarray(B)
    L = Bd.shape[1]
    cols = range(L) if columns is None else columns
    T = np.zeros((Bd.shape[0], len(cols)))
    its = np.zeros(len(cols), dtype=np.int64)
    rel = np.zeros(len(cols))
    for j, c in enumerate(cols):
        T[:, j], its[j], rel[j] = pcg(A, Bd[:, c], d, tol, maxit)
    return T, its, rel


def pcg_columns(A, Bm, d, tol=1e-8, maxit=50000):
    """``pcg`` applied to every column of Bm at once.

    Each column runs exactly the iteration of ``pcg`` (same steps, same stop
    rule); a column stops changing once it has converged.  Only the loop over
    columns is replaced by array arithmetic.  Returns (X, iterations, relres).
    """
    Bm = Bm.toarray() if sp.issparse(Bm) else np.asarray(Bm, dtype=np.float64)
    n, k = Bm.shape
    X = np.zeros((n, k))
    its = np.zeros(k, dtype=np.int64)
    bnorm = np.linalg.norm(Bm, axis=0)
    active = bnorm > 0.0
    R = Bm.copy()
    relres = np.where(active, 1.0, 0.0)
    Zm = R / d[:, None]
    P = Zm.copy()
    rho = (R * Zm).sum(axis=0)
    for it in range(1, maxit + 1):
        if not active.any():
            break
        Q = A @ P
        pq = (P * Q).sum(axis=0)
        if not (pq[active] > 0.0).all():
            raise NotConverged("p.Ap <= 0: the matrix is not positive definite")
        alpha = np.where(active, rho / np.where(active, pq, 1.0), 0.0)
        X += alpha * P
        R -= alpha * Q
        rn = np.linalg.norm(R, axis=0)
        done = active & (rn <= tol * bnorm)
        its[done] = it
        relres[done] = rn[done] / bnorm[done]
        active &= ~done
        Zm = R / d[:, None]
        rho_new = (R * Zm).sum(axis=0)
        beta = np.where(active, rho_new / np.where(active, rho, 1.0), 0.0)
        rho = np.where(active, rho_new, rho)
        P = np.where(active, Zm + beta * P, P)
    if active.any():
        raise NotConverged(f"no convergence in {maxit} iterations")
    return X, its, relres


def transfer_reference(A, B, tol=1e-12):
    """T = A^-1 B exact up to round-off: dense Cholesky for small systems,
    else ``pcg_columns`` with the Jacobi diagonal at a tight tolerance."""
    if A.shape[0] <= 12000:
        return transfer_direct(A, B)
    X, _, _ = pcg_columns(A, B, A.diagonal().copy(), tol=tol)
    return X
