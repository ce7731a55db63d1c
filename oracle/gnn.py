"""Oracle: the mesh-graph network of the learned PCG warm start (FP64 NumPy).

Test infrastructure only (see the package docstring).  The paper has no
learned component; this is the reference for the project's own network,
whose GPU forward and backward kernels are checked against it.

Graph: the mesh graph without self loops, aggregated with the symmetric
normalisation Ahat = D^-1/2 Adj D^-1/2 (D = node degrees), so the transpose
needed by the backward pass is Ahat itself.

Layer k (k = 0..K-1) with h_k aggregation hops (h_k >= 1) maps H_k
(n x F_k) to

    M_k     = Ahat^(h_k) H_k     (Ahat applied h_k times)
    Z_k     = H_k Ws_k + M_k Wn_k + b_k
    H_{k+1} = relu(Z_k)          (identity on the last layer)

Layers with many hops see far across the mesh: the potential change that a
conductivity perturbation causes is global, and polynomials in Ahat of high
degree act on the smooth part of the mesh graph's spectrum.

Prediction y = H_K[:, 0]; loss = sum_i (y_i - t_i)^2 / sum_i t_i^2.
Parameters per layer: Ws (F_k x F_{k+1}), Wn (F_k x F_{k+1}), b (F_{k+1}).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def normalized_adjacency(indptr, indices, n):
    """Ahat from a CSR structure that may contain the diagonal."""
    rows = np.repeat(np.arange(n), np.diff(indptr))
    keep = rows != indices
    r, c = rows[keep], indices[keep]
    deg = np.bincount(r, minlength=n).astype(np.float64)
    v = 1.0 / np.sqrt(deg[r] * deg[c])
    return sp.csr_matrix((v, (r, c)), shape=(n, n))


def init_params(dims, seed):
    """Glorot-uniform weights, zero biases; dims = [F_0, F_1, ..., F_K]."""
    rng = np.random.default_rng(seed)
    params = []
    for fi, fo in zip(dims[:-1], dims[1:]):
        lim = np.sqrt(6.0 / (fi + fo))
        params.append(dict(Ws=rng.uniform(-lim, lim, (fi, fo)),
                           Wn=rng.uniform(-lim, lim, (fi, fo)),
                           b=np.zeros(fo)))
    return params


def aggregate(Ahat, H, hops):
    """Ahat^hops H, one product at a time."""
    M = H
    for _ in range(hops):
        M = Ahat @ M
    return M


def forward(params, Ahat, X, hops=None):
    """Returns (prediction y, cache for backward); hops[k] per layer (1)."""
    H = X
    cache = []
    K = len(params)
    for k, p in enumerate(params):
        M = aggregate(Ahat, H, hops[k] if hops else 1)
        Z = H @ p["Ws"] + M @ p["Wn"] + p["b"]
        cache.append((H, M, Z))
        H = np.maximum(Z, 0.0) if k < K - 1 else Z
    return H[:, 0], cache


def loss(y, t):
    return float(((y - t) ** 2).sum() / (t ** 2).sum())


def backward(params, Ahat, cache, y, t, hops=None):
    """Gradients of the loss with respect to every parameter."""
    K = len(params)
    dH = np.zeros_like(cache[-1][2])
    dH[:, 0] = 2.0 * (y - t) / (t ** 2).sum()
    grads = [None] * K
    for k in range(K - 1, -1, -1):
        H, M, Z = cache[k]
        dZ = dH if k == K - 1 else dH * (Z > 0.0)
        grads[k] = dict(Ws=H.T @ dZ, Wn=M.T @ dZ, b=dZ.sum(axis=0))
        dM = dZ @ params[k]["Wn"].T
        dH = dZ @ params[k]["Ws"].T + aggregate(Ahat.T, dM, hops[k] if hops else 1)
    return grads


def adam_step(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), in place; state holds m, v and t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k, (p, g) in enumerate(zip(params, grads)):
        for name in ("Ws", "Wn", "b"):
            key = (k, name)
            m = state.setdefault(("m",) + key, np.zeros_like(p[name]))
            v = state.setdefault(("v",) + key, np.zeros_like(p[name]))
            m[...] = b1 * m + (1 - b1) * g[name]
            v[...] = b2 * v + (1 - b2) * g[name] ** 2
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            p[name] -= lr * mh / (np.sqrt(vh) + eps)
