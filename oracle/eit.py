"""Oracle: linearized EIT lead field (App. A.3).

Test infrastructure only (see the package docstring).

With G = 0 and injected currents I, Eq. (u_system) gives z = T v,
M v = I with M = C - B^T A^-1 B = C - B^T T, and the data y = R v, i.e.
y = R M^-1 I.  Differentiating with respect to the conductivity s_m of
element m (sigma = sum_m s_m chi_m):

    dy/ds_m = -R M^-1 B^T A^-1 (dA/ds_m) A^-1 B M^-1 I
            = -R M^-1 T^T (K1_m U),     U = T M^-1 I,

where K1_m = dA/ds_m is the element stiffness matrix of tet m with unit
conductivity (4 x 4, supported on the tet's vertices).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import element_gradients
from .leadfield import average_reference


def forward(T, B, C, I):
    """y = R M^-1 I for current patterns I (L x P)."""
    Bd = B.toarray() if sp.issparse(B) else np.asarray(B)
    M = np.diag(C) - Bd.T @ T
    return average_reference(T.shape[1]) @ np.linalg.solve(M, I)


def unit_element_matrices(nodes, tets, elems):
    g, vol = element_gradients(nodes, tets[elems])
    return vol[:, None, None] * np.einsum("eia,eja->eij", g, g)


def leadfield(T, B, C, I, nodes, tets, elems):
    """dy/ds_m for the listed elements: array (P, L, len(elems))."""
    Bd = B.toarray() if sp.issparse(B) else np.asarray(B)
    L = T.shape[1]
    M = np.diag(C) - Bd.T @ T
    Minv = np.linalg.inv(M)
    U = T @ (Minv @ I)                        # n x P
    K1 = unit_element_matrices(nodes, tets, elems)
    RMT = average_reference(L) @ Minv @ T.T   # L x n
    P = I.shape[1]
    out = np.zeros((P, L, len(elems)))
    for j, m in enumerate(elems):
        v = tets[m]
        for p in range(P):
            w = K1[j] @ U[v, p]                # K1_m U on the tet's vertices
            out[p, :, j] = -RMT[:, v] @ w
    return out
