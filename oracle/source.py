"""Oracle: the source matrix G for point dipoles (App. A.1, g_ij).

Test infrastructure only (see the package docstring).

The paper's G has entries g_ij = int psi_i (div w_j) dV for H(div) source
basis functions w_j (Sec. 2 "Primary current model"); the H(div)/PBO
coefficients are not given in the paper.  The reading used here is the
classical partial-integration point dipole: a unit dipole q = e_k at a point
x_0 inside tetrahedron d gives (G x)_i = int psi_i div J^p dV =
-q . grad psi_i(x_0), so

    G[i, 3 d + k] = -d psi_i / d x_k   on tetrahedron d,

four nonzeros per column, columns ordered "position 1 xyz, position 2 xyz,
..." as the Cartesian source orientations of Sec. 2.4.2 ("Mesh tool").
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import element_gradients


def point_dipole_matrix(nodes, tets, dipole_tets):
    """G as an (n x 3m) CSC matrix with sorted row indices."""
    d = np.asarray(dipole_tets, dtype=np.int64)
    m = d.shape[0]
    n = nodes.shape[0]
    g, _ = element_gradients(nodes, tets[d])          # (m, 4, 3)
    rows = np.repeat(tets[d].astype(np.int64)[:, None, :], 3, axis=1)  # (m, 3, 4)
    cols = np.broadcast_to((3 * np.arange(m)[:, None] + np.arange(3)[None, :])[:, :, None],
                           (m, 3, 4))
    vals = -np.transpose(g, (0, 2, 1))                # (m, 3[k], 4[i])
    G = sp.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())),
                      shape=(n, 3 * m)).tocsc()
    G.sort_indices()
    return G


def dipole_positions(nodes, tets, dipole_tets):
    """Centroids of the dipole tetrahedra (the source positions)."""
    return nodes[tets[np.asarray(dipole_tets, dtype=np.int64)]].mean(axis=1)
