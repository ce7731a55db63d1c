"""Pins of the oracle's point-dipole source matrix (App. A.1, g_ij)."""
import numpy as np

from oracle import source


def test_dipole_columns_reproduce_linear_gradients(head8):
    # For u(x) = a . x + c the P1 interpolant is exact, so for the column of
    # dipole d and direction k: sum_i G[i, 3d+k] u(x_i) = -du/dx_k = -a_k.
    H = head8
    G = source.point_dipole_matrix(H.nodes, H.tets, H.dipole_tets[:50]).toarray()
    a = np.array([0.3, -1.7, 2.2])
    u = H.nodes @ a + 0.9
    np.testing.assert_allclose(G.T @ u, -np.tile(a, 50), rtol=1e-10)
    # constants are annihilated: the gradients of the basis sum to zero
    np.testing.assert_allclose(G.sum(axis=0), 0.0, atol=1e-9 * np.abs(G).max())


def test_dipole_matrix_layout(head8):
    H = head8
    G = source.point_dipole_matrix(H.nodes, H.tets, H.dipole_tets[:7])
    assert G.shape == (H.n, 21)
    assert np.all(np.diff(G.indptr) == 4)
    for c in range(21):
        rows = G.indices[G.indptr[c]:G.indptr[c + 1]]
        assert np.all(np.diff(rows) > 0)
        np.testing.assert_array_equal(rows, np.sort(H.tets[H.dipole_tets[c // 3]]))
