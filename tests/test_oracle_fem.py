"""Pins of the oracle's FEM matrices (App. A.1) against closed forms.

None of these re-types the oracle's formulas: each compares with a value
derived another way (a hand-derived element matrix, a finite-difference
stencil, quadrature, a null vector of the continuous problem).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fem
from paper_1811_07717_amd import headmodel as hm


def test_kuhn_element_matrix_closed_form():
    # Path simplex (0,0,0)->(h,0,0)->(h,h,0)->(h,h,h): the basis gradients are
    # (-1,0,0)/h, (1,-1,0)/h, (0,1,-1)/h, (0,0,1)/h and the volume h^3/6, so
    # K = (sigma h / 6) * tridiag(-1, [1,2,2,1], -1).
    h, sigma = 0.004, 0.7
    nodes = np.array([[0, 0, 0], [h, 0, 0], [h, h, 0], [h, h, h]], dtype=np.float64)
    tets = np.array([[0, 1, 2, 3]], dtype=np.int32)
    K = fem.element_stiffness(nodes, tets, np.array([sigma]))[0]
    ref = sigma * h / 6.0 * np.array([[1, -1, 0, 0], [-1, 2, -1, 0],
                                      [0, -1, 2, -1], [0, 0, -1, 1]], dtype=np.float64)
    np.testing.assert_allclose(K, ref, rtol=1e-13, atol=1e-15 * sigma * h)


def test_gradients_against_barycentric_solve():
    # Independent route: psi_i(x) = [1 x y z] . c_i with [1 x_j]^T c_i = delta_ij.
    rng = np.random.default_rng(7)
    nodes = rng.normal(size=(40, 3))
    tets = rng.choice(40, size=(25, 4), replace=True)
    tets = np.array([t for t in tets if len(set(t)) == 4], dtype=np.int32)
    g, vol = fem.element_gradients(nodes, tets)
    for e, t in enumerate(tets):
        M = np.hstack([np.ones((4, 1)), nodes[t]])
        Cm = np.linalg.inv(M)                      # column i = coefficients of psi_i
        np.testing.assert_allclose(g[e], Cm[1:, :].T, rtol=1e-10, atol=1e-12)
        assert vol[e] == pytest.approx(abs(np.linalg.det(M)) / 6.0, rel=1e-12)


def test_anisotropic_tensor_reduces_to_scalar():
    H = hm.make_head(8.0, L=4, m=1, seed=3)
    s6 = np.zeros((H.e, 6))
    s6[:, :3] = H.sigma[:, None]
    K1 = fem.element_stiffness(H.nodes, H.tets[:200], H.sigma[:200])
    K6 = fem.element_stiffness(H.nodes, H.tets[:200], s6[:200])
    np.testing.assert_allclose(K6, K1, rtol=1e-14, atol=0)


def test_interior_row_is_seven_point_stencil():
    # Kuhn P1 stiffness with constant sigma equals sigma*h times the 7-point
    # finite-difference Laplacian: 6 on the diagonal, -1 for the 6 axis
    # neighbours and 0 for the 8 diagonal neighbours of the Kuhn graph.
    h_mm, sigma = 8.0, 0.5
    nodes, tets, sig, _, _ = hm.kuhn_sphere(h_mm, sigmas=(sigma,) * 4)
    K = fem.stiffness(nodes, tets, sig)
    i = int(np.argmin((nodes ** 2).sum(1)))
    h = h_mm * 1e-3
    cols = K.indices[K.indptr[i]:K.indptr[i + 1]]
    vals = K.data[K.indptr[i]:K.indptr[i + 1]]
    assert cols.size == 15
    off = np.rint((nodes[cols] - nodes[i]) / h).astype(int)
    for o, v in zip(off, vals):
        nz = np.abs(o).sum()
        expect = 6.0 if nz == 0 else (-1.0 if nz == 1 else 0.0)
        assert v == pytest.approx(expect * sigma * h, abs=1e-12 * sigma * h)


def test_stiffness_symmetric_zero_rowsum_positive_diag(sys8):
    K = sys8["K"]
    d = K.diagonal()
    assert (d > 0).all()
    asym = abs(K - K.T).max()
    assert asym <= 1e-13 * d.max()
    rs = np.abs(np.asarray(K.sum(axis=1)).ravel())
    assert (rs <= 1e-12 * d).all()


def test_structure_is_mesh_graph(head8, sys8):
    # nnz of the 8 mm sphere mesh graph, counted independently from the
    # generator's vertex pairs.
    t = head8.tets.astype(np.int64)
    pairs = np.unique(np.stack([np.repeat(t, 4, 1).ravel(), np.tile(t, (1, 4)).ravel()], 1), axis=0)
    assert sys8["A"].nnz == pairs.shape[0] == 103681


def _midpoint_quadrature(nodes, tri):
    """int psi_i psi_j and int psi_i over a triangle with the edge-midpoint
    rule (exact for quadratics); basis values from barycentric solves."""
    x = nodes[tri]
    area = 0.5 * np.linalg.norm(np.cross(x[1] - x[0], x[2] - x[0]))
    mids = [(x[0] + x[1]) / 2, (x[1] + x[2]) / 2, (x[0] + x[2]) / 2]
    # barycentric coordinates in the triangle's plane via least squares
    Mb = np.vstack([x.T, np.ones(3)])
    mass = np.zeros((3, 3))
    lin = np.zeros(3)
    for p in mids:
        lam = np.linalg.lstsq(Mb, np.append(p, 1.0), rcond=None)[0]
        mass += np.outer(lam, lam) * area / 3
        lin += lam * area / 3
    return mass, lin, area


def test_electrode_terms_against_quadrature():
    rng = np.random.default_rng(11)
    nodes = rng.normal(size=(5, 3)) * 0.01
    tris = np.array([[0, 1, 2], [1, 2, 3], [2, 3, 4]], dtype=np.int32)
    te = np.array([0, 0, 1], dtype=np.int32)
    Z = np.array([1500.0, 3000.0])
    (r, c, v), B, C, calA = fem.electrode_terms(nodes, tris, te, Z, 5)
    Acem = fem.to_csr(r, c, v, 5).toarray()
    ref_A = np.zeros((5, 5))
    ref_B = np.zeros((5, 2))
    areas = [_midpoint_quadrature(nodes, t)[2] for t in tris]
    cal = np.array([areas[0] + areas[1], areas[2]])
    for k, t in enumerate(tris):
        mass, lin, _ = _midpoint_quadrature(nodes, t)
        l = te[k]
        ref_A[np.ix_(t, t)] += mass / (Z[l] * cal[l])
        ref_B[t, l] += lin / (Z[l] * cal[l])
    np.testing.assert_allclose(Acem, ref_A, rtol=1e-12, atol=1e-20)
    np.testing.assert_allclose(B.toarray(), ref_B, rtol=1e-12, atol=1e-20)
    np.testing.assert_allclose(C, 1.0 / Z, rtol=1e-14)
    np.testing.assert_allclose(calA, cal, rtol=1e-13)


def test_single_triangle_closed_form():
    # One triangle, one electrode: 1/(Z calA) * |F|(1+delta)/12 = (1+delta)/(12 Z),
    # b = 1/(3Z) and c = 1/Z, independent of the triangle's shape and size.
    nodes = np.array([[0.0, 0, 0], [0.003, 0.0005, 0], [0.001, 0.002, 0.0004]])
    Z = 2000.0
    (r, c, v), B, C, _ = fem.electrode_terms(nodes, np.array([[0, 1, 2]]), np.array([0]),
                                             np.array([Z]), 3)
    Acem = fem.to_csr(r, c, v, 3).toarray()
    np.testing.assert_allclose(Acem, (np.ones((3, 3)) + np.eye(3)) / (12 * Z), rtol=1e-13)
    np.testing.assert_allclose(B.toarray().ravel(), np.full(3, 1 / (3 * Z)), rtol=1e-13)
    assert C[0] == pytest.approx(1 / Z, rel=1e-14)


def test_block_system_null_vector(head8):
    # Without grounding the CEM system of Eq. (u_system) annihilates the
    # constant: A0 1 - B 1 = 0 and -B^T 1 + C 1 = 0 (a constant potential with
    # equal electrode voltages carries no current).  This holds only with the
    # 1/(Z calA) scaling of B and C.
    H = head8
    S = fem.assemble(H.nodes, H.tets, H.sigma, H.tris, H.tri_electrode, H.Z)
    A0, B, C = S["A0"], S["B"], S["C"]
    one_n, one_L = np.ones(H.n), np.ones(H.L)
    top = A0 @ one_n - B @ one_L
    bot = -(B.T @ one_n) + C
    assert np.abs(top).max() <= 1e-12 * A0.diagonal().max()
    assert np.abs(bot).max() <= 1e-12 * C.max()


def test_grounded_matrices_spd(sys8, direct8):
    A = sys8["A"]
    sla.cholesky(A.toarray(), lower=True)           # raises if not SPD
    M = np.diag(sys8["C"]) - sys8["B"].T @ direct8
    M = 0.5 * (M + M.T)
    assert np.linalg.eigvalsh(M).min() > 0


def test_ground_node_rule(head8, sys8):
    g = sys8["ground"]
    bf = fem.boundary_faces(head8.tets, head8.n)
    bnodes = np.unique(bf)
    enodes = np.unique(head8.tris)
    assert g in bnodes and g not in enodes
    assert np.all(np.isin(bnodes[bnodes < g], enodes))
    A = sys8["A"]
    row = A.getrow(g)
    assert row.nnz == 15 or row.nnz > 1
    assert row[0, g] == 1.0 and abs(row).sum() == 1.0
    col = A.getcol(g)
    assert abs(col).sum() == 1.0


def test_boundary_faces_match_structural_generator(head8):
    bf = fem.boundary_faces(head8.tets, head8.n)
    bf = bf[np.lexsort((bf[:, 2], bf[:, 1], bf[:, 0]))]
    np.testing.assert_array_equal(bf, head8.boundary_tris)


def test_ldp_is_abs_row_sum(sys8):
    A = sys8["A"]
    d = fem.preconditioner_diag(A, "ldp")
    dense = np.abs(A.toarray()).sum(1)
    np.testing.assert_allclose(d, dense, rtol=1e-14)
