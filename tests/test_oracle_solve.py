"""Pins of the oracle's solves and lead field (App. A.2-A.4, Sec. 2.3.1)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fem, leadfield as lf, solve, source
from paper_1811_07717_amd import headmodel as hm


def test_pcg_iterations_match_scipy_cg(sys8):
    # Same preconditioner, same relative tolerance, x0 = 0: scipy's cg stops on
    # ||r|| <= rtol ||b|| as well, so the counts agree to within one.
    A, B = sys8["A"], sys8["B"].toarray()
    d = fem.preconditioner_diag(A)
    Minv = sp.diags(1.0 / d)
    for c in (0, 9, 31):
        x, its, rel = solve.pcg(A, B[:, c], d, tol=1e-8)
        count = [0]

        def cb(_):
            count[0] += 1
        xs, info = spla.cg(A, B[:, c], rtol=1e-8, atol=0.0, M=Minv, maxiter=10000, callback=cb)
        assert info == 0
        assert abs(its - count[0]) <= 1
        assert rel <= 1e-8
        np.testing.assert_allclose(x, xs, rtol=0, atol=1e-6 * np.abs(xs).max())


def test_pcg_matches_direct_solve(sys8, direct8):
    A, B = sys8["A"], sys8["B"]
    d = fem.preconditioner_diag(A)
    T, its, _ = solve.transfer_pcg(A, B, d, tol=1e-12, columns=[3, 17])
    ref = direct8[:, [3, 17]]
    assert np.abs(T - ref).max() <= 1e-9 * np.abs(ref).max()


def test_pcg_columns_equals_single_column_pcg(sys8):
    A, B = sys8["A"], sys8["B"]
    for kind in ("jacobi", "ldp"):
        d = fem.preconditioner_diag(A, kind)
        X, its, rel = solve.pcg_columns(A, B, d, tol=1e-8)
        T, its1, rel1 = solve.transfer_pcg(A, B, d, tol=1e-8, columns=[0, 5, 30])
        np.testing.assert_array_equal(its[[0, 5, 30]], its1)
        np.testing.assert_allclose(X[:, [0, 5, 30]], T, rtol=0, atol=1e-12 * np.abs(T).max())


def test_pcg_detects_indefinite():
    A = sp.csr_matrix(np.diag([1.0, -2.0, 3.0]))
    with pytest.raises(solve.NotConverged):
        solve.pcg(A, np.ones(3), np.ones(3))


def test_leadfield_column_sums_vanish(head8, sys8, direct8):
    G = source.point_dipole_matrix(head8.nodes, head8.tets, head8.dipole_tets)
    LF = lf.leadfield(direct8, sys8["B"], sys8["C"], G)
    assert LF.shape == (head8.L, 3 * head8.m)
    assert np.abs(LF.sum(axis=0)).max() <= 1e-10 * np.abs(LF).max()


def test_reciprocity_direct_block_solve(head8, sys8, direct8):
    # Eq. (aku) against a direct solve of Eq. (u_system) driven by the source.
    G = source.point_dipole_matrix(head8.nodes, head8.tets, head8.dipole_tets)
    LF = lf.leadfield(direct8, sys8["B"], sys8["C"], G)
    for c in (0, 1, 2, 1500, 2999):
        col = lf.leadfield_column_direct(sys8["A"], sys8["B"], sys8["C"],
                                         G[:, c].toarray().ravel())
        assert np.abs(col - LF[:, c]).max() <= 1e-10 * np.abs(LF[:, c]).max()


def test_ground_independence(head8, sys8, direct8):
    # Two admissible ground nodes give the same lead field (the fix only
    # removes the constant null vector of the CEM system).
    H = head8
    G = source.point_dipole_matrix(H.nodes, H.tets, H.dipole_tets[:40])
    LF1 = lf.leadfield(direct8, sys8["B"], sys8["C"], G)
    bf = np.unique(fem.boundary_faces(H.tets, H.n))
    other = int(np.setdiff1d(bf, np.unique(H.tris))[-1])
    assert other != sys8["ground"]
    S2 = fem.assemble(H.nodes, H.tets, H.sigma, H.tris, H.tri_electrode, H.Z, ground=other)
    T2 = solve.transfer_direct(S2["A"], S2["B"])
    LF2 = lf.leadfield(T2, S2["B"], S2["C"], G)
    assert np.abs(LF1 - LF2).max() <= 1e-10 * np.abs(LF1).max()
    # T itself depends on the ground node
    assert np.abs(T2 - direct8).max() > 1e-6 * np.abs(direct8).max()


def test_ungrounded_schur_is_singular(head8, sys8):
    # Without the fix, A0 1 = B 1 gives T 1 = 1 and S 1 = B^T 1 - C 1 = 0, so
    # the fix is required.  Check B^T 1 = C (the consequence used).
    one = np.ones(head8.n)
    np.testing.assert_allclose(sys8["B"].T @ one, sys8["C"], rtol=1e-12)


def _tiny_mesh():
    """A 2x2x2 block of Kuhn cubes (48 tets), two electrodes on the top."""
    h = 0.01
    g = np.arange(3)
    Zc, Yc, Xc = np.meshgrid(g, g, g, indexing="ij")
    nodes = np.stack([Xc.ravel(), Yc.ravel(), Zc.ravel()], 1).astype(float) * h
    idx = lambda x, y, z: (z * 3 + y) * 3 + x
    tets = []
    for cz in range(2):
        for cy in range(2):
            for cx in range(2):
                for p in hm.PERMS:
                    v = np.array([cx, cy, cz])
                    path = [v.copy()]
                    for ax in p:
                        v = v.copy()
                        v[ax] += 1
                        path.append(v)
                    tets.append([idx(*q) for q in path])
    tets = np.array(tets, dtype=np.int32)
    bf = fem.boundary_faces(tets, nodes.shape[0])
    top = bf[np.all(nodes[bf][:, :, 2] == 2 * h, axis=1)]
    cx = nodes[top].mean(1)[:, 0]
    tris = top.astype(np.int32)
    te = (cx > h).astype(np.int32)
    sigma = np.linspace(0.2, 0.9, tets.shape[0])
    return nodes, tets, sigma, tris, te


def test_brute_force_tiny_mesh():
    # Dense assembly by explicit loops with barycentric-solve gradients, the
    # full (n+L) block system of Eq. (u_system) solved with LAPACK, versus the
    # oracle's sparse pipeline.
    nodes, tets, sigma, tris, te = _tiny_mesh()
    n, L = nodes.shape[0], 2
    Z = np.array([1000.0, 2500.0])
    A = np.zeros((n, n))
    for e, t in enumerate(tets):
        M = np.hstack([np.ones((4, 1)), nodes[t]])
        grad = np.linalg.inv(M)[1:, :]             # column i = grad psi_i
        vol = abs(np.linalg.det(M)) / 6
        for a in range(4):
            for b in range(4):
                A[t[a], t[b]] += sigma[e] * vol * grad[:, a] @ grad[:, b]
    area = np.array([0.5 * np.linalg.norm(np.cross(nodes[t[1]] - nodes[t[0]],
                                                   nodes[t[2]] - nodes[t[0]])) for t in tris])
    calA = np.array([area[te == l].sum() for l in range(L)])
    B = np.zeros((n, L))
    C = np.zeros(L)
    for k, t in enumerate(tris):
        l = te[k]
        s = 1.0 / (Z[l] * calA[l])
        for a in range(3):
            B[t[a], l] += s * area[k] / 3
            for b in range(3):
                A[t[a], t[b]] += s * area[k] * (2 if a == b else 1) / 12
        C[l] += s * area[k]
    bf = fem.boundary_faces(tets, n)
    gnd = int(np.setdiff1d(np.unique(bf), np.unique(tris))[0])
    A[gnd, :] = 0
    A[:, gnd] = 0
    A[gnd, gnd] = 1
    dip = np.array([5, 20, 33])
    G = np.zeros((n, 9))
    for j, e in enumerate(dip):
        t = tets[e]
        grad = np.linalg.inv(np.hstack([np.ones((4, 1)), nodes[t]]))[1:, :]
        for k in range(3):
            G[t, 3 * j + k] = -grad[k, :]
    K = np.block([[A, -B], [-B.T, np.diag(C)]])
    sol = np.linalg.solve(K, np.vstack([-G, np.zeros((L, 9))]))
    LF_ref = lf.average_reference(L) @ sol[n:]

    S = fem.assemble(nodes, tets, sigma, tris, te, Z)
    assert S["ground"] == gnd
    np.testing.assert_allclose(S["A"].toarray(), A, rtol=1e-12, atol=1e-14 * np.abs(A).max())
    T = solve.transfer_direct(S["A"], S["B"])
    Gs = source.point_dipole_matrix(nodes, tets, dip)
    np.testing.assert_allclose(Gs.toarray(), G, rtol=1e-12, atol=1e-12 * np.abs(G).max())
    LF = lf.leadfield(T, S["B"], S["C"], Gs)
    np.testing.assert_allclose(LF, LF_ref, rtol=1e-9, atol=1e-12 * np.abs(LF_ref).max())


def test_single_electrode_leadfield_is_zero():
    # L = 1: the average reference R is the zero matrix, so the lead field is 0.
    H = hm.make_head(8.0, L=1, m=3, seed=2)
    S = fem.assemble(H.nodes, H.tets, H.sigma, H.tris, H.tri_electrode, H.Z)
    T = solve.transfer_direct(S["A"], S["B"])
    G = source.point_dipole_matrix(H.nodes, H.tets, H.dipole_tets)
    assert np.all(lf.leadfield(T, S["B"], S["C"], G) == 0.0)


def test_rdm_mag_definitions():
    a = np.array([[1.0, 0.0], [0.0, 2.0]])
    b = np.array([[2.0, 0.0], [0.0, 2.0]])
    np.testing.assert_allclose(lf.rdm(a, b), [0.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(lf.mag(a, b), [0.5, 1.0])
    c = np.array([[0.0], [1.0]])
    d = np.array([[1.0], [0.0]])
    assert lf.rdm(c, d)[0] == pytest.approx(np.sqrt(2.0))


def test_reciprocity_columns_match_eq_aku(head8, sys8, direct8):
    # Column-by-column lead field from the Schur system equals Eq. (aku).
    G = source.point_dipole_matrix(head8.nodes, head8.tets, head8.dipole_tets)
    LF = lf.leadfield(direct8, sys8["B"], sys8["C"], G)
    cols = [0, 4, 2999]
    got = lf.leadfield_columns_reciprocity(sys8["A"], sys8["B"], sys8["C"], G[:, cols])
    assert np.abs(got - LF[:, cols]).max() <= 1e-9 * np.abs(LF[:, cols]).max()
