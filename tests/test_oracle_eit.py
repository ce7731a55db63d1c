"""Pins of the oracle's linearized EIT lead field (App. A.3) and of the
anisotropic conductivity path (Sec. 2 "Conductivity distribution")."""
import numpy as np

from oracle import eit, fem, solve
from paper_1811_07717_amd import headmodel as hm


def _system(H, sigma):
    S = fem.assemble(H.nodes, H.tets, sigma, H.tris, H.tri_electrode, H.Z)
    return S, solve.transfer_direct(S["A"], S["B"])


def test_eit_leadfield_matches_finite_differences():
    # Central differences of the forward model y = R M^-1 I in s_m against
    # the closed-form derivative, for a few elements and two current patterns.
    H = hm.make_head(8.0, L=12, m=1, seed=4)
    S, T = _system(H, H.sigma)
    I = np.zeros((12, 2))
    I[0, 0], I[6, 0] = 1e-3, -1e-3
    I[3, 1], I[9, 1] = 1e-3, -1e-3
    elems = np.array([10, 5000, 20000, 37000])
    J = eit.leadfield(T, S["B"], S["C"], I, H.nodes, H.tets, elems)
    for j, m in enumerate(elems):
        h = 1e-4 * H.sigma[m]
        ys = []
        for sgn in (1, -1):
            s2 = H.sigma.copy()
            s2[m] += sgn * h
            S2, T2 = _system(H, s2)
            ys.append(eit.forward(T2, S2["B"], S2["C"], I))
        fd = (ys[0] - ys[1]) / (2 * h)            # L x P
        # central differences with h = 1e-4 s_m: truncation ~1e-8 relative,
        # cancellation ~eps |y| / h; entries near zero carry that noise
        np.testing.assert_allclose(J[:, :, j].T, fd, rtol=1e-5,
                                   atol=1e-4 * np.abs(fd).max())


def test_eit_forward_sums_to_zero():
    H = hm.make_head(8.0, L=10, m=1, seed=4)
    S, T = _system(H, H.sigma)
    I = np.zeros((10, 1))
    I[1, 0], I[7, 0] = 1.0, -1.0
    y = eit.forward(T, S["B"], S["C"], I)
    assert abs(y.sum()) <= 1e-10 * np.abs(y).max()


def _rotation(a, b, c):
    Rz = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
    Ry = np.array([[np.cos(b), 0, np.sin(b)], [0, 1, 0], [-np.sin(b), 0, np.cos(b)]])
    Rx = np.array([[1, 0, 0], [0, np.cos(c), -np.sin(c)], [0, np.sin(c), np.cos(c)]])
    return Rz @ Ry @ Rx


def _tensor_rows(S3):
    return np.stack([S3[:, 0, 0], S3[:, 1, 1], S3[:, 2, 2], S3[:, 0, 1], S3[:, 0, 2],
                     S3[:, 1, 2]], axis=1)


def test_anisotropic_element_matrix_is_rotation_invariant():
    # Rotating the geometry by Q and the tensor to Q S Q^T leaves every
    # element stiffness matrix unchanged.
    rng = np.random.default_rng(5)
    H = hm.make_head(8.0, L=4, m=1, seed=3)
    tets = H.tets[:300]
    A = rng.normal(size=(300, 3, 3))
    S3 = np.einsum("eij,ekj->eik", A, A) + 0.1 * np.eye(3)     # SPD tensors
    Q = _rotation(0.3, -1.1, 0.7)
    K = fem.element_stiffness(H.nodes, tets, _tensor_rows(S3))
    Kr = fem.element_stiffness(H.nodes @ Q.T, tets, _tensor_rows(Q @ S3 @ Q.T))
    np.testing.assert_allclose(Kr, K, rtol=1e-10, atol=1e-12 * np.abs(K).max())


def test_anisotropic_axis_scaling_matches_stretched_mesh():
    # A diagonal tensor diag(a, b, c) on a mesh equals the isotropic unit
    # conductivity on the mesh stretched by (1/sqrt(a), 1/sqrt(b), 1/sqrt(c)),
    # up to the volume factor sqrt(abc).
    H = hm.make_head(8.0, L=4, m=1, seed=3)
    tets = H.tets[:500]
    a, b, c = 2.0, 0.5, 3.0
    s6 = np.tile([a, b, c, 0.0, 0.0, 0.0], (500, 1))
    K = fem.element_stiffness(H.nodes, tets, s6)
    st = H.nodes / np.sqrt([a, b, c])
    Ks = fem.element_stiffness(st, tets, np.ones(500)) * np.sqrt(a * b * c)
    np.testing.assert_allclose(K, Ks, rtol=1e-10, atol=1e-12 * np.abs(K).max())
