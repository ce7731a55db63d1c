"""Oracle: finite-element matrices of the CEM system (App. A.1).

Test infrastructure only (see the package docstring).

Notation follows App. A.1 of the paper: psi_i are the linear nodal basis
functions, sigma the element-wise conductivity (Sec. 2 "Conductivity
distribution"), e_l the electrode patches, Z_l the contact impedances and
calA_l the contact areas.  The system of Eq. (u_system) is

    [  A   -B ] [z]   [-G x]
    [ -B^T  C ] [v] = [  I ]

with

    a_ij  = int sigma grad psi_i . grad psi_j dV
            + sum_l 1/(Z_l calA_l) int_{e_l} psi_i psi_j dS
    b_il  = 1/(Z_l calA_l) int_{e_l} psi_i dS
    c_ll  = 1/(Z_l calA_l) int_{e_l} dS = 1/Z_l

(the 1/(Z_l calA_l) factor of b and c is the reading that makes the block
system reproduce the weak form's 1/(Z calA^2) int u int v term; the printed
1/Z_l alone is dimensionally inconsistent with a_ij).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


# ---------------------------------------------------------------------------
# Element geometry
# ---------------------------------------------------------------------------

def element_gradients(nodes, tets):
    """Gradients of the four linear basis functions and the volume per tet.

    With J the 3x3 matrix whose rows are x_k - x_0 (k = 1, 2, 3), a point is
    x = x_0 + J^T lam, so the barycentric coordinates lam = J^-T (x - x_0)
    have gradients equal to the columns of J^-1; psi_0 = 1 - sum lam.

    Returns grads (e, 4, 3) and vol (e,) = |det J| / 6.
    """
    x = nodes[tets]                                  # (e, 4, 3)
    J = x[:, 1:, :] - x[:, :1, :]                    # (e, 3, 3) rows x_k - x_0
    Jinv = np.linalg.inv(J)
    g123 = np.transpose(Jinv, (0, 2, 1))             # row k-1 = column k-1 of J^-1
    g0 = -g123.sum(axis=1, keepdims=True)
    grads = np.concatenate([g0, g123], axis=1)
    vol = np.abs(np.linalg.det(J)) / 6.0
    return grads, vol


def sigma_tensor(sigma):
    """(e,) scalars or (e, 6) rows (s11, s22, s33, s12, s13, s23) -> (e, 3, 3).

    The row layout is the one given in Sec. 2 "Conductivity distribution".
    """
    sigma = np.asarray(sigma, dtype=np.float64)
    if sigma.ndim == 1:
        return sigma[:, None, None] * np.eye(3)[None]
    s = np.empty((sigma.shape[0], 3, 3))
    s[:, 0, 0], s[:, 1, 1], s[:, 2, 2] = sigma[:, 0], sigma[:, 1], sigma[:, 2]
    s[:, 0, 1] = s[:, 1, 0] = sigma[:, 3]
    s[:, 0, 2] = s[:, 2, 0] = sigma[:, 4]
    s[:, 1, 2] = s[:, 2, 1] = sigma[:, 5]
    return s


def element_stiffness(nodes, tets, sigma):
    """K^e_ij = int_T sigma grad psi_i . grad psi_j dV = vol * g_i^T S g_j.

    (App. A.1, first term of a_ij; gradients are constant on a tet.)
    """
    g, vol = element_gradients(nodes, tets)
    S = sigma_tensor(sigma)
    Sg = np.einsum("eab,ejb->eja", S, g)             # S g_j
    return vol[:, None, None] * np.einsum("eia,eja->eij", g, Sg)


def stiffness_triplets(nodes, tets, sigma):
    """(rows, cols, vals) of every element matrix entry, 16 per tetrahedron."""
    Ke = element_stiffness(nodes, tets, sigma)
    t = tets.astype(np.int64)
    rows = np.repeat(t, 4, axis=1).ravel()
    cols = np.tile(t, (1, 4)).ravel()
    return rows, cols, Ke.ravel()


def to_csr(rows, cols, vals, n):
    """Sum triplets into CSR.  Entries that sum to zero stay stored, so the
    structure is exactly the set of (row, col) pairs given."""
    M = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    M.sort_indices()
    return M


def stiffness(nodes, tets, sigma):
    """Assembled volume term of A as a CSR matrix.

    The sparsity structure is every (i, j) pair that shares a tetrahedron,
    diagonal included; entries that happen to sum to zero are kept as stored
    zeros so that the structure is the mesh graph.
    """
    return to_csr(*stiffness_triplets(nodes, tets, sigma), nodes.shape[0])


# ---------------------------------------------------------------------------
# Boundary
# ---------------------------------------------------------------------------

def boundary_faces(tets, n):
    """Faces that belong to exactly one tetrahedron, each sorted ascending."""
    t = tets.astype(np.int64)
    f = np.concatenate([t[:, [1, 2, 3]], t[:, [0, 2, 3]],
                        t[:, [0, 1, 3]], t[:, [0, 1, 2]]])
    f = np.sort(f, axis=1)
    if n < 2_000_000:
        key = (f[:, 0] * n + f[:, 1]) * n + f[:, 2]
        u, idx, cnt = np.unique(key, return_index=True, return_counts=True)
        return f[idx[cnt == 1]]
    u, cnt = np.unique(f, axis=0, return_counts=True)
    return u[cnt == 1]


def ground_node(tets, tris, n):
    """The index i' of App. A.1's ground fix.

    The paper asks for a node whose basis function peaks on the part of the
    boundary not covered by electrodes.  Reading used here: the smallest
    boundary node index that is not a vertex of any electrode triangle.
    """
    bf = boundary_faces(tets, n)
    bnode = np.zeros(n, dtype=bool)
    bnode[bf.ravel()] = True
    bnode[np.asarray(tris).ravel()] = False
    cand = np.flatnonzero(bnode)
    if cand.size == 0:
        raise ValueError("no boundary node outside the electrodes")
    return int(cand[0])


# ---------------------------------------------------------------------------
# Complete electrode model
# ---------------------------------------------------------------------------

def triangle_areas(nodes, tris):
    x = nodes[np.asarray(tris, dtype=np.int64)]
    c = np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0])
    return 0.5 * np.sqrt((c * c).sum(axis=1))


def electrode_terms(nodes, tris, tri_electrode, Z, n):
    """Surface terms of A, the matrix B and the diagonal of C (App. A.1).

    On a triangle F with P1 basis functions, int_F psi_i psi_j dS =
    (1 + delta_ij) |F| / 12 and int_F psi_i dS = |F| / 3.  Summed over the
    triangles of e_l and scaled by 1/(Z_l calA_l) with calA_l = sum |F|:

        (rows, cols, vals) of A_cem, B (n x L CSR), C (L,), calA (L,)
    """
    tris = np.asarray(tris, dtype=np.int64)
    te = np.asarray(tri_electrode, dtype=np.int64)
    Z = np.asarray(Z, dtype=np.float64)
    L = Z.shape[0]
    area = triangle_areas(nodes, tris)
    calA = np.bincount(te, weights=area, minlength=L)
    w = area / (Z[te] * calA[te])                    # |F| / (Z_l calA_l)
    mass = np.array([[2.0, 1.0, 1.0], [1.0, 2.0, 1.0], [1.0, 1.0, 2.0]]) / 12.0
    rows = np.repeat(tris, 3, axis=1).ravel()
    cols = np.tile(tris, (1, 3)).ravel()
    vals = (w[:, None, None] * mass[None]).ravel()
    brow = tris.ravel()
    bcol = np.repeat(te, 3)
    bval = np.repeat(w / 3.0, 3)
    B = sp.coo_matrix((bval, (brow, bcol)), shape=(n, L)).tocsr()
    C = np.bincount(te, weights=w, minlength=L)      # = 1 / Z_l
    return (rows, cols, vals), B, C, calA


def apply_ground(A, i):
    """Ground fix of App. A.1: a_{i'i'} = 1, a_{i'j} = 0 (j != i').

    The column is zeroed as well so that A stays symmetric for CG; this gives
    the same lead field because row i' of B is zero (i' is on no electrode),
    so the i'-th entry of every transfer column is zero anyway.
    Stored structure is preserved (zeros stay stored).
    """
    A = A.tocsr(copy=True)
    A.sort_indices()
    start, end = A.indptr[i], A.indptr[i + 1]
    A.data[start:end] = 0.0
    hit = A.indices == i
    A.data[hit] = 0.0
    diag = start + np.flatnonzero(A.indices[start:end] == i)[0]
    A.data[diag] = 1.0
    return A


def preconditioner_diag(A, kind="jacobi"):
    """Diagonal D of the PCG preconditioner.

    "jacobi": D_ii = a_ii.  "ldp": the lumped diagonal of Sec. 2.3.1,
    D_ii = sum_j |a_ij|.
    """
    if kind == "jacobi":
        return A.diagonal().copy()
    if kind == "ldp":
        return np.asarray(abs(A).sum(axis=1)).ravel()
    raise ValueError(kind)


def assemble(nodes, tets, sigma, tris, tri_electrode, Z, ground=None):
    """The grounded system of Eq. (u_system): dict with A, B, C, ground, ...

    ``ground`` None selects the node of ``ground_node``.
    """
    n = nodes.shape[0]
    kr, kc, kv = stiffness_triplets(nodes, tets, sigma)
    (er, ec, ev), B, C, calA = electrode_terms(nodes, tris, tri_electrode, Z, n)
    K = to_csr(kr, kc, kv, n)
    A0 = to_csr(np.concatenate([kr, er]), np.concatenate([kc, ec]),
                np.concatenate([kv, ev]), n)
    # The surface terms add no structure because every electrode triangle is
    # a face of a tetrahedron; check it rather than assume it.
    if A0.nnz != K.nnz:
        raise ValueError("electrode triangle is not a mesh face")
    g = ground_node(tets, tris, n) if ground is None else int(ground)
    A = apply_ground(A0, g)
    return dict(A=A, A0=A0, K=K, B=B, C=C, calA=calA, ground=g)
