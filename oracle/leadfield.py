"""Oracle: the EEG lead field (App. A.2, Eq. (aku)).

Test infrastructure only (see the package docstring).

    L = R (B^T A^-1 B - C)^-1 B^T A^-1 G

with R the average-reference matrix of App. A.1 (r_jj = 1 - 1/L,
r_ij = -1/L).  With T = A^-1 B (App. A.4) and A symmetric, B^T A^-1 = T^T.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def average_reference(L):
    """R of App. A.1: y = R v is the zero-mean electrode voltage vector."""
    return np.eye(L) - np.full((L, L), 1.0 / L)


def schur(T, B, C):
    """S = B^T A^-1 B - C = B^T T - C (L x L)."""
    Bd = B.toarray() if sp.issparse(B) else np.asarray(B)
    return Bd.T @ T - np.diag(C)


def leadfield(T, B, C, G):
    """Eq. (aku) with B^T A^-1 G = T^T G:  R S^-1 (T^T G), L x 3m."""
    L = T.shape[1]
    S = schur(T, B, C)
    TG = np.asarray((sp.csr_matrix(G).T @ T).T) if sp.issparse(G) else T.T @ G
    return average_reference(L) @ np.linalg.solve(S, TG)


def block_system_solve(A, B, C, rhs_top, I=None):
    """Solve Eq. (u_system) directly for one right-hand side: returns (z, v).

    The full (n+L) x (n+L) sparse matrix [A -B; -B^T C] is factorised with a
    sparse LU.  Used for the reciprocity check (T^T G against a direct
    solve driven by the source itself).
    """
    import scipy.sparse.linalg as spla
    n, L = B.shape
    Bs = sp.csr_matrix(B)
    K = sp.bmat([[A, -Bs], [-Bs.T, sp.diags(C)]], format="csc")
    rhs = np.concatenate([np.asarray(rhs_top, dtype=np.float64).ravel(),
                          np.zeros(L) if I is None else np.asarray(I, float)])
    sol = spla.splu(K).solve(rhs)
    return sol[:n], sol[n:]


def leadfield_column_direct(A, B, C, g):
    """One EEG lead-field column by solving Eq. (u_system) with x = e_j:
    the top right-hand side is -G x = -g, the currents I are zero, and the
    electrode voltages are y = R v."""
    _, v = block_system_solve(A, B, C, -np.asarray(g).ravel())
    return average_reference(B.shape[1]) @ v


def rdm(a, b):
    """Relative difference measure ||a/||a|| - b/||b|| ||_2 per column."""
    a = np.asarray(a)
    b = np.asarray(b)
    na = np.linalg.norm(a, axis=0)
    nb = np.linalg.norm(b, axis=0)
    return np.linalg.norm(a / na - b / nb, axis=0)


def mag(a, b):
    """Magnitude ratio ||a|| / ||b|| per column."""
    return np.linalg.norm(np.asarray(a), axis=0) / np.linalg.norm(np.asarray(b), axis=0)


def leadfield_columns_reciprocity(A, B, C, Gcols, tol=1e-12, maxit=200000):
    """Selected EEG lead-field columns, one sparse solve each (App. A.1-A.2).

    With I = 0 the second block row of Eq. (u_system) gives v = C^-1 B^T z;
    substituting into the first, (A - B C^-1 B^T) z = -G x.  That matrix is
    symmetric positive definite once A carries the ground fix, so each column
    is one preconditioned CG solve (``solve.pcg_columns``, Jacobi diagonal)
    followed by y = R v.  Gcols is n x k (the chosen columns of G).
    """
    from .solve import pcg_columns
    Bs = sp.csr_matrix(B)
    K = (sp.csr_matrix(A) - Bs @ sp.diags(1.0 / np.asarray(C)) @ Bs.T).tocsr()
    rhs = -(Gcols.toarray() if sp.issparse(Gcols) else np.asarray(Gcols))
    Zc, _, _ = pcg_columns(K, rhs, K.diagonal().copy(), tol=tol, maxit=maxit)
    V = (Bs.T @ Zc) / np.asarray(C)[:, None]
    return average_reference(B.shape[1]) @ V
