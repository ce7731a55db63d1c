"""Parity at the largest single-GPU size: the 1 mm four-layer sphere
(3.34 M nodes, 19.6 M tets), 256 electrodes, 100 000 dipoles x 3 orientations
(300 000 lead-field columns), in the launch configuration bench.py times.

The oracle cannot assemble and solve this size inside a test, so the expected
values come from tests/golden/fullsize_sphere1mm_L256.json (written by
make_fullsize.py, oracle only): SHA-256 of the oracle's CSR structure, the
ground node, 2000 sampled CSR values, oracle PCG iteration counts of two
electrode columns and six lead-field columns by reciprocity (App. A.1-A.2,
Eq. (aku), solved at 1e-12).

The transfer matrix T = A^-1 B (App. A.4) is checked against the oracle's
own matrix on sampled rows: the oracle assembles the rows of every node that
carries an electrode term, the ground node and 20 000 random nodes from the
tets and electrode triangles that touch them (a row of A depends on nothing
else), and b - A t restricted to those rows, whose norm can only be smaller
than the whole residual's, must meet the solve's bound for every column.
"""
import hashlib
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem, leadfield as lf
from paper_1811_07717_amd import headmodel as hm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NAME = "sphere1mm_L256"
GOLD = os.path.join(os.path.dirname(__file__), "golden", f"fullsize_{NAME}.json")


def say(*a):
    print(*a, flush=True)


def sha(t):
    return hashlib.sha256(np.ascontiguousarray(t.cpu().numpy()).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def full():
    from paper_1811_07717_amd import zi
    with open(GOLD) as f:
        gold = json.load(f)
    H = hm.workload(NAME)
    say(f"[case] {NAME}: n={H.n} e={H.e} L={H.L} m={H.m}")
    assert (H.n, H.e, H.L, 3 * H.m) == (gold["n"], gold["e"], gold["L"], 300000)
    say("[gpu] zi_assemble 1 mm")
    g = zi.System.from_head(H)
    say("[gpu] zi_transfer_solve 1 mm, 256 columns, tol 1e-8, automatic tile")
    T, st = g.transfer_solve(tol=1e-8)
    say(f"[1mm] iterations {st['iters'].min()}..{st['iters'].max()}, {st['seconds']:.2f} s")
    say("[gpu] zi_point_dipoles + zi_leadfield 1 mm, 300 000 columns")
    G = g.point_dipoles(torch.from_numpy(H.dipole_tets).cuda())
    LF = g.leadfield(T, G)
    yield dict(H=H, g=g, T=T, st=st, G=G, LF=LF, gold=gold)
    g.close()


@pytest.fixture(scope="module")
def oracle_rows(full):
    """Oracle rows of A (ground fix included) and of B for a row sample."""
    H, gold = full["H"], full["gold"]
    (er, ec, ev), B, C, calA = fem.electrode_terms(H.nodes, H.tris, H.tri_electrode, H.Z, H.n)
    rng = np.random.default_rng(1814)
    rows = np.unique(np.concatenate([np.unique(H.tris), [gold["ground"]],
                                     rng.choice(H.n, size=20000, replace=False)]))
    touch = np.zeros(H.n, dtype=bool)
    touch[rows] = True
    keep = touch[H.tets].any(axis=1)
    kr, kc, kv = fem.stiffness_triplets(H.nodes, H.tets[keep], H.sigma[keep])
    A = fem.to_csr(np.concatenate([kr, er]), np.concatenate([kc, ec]),
                   np.concatenate([kv, ev]), H.n)
    A = fem.apply_ground(A, gold["ground"])
    say(f"[oracle] {rows.size} sampled rows from {int(keep.sum())} tets")
    return rows, A[rows], sp.csr_matrix(B)[rows]


def test_structure_and_values(full):
    g, gold = full["g"], full["gold"]
    v = g.view()
    assert g.nnz == gold["nnz"]
    assert g.ground == gold["ground"]
    assert sha(v["row_ptr"]) == gold["row_ptr_sha256"]
    assert sha(v["col"]) == gold["col_sha256"]
    val = v["val"].cpu().numpy()[gold["sample_pos"]]
    ref = np.array(gold["sample_val"])
    assert np.abs(val - ref).max() <= 1e-13 * np.abs(ref).max()


def test_iteration_counts(full):
    its = full["st"]["iters"]
    for c, k in full["gold"]["pcg_iters"].items():
        assert abs(int(its[int(c)]) - k) <= max(3, 0.02 * k), (c, its[int(c)], k)


def _sampled_residual(T, rows_A, rows_B):
    cols = np.unique(rows_A.indices)
    Tc = T[torch.from_numpy(cols).to(T.device)].cpu().numpy()
    Ac = rows_A[:, cols]
    Bd = rows_B.toarray()
    return np.linalg.norm(Bd - Ac @ Tc, axis=0) / np.linalg.norm(Bd, axis=0)


def test_true_residual_on_oracle_rows(full, oracle_rows):
    _, Ar, Br = oracle_rows
    res = _sampled_residual(full["T"], Ar, Br)
    say(f"[1mm] residual on the oracle's sampled rows: max {res.max():.3e}")
    assert res.max() <= 1.5e-8
    assert full["st"]["relres_true"].max() <= 1.5e-8


def test_sampled_leadfield_columns(full):
    gold = full["gold"]
    got = full["LF"][:, gold["lf_columns"]].cpu().numpy()
    ref = np.array(gold["lf_values"]).T
    r = lf.rdm(got, ref)
    m = np.abs(lf.mag(got, ref) - 1)
    say(f"[1mm] sampled LF columns: RDM max {r.max():.3e}, |MAG-1| max {m.max():.3e}")
    assert r.max() <= 1e-4 and m.max() <= 1e-4


def test_mixed_precision_full_size(full, oracle_rows):
    # FP32 directions and products, FP64 recurrences and refinement, on the
    # same workload: the same checks against the oracle.
    g, gold = full["g"], full["gold"]
    _, Ar, Br = oracle_rows
    say("[gpu] mixed-precision solve 1 mm")
    T, st = g.transfer_solve(tol=1e-8, precision="fp32_spmm_ir")
    say(f"[1mm] mixed: iterations {st['iters'].min()}..{st['iters'].max()}, "
        f"refinements {st['refinements']}, {st['seconds']:.2f} s")
    res = _sampled_residual(T, Ar, Br)
    say(f"[1mm] mixed: residual on the oracle's sampled rows: max {res.max():.3e}")
    assert res.max() <= 1.5e-8
    LF = g.leadfield(T, full["G"])
    got = LF[:, gold["lf_columns"]].cpu().numpy()
    ref = np.array(gold["lf_values"]).T
    r = lf.rdm(got, ref)
    m = np.abs(lf.mag(got, ref) - 1)
    say(f"[1mm] mixed: sampled LF columns RDM max {r.max():.3e}, |MAG-1| max {m.max():.3e}")
    assert r.max() <= 1e-4 and m.max() <= 1e-4
