"""Parity at the benchmark's full size (2 mm sphere, 128 electrodes, 30 000
lead-field columns) in the launch configuration bench.py times.

The oracle cannot solve all 128 columns in seconds, so the expected values
come from tests/golden/fullsize_sphere2mm_L128.json (written by
make_fullsize.py, oracle only): structure hashes, sampled CSR values, oracle
PCG iteration counts of two columns and six lead-field columns by
reciprocity.  The transfer matrix is checked by its true residual against the
oracle's assembled A (a property that holds at any size).
"""
import hashlib
import json
import os

import numpy as np
import pytest

from oracle import fem, leadfield as lf
from paper_1811_07717_amd import headmodel as hm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NAME = "sphere2mm_L128"
GOLD = os.path.join(os.path.dirname(__file__), "golden", f"fullsize_{NAME}.json")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def full():
    from paper_1811_07717_amd import zi
    with open(GOLD) as f:
        gold = json.load(f)
    H = hm.workload(NAME)
    say(f"[case] {NAME}: n={H.n} e={H.e} L={H.L} m={H.m}")
    say("[gpu] zi_assemble 2 mm")
    g = zi.System.from_head(H)
    say("[gpu] zi_transfer_solve 2 mm, tol 1e-8, automatic tile")
    T, st = g.transfer_solve(tol=1e-8)
    say(f"[2mm] iterations {st['iters'].min()}..{st['iters'].max()}, {st['seconds']:.2f} s")
    say("[gpu] zi_point_dipoles + zi_leadfield 2 mm")
    G = g.point_dipoles(torch.from_numpy(H.dipole_tets).cuda())
    LF = g.leadfield(T, G)
    yield dict(H=H, g=g, T=T, st=st, LF=LF, gold=gold)
    g.close()


def sha(t):
    return hashlib.sha256(np.ascontiguousarray(t.cpu().numpy()).tobytes()).hexdigest()


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


def test_true_residual_with_oracle_matrix(full):
    H = full["H"]
    S = fem.assemble(H.nodes, H.tets, H.sigma, H.tris, H.tri_electrode, H.Z)
    T = full["T"].cpu().numpy()
    Bd = S["B"].toarray()
    res = np.linalg.norm(Bd - S["A"] @ T, axis=0) / np.linalg.norm(Bd, axis=0)
    say(f"[2mm] true relative residual max {res.max():.3e}")
    assert res.max() <= 1.5e-8
    np.testing.assert_allclose(full["st"]["relres_true"], res, rtol=1e-3, atol=1e-12)


def test_sampled_leadfield_columns(full):
    gold = full["gold"]
    LF = full["LF"].cpu().numpy()
    got = LF[:, gold["lf_columns"]]
    ref = np.array(gold["lf_values"]).T
    r = lf.rdm(got, ref)
    m = np.abs(lf.mag(got, ref) - 1)
    say(f"[2mm] sampled LF columns: RDM max {r.max():.3e}, |MAG-1| max {m.max():.3e}")
    assert r.max() <= 1e-4 and m.max() <= 1e-4


def test_leadfield_properties(full):
    LF = full["LF"]
    assert torch.isfinite(LF).all()
    cs = LF.sum(dim=0).abs().max().item()
    assert cs <= 1e-9 * LF.abs().max().item()


def test_mixed_precision_full_size(full):
    # The same workload with FP32 products and FP64 refinement: true residual
    # against the oracle's A and the sampled lead-field columns, per electrode.
    H, g, gold = full["H"], full["g"], full["gold"]
    say("[gpu] mixed-precision solve 2 mm")
    T, st = g.transfer_solve(tol=1e-8, precision="fp32_spmm_ir")
    say(f"[2mm] mixed: iterations {st['iters'].min()}..{st['iters'].max()}, "
        f"refinements {st['refinements']}, {st['seconds']:.2f} s")
    S = fem.assemble(H.nodes, H.tets, H.sigma, H.tris, H.tri_electrode, H.Z)
    Tn = T.cpu().numpy()
    Bd = S["B"].toarray()
    res = np.linalg.norm(Bd - S["A"] @ Tn, axis=0) / np.linalg.norm(Bd, axis=0)
    assert res.max() <= 1.5e-8
    d64 = np.linalg.norm(Tn - full["T"].cpu().numpy(), axis=0) / np.linalg.norm(Tn, axis=0)
    say(f"[2mm] mixed vs FP64 transfer columns: max relative difference {d64.max():.2e}")
    G = g.point_dipoles(torch.from_numpy(H.dipole_tets).cuda())
    LF = g.leadfield(T, G).cpu().numpy()
    got = LF[:, gold["lf_columns"]]
    ref = np.array(gold["lf_values"]).T
    assert lf.rdm(got, ref).max() <= 1e-4
    assert np.abs(lf.mag(got, ref) - 1).max() <= 1e-4
