"""hipGraph replay, batched multi-head solves and the SpMM autotuner.

Graph replays and batches run exactly the kernels of the eager solve, so
their transfer matrices and iteration counts must be bit-identical to it;
the eager solve itself is pinned to the oracle in test_gpu_parity.py.  Each
graph here is replayed many times with host synchronisation between replays.
"""
import numpy as np
import pytest

from oracle import fem, solve
from paper_1811_07717_amd import headmodel as hm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def test_graph_replay_matches_eager():
    from paper_1811_07717_amd import zi
    H = hm.workload("sphere8mm_L37")
    g = zi.System.from_head(H)
    say("[gpu] eager vs graph solve, 8 mm L37")
    T1, s1 = g.transfer_solve(tol=1e-8)
    T2, s2 = g.transfer_solve(tol=1e-8, graph=True, check_every=16)
    assert torch.equal(T1, T2)
    np.testing.assert_array_equal(s1["iters"], s2["iters"])
    T5, s5 = g.transfer_solve(tol=1e-8, form="classic")
    T6, s6 = g.transfer_solve(tol=1e-8, graph=True, check_every=16, form="classic")
    assert torch.equal(T5, T6)
    np.testing.assert_array_equal(s5["iters"], s6["iters"])
    T3, s3 = g.transfer_solve(tol=1e-8, graph=True, precision="fp32_spmm_ir")
    T4, s4 = g.transfer_solve(tol=1e-8, precision="fp32_spmm_ir")
    assert torch.equal(T3, T4)
    assert s3["refinements"] == s4["refinements"]
    g.close()


def test_batch_matches_individual_solves_and_oracle():
    from paper_1811_07717_amd import zi
    heads = [hm.make_head(8.0, L=8, m=1, seed=1), hm.make_head(6.0, L=21, m=1, seed=2),
             hm.make_head(8.0, L=40, m=1, seed=3, scale=0.93),
             hm.make_head(7.0, L=16, m=1, seed=4, sigmas=(0.2, 1.0, 0.01, 0.5))]
    systems = [zi.System.from_head(H) for H in heads]
    say("[gpu] batch of 4 uneven heads")
    Ts, stats, rc = zi.transfer_solve_batch(systems, tol=1e-8, check_every=8)
    assert rc == zi.ZI_OK
    for H, g, T, st in zip(heads, systems, Ts, stats):
        T1, s1 = g.transfer_solve(tol=1e-8)
        assert torch.equal(T, T1)
        np.testing.assert_array_equal(st["iters"], s1["iters"])
        S = fem.assemble(H.nodes, H.tets, H.sigma, H.tris, H.tri_electrode, H.Z)
        Tn = T.cpu().numpy()
        Bd = S["B"].toarray()
        res = np.linalg.norm(Bd - S["A"] @ Tn, axis=0) / np.linalg.norm(Bd, axis=0)
        assert res.max() <= 1.5e-8
        ref = solve.transfer_direct(S["A"], S["B"])
        err = np.linalg.norm(Tn - ref, axis=0) / np.linalg.norm(ref, axis=0)
        assert err.max() <= 1e-5
    for g in systems:
        g.close()


def test_batch_mixed_precision():
    from paper_1811_07717_amd import zi
    heads = [hm.make_head(8.0, L=12, m=1, seed=5), hm.make_head(7.0, L=9, m=1, seed=6)]
    systems = [zi.System.from_head(H) for H in heads]
    Ts, stats, rc = zi.transfer_solve_batch(systems, tol=1e-8, precision="fp32_spmm_ir")
    assert rc == zi.ZI_OK
    for H, g, T, st in zip(heads, systems, Ts, stats):
        T1, s1 = g.transfer_solve(tol=1e-8, precision="fp32_spmm_ir")
        assert torch.equal(T, T1)
        assert st["refinements"] == s1["refinements"]
    for g in systems:
        g.close()


def test_autotuner_picks_a_tile_and_results_do_not_change():
    from paper_1811_07717_amd import zi
    H = hm.workload("sphere8mm_L32")
    g = zi.System.from_head(H)
    T0, s0 = g.transfer_solve(tol=1e-8, tile=0)
    best, ms = g.autotune()
    say(f"[autotune] best tile {best} ({zi.tile_names()[best]}), ms {np.round(ms, 4).tolist()}")
    assert 0 <= best < len(ms) and ms[best] == ms.min() and np.all(ms > 0)
    T1, s1 = g.transfer_solve(tol=1e-8)
    assert s1["tile"] == best
    # the timing-driven pick cannot change a bit of the result
    assert torch.equal(T0, T1)
    assert np.array_equal(s0["iters"], s1["iters"])
    g.close()


@pytest.mark.parametrize("form,precision", [("single", "fp64"), ("classic", "fp64"),
                                            ("auto", "fp32_spmm_ir")])
def test_every_tile_gives_the_same_bits(form, precision):
    # Products are summed row by row in column order whatever the tile, the
    # streaming kernels run with one geometry, and the SpMM's dot product is
    # summed on fixed grids: T and the iteration counts are bitwise the same
    # for all tiles (ragged 37 columns: padding and partial chunks included).
    from paper_1811_07717_amd import zi
    H = hm.workload("sphere8mm_L37")
    g = zi.System.from_head(H)
    say(f"[case] every tile, {form} {precision}, L={H.L}")
    T0, s0 = g.transfer_solve(tol=1e-8, tile=0, form=form, precision=precision)
    for t, name in enumerate(zi.tile_names()):
        if t == 0:
            continue
        T, st = g.transfer_solve(tol=1e-8, tile=t, form=form, precision=precision)
        assert np.array_equal(st["iters"], s0["iters"]), (t, zi.tile_names()[t])
        assert torch.equal(T, T0), (t, zi.tile_names()[t], (T - T0).abs().max().item())
    g.close()
