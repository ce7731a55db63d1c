"""The LDS ring SpMM tile of the solver (App. A.4, Sec. 2.3.1): T and the
iteration counts must be bitwise those of a front tile, in the
single-reduction and classic FP64 forms and in mixed precision (float32
vectors, 32 columns per chunk), since every tile forms the products in CSR
order and sums the dot products on fixed grids.  Cases: the 2 mm sphere (the
window covers almost every reference), tensor conductivity (many rows of
more than eight entries, the ring kernel's path that reads memory in the row
loop), a mesh stretched along z (pencil layers longer than the window: most
references come from the halo lists or, where a list is full, from memory),
a ragged column count, batched heads, and zi_spmm, which the tile does not
serve."""
import numpy as np
import pytest

from paper_1811_07717_amd import headmodel as hm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RING = "ring_g64_cw16"
FRONT = "lpr32_nv2_cw128_front"


def say(*a):
    print(*a, flush=True)


def _tiles():
    from paper_1811_07717_amd import zi
    names = zi.tile_names()
    return names.index(RING), names.index(FRONT)


def _same_as_front(g, what, **kw):
    ring, front = _tiles()
    kw.setdefault("form", "single")
    T0, s0 = g.transfer_solve(tol=1e-8, tile=front, **kw)
    T1, s1 = g.transfer_solve(tol=1e-8, tile=ring, **kw)
    say(f"[ring] {what}: iterations {s1['iters'].min()}..{s1['iters'].max()}, "
        f"true residual max {s1['relres_true'].max():.2e}")
    assert s1["tile"] == ring and s0["tile"] == front
    assert np.array_equal(s0["iters"], s1["iters"])
    assert torch.equal(T0, T1), (T0 - T1).abs().max().item()
    assert s1["relres_true"].max() <= 1.5e-8
    return T1


def test_ring_2mm_matches_front():
    from paper_1811_07717_amd import zi
    H = hm.workload("sphere2mm_L128")
    say(f"[case] ring tile, 2 mm sphere: n={H.n} L={H.L}")
    g = zi.System.from_head(H)
    _same_as_front(g, "2 mm, single-reduction")
    _same_as_front(g, "2 mm, mixed precision", form="auto", precision="fp32_spmm_ir")
    g.close()


@pytest.mark.parametrize("form,precision", [("classic", "fp64"), ("auto", "fp32_spmm_ir")])
def test_ring_classic_and_mixed_ragged(form, precision):
    from paper_1811_07717_amd import zi
    H = hm.workload("sphere8mm_L37")
    say(f"[case] ring tile, {form} {precision}, L={H.L}")
    g = zi.System.from_head(H)
    _same_as_front(g, f"{form} {precision}", form=form, precision=precision)
    g.close()


def test_ring_tensor_conductivity():
    from paper_1811_07717_amd import zi
    H = hm.make_head(8.0, L=24, m=1, seed=21)
    cen = H.nodes[H.tets].mean(1)
    r = cen / np.linalg.norm(cen, axis=1, keepdims=True)
    S = H.sigma[:, None, None] * np.eye(3)[None]
    sk = H.labels == 3
    rr = np.einsum("ei,ej->eij", r[sk], r[sk])
    S[sk] = H.sigma[sk, None, None] * (rr + 10.0 * (np.eye(3)[None] - rr))
    s6 = np.ascontiguousarray(np.stack([S[:, 0, 0], S[:, 1, 1], S[:, 2, 2], S[:, 0, 1],
                                        S[:, 0, 2], S[:, 1, 2]], axis=1))
    say(f"[case] ring tile, tensor skull 8 mm: n={H.n} L={H.L}")
    c = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    g = zi.System(c(H.nodes), c(H.tets), c(s6), c(H.tris), c(H.tri_electrode), H.Z)
    # the skull's rows keep all 15 couplings in the solver's matrix: a mean
    # above 8 entries per row means rows of more than 8 entries
    say(f"[ring] solver entries per row: {g.nnz_solver / g.n:.2f}")
    assert g.nnz_solver > 8 * g.n
    _same_as_front(g, "tensor skull")
    g.close()


def test_ring_stretched_mesh():
    from paper_1811_07717_amd import zi
    H = hm.make_head(8.0, L=16, m=1, seed=41)
    nodes = H.nodes * np.array([1.0, 1.0, 6.0])
    say(f"[case] ring tile, 8 mm sphere stretched 6x along z: n={H.n}")
    c = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    g = zi.System(c(nodes), c(H.tets), c(H.sigma), c(H.tris), c(H.tri_electrode), H.Z)
    _same_as_front(g, "stretched")
    _same_as_front(g, "stretched, mixed precision", form="auto", precision="fp32_spmm_ir")
    g.close()


def test_ring_batched_heads():
    from paper_1811_07717_amd import zi
    ring, _ = _tiles()
    heads = [hm.make_head(h, L=L, m=1, seed=sd) for h, L, sd in
             ((8.0, 32, 51), (6.0, 24, 52), (8.0, 37, 53))]
    say(f"[case] ring tile, {len(heads)} batched heads")
    gs = [zi.System.from_head(H) for H in heads]
    Ts, sts, _ = zi.transfer_solve_batch(gs, tol=1e-8, tile=ring, form="single")
    for g, T, st in zip(gs, Ts, sts):
        T1, s1 = g.transfer_solve(tol=1e-8, tile=ring, form="single")
        assert np.array_equal(st["iters"], s1["iters"])
        assert torch.equal(T, T1)
        g.close()


def test_ring_not_for_zi_spmm():
    from paper_1811_07717_amd import zi
    ring, _ = _tiles()
    H = hm.workload("sphere8mm_L32")
    g = zi.System.from_head(H)
    X = torch.zeros((H.n, 32), dtype=torch.float64, device="cuda")
    with pytest.raises(zi.ZiError, match="solver's products only"):
        g.spmm(X, tile=ring)
    # both precisions score it
    for prec in ("fp64", "fp32_spmm_ir"):
        best, ms = g.autotune(precision=prec)
        assert ms[ring] > 0
    g.close()
