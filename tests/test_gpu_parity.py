"""Parity of the HIP path against the FP64 oracle on small seeded heads.

Every product value comes from libzi through the C-ABI (paper_1811_07717_amd.zi);
every expected value comes from oracle/.  Integer outputs (CSR structure,
ground node, boundary flags, B structure, G structure) must match bit for bit;
floating-point outputs within the bounds stated per test.
"""
import numpy as np
import pytest

from oracle import fem, leadfield as lf, solve, source
from paper_1811_07717_amd import headmodel as hm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = ["sphere8mm_L32", "sphere8mm_L37"]


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", params=CASES)
def case(request):
    from paper_1811_07717_amd import zi
    H = hm.workload(request.param)
    say(f"[case] {request.param}: n={H.n} e={H.e} L={H.L} m={H.m}")
    S = fem.assemble(H.nodes, H.tets, H.sigma, H.tris, H.tri_electrode, H.Z)
    Tref = solve.transfer_direct(S["A"], S["B"])
    G = source.point_dipole_matrix(H.nodes, H.tets, H.dipole_tets)
    LFref = lf.leadfield(Tref, S["B"], S["C"], G)
    say(f"[gpu] zi_assemble {request.param}")
    sysg = zi.System.from_head(H)
    yield dict(name=request.param, H=H, S=S, Tref=Tref, G=G, LFref=LFref, sys=sysg)
    sysg.close()


def test_structure_bitwise(case):
    S, g = case["S"], case["sys"]
    v = g.view()
    A = S["A"]
    assert g.nnz == A.nnz
    np.testing.assert_array_equal(v["row_ptr"].cpu().numpy(), A.indptr)
    np.testing.assert_array_equal(v["col"].cpu().numpy(), A.indices)
    assert g.ground == S["ground"]
    H = case["H"]
    bnodes = np.zeros(H.n, dtype=np.uint8)
    bnodes[fem.boundary_faces(H.tets, H.n).ravel()] = 1
    np.testing.assert_array_equal(v["boundary"].cpu().numpy(), bnodes)
    B = S["B"].tocsr()
    B.sort_indices()
    np.testing.assert_array_equal(v["b_ptr"].cpu().numpy(), B.indptr)
    np.testing.assert_array_equal(v["b_col"].cpu().numpy(), B.indices)


def test_values(case):
    S, g = case["S"], case["sys"]
    v = g.view()
    A = S["A"]
    val = v["val"].cpu().numpy()
    rowmax = np.maximum.reduceat(np.abs(A.data), A.indptr[:-1])
    scale = np.repeat(rowmax, np.diff(A.indptr))
    err = np.abs(val - A.data) / scale
    say(f"[{case['name']}] max CSR value error / row max = {err.max():.3e}")
    assert err.max() <= 1e-13
    B = S["B"].tocsr()
    B.sort_indices()
    np.testing.assert_allclose(v["b_val"].cpu().numpy(), B.data, rtol=1e-13)
    np.testing.assert_allclose(v["C"].cpu().numpy(), S["C"], rtol=1e-14)
    np.testing.assert_allclose(v["calA"].cpu().numpy(), S["calA"], rtol=1e-13)


def test_point_dipoles(case):
    H, g, G = case["H"], case["sys"], case["G"]
    cp, ri, gv = g.point_dipoles(torch.from_numpy(H.dipole_tets).cuda())
    np.testing.assert_array_equal(cp.cpu().numpy(), G.indptr)
    np.testing.assert_array_equal(ri.cpu().numpy(), G.indices)
    np.testing.assert_allclose(gv.cpu().numpy(), G.data, rtol=1e-12,
                               atol=1e-14 * np.abs(G.data).max())


@pytest.mark.parametrize("k", [2, 32, 38, 128])
def test_spmm(case, k):
    g, A = case["sys"], case["S"]["A"]
    rng = np.random.default_rng(k)
    X = rng.standard_normal((g.n, k))
    Y, _ = g.spmm(torch.from_numpy(X).cuda())
    ref = A @ X
    err = np.abs(Y.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err <= 1e-14


def test_spmm_every_tile(case):
    from paper_1811_07717_amd import zi
    g, A = case["sys"], case["S"]["A"]
    X = np.random.default_rng(3).standard_normal((g.n, 40))
    ref = A @ X
    Xd = torch.from_numpy(X).cuda()
    outs = []
    for t, name in enumerate(zi.tile_names()):
        if name.startswith("ring"):
            continue   # the ring SpMM serves the solver's products only
        Y, _ = g.spmm(Xd, tile=t)
        Y = Y.cpu().numpy()
        assert np.abs(Y - ref).max() <= 1e-14 * np.abs(ref).max()
        outs.append(Y)
    for Y in outs[1:]:
        np.testing.assert_array_equal(Y, outs[0])      # same order of summation


def test_transfer_solve_against_oracle(case):
    g, S, Tref = case["sys"], case["S"], case["Tref"]
    say(f"[gpu] zi_transfer_solve {case['name']} tol 1e-8")
    T, st = g.transfer_solve(tol=1e-8)
    T = T.cpu().numpy()
    d = fem.preconditioner_diag(S["A"])
    _, its_o, _ = solve.pcg_columns(S["A"], S["B"], d, tol=1e-8)
    diff = np.abs(st["iters"] - its_o)
    say(f"[{case['name']}] iterations gpu {st['iters'].min()}..{st['iters'].max()}, "
        f"oracle {its_o.min()}..{its_o.max()}, max diff {diff.max()}")
    assert (diff <= np.maximum(3, 0.02 * its_o)).all()
    Bd = S["B"].toarray()
    res = np.linalg.norm(Bd - S["A"] @ T, axis=0) / np.linalg.norm(Bd, axis=0)
    assert res.max() <= 1.5e-8
    np.testing.assert_allclose(st["relres_true"], res, rtol=1e-3, atol=1e-12)
    assert (st["relres_rec"] <= 1e-8).all()
    colerr = np.linalg.norm(T - Tref, axis=0) / np.linalg.norm(Tref, axis=0)
    say(f"[{case['name']}] T column error vs direct: max {colerr.max():.3e}")
    assert colerr.max() <= 1e-5


def test_transfer_solve_tight(case):
    g, Tref = case["sys"], case["Tref"]
    T, st = g.transfer_solve(tol=1e-13, precond="ldp")
    colerr = np.linalg.norm(T.cpu().numpy() - Tref, axis=0) / np.linalg.norm(Tref, axis=0)
    assert colerr.max() <= 1e-9


def test_ldp_iterations(case):
    g, S = case["sys"], case["S"]
    T, st = g.transfer_solve(tol=1e-8, precond="ldp")
    d = fem.preconditioner_diag(S["A"], "ldp")
    _, its_o, _ = solve.pcg_columns(S["A"], S["B"], d, tol=1e-8)
    assert (np.abs(st["iters"] - its_o) <= np.maximum(3, 0.02 * its_o)).all()


def test_deterministic(case):
    g = case["sys"]
    T1, s1 = g.transfer_solve(tol=1e-8)
    T2, s2 = g.transfer_solve(tol=1e-8)
    assert torch.equal(T1, T2)
    np.testing.assert_array_equal(s1["iters"], s2["iters"])


def test_single_reduction_matches_classic(case):
    # The single-reduction form (the FP64 default) and the classic form produce
    # the same iterates in exact arithmetic: equal iteration counts up to a
    # column that sits at the stopping threshold, and equal T up to rounding.
    g = case["sys"]
    say(f"[gpu] classic vs single-reduction PCG {case['name']}")
    T1, s1 = g.transfer_solve(tol=1e-8, form="classic", timing=True)
    T2, s2 = g.transfer_solve(tol=1e-8, form="single", timing=True)
    assert set(s1["kernels"]) == {"spmm_pq", "update", "pupdate", "xflush"}
    assert set(s2["kernels"]) == {"spmm_sr", "update", "pflush"}
    di = np.abs(s1["iters"] - s2["iters"])
    d = ((T1 - T2).norm(dim=0) / T1.norm(dim=0)).cpu().numpy()
    say(f"[{case['name']}] iteration difference max {di.max()}, T difference max {d.max():.2e}")
    assert di.max() <= 1
    assert d[di == 0].max() <= 1e-9 and d.max() <= 1e-6
    T3, s3 = g.transfer_solve(tol=1e-8)
    assert torch.equal(T3, T2)
    np.testing.assert_array_equal(s3["iters"], s2["iters"])


@pytest.mark.parametrize("form,precision", [("single", "fp64"), ("classic", "fp64"),
                                            ("auto", "fp32_spmm_ir")])
def test_initial_iterate(case, form, precision):
    # x0 = the oracle's direct solution already meets the tolerance: no
    # iteration, T is x0 exactly.  x0 = 0.9 of it: the solve reaches the
    # tolerance in fewer iterations than from zero.
    g, S, Tref = case["sys"], case["S"], case["Tref"]
    say(f"[gpu] initial iterates, {form} / {precision} {case['name']}")
    x0 = torch.from_numpy(np.ascontiguousarray(Tref)).cuda()
    T, st = g.transfer_solve(tol=1e-8, x0=x0, form=form, precision=precision)
    assert (st["iters"] == 0).all()
    assert torch.equal(T, x0)
    T0, st0 = g.transfer_solve(tol=1e-8, form=form, precision=precision)
    T1, st1 = g.transfer_solve(tol=1e-8, x0=0.9 * x0, form=form, precision=precision)
    Tn = T1.cpu().numpy()
    Bd = S["B"].toarray()
    res = np.linalg.norm(Bd - S["A"] @ Tn, axis=0) / np.linalg.norm(Bd, axis=0)
    say(f"[{case['name']}] from 0.9 x*: iterations {st1['iters'].max()} (from zero "
        f"{st0['iters'].max()}), true residual max {res.max():.2e}")
    assert res.max() <= 1.5e-8
    assert (st1["iters"] <= st0["iters"]).all()


def test_not_converged_returns_last_iterate(case):
    from paper_1811_07717_amd import zi
    g = case["sys"]
    T, st = g.transfer_solve(tol=1e-8, maxit=3, raise_on_error=False)
    assert st["status"] == zi.ZI_ENOTCONV
    assert (st["iters"] == 3).all()
    assert torch.isfinite(T).all() and T.abs().max() > 0


def test_leadfield_against_oracle(case):
    g, H = case["sys"], case["H"]
    say(f"[gpu] full lead field {case['name']}")
    T, _ = g.transfer_solve(tol=1e-8)
    G = g.point_dipoles(torch.from_numpy(H.dipole_tets).cuda())
    LF = g.leadfield(T, G).cpu().numpy()
    ref = case["LFref"]
    r = lf.rdm(LF, ref)
    m = np.abs(lf.mag(LF, ref) - 1)
    say(f"[{case['name']}] LF vs oracle: RDM max {r.max():.3e}, |MAG-1| max {m.max():.3e}")
    assert r.max() <= 1e-4 and m.max() <= 1e-4
    assert np.abs(LF.sum(axis=0)).max() <= 1e-9 * np.abs(LF).max()


def test_leadfield_exact_given_tight_solve(case):
    g, H = case["sys"], case["H"]
    T, _ = g.transfer_solve(tol=1e-13, precond="ldp")
    G = g.point_dipoles(torch.from_numpy(H.dipole_tets).cuda())
    LF = g.leadfield(T, G).cpu().numpy()
    ref = case["LFref"]
    assert np.abs(LF - ref).max() <= 1e-8 * np.abs(ref).max()


def test_leadfield_fp32_matrix_cores(case):
    g, H = case["sys"], case["H"]
    T, _ = g.transfer_solve(tol=1e-8)
    G = g.point_dipoles(torch.from_numpy(H.dipole_tets).cuda())
    LF = g.leadfield(T, G, precision=1).cpu().numpy()
    ref = case["LFref"]
    r = lf.rdm(LF, ref)
    m = np.abs(lf.mag(LF, ref) - 1)
    say(f"[{case['name']}] fp32 LF: RDM max {r.max():.3e}, |MAG-1| max {m.max():.3e}")
    assert r.max() <= 1e-4 and m.max() <= 1e-4


def test_mixed_precision_refinement(case):
    # FP32 matrix products inside FP64 recurrences, FP64 iterative refinement:
    # the true FP64 residual must still reach the tolerance, and the lead field
    # must match the oracle to the same bar as the FP64 solve.
    g, S, H = case["sys"], case["S"], case["H"]
    say(f"[gpu] mixed-precision solve {case['name']}")
    T, st = g.transfer_solve(tol=1e-8, precision="fp32_spmm_ir")
    Tn = T.cpu().numpy()
    Bd = S["B"].toarray()
    res = np.linalg.norm(Bd - S["A"] @ Tn, axis=0) / np.linalg.norm(Bd, axis=0)
    colerr = np.linalg.norm(Tn - case["Tref"], axis=0) / np.linalg.norm(case["Tref"], axis=0)
    say(f"[{case['name']}] mixed: iters {st['iters'].min()}..{st['iters'].max()}, "
        f"refinements {st['refinements']}, true residual max {res.max():.2e}, "
        f"T column error max {colerr.max():.2e}")
    assert res.max() <= 1.5e-8
    assert colerr.max() <= 1e-5
    G = g.point_dipoles(torch.from_numpy(H.dipole_tets).cuda())
    LF = g.leadfield(T, G).cpu().numpy()
    r = lf.rdm(LF, case["LFref"])
    m = np.abs(lf.mag(LF, case["LFref"]) - 1)
    assert r.max() <= 1e-4 and m.max() <= 1e-4


@pytest.mark.parametrize("graph", [False, True])
def test_mixed_refinement_cycles(case, graph):
    # Float32 cycles stopped after a residual reduction of 1e-3 force FP64
    # refinement restarts at iterations that fall inside an X-flush window;
    # the restarted solve must still meet the tolerance against the oracle.
    from paper_1811_07717_amd import zi
    g, S, Tref = case["sys"], case["S"], case["Tref"]
    say(f"[gpu] mixed precision with refinement cycles (graph={graph}) {case['name']}")
    T, st = g.transfer_solve(tol=1e-8, precision="fp32_spmm_ir", refine_eta=1e-3, graph=graph)
    Tn = T.cpu().numpy()
    Bd = S["B"].toarray()
    res = np.linalg.norm(Bd - S["A"] @ Tn, axis=0) / np.linalg.norm(Bd, axis=0)
    colerr = np.linalg.norm(Tn - Tref, axis=0) / np.linalg.norm(Tref, axis=0)
    say(f"[{case['name']}] refinements {st['refinements']}, block iterations {st['block_iters']}, "
        f"true residual max {res.max():.2e}, T error max {colerr.max():.2e}")
    assert st["refinements"] >= 2
    assert res.max() <= 1.5e-8 and colerr.max() <= 1e-5
    _, st = g.transfer_solve(tol=1e-8, precision="fp32_spmm_ir", refine_eta=1.5,
                             raise_on_error=False)
    assert st["status"] == zi.ZI_EINVAL
