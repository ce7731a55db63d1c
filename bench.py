"""Lead-field build benchmark on one MI355X.

One step = the whole hot path on device-resident inputs:
zi_assemble (stiffness + CEM + ground) -> zi_transfer_solve (Jacobi PCG on all
electrode columns to relative residual 1e-8) -> zi_leadfield (Schur complement,
Cholesky, T^T G, matrix-core product).  The dipole source matrix G is built
once before timing (it is an input of the lead-field stage).

Prints one JSON line (rank 0).  Default workload: the 1 mm four-layer sphere
(3.34 M nodes, 19.6 M tets) with 256 electrodes and 100 000 dipoles x 3
orientations, in FP64; ``--workload sphere2mm_L128`` runs the 2 mm sphere with
128 electrodes, ``--mixed`` also times the mixed-precision solve.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

def log(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


METRIC = "LF build s and electrode-solves/s at rel.resid 1e-8; SpMM HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="sphere1mm_L256")
    p.add_argument("--tile", type=int, default=-1)
    p.add_argument("--precond", default="jacobi")
    p.add_argument("--precision", default="fp64", choices=["fp64", "fp32_spmm_ir"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-batch", dest="batch", action="store_false",
                   help="skip the batched-heads measurement (64 uneven heads, one after the "
                        "other and in one zi_transfer_solve_batch call)")
    p.add_argument("--mixed", action="store_true",
                   help="also time the same builds with the mixed-precision solve (fp32 "
                        "search directions and products, fp64 recurrences)")
    p.add_argument("--sweep-tiles", action="store_true",
                   help="also time zi_spmm with every tile on an n x L block")
    p.add_argument("--calib-copy-mb", type=int, default=0,
                   help="also run one torch copy of this many MiB (counter calibration)")
    p.add_argument("--columns", type=int, default=0,
                   help="solve only the first K electrode columns (one GPU's share of a "
                        "build sharded by column) and skip the lead field, which needs all")
    p.add_argument("--no-autotune", dest="autotune", action="store_false",
                   help="skip zi_autotune (default: tune the tile once before timing)")
    return p.parse_args()


def traffic_for(kernel, workload, tile):
    """HBM bytes per product from the committed counter summary, if it was
    taken on the current kernel source (and, for the SpMM, the same tile);
    else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    key = f"{kernel}@{tile}" if kernel.startswith("spmm") else kernel
    e = d.get(workload, {}).get(key)
    from paper_1811_07717_amd.counters import source_hash
    if not e or e.get("source_hash") != source_hash():
        return None
    return e.get("bytes_per_launch")


def copy_bandwidth(torch, dev, mib=2048):
    """Achievable HBM bandwidth of the library's plain 16-byte streaming copy
    (read + write bytes / s, best of 5)."""
    from paper_1811_07717_amd import zi
    x = torch.ones((mib << 20) // 8, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    ms = min(zi.copy_probe(x, y) for _ in range(6))
    return 2 * (mib << 20) / (ms * 1e-3) / 1e9


def _oracle_pcg_worker(path, seed, iters):
    """One worker of the CPU baseline: ``iters`` iterations of the oracle's
    PCG (one electrode-like column) on the sampled oracle matrix; returns the
    wall time of those iterations."""
    import numpy as np
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits

    from oracle import solve
    z = np.load(path)
    A = sp.csr_matrix((z["data"], z["indices"], z["indptr"]), shape=tuple(z["shape"]))
    d = z["d"]
    b = np.random.default_rng(seed).standard_normal(A.shape[0])
    with threadpool_limits(1):
        t0 = time.perf_counter()
        try:
            solve.pcg(A, b, d, tol=1e-300, maxit=iters)
        except solve.NotConverged:
            pass
        return time.perf_counter() - t0


def host_cpu():
    """(logical cores, CPU model) of this host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    if model == "unknown":
        try:
            import subprocess
            out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
            for line in out.splitlines():
                if line.startswith("Model name:"):
                    model = line.split(":", 1)[1].strip()
                    break
        except Exception:
            pass
    return os.cpu_count() or 1, model


def cpu_baseline_sample(H, workers=None, iters=40, slabs=8):
    """Time the oracle (plain NumPy/SciPy FP64) on a bounded sample of the
    workload's own mesh, before anything touches the GPU.

    Sample: the tets whose centroid lies in the central z-slab that holds
    1/``slabs`` of them (its own nodes renumbered).  The oracle assembles that
    sub-mesh (stiffness, electrode terms of its triangles, ground fix:
    ``fem.assemble``), then ``workers`` processes each run ``iters`` oracle PCG
    iterations on it at once (one column each, one thread each; the electrode
    columns of a build are independent, so this is the oracle's throughput on
    all cores).  ``cpu_baseline`` scales the times to the whole mesh by the
    tet and nonzero counts and to the iteration counts of the GPU build."""
    import concurrent.futures
    import multiprocessing as mp
    import tempfile

    from oracle import fem
    cores, model = host_cpu()
    workers = workers or min(cores, 16)
    cz = H.nodes[H.tets, 2].mean(axis=1)
    lo, hi = np.quantile(cz, [0.5 - 0.5 / slabs, 0.5 + 0.5 / slabs])
    keep = (cz >= lo) & (cz <= hi)
    tets = H.tets[keep]
    used = np.unique(tets)
    new = np.full(H.n, -1, dtype=np.int64)
    new[used] = np.arange(used.size)
    tets_s = new[tets].astype(np.int32)
    # electrode triangles that are faces of a kept tet
    tri = np.sort(H.tris, axis=1)
    f = np.sort(np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]], tets[:, [0, 1, 3]],
                                tets[:, [0, 1, 2]]]), axis=1)
    f = f[np.isin(f[:, 0], tri[:, 0])]
    faces = set(map(tuple, f.tolist()))
    tri_ok = np.array([tuple(t) in faces for t in tri.tolist()], dtype=bool)
    tris_s = new[H.tris[tri_ok]].astype(np.int32)
    tre_s = H.tri_electrode[tri_ok]
    sigma_s = H.sigma[keep]
    t0 = time.perf_counter()
    S = fem.assemble(H.nodes[used], tets_s, sigma_s, tris_s, tre_s, H.Z)
    t_asm = time.perf_counter() - t0
    A = S["A"]
    d = fem.preconditioner_diag(A)
    tmp = tempfile.mkdtemp(prefix="zi_cpu_baseline_")
    path = os.path.join(tmp, "A.npz")
    np.savez(path, data=A.data, indices=A.indices, indptr=A.indptr,
             shape=np.array(A.shape), d=d)
    try:
        ctx = mp.get_context("spawn")
        with concurrent.futures.ProcessPoolExecutor(workers, mp_context=ctx) as ex:
            list(ex.map(_oracle_pcg_worker, [path] * workers, range(workers), [2] * workers))
            t0 = time.perf_counter()
            per = list(ex.map(_oracle_pcg_worker, [path] * workers, range(workers),
                              [iters] * workers))
            t_wall = time.perf_counter() - t0
    finally:
        os.remove(path)
        os.rmdir(tmp)
    return dict(cores=workers, host_cores=cores, model=model, t_asm=t_asm, e_s=int(keep.sum()),
                n_s=int(used.size), nnz_s=int(A.nnz), t_iter=t_wall / iters,
                t_iter_single=float(np.median(per)) / iters, iters=iters, slabs=slabs)


def cpu_baseline(smp, H, nnz, iters, L):
    """The oracle's electrode-solves/s for one whole lead-field build,
    scaled from ``cpu_baseline_sample``: assembly time x (tets / sampled
    tets), and per column the GPU build's iteration count x the time of one
    oracle PCG iteration x (nonzeros / sampled nonzeros), with ``cores``
    columns in flight at once."""
    t_asm = smp["t_asm"] * H.e / smp["e_s"]
    t_it = smp["t_iter"] * nnz / smp["nnz_s"]
    t_cols = float(np.sum(iters)) * t_it / smp["cores"]
    t_step = t_asm + t_cols
    return {"value": L / t_step, "unit": "electrode-solves/s", "cores": smp["cores"],
            "kind": "oracle", "host_cores": smp["host_cores"], "host_cpu": smp["model"],
            "seconds_per_build": t_step,
            "sample": (f"central z-slab of the mesh holding 1/{smp['slabs']} of its tets "
                       f"({smp['e_s']} tets, {smp['n_s']} nodes, {smp['nnz_s']} nonzeros): "
                       f"oracle assembly {smp['t_asm']:.1f} s, then {smp['cores']} worker "
                       f"processes running {smp['iters']} oracle PCG iterations each at once "
                       f"({smp['t_iter'] * 1e3:.1f} ms per iteration with all of them running, "
                       f"{smp['t_iter_single'] * 1e3:.1f} ms median per worker); scaled to "
                       f"{H.e} tets and {nnz} nonzeros and to the GPU build's "
                       f"{int(np.sum(iters))} column-iterations over {L} columns"),
            "seconds_assembly": t_asm, "seconds_per_column_iteration": t_it}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the lead-field build "
              "shards by electrode column across GPUs by design but that path is not built.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1811_07717_amd import headmodel as hm, zi

    t_start = time.perf_counter()
    H = hm.workload(a.workload)
    log(f"workload {a.workload}: n={H.n} e={H.e} L={H.L} ({time.perf_counter() - t_start:.1f} s)")
    # the oracle's sample runs first, in worker processes, before anything
    # touches the GPU
    smp = None if a.no_cpu_baseline else cpu_baseline_sample(H)
    if smp is not None:
        log(f"oracle sample done ({smp['cores']} workers, {time.perf_counter() - t_start:.1f} s)")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(0)
    nodes = torch.from_numpy(H.nodes).to(dev)
    tets = torch.from_numpy(H.tets).to(dev)
    sigma = torch.from_numpy(np.ascontiguousarray(H.sigma)).to(dev)
    tris = torch.from_numpy(H.tris).to(dev)
    tre = torch.from_numpy(H.tri_electrode).to(dev)
    dip = torch.from_numpy(H.dipole_tets).to(dev)
    L = H.L
    if not 0 <= a.columns <= L:
        sys.exit(f"--columns must be in [0, {L}]")
    cols = list(range(a.columns)) if a.columns else None
    K = a.columns or L
    T = torch.empty((H.n, K), dtype=torch.float64, device=dev)
    LF = torch.empty((L, 3 * H.m), dtype=torch.float64, device=dev)
    s0 = zi.System(nodes, tets, sigma, tris, tre, H.Z)
    G = s0.point_dipoles(dip)
    tuned = None
    if a.autotune:
        best, ms = s0.autotune(a.precision)
        tuned = {"tile": zi.tile_names()[best], "ms": {n: float(v) for n, v in
                                                      zip(zi.tile_names(), ms)}}
        if a.tile < 0 and cols is None:   # tuned for all L columns
            a.tile = best
    s0.close()
    torch.cuda.synchronize()
    log(f"set-up done, tile {a.tile} ({time.perf_counter() - t_start:.1f} s)")

    # Every library call synchronises its stream before returning, so the
    # wall clock between calls splits a build into its stages without adding
    # synchronisation.
    stage_names = ("assemble", "transfer_solve", "leadfield", "destroy")

    def step():
        t = [time.perf_counter()]
        s = zi.System(nodes, tets, sigma, tris, tre, H.Z)
        t.append(time.perf_counter())
        _, st = s.transfer_solve(tol=1e-8, precond=a.precond, precision=a.precision,
                                 timing=True, tile=a.tile, out=T, columns=cols)
        t.append(time.perf_counter())
        if cols is None:
            s.leadfield(T, G, out=LF)
        t.append(time.perf_counter())
        s.close()
        t.append(time.perf_counter())
        st["stages"] = [t[i + 1] - t[i] for i in range(4)]
        return st

    for w in range(a.warmup):
        step()
        log(f"warm-up {w + 1}/{a.warmup}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    step_s = []
    for k in range(a.steps):
        ts = time.perf_counter()
        stats.append(step())
        step_s.append(time.perf_counter() - ts)
        log(f"step {k + 1}/{a.steps}: {step_s[-1]:.3f} s")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps

    mixed = None
    if a.precision == "fp64" and cols is None and a.mixed:
        # the same builds with ZI_FP32_SPMM_IR, timed separately; the lead field
        # is compared with the FP64 one just computed
        LF64 = LF.clone()
        s1 = zi.System(nodes, tets, sigma, tris, tre, H.Z)
        bm, _ = s1.autotune("fp32_spmm_ir")
        s1.close()

        def mstep():
            s = zi.System(nodes, tets, sigma, tris, tre, H.Z)
            _, st = s.transfer_solve(tol=1e-8, precond=a.precond, precision="fp32_spmm_ir",
                                     tile=bm, out=T)
            s.leadfield(T, G, out=LF)
            s.close()
            return st

        for _ in range(a.warmup):
            mstep()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mst = [mstep() for _ in range(a.steps)]
        torch.cuda.synchronize()
        dtm = (time.perf_counter() - t0) / a.steps
        n64 = LF64.norm(dim=0)
        nm = LF.norm(dim=0)
        rdm = (LF / nm - LF64 / n64).norm(dim=0)
        mixed = {"value": L / dtm, "ms_per_step": dtm * 1e3, "tile": zi.tile_names()[bm],
                 "pcg_iters": {"median": int(np.median(mst[-1]["iters"])),
                               "max": int(mst[-1]["iters"].max()),
                               "refinements": int(mst[-1]["refinements"])},
                 "true_relres_max": float(max(np.max(x["relres_true"]) for x in mst)),
                 "lf_rdm_vs_fp64_max": float(rdm.max()),
                 "lf_mag_vs_fp64_max": float((nm / n64 - 1).abs().max()),
                 "dtype": "f32 search directions and products; f64 matrix values, sums, "
                          "dots and recurrences"}
        del LF64

    if a.calib_copy_mb:
        x = torch.ones((a.calib_copy_mb << 20) // 8, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        zi.copy_probe(x, y)
        torch.cuda.synchronize()

    tiles = None
    if a.sweep_tiles:
        s1 = zi.System(nodes, tets, sigma, tris, tre, H.Z)
        X = torch.randn((H.n, L + (L & 1)), dtype=torch.float64, device=dev)
        nb = 12 * s1.nnz_solver + 4 * (H.n + 1) + 16 * H.n * X.shape[1]
        tiles = {}
        for t, name in enumerate(zi.tile_names()):
            Y, _ = s1.spmm(X, tile=t)
            ms = min(s1.spmm(X, tile=t, out=Y)[1] for _ in range(5))
            tiles[name] = {"ms": ms, "gbs": nb / (ms * 1e-3) / 1e9}
        s1.close()
        del X

    # dominant kernel: the largest (average launch time x launches); the
    # library times a sample of the launches
    ktot = {}
    for st in stats:
        for k, v in st["kernels"].items():
            e = ktot.setdefault(k, dict(ms=0.0, launches=0, calls=0, bytes=v["bytes"]))
            e["ms"] += v["ms"]
            e["launches"] += v["launches"]
            e["calls"] += v["calls"]
    dom = max(ktot, key=lambda k: ktot[k]["ms"] / max(ktot[k]["launches"], 1) * ktot[k]["calls"])
    avg_ms = ktot[dom]["ms"] / ktot[dom]["launches"]
    gbs = ktot[dom]["bytes"] / (avg_ms * 1e-3) / 1e9
    iters = stats[-1]["iters"]
    out = {
        "metric": METRIC,
        "value": K / dt,
        "unit": "electrode-solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == "fp64" else "f32 products, f64 recurrences",
        "data": "synthetic",
        "config": {"workload": a.workload, "h_mm": H.h_mm, "n_nodes": H.n, "n_tets": H.e,
                   "nnz": int(s0.nnz), "nnz_solver": int(s0.nnz_solver), "electrodes": L, "lf_columns": 3 * H.m,
                   "tol": 1e-8, "precond": a.precond, "precision": a.precision,
                   "tile": stats[-1]["tile"], "tile_name": zi.tile_names()[stats[-1]["tile"]],
                   "columns_solved": K,
                   "leadfield": cols is None},
        "lf_build_s": dt,
        "lf_build_s_median": float(np.median(step_s)),
        "stages_median_s": {nm: float(np.median([x["stages"][i] for x in stats]))
                            for i, nm in enumerate(stage_names)},
        "electrode_solves_per_s_solve_only":
            K / float(np.median([x["stages"][1] for x in stats])),
        "pcg_iters": {"median": int(np.median(iters)), "max": int(iters.max()),
                      "block_loop": int(stats[-1]["block_iters"]),
                      "refinements": int(stats[-1]["refinements"])},
        "solver_kernels": {k: {"avg_ms": v["ms"] / v["launches"],
                               "gbs": v["bytes"] / (v["ms"] / v["launches"] * 1e-3) / 1e9,
                               "bytes_per_launch": v["bytes"],
                               "launches_per_step": v["calls"] // a.steps,
                               "timed_launches": v["launches"]} for k, v in ktot.items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                     "traffic": traffic_for(dom, a.workload + ("" if a.precision == "fp64" else "_mixed"),
                                            zi.tile_names()[stats[-1]["tile"]])},
    }
    rf = out["roofline"]
    if rf["traffic"]:
        # measured HBM bytes of the same kernel over the same average time
        rf["traffic_gbs"] = rf["traffic"] / (avg_ms * 1e-3) / 1e9
        rf["traffic_frac"] = rf["traffic_gbs"] / HBM_PEAK_GBS
    # the plain SpMM's unit of work, Y = A X on the mesh graph with K columns:
    # 12 nnz + 4 (n + 1) + 16 n K bytes, over the same kernel time
    if dom.startswith("spmm"):
        unit_bytes = 12 * int(s0.nnz) + 4 * (H.n + 1) + 16 * H.n * K
        rf["spmm_unit_bytes"] = unit_bytes
        rf["spmm_unit_frac"] = unit_bytes / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
    out["hbm_copy_gbs"] = copy_bandwidth(torch, dev)
    if tiles:
        out["spmm_tiles"] = tiles
    if tuned:
        out["autotune"] = tuned
    if smp is not None:
        out["cpu_baseline"] = cpu_baseline(smp, H, int(s0.nnz), iters, K)
    if a.batch:
        T = LF = None   # the 1 mm blocks go back before the heads are built
        torch.cuda.empty_cache()
        zi.release_cached_memory()
        import bench_batch
        out["batched_heads"] = bench_batch.measure(64, "fp64", log=log)
    if mixed is not None:
        out["mixed_precision"] = mixed
    print(json.dumps(out))


if __name__ == "__main__":
    main()
