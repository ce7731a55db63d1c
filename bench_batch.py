"""Batched uneven heads: 64 four-layer spheres with jittered radii (x U[0.9,
1.1]), layer conductivities x exp(U[ln 0.5, ln 2]), grid 2.5-6 mm and 32-128
electrodes each.  Times the transfer matrices of all heads (a) one head after
the other with eager launches and (b) with zi_transfer_solve_batch (every
head's iterations in graphs of eight heads, one branch per head, the next
replay queued while the host reads the flags of the last), after autotuning
each head's SpMM tile.  Prints one JSON line; bench.py reports the same
figures in its `batched_heads` field.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))


def measure(count=64, precision="fp64", log=None, markers=False):
    """Solve the transfer matrices of `count` uneven heads one after the other
    and then in one zi_transfer_solve_batch call; returns the figures.
    markers: launch the library's copy kernel on a small block before, between
    and after the two phases, so that a kernel trace can be cut into them."""
    import torch

    from paper_1811_07717_amd import headmodel as hm, zi
    say = log or (lambda m: print(f"[batch] {m}", file=sys.stderr, flush=True))
    say(f"generating {count} heads")
    heads = hm.batch_heads(count=count)
    systems = [zi.System.from_head(H) for H in heads]
    tiles = [g.autotune(precision)[0] for g in systems]
    torch.cuda.synchronize()
    solves = sum(H.L for H in heads)
    mark_src = torch.zeros(1 << 16, dtype=torch.float64, device="cuda")
    mark_dst = torch.empty_like(mark_src)

    def mark():
        if markers:
            zi.copy_probe(mark_src, mark_dst)
            torch.cuda.synchronize()

    mark()
    say("sequential")
    t0 = time.perf_counter()
    seq_iters = []
    seq_T = []
    for g in systems:
        T, st = g.transfer_solve(tol=1e-8, precision=precision)
        seq_iters.append(int(st["iters"].max()))
        seq_T.append(T)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    mark()
    say("one batch")
    t0 = time.perf_counter()
    Ts, stats, rc = zi.transfer_solve_batch(systems, tol=1e-8, precision=precision)
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    mark()
    res = max(float(s["relres_true"].max()) for s in stats)
    same = all(torch.equal(a, b) for a, b in zip(Ts, seq_T))
    out = {"heads": count, "precision": precision, "electrode_solves": solves,
           "nodes_min": min(H.n for H in heads), "nodes_max": max(H.n for H in heads),
           "sequential_s": t_seq, "batched_s": t_bat,
           "sequential_solves_per_s": solves / t_seq, "batched_solves_per_s": solves / t_bat,
           "speedup": t_seq / t_bat, "max_true_relres": res, "status": rc,
           "batched_equals_sequential": same,
           "tiles": sorted(set(zi.tile_names()[t] for t in tiles)),
           "iters_max": max(seq_iters)}
    for g in systems:
        g.close()
    return out


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--heads", type=int, default=64)
    p.add_argument("--precision", default="fp64", choices=["fp64", "fp32_spmm_ir"])
    p.add_argument("--markers", action="store_true",
                   help="mark the phases with copy kernels (for a kernel trace)")
    a = p.parse_args()
    out = measure(a.heads, a.precision, markers=a.markers)
    out["metric"] = "electrode-solves/s at rel.resid 1e-8, uneven heads"
    print(json.dumps(out))


if __name__ == "__main__":
    main()
