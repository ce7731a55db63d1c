"""Learned warm start on the 2 mm four-layer sphere with perturbed
conductivity (log-normal, sd 0.2, smoothed with an 8 mm Gaussian).

Generates training data with the method itself (mixed-precision transfer
columns of random electrodes for random fields), trains the 6-layer mesh-graph
network (hidden 64, float32, layers aggregating over 1, 4, 16, 64, 16, 4 hops;
features, targets and x0 from library kernels) with the library's
forward/backward kernels, and
reports PCG iterations and wall time to relative residual 1e-8 on held-out
fields from x0 = 0, from the unperturbed head's transfer column, and from the
network.  Prints one JSON line; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--workload", default="sphere2mm_L128")
    p.add_argument("--fields", type=int, default=250)
    p.add_argument("--per-field", type=int, default=8)
    p.add_argument("--epochs", type=int, default=3)
    p.add_argument("--eval-fields", type=int, default=200)
    p.add_argument("--lr", type=float, default=1e-3)
    a = p.parse_args()
    from paper_1811_07717_amd import headmodel as hm, warmstart

    log = lambda m: print(m, file=sys.stderr, flush=True)
    H = hm.workload(a.workload)
    t0 = time.time()
    ws = warmstart.WarmStart(H, seed=1, log=log)
    data = ws.make_dataset(a.fields, a.per_field, seed=11)
    t_data = time.time() - t0
    t1 = time.time()
    hist = ws.train(data, epochs=a.epochs, lr=a.lr)
    t_train = time.time() - t1
    del data
    log("[warmstart] evaluating")
    rows = ws.evaluate(a.eval_fields, seed=77)
    out = {"metric": "PCG iterations to rel.resid 1e-8 from a learned x0 vs zero start",
           "workload": a.workload, "n_nodes": H.n, "train_solves": a.fields * a.per_field,
           "epochs": a.epochs, "train_loss": hist, "data_s": t_data, "train_s": t_train,
           "eval_fields": a.eval_fields}
    for k in ("zero", "t0", "gnn"):
        its = np.array([r[k][0] for r in rows])
        out[k] = {"iters_mean": float(its.mean()), "iters_median": float(np.median(its)),
                  "iters_max": int(its.max()),
                  "seconds_mean": float(np.mean([r[k][2] for r in rows])),
                  "true_relres_max": float(max(r[k][1] for r in rows))}
    out["gain_vs_zero_iters"] = 1.0 - out["gnn"]["iters_mean"] / out["zero"]["iters_mean"]
    out["gain_vs_t0_iters"] = 1.0 - out["gnn"]["iters_mean"] / out["t0"]["iters_mean"]
    print(json.dumps(out))
    ws.close()


if __name__ == "__main__":
    main()
