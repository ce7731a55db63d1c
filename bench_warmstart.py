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
    p.add_argument("--ceiling", type=int, default=0,
                   help="instead of training: on this many held-out fields, PCG iterations "
                        "from t0 plus a fraction of the true correction, the true correction "
                        "smoothed over the mesh graph, and the true correction plus noise")
    a = p.parse_args()
    if a.ceiling:
        return ceiling(a)
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


def ceiling(a):
    """What an initial iterate would have to achieve: the true transfer column t
    (PCG to 1e-12) against t0 on held-out fields, then the iterations to 1e-8
    from t0 + c (t - t0), from t0 + Ahat^h (t - t0) (the network's own
    aggregation, a one-layer network with unit neighbour weight) and from
    t + white noise of a fraction of max |t - t0|."""
    import torch
    from paper_1811_07717_amd import headmodel as hm, warmstart, zi

    log = lambda m: print(m, file=sys.stderr, flush=True)
    H = hm.workload(a.workload)
    ws = warmstart.WarmStart(H, seed=1, log=log)
    hops = (2, 8, 32, 128)
    smooth = {}
    for h in hops:
        m = zi.MeshGNN(ws.base, (2, 1), (h,))
        m.set_params(np.array([0, 0, 1, 0, 0], dtype=np.float32))
        smooth[h] = m

    def iters(s, l, x0):
        _, st = s.transfer_solve(tol=1e-8, columns=[l], x0=x0, graph=True)
        return int(st["iters"][0])

    rng = np.random.default_rng(5)
    rows = []
    for f in range(a.ceiling):
        sig = torch.from_numpy(hm.perturbed_sigma(H, seed=77 * 100003 + f)).cuda()
        s = ws.system(sig)
        l = int(rng.integers(H.L))
        t, _ = s.transfer_solve(tol=1e-12, columns=[l], graph=True)
        t0 = ws.T0[:, [l]].contiguous()
        d = t - t0
        r = {"zero": iters(s, l, None), "t0": iters(s, l, t0)}
        for c in (0.5, 0.9, 0.99):
            r[f"t0+{c}(t-t0)"] = iters(s, l, (t0 + c * d).contiguous())
        for h in hops:
            X = torch.zeros((H.n, 2), dtype=torch.float32, device="cuda")
            X[:, 0] = d[:, 0].float()
            r[f"t0+Ahat^{h}(t-t0)"] = iters(s, l, (t0 + smooth[h].forward(X).double()[:, None])
                                            .contiguous())
        g = torch.Generator(device="cuda")
        g.manual_seed(f)
        for e in (0.01, 0.1):
            noise = torch.randn(t.shape, device="cuda", dtype=torch.float64, generator=g)
            r[f"t+noise{e}"] = iters(s, l, (t + e * d.abs().max() * noise).contiguous())
        s.close()
        rows.append(r)
        log(f"[ceiling] field {f + 1}/{a.ceiling}: {r}")
    out = {"metric": "mean PCG iterations to rel.resid 1e-8 from constructed initial iterates",
           "workload": a.workload, "fields": a.ceiling,
           "iters_mean": {k: float(np.mean([r[k] for r in rows])) for k in rows[0]}}
    print(json.dumps(out))
    ws.close()


if __name__ == "__main__":
    main()
