"""Learned PCG initial iterates for perturbed-conductivity heads.

A mesh-graph network (zi_gnn, the library's own forward/backward kernels) is
trained on transfer columns that the method itself produces for randomly
perturbed conductivity fields, and then proposes x0 for zi_transfer_solve.
The PCG always runs to the same tolerance; the network only changes where it
starts.

For electrode l and a head whose conductivity differs from the base head's,
the network sees per node the ten features of zi_gnn_features (the
right-hand side, the conductivity change seen by the node, the base head's
transfer column t0_l, position, distance to the electrode, a compartment mark,
the residual b_l - A t0_l of t0_l for this head, each scaled to O(1), and a
constant),
and predicts g (t_l - t0_l) / s_l with s_l = max |t0_l| and g a fixed gain that
gives the training targets unit RMS (zi_gnn_target); the proposed initial
iterate is x0 = t0_l + s_l * prediction / g (zi_gnn_x0).  The layers
aggregate over 1, 4, 16, 64, 16 and 4 mesh-graph hops, so the output sees the
whole head: the change of the potential caused by a conductivity change is
global.  The output layer starts at zero, so the untrained network proposes
x0 = t0_l.  Feature construction, targets and x0 run in library kernels; this
module only orchestrates (device memory, which column, when to train).
"""
from __future__ import annotations

import time

import numpy as np

from . import headmodel as hm
from . import zi

N_FEATURES = 10
DIMS = (N_FEATURES, 64, 64, 64, 64, 64, 1)
HOPS = (1, 4, 16, 64, 16, 4)


def glorot_params(dims, seed, zero_last=False):
    """Flat float32 parameters in the zi_gnn layout (Glorot-uniform weights;
    with zero_last the output layer starts at zero, so the untrained network
    predicts no correction)."""
    rng = np.random.default_rng(seed)
    out = []
    K = len(dims) - 1
    for k, (fi, fo) in enumerate(zip(dims[:-1], dims[1:])):
        lim = 0.0 if (zero_last and k == K - 1) else np.sqrt(6.0 / (fi + fo))
        out += [rng.uniform(-lim, lim, fi * fo), rng.uniform(-lim, lim, fi * fo), np.zeros(fo)]
    return np.concatenate(out).astype(np.float32)


class WarmStart:
    def __init__(self, H, dims=DIMS, hops=HOPS, seed=0, log=print):
        import torch
        self.torch = torch
        self.H = H
        self.dims = list(dims)
        self.hops = list(hops) if hops is not None else None
        self.log = log
        self.base = zi.System.from_head(H)
        T0, _ = self.base.transfer_solve(tol=1e-8, graph=True)
        self.T0 = T0
        self.R = float(np.linalg.norm(H.nodes, axis=1).max())
        self.net = zi.MeshGNN(self.base, self.dims, self.hops)
        self.net.set_params(glorot_params(self.dims, seed, zero_last=True))
        self.gain = 1.0

    def close(self):
        self.net.close()
        self.base.close()

    def system(self, sigma):
        """The head with per-tet conductivities sigma (device tensor)."""
        k = self.base._keep
        return zi.System(k[0], k[1], sigma, k[3], k[4], self.H.Z)

    def features(self, sys_p, l):
        return zi.gnn_features(self.base, sys_p, self.T0, l, self.H.centres[l], self.R)

    def predict_x0(self, sys_p, ls):
        torch = self.torch
        x0 = torch.empty((self.H.n, len(ls)), dtype=torch.float64, device="cuda")
        for j, l in enumerate(ls):
            y = self.net.forward(self.features(sys_p, l))
            zi.gnn_x0(y, self.T0, l, self.gain, x0, j)
        return x0

    # -- data, training, evaluation -----------------------------------------
    def make_dataset(self, n_fields, per_field, seed, precision="fp32_spmm_ir"):
        torch = self.torch
        rng = np.random.default_rng(seed)
        data = []
        t0 = time.time()
        for f in range(n_fields):
            sig = torch.from_numpy(hm.perturbed_sigma(self.H, seed=seed * 100003 + f)).cuda()
            s = self.system(sig)
            ls = rng.choice(self.H.L, size=per_field, replace=False)
            T, _ = s.transfer_solve(tol=1e-8, precision=precision, columns=ls, graph=True)
            if f == 0:
                # the gain that gives the targets unit RMS, from the first field
                ss = sum(zi.gnn_target(T, j, self.T0, int(l))[1] for j, l in enumerate(ls))
                rms = np.sqrt(ss / (len(ls) * self.H.n))
                self.gain = 1.0 / rms if rms > 0 else 1.0
                self.log(f"[warmstart] target gain {self.gain:.3g}")
            for j, l in enumerate(ls):
                data.append((self.features(s, int(l)),
                             zi.gnn_target(T, j, self.T0, int(l), self.gain)[0]))
            s.close()
            if (f + 1) % max(1, n_fields // 10) == 0:
                self.log(f"[warmstart] data: field {f + 1}/{n_fields} ({time.time() - t0:.0f} s)")
        return data

    def train(self, data, epochs, lr=1e-3, seed=0):
        rng = np.random.default_rng(seed)
        hist = []
        t0 = time.time()
        for ep in range(epochs):
            order = rng.permutation(len(data))
            tot = 0.0
            rate = lr * (0.5 ** ep)
            for i, k in enumerate(order):
                X, t = data[k]
                loss, _ = self.net.loss_grad(X, t)
                self.net.adam_step(rate)
                tot += loss
                if (i + 1) % max(1, len(data) // 4) == 0 and i + 1 < len(data):
                    self.log(f"[warmstart] epoch {ep + 1}: {i + 1}/{len(data)} steps, "
                             f"mean loss {tot / (i + 1):.4f} ({time.time() - t0:.0f} s)")
            hist.append(tot / len(data))
            self.log(f"[warmstart] epoch {ep + 1}/{epochs}: mean loss {hist[-1]:.4f} "
                     f"({time.time() - t0:.0f} s)")
        return hist

    def evaluate(self, n_fields, seed, tol=1e-8):
        """PCG iterations to tol from x0 = 0, from t0 and from the network;
        the network's time includes its features and x0."""
        torch = self.torch
        rng = np.random.default_rng(seed)
        rows = []
        for f in range(n_fields):
            sig = torch.from_numpy(hm.perturbed_sigma(self.H, seed=seed * 100003 + f)).cuda()
            s = self.system(sig)
            l = int(rng.integers(self.H.L))
            res = {}
            for name in ("zero", "t0", "gnn"):
                x0 = None
                torch.cuda.synchronize()
                ta = time.perf_counter()
                if name == "t0":
                    x0 = self.T0[:, [l]].contiguous()
                elif name == "gnn":
                    x0 = self.predict_x0(s, [l])
                _, st = s.transfer_solve(tol=tol, columns=[l], x0=x0, graph=True)
                torch.cuda.synchronize()
                res[name] = (int(st["iters"][0]), float(st["relres_true"][0]),
                             time.perf_counter() - ta)
            s.close()
            rows.append(res)
            if (f + 1) % max(1, n_fields // 10) == 0:
                self.log(f"[warmstart] eval: field {f + 1}/{n_fields}")
        return rows
