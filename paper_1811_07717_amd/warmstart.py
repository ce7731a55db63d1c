"""Learned PCG initial iterates for perturbed-conductivity heads.

A mesh-graph network (zi_gnn, the library's own forward/backward kernels) is
trained on transfer columns that the method itself produces for randomly
perturbed conductivity fields, and then proposes x0 for zi_transfer_solve.
The PCG always runs to the same tolerance; the network only changes where it
starts.

For electrode l and conductivity field sigma the network sees, per node:
  0  b_l / max b_l                       (the right-hand side)
  1  mean over incident tets of log(sigma / sigma_ref)   (the perturbation)
  2  t0_l / s_l                          (the unperturbed head's transfer column)
  3-5 node position / outer radius
  6  distance to electrode l's centre / outer radius
  7  mean over incident tets of log(sigma_ref / 0.33)    (the compartment)
and predicts g (t_l - t0_l) / s_l with s_l = max |t0_l| and g a fixed gain
that gives the training targets unit RMS; the proposed initial iterate is
x0 = t0_l + s_l * prediction / g.  The output layer starts at zero, so the
untrained network proposes x0 = t0_l.
"""
from __future__ import annotations

import time

import numpy as np

from . import headmodel as hm
from . import zi

N_FEATURES = 8


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


def _node_mean(H, values):
    cnt = np.bincount(H.tets.ravel(), minlength=H.n).astype(np.float64)
    return np.bincount(H.tets.ravel(), weights=np.repeat(values, 4), minlength=H.n) / cnt


def _incidence(H):
    """Node -> incident tets in ascending order, padded with -1 (n x max degree)."""
    flat = H.tets.ravel().astype(np.int64)
    order = np.argsort(flat, kind="stable")
    cnt = np.bincount(flat, minlength=H.n)
    start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    pos = np.arange(flat.size) - np.repeat(start, cnt)
    inc = np.full((H.n, int(cnt.max())), -1, dtype=np.int64)
    inc[flat[order], pos] = order // 4
    return inc, cnt


class WarmStart:
    def __init__(self, H, dims=(N_FEATURES, 64, 64, 64, 64, 64, 1), seed=0, log=print):
        import torch
        self.torch = torch
        self.H = H
        self.dims = list(dims)
        self.log = log
        self.base = zi.System.from_head(H)
        T0, st = self.base.transfer_solve(tol=1e-8, graph=True)
        self.T0 = T0
        self.scale = T0.abs().max(dim=0).values                       # s_l
        R = float(np.linalg.norm(H.nodes, axis=1).max())
        self.R = R
        v = self.base.view()
        rows = torch.repeat_interleave(torch.arange(H.n, device="cuda"),
                                       (v["b_ptr"][1:] - v["b_ptr"][:-1]).long())
        self.b_rows, self.b_col, self.b_val = rows, v["b_col"].long(), v["b_val"]
        self.static = torch.from_numpy(np.concatenate(
            [H.nodes / R, _node_mean(H, np.log(H.sigma / 0.33))[:, None]], axis=1)).cuda()
        inc, cnt = _incidence(H)
        self.inc = torch.from_numpy(inc).cuda()
        self.inc_valid = self.inc >= 0
        self.inc_cnt = torch.from_numpy(cnt.astype(np.float64)).cuda()
        self.sig_ref_log = torch.log(torch.from_numpy(H.sigma).cuda())
        self.net = zi.MeshGNN(self.base, self.dims)
        self.net.set_params(glorot_params(self.dims, seed, zero_last=True))
        self.gain = 1.0

    def close(self):
        self.net.close()
        self.base.close()

    def log_perturbation(self, sigma):
        """Per-node mean over the incident tets of log(sigma / sigma_ref), on the
        device (sigma: per-tet conductivities, numpy or a device tensor)."""
        torch = self.torch
        sig = sigma if isinstance(sigma, torch.Tensor) else torch.from_numpy(sigma)
        d = torch.log(sig.cuda()) - self.sig_ref_log
        g = torch.where(self.inc_valid, d[self.inc.clamp(min=0)], torch.zeros((), dtype=d.dtype,
                                                                               device=d.device))
        return g.sum(dim=1) / self.inc_cnt

    def features(self, sigma, l, pert=None):
        torch = self.torch
        H = self.H
        n = H.n
        X = torch.zeros((n, N_FEATURES), dtype=torch.float64, device="cuda")
        sel = self.b_col == l
        b = torch.zeros(n, dtype=torch.float64, device="cuda")
        b[self.b_rows[sel]] = self.b_val[sel]
        X[:, 0] = b / b.abs().max()
        if pert is None:
            pert = self.log_perturbation(sigma)
        X[:, 1] = pert
        X[:, 2] = self.T0[:, l] / self.scale[l]
        X[:, 3:6] = self.static[:, 0:3]
        c = torch.from_numpy(H.centres[l] / self.R).cuda()
        X[:, 6] = (self.static[:, 0:3] - c).norm(dim=1)
        X[:, 7] = self.static[:, 3]
        return X.float().contiguous()

    def target(self, t, l):
        return ((t - self.T0[:, l]) / self.scale[l]).float().contiguous()   # times gain later

    def predict_x0(self, sigma, ls):
        torch = self.torch
        pert = self.log_perturbation(sigma)
        cols = []
        for l in ls:
            y = self.net.forward(self.features(sigma, l, pert)).double()
            cols.append(self.T0[:, l] + self.scale[l] * y / self.gain)
        return torch.stack(cols, dim=1).contiguous()

    # -- data, training, evaluation -----------------------------------------
    def make_dataset(self, n_fields, per_field, seed, precision="fp32_spmm_ir"):
        torch = self.torch
        rng = np.random.default_rng(seed)
        data = []
        t0 = time.time()
        for f in range(n_fields):
            sig = torch.from_numpy(hm.perturbed_sigma(self.H, seed=seed * 100003 + f)).cuda()
            s = zi.System(self.base._keep[0], self.base._keep[1], sig, self.base._keep[3],
                          self.base._keep[4], self.H.Z)
            ls = rng.choice(self.H.L, size=per_field, replace=False)
            T, _ = s.transfer_solve(tol=1e-8, precision=precision, columns=ls, graph=True)
            s.close()
            pert = self.log_perturbation(sig)
            for j, l in enumerate(ls):
                data.append((self.features(sig, int(l), pert), self.target(T[:, j], int(l))))
            if (f + 1) % max(1, n_fields // 10) == 0:
                self.log(f"[warmstart] data: field {f + 1}/{n_fields} ({time.time() - t0:.0f} s)")
        rms = float(np.sqrt(np.mean([float((t.double() ** 2).mean()) for _, t in data])))
        self.gain = 1.0 / rms if rms > 0 else 1.0
        data = [(X, (t * self.gain).contiguous()) for X, t in data]
        self.log(f"[warmstart] target gain {self.gain:.3g}")
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
        """PCG iterations to tol from x0 = 0, from t0 and from the network."""
        torch = self.torch
        rng = np.random.default_rng(seed)
        rows = []
        for f in range(n_fields):
            sig = torch.from_numpy(hm.perturbed_sigma(self.H, seed=seed * 100003 + f)).cuda()
            s = zi.System(self.base._keep[0], self.base._keep[1], sig, self.base._keep[3],
                          self.base._keep[4], self.H.Z)
            l = int(rng.integers(self.H.L))
            res = {}
            for name in ("zero", "t0", "gnn"):
                x0 = None
                torch.cuda.synchronize()
                ta = time.perf_counter()
                if name == "t0":
                    x0 = self.T0[:, [l]].contiguous()
                elif name == "gnn":
                    x0 = self.predict_x0(sig, [l])     # network time is included
                _, st = s.transfer_solve(tol=tol, columns=[l], x0=x0, graph=True)
                torch.cuda.synchronize()
                res[name] = (int(st["iters"][0]), float(st["relres_true"][0]),
                             time.perf_counter() - ta)
            s.close()
            rows.append(res)
            if (f + 1) % max(1, n_fields // 10) == 0:
                self.log(f"[warmstart] eval: field {f + 1}/{n_fields}")
        return rows
