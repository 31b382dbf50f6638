"""Learned Newton initial guess: training on the solver's own time steps, and evaluation
against the plain guesses at an equal Newton target.

The network (include/fsi_guess.h) corrects the linear extrapolation 2 y_{n-1} - y_{n-2};
features, targets, forward and backward passes and Adam steps all run in the library's
kernels.  Host NumPy only draws the initial weights and fits the 21 feature/output
scales (root mean squares over the training snapshots, read back once).

Evaluation at one step n (the same for every guess): Newton runs from the guess, with
Dirichlet values imposed, until ||F|| <= 1e-6 ||F(y_{n-1})|| -- an absolute target fixed
by the previous solution, so that a better guess is not held to a smaller relative base.

Run as a module for the comparison on the depth-1 tree:
    python -m paper_1810_04289_amd.guess --train-steps 40 --eval-steps 12
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import fsi
from . import workload as W

PERIOD, U_MEAN, U_AMP = 0.8, 30.0, 15.0


def phase_features(t: float, dt: float, amp: float) -> np.ndarray:
    """Four features of the inflow at step time t: phase (sin, cos), peak velocity and its
    rate of change, both relative to the mean inflow."""
    w = 2.0 * math.pi / PERIOD
    U = W.inflow_peak(t, amp=amp)
    dU = W.inflow_peak(t, amp=amp) - W.inflow_peak(t - dt, amp=amp)
    return np.array([math.sin(w * t), math.cos(w * t), U / U_MEAN, dU / (dt * w * U_AMP)], dtype=np.float32)


def init_params(dims, seed: int = 0, last_scale: float = 0.1) -> np.ndarray:
    """Glorot-uniform weights, zero biases; the last layer scaled down so that the untrained
    network barely moves the extrapolation."""
    rng = np.random.default_rng(seed)
    out = []
    for l, (a, b) in enumerate(dims):
        lim = math.sqrt(6.0 / (a + b)) * (last_scale if l == len(dims) - 1 else 1.0)
        out.append(rng.uniform(-lim, lim, a * b))
        out.append(np.zeros(b))
    return np.concatenate(out).astype(np.float32)


def layer_dims(nin=fsi.GUESS_NIN, hidden=128, nlayers=4, nout=7):
    return [(nin if l == 0 else hidden, nout if l == nlayers - 1 else hidden) for l in range(nlayers)]


class LearnedGuess:
    def __init__(self, V: int, hidden: int = 128, nlayers: int = 4, seed: int = 0):
        self.V = V
        self.dims = layer_dims(hidden=hidden, nlayers=nlayers)
        self.net = fsi.MLP(fsi.GUESS_NIN, hidden, nlayers, 7, nmax=V)
        self.net.set_params(init_params(self.dims, seed))
        self.scales = np.ones(21, dtype=np.float32)

    def fit_scales(self, triples):
        """triples: [(y_{n-2}, y_{n-1}, y_n)] device tensors [7V]."""
        a = np.stack([t[1].cpu().numpy().reshape(-1, 7) for t in triples])
        d = np.stack([(t[1] - t[2]).cpu().numpy().reshape(-1, 7) for t in triples])
        r = np.stack([(t[2] - 2 * t[1] + t[0]).cpu().numpy().reshape(-1, 7) for t in triples])
        rms = lambda x: np.sqrt(np.mean(x.reshape(-1, 7) ** 2, axis=0))
        sc = np.concatenate([rms(a), rms(d), rms(r)])
        sc = np.where(sc > 0, sc, 1.0)
        self.scales = sc.astype(np.float32)
        self.net.set_scales(self.scales)

    def train(self, samples, steps: int = 300, lr: float = 1e-3, seed: int = 0, log=None):
        """samples: [(y_{n-2}, y_{n-1}, y_n, tfeat)]; one Adam step per snapshot, snapshots in
        a seeded random order per epoch.  Returns the loss history."""
        data = []
        for y2, y1, y, tf in samples:
            # features from (y1, y2) and the target; kept on the device for the epochs
            data.append((self.net.features(y1, y2, tf), self.net.target(y, y1, y2)))
        rng = np.random.default_rng(seed)
        hist, k = [], 0
        while k < steps:
            for i in rng.permutation(len(data)):
                if k >= steps:
                    break
                hist.append(self.net.train_step(data[i][0], data[i][1], lr=lr))
                k += 1
            if log:
                log(f"[guess] train step {k}: loss {np.mean(hist[-len(data):]):.4e}")
        return hist

    def predict(self, y1, y2, tfeat=None):
        return self.net.predict(y1, y2, tfeat)


def _norm(s, y, F):
    s.residual(y, F, check=False)
    return float(F.norm())


def run(depth=1, train_steps=40, eval_steps=12, amp_eval=18.0, nsub=None, ilu=3, train_iters=400, seed=0,
        log=print):
    import torch
    dt = 1e-3
    mesh = W.tree_mesh(depth=depth, h=W.TREE_H[depth])
    if nsub is None:
        nsub = max(1, round(256 * mesh.nverts / 202715))
    ph = W.physics_config1()
    s = fsi.Solver(mesh, ph, dict(nsub=nsub, overlap=1, ilu_level=ilu, gmres_maxit=600, newton_maxit=30))
    dev = s.device
    rigid = W.rigid_wall_mask(mesh)

    def trajectory(amp, nsteps, on_step=None):
        ys = [torch.zeros(s.n, dtype=torch.float64, device=dev)]
        for k in range(nsteps):
            t = (k + 1) * dt
            g = torch.as_tensor(W.dirichlet_values(mesh, W.inflow_peak(t, amp=amp))).to(dev)
            s.set_step(t, dt, ys[-1], g, None, rigid if k < 2 else None)
            if on_step is not None and k >= 4:
                on_step(k, t, ys, amp)
            s.set_newton_tol(1e-6, 0.0)
            y = ys[-1].clone()
            st, rc = s.newton_solve(y, check=False)
            if rc:
                raise RuntimeError(f"plain step {k} failed: {rc}")
            ys.append(y)
        return ys

    # training data: the plain solver's own steps (compliant steps from k = 4 on)
    t0 = time.perf_counter()
    ys = trajectory(U_AMP, train_steps + 4)
    samples = [(ys[k - 1], ys[k], ys[k + 1], phase_features((k + 1) * dt, dt, U_AMP)) for k in range(4, len(ys) - 1)]
    lg = LearnedGuess(mesh.nverts, seed=seed)
    lg.fit_scales([(a, b, c) for a, b, c, _ in samples])
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    hist = lg.train(samples, steps=train_iters, seed=seed, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0

    # evaluation on a perturbed inflow: each guess solved to the same absolute target
    F = torch.empty(s.n, dtype=torch.float64, device=dev)
    rec = {"previous": [], "extrapolation": [], "learned": []}
    f0s = {"previous": [], "extrapolation": [], "learned": []}

    def compare(k, t, ys_, amp):
        y1, y2 = ys_[-1], ys_[-2]
        tmp = y1.clone()
        s.impose_dirichlet(tmp)
        target = 1e-6 * _norm(s, tmp, F)
        guesses = {"previous": y1.clone(), "extrapolation": lg.predict(y1, y2),
                   "learned": lg.predict(y1, y2, phase_features(t, dt, amp))}
        for name, g in guesses.items():
            tmp.copy_(g)
            s.impose_dirichlet(tmp)
            f0s[name].append(_norm(s, tmp, F))
            s.set_newton_tol(0.0, target)
            torch.cuda.synchronize()
            tt = time.perf_counter()
            st, rc = s.newton_solve(g, check=False)
            torch.cuda.synchronize()
            rec[name].append(dict(rc=rc, NI=st["newton_iters"], LI=st["linear_iters"], sec=time.perf_counter() - tt))

    trajectory(amp_eval, eval_steps + 4, on_step=compare)
    summary = {"depth": depth, "vertices": mesh.nverts, "unknowns": s.n, "nsub": nsub, "ilu": ilu,
               "train_snapshots": len(samples), "train_adam_steps": train_iters, "eval_steps": len(rec["learned"]),
               "amp_train": U_AMP, "amp_eval": amp_eval, "data_s": round(t_data, 2), "train_s": round(t_train, 2),
               "loss_first": hist[0], "loss_last": float(np.mean(hist[-len(samples):]))}
    for name, r in rec.items():
        summary[name] = {"failures": sum(1 for x in r if x["rc"]), "NI": float(np.mean([x["NI"] for x in r])),
                         "LI_per_step": float(np.mean([x["LI"] for x in r])),
                         "s_per_step": float(np.mean([x["sec"] for x in r])),
                         "F0_rel": float(np.mean(np.array(f0s[name]) / np.array(f0s["previous"])))}
    s.close()
    lg.net.close()
    return summary


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--depth", type=int, default=1)
    ap.add_argument("--train-steps", type=int, default=40)
    ap.add_argument("--eval-steps", type=int, default=12)
    ap.add_argument("--amp-eval", type=float, default=18.0)
    ap.add_argument("--train-iters", type=int, default=400)
    a = ap.parse_args()
    out = run(depth=a.depth, train_steps=a.train_steps, eval_steps=a.eval_steps, amp_eval=a.amp_eval,
              train_iters=a.train_iters, log=lambda *x: print(*x, file=sys.stderr, flush=True))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
