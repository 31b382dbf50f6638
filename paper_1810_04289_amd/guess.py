"""Learned Newton initial guess: training on the solver's own time steps, and evaluation
against the plain guesses at an equal Newton target.

The network (include/fsi_guess.h) corrects the linear extrapolation 2 y_{n-1} - y_{n-2};
features, targets, forward and backward passes and Adam steps all run in the library's
kernels.  Host NumPy only draws the initial weights and fits the 21 feature/output scales
(root mean squares over the training snapshots, read back once); torch holds the pooled
training rows and shuffles them into mini-batches.

The guess handed to Newton is whichever of the extrapolation, the network's guess and their
residual-optimal blend has the smallest nonlinear residual (at most three residual
evaluations): the residual test of §3 judges the network, and the extrapolation is the
fallback.

Evaluation at one step n, the same for every guess: Newton runs from the guess, with
Dirichlet values imposed, until ||F|| <= 1e-6 ||F(y_{n-1})||.  The absolute target is fixed
by the previous solution, so that a better guess is not held to a smaller relative base;
for the previous-state guess it is exactly the plain solver's relative test.

Run as a module for the comparison:
    python -m paper_1810_04289_amd.guess --case tube
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

CASES = {
    # straight compliant tube, ~2.1k vertices; ILU(3): with ILU(2) GMRES stagnates at the
    # first compliant step after the rigid start
    "tube": dict(mesh=lambda: W.tube_mesh(), opts=dict(nsub=4, overlap=1, ilu_level=3)),
    # depth-1 tree, subdomains of the depth-3 benchmark's size
    "tree1": dict(mesh=lambda: W.tree_mesh(depth=1, h=W.TREE_H[1]), opts=dict(nsub=33, overlap=1, ilu_level=3)),
    # depth-4 tree, ~593k vertices, subdomains of the depth-3 benchmark's size
    "tree4": dict(mesh=lambda: W.tree_mesh(depth=4, h=W.TREE_H[4]), opts=dict(nsub=768, overlap=1, ilu_level=3)),
}


def phase_features(t: float, dt: float, amp: float) -> np.ndarray:
    """Four features of the inflow at step time t: phase (sin, cos), peak velocity and its
    change over the step, both relative to the mean inflow and the base amplitude."""
    w = 2.0 * math.pi / PERIOD
    U = W.inflow_peak(t, amp=amp)
    dU = U - W.inflow_peak(t - dt, amp=amp)
    return np.array([math.sin(w * t), math.cos(w * t), U / U_MEAN, dU / (dt * w * U_AMP)], dtype=np.float32)


def layer_dims(nin=fsi.GUESS_NIN, hidden=128, nlayers=4, nout=7):
    return [(nin if l == 0 else hidden, nout if l == nlayers - 1 else hidden) for l in range(nlayers)]


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


class LearnedGuess:
    """The network, its scales and its training on pooled snapshot rows."""

    def __init__(self, V: int, hidden: int = 128, nlayers: int = 4, batch: int = 8192, seed: int = 0):
        self.V, self.batch = V, batch
        self.dims = layer_dims(hidden=hidden, nlayers=nlayers)
        self.net = fsi.MLP(fsi.GUESS_NIN, hidden, nlayers, 7, nmax=max(V, batch))
        self.net.set_params(init_params(self.dims, seed))
        self.scales = np.ones(21, dtype=np.float32)

    def close(self):
        self.net.close()

    def fit_scales(self, samples):
        """samples: [(y_{n-2}, y_{n-1}, y_n, tfeat)] with device state vectors [7V].  s is the
        RMS of y_{n-1} over the snapshots, the sigma floor 1e-3 of the mean step change, and
        the output gains start at 1."""
        def rms(v):
            return np.sqrt((v.reshape(-1, 7) ** 2).mean(0).cpu().numpy())
        s = np.sqrt(np.mean([rms(y1) ** 2 for _, y1, _, _ in samples], axis=0))
        sig = np.mean([rms(y1 - y2) for y2, y1, _, _ in samples], axis=0)
        sc = np.concatenate([np.where(s > 0, s, 1.0), 1e-3 * sig + 1e-30, np.ones(7)])
        self.scales = sc.astype(np.float32)
        self.net.set_scales(self.scales)

    GROUPS = {"u": (0, 1, 2), "p": (3,), "d": (4, 5, 6)}

    def fit_gains(self, samples, groups=("u",)):
        """Per component group (velocity u, pressure p, displacement d) the least-squares
        weight of the network's correction on held-out snapshots, clipped to [0, 1]; groups
        not listed get no correction.  By default only the velocity is corrected: pressure
        and displacement, well predicted within the training period, carry that period's
        start-up transient and come out worse than the extrapolation in the next one."""
        import torch
        num, den = np.zeros(7), np.zeros(7)
        for y2, y1, y, tf in samples:
            T = self.net.target(y, y1, y2)
            out = self.net.forward(self.net.features(y1, y2, tf))
            num += (T * out).sum(0).double().cpu().numpy()
            den += (out * out).sum(0).double().cpu().numpy()
        gain = np.zeros(7)
        for name in groups:
            g = list(self.GROUPS[name])
            gain[g] = np.clip(num[g].sum() / max(den[g].sum(), 1e-300), 0.0, 1.0)
        self.scales[14:21] = gain
        self.net.set_scales(self.scales)
        return gain

    def train(self, samples, steps: int = 2000, lr: float = 2e-3, lr_end: float = 1e-4, seed: int = 0, log=None):
        """Adam on mini-batches of rows drawn without replacement from all snapshots (a new
        permutation per epoch), learning rate on a cosine from lr to lr_end.  Returns the
        loss history."""
        import torch
        X = torch.cat([self.net.features(y1, y2, tf) for y2, y1, _, tf in samples])
        T = torch.cat([self.net.target(y, y1, y2) for y2, y1, y, _ in samples])
        N = X.shape[0]
        B = min(self.batch, N)
        gen = torch.Generator(device=X.device)
        gen.manual_seed(seed)
        hist, k, epoch = [], 0, 0
        while k < steps:
            perm = torch.randperm(N, generator=gen, device=X.device)
            Xp, Tp = X[perm].contiguous(), T[perm].contiguous()
            for b0 in range(0, N - B + 1, B):
                lr_k = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * k / steps))
                hist.append(self.net.train_step(Xp[b0:b0 + B], Tp[b0:b0 + B], lr=lr_k))
                k += 1
                if k >= steps:
                    break
            epoch += 1
            if log and (epoch % 10 == 0 or k >= steps):
                log(f"[guess] epoch {epoch} step {k}: loss {np.mean(hist[-(N // B):]):.4e}")
        return hist

    def predict(self, y1, y2, tfeat=None):
        return self.net.predict(y1, y2, tfeat)


def choose_guess(S, ge, gn):
    """The learned start: of the extrapolation ge, the network's guess gn and their blend
    ge + a (gn - ge), the one with the smallest residual.  a minimizes the residual's norm
    along the line through the two residuals, F(ge) + a (F(gn) - F(ge)), clipped to [0, 1];
    it costs one more residual evaluation.  Returns the guess, the network's residual norm
    and the a taken (0: extrapolation, 1: network)."""
    import torch
    Fe, Fn = S.residual(ge), S.residual(gn)
    if Fe is None:
        return gn.clone(), (math.inf if Fn is None else float(Fn.norm())), 1.0
    fe = float(Fe.norm())
    if Fn is None:
        return ge.clone(), math.inf, 0.0
    fn = float(Fn.norm())
    D = Fn - Fe
    dd = float(torch.dot(D, D))
    a = min(1.0, max(0.0, -float(torch.dot(Fe, D)) / dd)) if dd > 0 else 0.0
    best, g_best, a_best = fe, ge, 0.0
    if fn < best:
        best, g_best, a_best = fn, gn, 1.0
    if 0.0 < a < 1.0:
        gb = ge + a * (gn - ge)
        Fb = S.residual(gb)
        if Fb is not None and float(Fb.norm()) < best:
            best, g_best, a_best = float(Fb.norm()), gb, a
    return g_best.clone(), fn, a_best


class Stepper:
    """The plain solver on one case: backward Euler steps with the pulsatile inflow, the
    wall held rigid for the first two steps of a run from rest."""

    def __init__(self, case: str, dt: float):
        c = CASES[case]
        self.mesh = c["mesh"]()
        opts = dict(c["opts"], gmres_maxit=600, newton_maxit=30)
        self.s = fsi.Solver(self.mesh, W.physics_config1(), opts)
        self.dt = dt
        self.rigid = W.rigid_wall_mask(self.mesh)
        self.F = self.s.vec()

    def close(self):
        self.s.close()

    def set_step(self, k: int, amp: float, y_prev):
        import torch
        t = (k + 1) * self.dt
        g = torch.as_tensor(W.dirichlet_values(self.mesh, W.inflow_peak(t, amp=amp))).to(self.s.device)
        self.s.set_step(t, self.dt, y_prev, g, None, self.rigid if k < 2 else None)
        return t

    def fnorm(self, y):
        """||F(y)|| with the step's Dirichlet values imposed on a copy of y (infinite where
        the residual is undefined, e.g. an inverted element)."""
        tmp = y.clone()
        self.s.impose_dirichlet(tmp)
        if self.s.residual(tmp, self.F, check=False):
            return math.inf
        return float(self.F.norm())

    def residual(self, y):
        """F(y) with the step's Dirichlet values imposed on a copy of y (a new vector), or
        None where the residual is undefined."""
        tmp = y.clone()
        self.s.impose_dirichlet(tmp)
        if self.s.residual(tmp, self.F, check=False):
            return None
        return self.F.clone()

    def solve(self, y, rtol=1e-6, atol=0.0):
        self.s.set_newton_tol(rtol, atol)
        st, rc = self.s.newton_solve(y, check=False)
        return st, rc


def run(case="tube", dt=2e-3, train_steps=400, eval_steps=60, amp_eval=18.0, train_iters=2000, batch=8192, seed=0,
        skip=0, eval_offset=0, groups=("u",), log=print):
    """Trains on one inflow period of the plain solver's steps (amplitude 15 cm/s; the first
    `skip` steps of the start from rest left out), continues with amplitude amp_eval, and
    compares the guesses over eval_steps steps from eval_offset steps into the next period."""
    import torch
    S = Stepper(case, dt)
    V = S.mesh.nverts

    # the plain solver's trajectory; training uses steps 4 .. train_steps (wall compliant
    # for both previous states)
    t0 = time.perf_counter()
    ys = [S.s.vec()]
    for k in range(train_steps):
        S.set_step(k, U_AMP, ys[-1])
        y = ys[-1].clone()
        st, rc = S.solve(y)
        if rc:
            raise RuntimeError(f"plain step {k} failed: {rc}")
        ys.append(y)
        if log and (k + 1) % 50 == 0:
            log(f"[guess] plain step {k + 1}: NI {st['newton_iters']} LI {st['linear_iters']}")
    samples = [(ys[k - 1], ys[k], ys[k + 1], phase_features((k + 1) * dt, dt, U_AMP))
               for k in range(max(4, skip), train_steps)]
    t_data = time.perf_counter() - t0

    lg = LearnedGuess(V, batch=batch, seed=seed)
    lg.fit_scales(samples)
    # every tenth snapshot is held out for the gains
    fit = [x for i, x in enumerate(samples) if i % 10 != 5]
    held = [x for i, x in enumerate(samples) if i % 10 == 5]
    t0 = time.perf_counter()
    hist = lg.train(fit, steps=train_iters, seed=seed, log=log)
    gain = lg.fit_gains(held, groups)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    if log:
        log(f"[guess] output gains (u, p, d): {gain[0]:.3f} {gain[3]:.3f} {gain[4]:.3f}")

    names = ("previous", "extrapolation", "learned")
    rec = {n: [] for n in names}
    net_f0, picked, alphas, l2 = [], 0, [], {"extrapolation": [], "network": []}
    y1, y2 = ys[-1], ys[-2]
    nfit = len(fit)
    del ys, samples, fit, held
    for j in range(eval_offset):  # plain steps into the next period
        S.set_step(train_steps + j, amp_eval, y1)
        y = y1.clone()
        st, rc = S.solve(y)
        if rc:
            raise RuntimeError(f"plain step {train_steps + j} failed: {rc}")
        y2, y1 = y1, y
    for j in range(eval_steps):
        k = train_steps + eval_offset + j
        t = S.set_step(k, amp_eval, y1)
        target = 1e-6 * S.fnorm(y1)
        f_prev = S.fnorm(y1)
        out = {}
        for name in names:
            torch.cuda.synchronize()
            tt = time.perf_counter()
            if name == "previous":
                g = y1.clone()
            elif name == "extrapolation":
                g = lg.predict(y1, y2)
            else:
                ge = lg.predict(y1, y2)
                gn = lg.predict(y1, y2, phase_features(t, dt, amp_eval))
                g, fn, a = choose_guess(S, ge, gn)
                net_f0.append(fn / f_prev)
                alphas.append(a)
                picked += a > 0.0
            f0 = S.fnorm(g)
            st, rc = S.solve(g, rtol=0.0, atol=target)
            torch.cuda.synchronize()
            rec[name].append(dict(rc=rc, NI=st["newton_iters"], LI=st["linear_iters"], F0=f0 / f_prev,
                                  fnorm=st["fnorm"] / target, sec=time.perf_counter() - tt))
            out[name] = g
        # errors of the two predictions against the solution, relative to the step's change,
        # per component group (velocity, pressure, displacement)
        dy = (out["previous"] - y1).view(-1, 7)
        for nm, gg in (("extrapolation", ge), ("network", gn)):
            e = (gg - out["previous"]).view(-1, 7)
            l2[nm].append([float(e[:, a:b].norm() / max(float(dy[:, a:b].norm()), 1e-300))
                           for a, b in ((0, 3), (3, 4), (4, 7))])
        # the trajectory continues from the plain solver's solution
        y2, y1 = y1, out["previous"]
        if log and (j + 1) % 10 == 0:
            log(f"[guess] eval step {j + 1}: " + ", ".join(f"{n} NI {rec[n][-1]['NI']}" for n in names))

    summary = {"case": case, "groups": "".join(groups), "vertices": V, "unknowns": S.s.n, "dt": dt, "train_snapshots": nfit,
               "train_rows": nfit * V, "skip": skip, "adam_steps": train_iters, "batch": batch,
               "eval_steps": eval_steps, "amp_train": U_AMP, "amp_eval": amp_eval, "data_s": round(t_data, 2),
               "train_s": round(t_train, 2), "loss_first": float(np.mean(hist[:10])),
               "loss_last": float(np.mean(hist[-10:])), "gains_upd": [float(gain[0]), float(gain[3]), float(gain[4])],
               "network_F0_rel": float(np.mean(net_f0)), "eval_offset": eval_offset,
               "rel_err_upd": {nm: np.mean(v, axis=0).tolist() for nm, v in l2.items()},
               "network_picked": picked, "blend_a_mean": float(np.mean(alphas)) if alphas else None}
    for name, r in rec.items():
        summary[name] = {"failures": sum(1 for x in r if x["rc"]),
                         "max_fnorm_over_target": float(max(x["fnorm"] for x in r)),
                         "NI": float(np.mean([x["NI"] for x in r])),
                         "LI_per_step": float(np.mean([x["LI"] for x in r])),
                         "s_per_step": float(np.mean([x["sec"] for x in r])),
                         "F0_rel": float(np.mean([x["F0"] for x in r]))}
    S.close()
    lg.close()
    return summary


GUESS_NAMES = ("previous", "extrapolation", "learned")


def _summarize(rec, net_f0, picked, l2):
    out = {"network_F0_rel": float(np.mean(net_f0)) if net_f0 else None, "network_picked": int(picked),
           "rel_err_upd": {nm: np.mean(v, axis=0).tolist() for nm, v in l2.items() if v}}
    for name, r in rec.items():
        out[name] = {"failures": sum(1 for x in r if x["rc"]),
                     "max_fnorm_over_target": float(max(x["fnorm"] for x in r)),
                     "NI": float(np.mean([x["NI"] for x in r])),
                     "LI_per_step": float(np.mean([x["LI"] for x in r])),
                     "s_per_step": float(np.mean([x["sec"] for x in r])),
                     "F0_rel": float(np.mean([x["F0"] for x in r]))}
    return out


def run_resumable(case="tree4", state_in=None, state_out="guess_state.npz", budget_s=1000.0, dt=2e-3,
                  train_steps=400, eval_steps=40, amp_eval=18.0, train_iters=2000, batch=8192, skip=100,
                  eval_offset=100, groups=("u",), ksub=1024, seed=0, log=print):
    """The comparison of `run` split over several processes, for meshes whose period of
    plain steps takes longer than one process may run.  Each call continues from
    `state_in` (none: from rest), works until about `budget_s` seconds have passed, and
    writes its state to `state_out` (a NumPy archive without pickled objects):

    - while the trajectory is generated: the plain state y_k in FP64 and, for a seeded set
      of `ksub` vertices, their states at every step so far, which are the training rows
      (the network is node-wise, so a vertex subset gives whole training rows);
    - once it is complete, the network is trained on those rows in the same call, and the
      evaluation carries y_{n-1} in FP64, y_{n-1} - y_{n-2} in FP32 (the extrapolation's
      second state is rebuilt from it), the trained parameters and the records so far.

    Returns {"status": "partial", ...} or, after the last evaluation step, the summary of
    `run` with the plain steps' NI, LI and seconds added."""
    import torch
    t_start = time.perf_counter()
    elapsed = lambda: time.perf_counter() - t_start
    S = Stepper(case, dt)
    V = S.mesh.nverts
    dev = S.s.device
    st = dict(np.load(state_in, allow_pickle=False)) if state_in else {}
    if log:
        log(f"[guess] {case}: V={V}, solver ready after {elapsed():.0f}s; "
            + (f"resuming phase {int(st['phase'])} at {int(st['k'])}" if st else "starting from rest"))

    def save(**kw):
        np.savez(state_out, **kw)

    phase = int(st.get("phase", 0))
    plain = list(map(tuple, st["plain"])) if "plain" in st else []
    info = json.loads(str(st["info"])) if "info" in st else {}
    if phase == 0:
        k = int(st.get("k", 0))
        y = torch.as_tensor(st["y"]).to(dev) if "y" in st else S.s.vec()
        sub = st["sub"] if "sub" in st else np.sort(np.random.default_rng(seed).choice(V, ksub, replace=False))
        isub = torch.as_tensor(sub, device=dev)
        traj = list(st["traj"]) if "traj" in st else [y.view(-1, 7)[isub].cpu().numpy()]
        y_prev, per, k0 = None, 0.0, k
        while k < train_steps:
            # room for this step and the checkpoint; the last step also needs room for the
            # training and one evaluation step (about four plain steps)
            need = 1.5 * per + 30.0 + (120.0 + 4.0 * per if k == train_steps - 1 else 0.0)
            if k > k0 and elapsed() + need > budget_s:
                save(phase=0, k=k, y=y.cpu().numpy(), sub=sub, traj=np.array(traj), plain=np.array(plain))
                return {"status": "partial", "phase": 0, "k": k, "elapsed_s": round(elapsed(), 1)}
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S.set_step(k, U_AMP, y)
            yn = y.clone()
            stt, rc = S.solve(yn)
            torch.cuda.synchronize()
            per = time.perf_counter() - t0
            if rc:
                raise RuntimeError(f"plain step {k} failed: {rc}")
            plain.append((stt["newton_iters"], stt["linear_iters"], per))
            y_prev, y = y, yn
            traj.append(y.view(-1, 7)[isub].cpu().numpy())
            k += 1
            if log and k % 10 == 0:
                log(f"[guess] plain step {k}: NI {stt['newton_iters']} LI {stt['linear_iters']} {per:.2f}s "
                    f"(elapsed {elapsed():.0f}s)")
        # the trajectory is complete: train on the subset's rows
        tr = [torch.as_tensor(a).to(dev).reshape(-1) for a in traj]
        samples = [(tr[j - 1], tr[j], tr[j + 1], phase_features((j + 1) * dt, dt, U_AMP))
                   for j in range(max(4, skip), train_steps)]
        lg = LearnedGuess(V, batch=batch, seed=seed)
        lg.fit_scales(samples)
        fit = [x for i, x in enumerate(samples) if i % 10 != 5]
        held = [x for i, x in enumerate(samples) if i % 10 == 5]
        t0 = time.perf_counter()
        hist = lg.train(fit, steps=train_iters, seed=seed, log=log)
        gain = lg.fit_gains(held, groups)
        torch.cuda.synchronize()
        info = {"train_snapshots": len(fit), "train_rows": len(fit) * len(sub), "subset_vertices": len(sub),
                "train_s": round(time.perf_counter() - t0, 2), "loss_first": float(np.mean(hist[:10])),
                "loss_last": float(np.mean(hist[-10:])), "gains_upd": [float(gain[0]), float(gain[3]), float(gain[4])]}
        if log:
            log(f"[guess] trained: {info}")
        params, scales = lg.net.get_params()[0], lg.scales.copy()
        y1, y2 = y, y_prev
        j0, evals = -eval_offset, np.zeros((0, 3, 6))
        net_f0, picked, alphas, l2e, l2n = [], 0, [], [], []
        del tr, samples, fit, held, traj
    else:
        lg = LearnedGuess(V, batch=batch, seed=seed)
        params, scales = st["params"], st["scales"]
        lg.net.set_params(params)
        lg.scales = scales.astype(np.float32)
        lg.net.set_scales(lg.scales)
        y1 = torch.as_tensor(st["y"]).to(dev)
        y2 = y1 - torch.as_tensor(st["dy"]).to(dev).double()
        j0, evals = int(st["k"]), st["evals"]
        net_f0, picked, alphas = list(st["net_f0"]), int(st["picked"]), list(st["alphas"])
        l2e, l2n = list(st["l2e"]), list(st["l2n"])
    evals = list(evals)
    per = 0.0
    for j in range(j0, eval_steps):
        if j > j0 and elapsed() + 1.3 * per + 30.0 + (3.0 * per if j == 0 else 0.0) > budget_s:
            save(phase=1, k=j, y=y1.cpu().numpy(), dy=(y1 - y2).float().cpu().numpy(), params=params, scales=scales,
                 evals=np.array(evals), net_f0=np.array(net_f0), picked=picked, alphas=np.array(alphas),
                 l2e=np.array(l2e), l2n=np.array(l2n),
                 plain=np.array(plain), info=np.array(json.dumps(info)))
            return {"status": "partial", "phase": 1, "k": j, "elapsed_s": round(elapsed(), 1)}
        te = time.perf_counter()
        k = train_steps + eval_offset + j
        t = S.set_step(k, amp_eval, y1)
        if j < 0:  # plain steps into the next period before the comparison
            y = y1.clone()
            stt, rc = S.solve(y)
            if rc:
                raise RuntimeError(f"plain step {k} failed: {rc}")
            y2, y1 = y1, y
            per = time.perf_counter() - te
            if log and (j + eval_offset + 1) % 10 == 0:
                log(f"[guess] plain step {k + 1} (amplitude {amp_eval}): NI {stt['newton_iters']} "
                    f"LI {stt['linear_iters']} {per:.2f}s (elapsed {elapsed():.0f}s)")
            continue
        f_prev = S.fnorm(y1)
        target = 1e-6 * f_prev
        row, out = [], {}
        for name in GUESS_NAMES:
            torch.cuda.synchronize()
            tt = time.perf_counter()
            if name == "previous":
                g = y1.clone()
            elif name == "extrapolation":
                g = lg.predict(y1, y2)
            else:
                ge = lg.predict(y1, y2)
                gn = lg.predict(y1, y2, phase_features(t, dt, amp_eval))
                g, fn, a = choose_guess(S, ge, gn)
                net_f0.append(fn / f_prev)
                alphas.append(a)
                picked += a > 0.0
            f0 = S.fnorm(g)
            stt, rc = S.solve(g, rtol=0.0, atol=target)
            torch.cuda.synchronize()
            row.append((rc, stt["newton_iters"], stt["linear_iters"], f0 / f_prev, stt["fnorm"] / target,
                        time.perf_counter() - tt))
            out[name] = g
        evals.append(row)
        dy = (out["previous"] - y1).view(-1, 7)
        for lst, gg in ((l2e, ge), (l2n, gn)):
            e = (gg - out["previous"]).view(-1, 7)
            lst.append([float(e[:, a:b].norm() / max(float(dy[:, a:b].norm()), 1e-300))
                        for a, b in ((0, 3), (3, 4), (4, 7))])
        y2, y1 = y1, out["previous"]
        per = time.perf_counter() - te
        if log:
            log(f"[guess] eval step {j + 1}: " + ", ".join(f"{n} NI {r[1]} LI {r[2]} {r[5]:.2f}s"
                                                           for n, r in zip(GUESS_NAMES, row))
                + f" (elapsed {elapsed():.0f}s)")
    rec = {n: [dict(rc=r[i][0], NI=r[i][1], LI=r[i][2], F0=r[i][3], fnorm=r[i][4], sec=r[i][5]) for r in evals]
           for i, n in enumerate(GUESS_NAMES)}
    pl = np.array(plain)
    summary = {"case": case, "groups": "".join(groups), "vertices": V, "unknowns": S.s.n, "dt": dt,
               "train_steps": train_steps, "skip": skip, "adam_steps": train_iters, "batch": batch,
               "eval_steps": eval_steps, "eval_offset": eval_offset, "amp_train": U_AMP, "amp_eval": amp_eval,
               "plain_period": {"NI": float(pl[:, 0].mean()), "LI_per_step": float(pl[:, 1].mean()),
                                "s_per_step": float(pl[:, 2].mean())},
               **info, **_summarize(rec, net_f0, picked, {"extrapolation": l2e, "network": l2n}),
               "blend_a_mean": float(np.mean(alphas)) if alphas else None}
    S.close()
    lg.close()
    return {"status": "done", **summary}


def train_bench(batch=8192, steps=200, warmup=20, hidden=128, nlayers=4, seed=0):
    """Adam steps of the guess network on one seeded synthetic batch (FP32 rows of unit
    variance): time per step and the dense-layer FLOP rate it implies."""
    import torch
    rng = np.random.default_rng(seed)
    dims = layer_dims(hidden=hidden, nlayers=nlayers)
    net = fsi.MLP(fsi.GUESS_NIN, hidden, nlayers, 7, nmax=batch)
    net.set_params(init_params(dims, seed))
    X = torch.as_tensor(rng.standard_normal((batch, fsi.GUESS_NIN)).astype(np.float32)).cuda()
    T = torch.as_tensor(rng.standard_normal((batch, 7)).astype(np.float32)).cuda()
    for _ in range(warmup):
        net.train_step(X, T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        loss = net.train_step(X, T)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    # forward, weight gradients and input gradients (all layers but the first)
    mac = sum(a * b for a, b in dims)
    flops = 2.0 * batch * (2 * mac + sum(a * b for a, b in dims[1:]))
    net.close()
    return {"batch": batch, "dims": dims, "steps": steps, "ms_per_step": sec * 1e3, "gflop_per_step": flops / 1e9,
            "tflops": flops / sec / 1e12, "loss": loss}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", default="tube", choices=sorted(CASES))
    ap.add_argument("--dt", type=float, default=2e-3)
    ap.add_argument("--train-steps", type=int, default=400)
    ap.add_argument("--eval-steps", type=int, default=60)
    ap.add_argument("--amp-eval", type=float, default=18.0)
    ap.add_argument("--train-iters", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--skip", type=int, default=0, help="start-up steps left out of training")
    ap.add_argument("--eval-offset", type=int, default=0, help="plain steps into the next period before comparing")
    ap.add_argument("--groups", default="u", help="component groups the network corrects, e.g. u or upd")
    ap.add_argument("--train-bench", action="store_true", help="time Adam steps on a synthetic batch only")
    ap.add_argument("--resumable", action="store_true", help="run in parts that end after --budget seconds")
    ap.add_argument("--state-in", default=None, help="state written by the previous part")
    ap.add_argument("--state-out", default="guess_state.npz")
    ap.add_argument("--budget", type=float, default=1000.0)
    a = ap.parse_args()
    if a.train_bench:
        print(json.dumps(train_bench(batch=a.batch)), flush=True)
        return
    if a.resumable:
        out = run_resumable(case=a.case, state_in=a.state_in, state_out=a.state_out, budget_s=a.budget, dt=a.dt,
                            train_steps=a.train_steps, eval_steps=a.eval_steps, amp_eval=a.amp_eval,
                            train_iters=a.train_iters, batch=a.batch, skip=a.skip, eval_offset=a.eval_offset,
                            groups=tuple(a.groups), log=lambda *x: print(*x, file=sys.stderr, flush=True))
        print(json.dumps(out), flush=True)
        return
    out = run(case=a.case, dt=a.dt, train_steps=a.train_steps, eval_steps=a.eval_steps, amp_eval=a.amp_eval,
              train_iters=a.train_iters, batch=a.batch, skip=a.skip, eval_offset=a.eval_offset, groups=tuple(a.groups),
              log=lambda *x: print(*x, file=sys.stderr, flush=True))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
