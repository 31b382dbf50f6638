"""Batched Schwarz on uneven subdomains: setup, sweeps and GMRES on one MI355X.

Workload: a bifurcating tree (depth 5 by default: about 1.47M vertices) cut into 512
subdomains of seeded lognormal size (log-standard deviation 0.5, mean about 2,900
vertices), overlap 2, ILU(l) (0 by default), sweeps in FP32 from rounded factors under FP64
GMRES.  The Jacobian is the first time step's from rest with the wall held rigid, or
(--compliant) the first compliant step's after two rigid-wall steps from rest.

Every subdomain's factorization is one launch (one workgroup per subdomain), and each
sweep is one launch over all subdomains; the sweep schedule is picked by the library's
tuner.  Prints one JSON line: subdomain sizes, factorization and sweep times, the sweeps'
algorithmic bytes and rate, and GMRES iterations and time.

    python -m paper_1810_04289_amd.schwarz_bench [--depth 5] [--nsub 512] [--ilu 0] [--compliant]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import fsi
from . import workload as W
from .metrics import sweep_bytes

HBM_PEAK = 8000.0  # GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run(depth=5, h=None, nsub=512, sigma=0.5, overlap=2, ilu=0, precision=fsi.PREC_FP32, seed=0, reps=20,
        compliant=False):
    import torch
    t0 = time.perf_counter()
    mesh = W.tree_mesh(depth=depth, h=W.TREE_H[depth] if h is None else h)
    part = W.uneven_partition(mesh, nsub, sigma=sigma, seed=seed)
    log(f"[schwarz] mesh V={mesh.nverts} E={mesh.ntets}, {nsub} subdomains ({time.perf_counter() - t0:.0f}s)")
    t0 = time.perf_counter()
    s = fsi.Solver(mesh, W.physics_config1(), dict(nsub=nsub, overlap=overlap, ilu_level=ilu, part=part,
                                                   precision=precision, gmres_maxit=600))
    log(f"[schwarz] solver set up ({time.perf_counter() - t0:.0f}s)")
    dt = 1e-3
    y_old = s.vec()
    k0 = 0
    if compliant:  # two rigid-wall steps from rest, then the first compliant step's Jacobian
        for k0 in range(2):
            s.set_step((k0 + 1) * dt, dt, y_old, s.vec(W.dirichlet_values(mesh, W.inflow_peak((k0 + 1) * dt))), None,
                       W.rigid_wall_mask(mesh))
            y = y_old.clone()
            st0, rc = s.newton_solve(y, check=False)
            log(f"[schwarz] rigid start step {k0}: rc {rc} NI {st0['newton_iters']} "
                f"LI {st0['lin_hist'][:st0['newton_iters']]}")
            if rc:
                raise RuntimeError(f"rigid start step {k0} failed with status {rc}")
            y_old = y
        k0 = 2
    g = s.vec(W.dirichlet_values(mesh, W.inflow_peak((k0 + 1) * dt)))
    s.set_step((k0 + 1) * dt, dt, y_old, g, None, None if compliant else W.rigid_wall_mask(mesh))
    y = y_old.clone()
    s.impose_dirichlet(y)
    F = s.vec()
    s.residual(y, F)
    s.jacobian(y)

    def timed(fn, n):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / n

    s.pc_setup()
    t_setup = timed(s.pc_setup, 3)
    best, us = s.pc_tune(3)
    z = s.vec()
    t_apply = timed(lambda: s.pc_apply(F, z), reps)
    s.prof_enable(True)
    for _ in range(reps):
        s.pc_apply(F, z)
    torch.cuda.synchronize()
    kern = {k: s.prof_get(k) for k in ("ilu_fwd", "ilu_bwd")}
    s.prof_enable(False)
    rhs = -F
    x = s.vec()
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = s.gmres(rhs, x)
    torch.cuda.synchronize()
    t_gmres = time.perf_counter() - t
    sw = sweep_bytes(s, precision)
    pc = s.pc_get(factors=False)
    owned = np.bincount(part, minlength=nsub)
    ext = np.diff(pc["sub_ptr"])
    out = {"workload": f"tree depth {depth}, {mesh.nverts} vertices, {s.n} unknowns, {nsub} uneven subdomains "
                       f"(lognormal sigma {sigma}, mean {mesh.nverts / nsub:.0f} vertices), overlap {overlap}, "
                       f"ILU({ilu}), sweeps {['FP64', 'FP32', 'BF16 factors'][precision]}, "
                       + ("compliant wall, first compliant step after two rigid ones" if compliant
                          else "rigid wall, first step"),
           "owned": {"min": int(owned.min()), "mean": float(owned.mean()), "max": int(owned.max())},
           "extended": {"min": int(ext.min()), "mean": float(ext.mean()), "max": int(ext.max())},
           "local_blocks": sw["local_blocks"], "pc_setup_ms": round(1e3 * t_setup, 2),
           "sweep_schedule": {"best_blocks_per_task": best, "us_per_apply": {str(k): round(v, 1) for k, v in us.items()}},
           "pc_apply_ms": round(1e3 * t_apply, 3)}
    for k, (ms, cnt) in kern.items():
        avg = ms / cnt * 1e-3
        out[k] = {"avg_us": round(1e6 * avg, 1), "bytes": sw[k], "GBs": round(sw[k] / avg / 1e9, 1),
                  "frac_hbm": round(sw[k] / avg / 1e9 / HBM_PEAK, 4)}
    out["gmres"] = {"iters": st["iters"], "converged": st["converged"],
                    "true_rel": st["rnorm_true"] / st["rnorm0"], "s": round(t_gmres, 4)}
    s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--depth", type=int, default=5)
    ap.add_argument("--h", type=float, default=None, help="lattice spacing (default: the depth's workload spacing)")
    ap.add_argument("--nsub", type=int, default=512)
    ap.add_argument("--compliant", action="store_true")
    ap.add_argument("--ilu", type=int, default=0)
    ap.add_argument("--overlap", type=int, default=2)
    ap.add_argument("--precision", type=int, default=fsi.PREC_FP32)
    a = ap.parse_args()
    print(json.dumps(run(depth=a.depth, h=a.h, nsub=a.nsub, overlap=a.overlap, ilu=a.ilu,
                         precision=a.precision, compliant=a.compliant)), flush=True)


if __name__ == "__main__":
    main()
