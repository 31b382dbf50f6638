"""Benchmark: seconds per implicit FSI time step at Newton rtol 1e-6 on one MI355X.

Workload: the seeded synthetic bifurcating compliant tree of depth 3 (8 outlets, radius
ratio 0.79, branch angles 25-45 deg, one-lattice-cell wall), about 203k vertices and 1.37M
active unknowns, pulsatile inflow 30 + 15 sin(2 pi t / 0.8) cm/s, traction-free planar outlets,
dt = 1e-3 s, 256 restricted additive Schwarz subdomains (one per compute unit) with overlap
1 and block ILU(l) subdomain solves (l = 3 by default: lower fill levels stall GMRES(30) on
this wall with 64 subdomains, and are slower with 256).

A step is one whole Newton-Krylov-Schwarz solve (residuals, exact Jacobians, Schwarz
setups, GMRES iterations, line searches) through the library's C ABI.  Before the warmup
the flow is started by two rigid-wall steps from rest (untimed setup of the initial
state).  Inputs (mesh, step Dirichlet data) are resident in HBM before timing starts.

Prints one JSON line.  With --gpus N > 1 it exits: the library runs on one GPU.
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

from paper_1810_04289_amd import workload as W  # noqa: E402
from paper_1810_04289_amd.metrics import spmv_bytes, sweep_bytes  # noqa: E402

METRIC = "sec per implicit FSI time step @1e-6 Newton rtol; SpMV/ILU HBM GB/s %peak"
HBM_PEAK = 8000.0  # GB/s, MI355X published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stored_traffic(kernel: str, precision: int, config: dict):
    """HBM bytes per launch measured with rocprofv3 counters, from a profile on record
    (profiles/ilu_sweep_traffic_tree3*.json, one per sweep schedule) taken with the current
    sweep source, the same sweep precision and the same Schwarz configuration (subdomains,
    fill level, overlap, ordering, sweep schedule); None if there is none."""
    import glob
    import hashlib
    src = open(os.path.join(ROOT, "paper_1810_04289_amd", "csrc", "ilu.hip"), "rb").read()
    sha = hashlib.sha256(src).hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "ilu_sweep_traffic_tree3*.json"))):
        try:
            rec = json.load(open(path))
        except (OSError, ValueError):
            continue
        if rec.get("ilu_hip_sha256") != sha or rec.get("precision", 0) != precision:
            continue
        rec_cfg = rec.get("config", {"nsub": 256, "ilu_level": 3, "overlap": 1, "ordering": 0})
        if any(rec_cfg.get(k) != config.get(k) for k in ("nsub", "ilu_level", "overlap", "ordering", "sweep_mb")):
            continue
        k = rec.get("kernels", {}).get(kernel)
        if k is not None:
            return k.get("hbm_bytes_per_launch")
    return None


ORDERING = {0: "RCM", 1: "1WD"}


def cpu_baseline(counts: dict, ilu_level: int, V_work: int, nsub_work: int, overlap: int = 1,
                 ordering: int = 0) -> dict:
    """The oracle (1 host core) timed on a bounded sample and scaled to the workload.

    Sample: the depth-1 tree (about 26k vertices, cut into subdomains of the workload's
    size), one call each of FuncEval, JacEval and PCSetUp and 8 GMRES iterations; the
    per-call times are combined with the GPU run's per-step call counts and scaled by the
    vertex ratio (every phase is linear in the mesh size at fixed subdomain size).
    """
    import oracle as O
    O.build()
    m = W.tree_mesh(depth=1, h=W.TREE_H[1])
    ph = W.physics_config1()
    ns = max(1, round(nsub_work * m.nverts / V_work))
    o = O.Oracle(m, ph, dict(nsub=ns, overlap=overlap, ilu_level=ilu_level, ordering=ordering, gmres_rtol=0.0,
                             gmres_maxit=8))
    g = W.dirichlet_values(m, 30.0)
    y0 = W.perturbed_state(m, np.zeros(m.n), seed=1)
    o.set_step(1e-3, 1e-3, np.zeros(m.n), g)
    y = o.impose_dirichlet(y0)
    t0 = time.perf_counter()
    F = o.residual(y)
    t_fe = time.perf_counter() - t0
    t0 = time.perf_counter()
    o.jacobian(y)
    t_je = time.perf_counter() - t0
    t0 = time.perf_counter()
    o.pc_setup()
    t_ps = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, st = o.gmres(-F)
    t_it = (time.perf_counter() - t0) / max(st["iters"], 1)
    per_step = (counts["funceval"] * t_fe + counts["jaceval"] * t_je + counts["pcsetup"] * t_ps +
                counts["gmres_iters"] * t_it)
    scale = V_work / m.nverts
    return {"value": per_step * scale, "unit": "s/step", "cores": 1, "kind": "oracle",
            "sample": (f"oracle phases on the depth-1 tree ({m.nverts} vertices, {ns} subdomains, ILU({ilu_level}), "
                       f"{ORDERING[ordering]} ordering): "
                       f"FuncEval {t_fe:.3f}s, JacEval {t_je:.3f}s, PCSetUp {t_ps:.3f}s, GMRES iter {t_it:.4f}s; "
                       f"combined with the GPU run's per-step counts {counts} and scaled by {scale:.2f} "
                       f"(vertex ratio)"),
            "cpu": _cpu_model()}


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--depth", type=int, default=3)
    ap.add_argument("--nsub", type=int, default=256)
    ap.add_argument("--ilu", type=int, default=3)
    ap.add_argument("--dt", type=float, default=1e-3)
    ap.add_argument("--overlap", type=int, default=1)
    ap.add_argument("--ordering", type=int, default=0, help="subdomain ordering: 0 RCM, 1 one-way dissection")
    ap.add_argument("--jac-lag", type=int, default=1, help="Newton iterations per Jacobian and Schwarz setup")
    ap.add_argument("--precision", type=int, default=0,
                    help="Schwarz sweep precision: 0 FP64, 1 FP32 factors and sweeps, 2 BF16 factors, FP32 sweeps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the row-length rule's sweep schedule")
    ap.add_argument("--sweep-mb", type=int, default=0,
                    help="use this sweep schedule (blocks per task) instead of tuning, e.g. to take "
                         "counters on the schedule a tuned run chose")
    ap.add_argument("--graphs", action="store_true", help="GMRES Arnoldi steps as captured graphs")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before timing, run a plain elementwise copy of this many MiB three times "
                         "(reference dispatch for scaling rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library does not "
              "shard the Schwarz subdomains over several GPUs.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1810_04289_amd import fsi
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)

    t0 = time.perf_counter()
    mesh = W.tree_mesh(depth=args.depth, h=W.TREE_H[args.depth])
    ph = W.physics_config1()
    opts = dict(nsub=args.nsub, overlap=args.overlap, ilu_level=args.ilu, ordering=args.ordering, jac_lag=args.jac_lag,
                gmres_restart=30,
                gmres_maxit=600,
                gmres_rtol=1e-3, newton_rtol=1e-6, newton_maxit=20, precision=args.precision)
    s = fsi.Solver(mesh, ph, opts)
    if args.graphs:
        s.set_graphs(True)
    log(f"[bench] mesh V={mesh.nverts} E={mesh.ntets} n={s.n} nnzb={s.nnzb} setup {time.perf_counter() - t0:.1f}s")

    dt = args.dt
    nsteps = 2 + args.warmup + args.steps
    G = [torch.as_tensor(W.dirichlet_values(mesh, W.inflow_peak((k + 1) * dt))).to(dev) for k in range(nsteps + 1)]
    rigid = W.rigid_wall_mask(mesh)
    y_old = torch.zeros(s.n, dtype=torch.float64, device=dev)
    y = torch.empty_like(y_old)

    def step(k, mask=None):
        s.set_step((k + 1) * dt, dt, y_old, G[k], None, mask)
        y.copy_(y_old)
        st, rc = s.newton_solve(y, check=False)
        if rc != 0:
            raise RuntimeError(f"step {k} failed with status {rc}: {st}")
        y_old.copy_(y)
        return st

    for k in range(2):
        st = step(k, rigid)
        log(f"[bench] rigid start step {k}: NI {st['newton_iters']} LI {st['lin_hist'][:st['newton_iters']]}")
    for k in range(2, 2 + args.warmup):
        st = step(k)
        log(f"[bench] warmup step {k}: NI {st['newton_iters']} LI {st['lin_hist'][:st['newton_iters']]}")

    tune = None
    if args.sweep_mb:
        s.pc_select(args.sweep_mb)
        tune = {"best_blocks_per_task": args.sweep_mb, "selected": True}
        log(f"[bench] sweep schedule selected: {args.sweep_mb} blocks per task")
    elif not args.no_tune:  # sweep schedule timed on the last step's factors, outside the timed steps
        best, us = s.pc_tune(3)
        tune = {"best_blocks_per_task": best, "us_per_apply": {str(k): round(v, 1) for k, v in us.items()}}
        log(f"[bench] sweep schedule: {tune}")

    if args.calib_copy_mib > 0:
        a = torch.ones(args.calib_copy_mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b

    # kernel times from HIP events over the timed steps; with graphs (whose kernels events
    # cannot bracket) from one more, eager, step after them
    s.prof_enable(not args.graphs)
    torch.cuda.synchronize()
    stats = []
    t_start = time.perf_counter()
    for k in range(2 + args.warmup, nsteps):
        stats.append(step(k))
        log(f"[bench] step {k}: NI {stats[-1]['newton_iters']} LI {stats[-1]['lin_hist'][:stats[-1]['newton_iters']]} "
            f"cuts {stats[-1]['line_search_cuts']}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    sec_per_step = elapsed / args.steps
    if args.graphs:
        s.prof_enable(True)
        step(nsteps)
        torch.cuda.synchronize()

    kernels = {}
    for name in ("ilu_fwd", "ilu_bwd", "ilu_factor", "spmv", "elem_jac_fluid", "elem_jac_solid", "jac_gather",
                 "elem_res_fluid", "elem_res_solid", "res_gather", "mdot", "vupdate", "vupdate_mdot",
                 "vupdate_sqnorm"):
        ms, cnt = s.prof_get(name)
        kernels[name] = {"total_ms": round(ms, 3), "count": cnt, "avg_us": round(1e3 * ms / cnt, 2) if cnt else None}
    s.prof_enable(False)

    sw = sweep_bytes(s, args.precision)
    dom = max(("ilu_fwd", "ilu_bwd"), key=lambda k: kernels[k]["total_ms"])
    t_dom = kernels[dom]["avg_us"]
    achieved = sw[dom] / (t_dom * 1e-6) / 1e9 if t_dom else None
    other = "ilu_bwd" if dom == "ilu_fwd" else "ilu_fwd"
    t_other = kernels[other]["avg_us"]
    sb = spmv_bytes(s)
    spmv_gbs = sb / (kernels["spmv"]["avg_us"] * 1e-6) / 1e9 if kernels["spmv"]["avg_us"] else None

    NI = float(np.mean([x["newton_iters"] for x in stats]))
    LI = float(np.sum([x["linear_iters"] for x in stats]) / max(1, np.sum([x["newton_iters"] for x in stats])))
    counts = {
        "funceval": float(np.mean([x["newton_iters"] + 1 + x["line_search_cuts"] for x in stats])),
        "jaceval": float(np.mean([-(-x["newton_iters"] // args.jac_lag) for x in stats])),
        "pcsetup": float(np.mean([-(-x["newton_iters"] // args.jac_lag) for x in stats])),
        "gmres_iters": float(np.mean([x["linear_iters"] for x in stats])),
    }
    phases = {k: float(np.mean([x[k] for x in stats])) for k in
              ("t_funceval", "t_jaceval", "t_pcsetup", "t_pcapply", "t_kspsolve", "t_kspsetup")}
    schwarz_cfg = dict(nsub=args.nsub, ilu_level=args.ilu, overlap=args.overlap, ordering=args.ordering,
                       sweep_mb=tune["best_blocks_per_task"] if tune else None)
    out = {
        "metric": METRIC, "value": round(sec_per_step, 5), "unit": "s/step", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * sec_per_step, 2), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {0: "f64", 1: "f64 (f32 Schwarz sweeps)", 2: "f64 (bf16 factors, f32 Schwarz sweeps)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"bifurcating compliant tree depth {args.depth}, {mesh.nverts} vertices, "
                               f"{mesh.ntets} tets, {s.n} unknowns, dt {dt}, {args.nsub} RAS subdomains overlap {args.overlap}, "
                               f"ILU({args.ilu}), {ORDERING[args.ordering]} ordering, GMRES(30) rtol 1e-3, Newton rtol 1e-6"
                               + {0: "", 1: ", FP32 sweeps", 2: ", BF16 factors with FP32 sweeps"}[args.precision],
                   "nverts": mesh.nverts, "ntets": mesh.ntets, "n": s.n, "nnzb": s.nnzb, "nsub": args.nsub,
                   "ilu_level": args.ilu, "overlap": args.overlap, "ordering": args.ordering, "jac_lag": args.jac_lag,
                   "dt": dt, "local_blocks": sw["local_blocks"],
                   "local_rows": sw["local_rows"]},
        "NI": NI, "LI": round(LI, 2), "sweep_schedule": tune, "graphs": bool(args.graphs),
        "kernel_times_from": "one eager step after the timed steps" if args.graphs else "the timed steps", "phases_s_per_step": {k: round(v, 5) for k, v in phases.items()},
        "roofline": {"bound": "hbm", "kernel": dom,
                     "achieved": round(achieved, 1) if achieved else None, "peak": HBM_PEAK, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK, 4) if achieved else None,
                     "traffic": stored_traffic(dom, args.precision, schwarz_cfg), "bytes_per_launch": sw[dom], "avg_us": t_dom,
                     "other_sweep": {"kernel": other, "bytes_per_launch": sw[other], "avg_us": t_other,
                                     "achieved": round(sw[other] / (t_other * 1e-6) / 1e9, 1) if t_other else None,
                                     "traffic": stored_traffic(other, args.precision, schwarz_cfg)}},
        "spmv": {"achieved_GBs": round(spmv_gbs, 1) if spmv_gbs else None, "bytes": sb,
                 "frac": round(spmv_gbs / HBM_PEAK, 4) if spmv_gbs else None},
        "kernels": kernels,
    }
    if args.precision != 0:
        out["error_vs_fp64"] = error_vs_fp64(s, fsi, mesh, ph, opts, G, rigid, dt, nsteps, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(counts, args.ilu, mesh.nverts, args.nsub, args.overlap, args.ordering)
    print(json.dumps(out), flush=True)
    s.close()


def error_vs_fp64(s, fsi, mesh, ph, opts, G, rigid, dt, nsteps, dev):
    """Outside the timed steps: every step of the run taken from the same state (the FP64
    path's) by the rounded-preconditioner solver s and by an FP64 solver; the relative
    2-norm difference of their results per step, and the Newton tolerance both meet."""
    import torch
    s64 = fsi.Solver(mesh, ph, dict(opts, precision=0))
    y_old = torch.zeros(s.n, dtype=torch.float64, device=dev)
    ya, yb = torch.empty_like(y_old), torch.empty_like(y_old)
    rel = []
    for k in range(nsteps):
        mask = rigid if k < 2 else None
        for solver, y in ((s64, ya), (s, yb)):
            solver.set_step((k + 1) * dt, dt, y_old, G[k], None, mask)
            y.copy_(y_old)
            st, rc = solver.newton_solve(y, check=False)
            if rc != 0:
                raise RuntimeError(f"comparison step {k} failed with status {rc}")
        rel.append(float(torch.linalg.vector_norm(yb - ya) / torch.linalg.vector_norm(ya)))
        y_old.copy_(ya)
        log(f"[bench] step {k}: rounded-preconditioner state vs FP64 rel {rel[-1]:.3e}")
    s64.close()
    return {"per_step_rel_2norm": [float(f"{r:.3e}") for r in rel], "max": float(f"{max(rel):.3e}"),
            "newton_rtol": opts["newton_rtol"],
            "note": "each step from the FP64 path's previous state; both solves meet the same Newton tolerance"}


if __name__ == "__main__":
    main()
