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


def oracle_phase_times(m, nsub: int, ilu_level: int, overlap: int, ordering: int) -> dict:
    """Seconds of one oracle call of FuncEval, JacEval and PCSetUp on mesh m, and of one GMRES
    iteration averaged over a whole restart cycle of 30 (the Gram-Schmidt cost grows with
    the basis index), at a perturbed rest state of the first step."""
    import oracle as O
    O.build()
    ph = W.physics_config1()
    o = O.Oracle(m, ph, dict(nsub=nsub, overlap=overlap, ilu_level=ilu_level, ordering=ordering, gmres_rtol=0.0,
                             gmres_maxit=30, gmres_restart=30))
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
    return {"funceval": t_fe, "jaceval": t_je, "pcsetup": t_ps, "gmres_iter": t_it, "gmres_iters_timed": st["iters"]}


def per_step(t: dict, counts: dict) -> float:
    return (counts["funceval"] * t["funceval"] + counts["jaceval"] * t["jaceval"] + counts["pcsetup"] * t["pcsetup"] +
            counts["gmres_iters"] * t["gmres_iter"])


def cpu_baseline(counts: dict, ilu_level: int, V_work: int, nsub_work: int, overlap: int = 1,
                 ordering: int = 0, small_mesh=None) -> dict:
    """The oracle (1 host core) timed on a bounded sample and scaled to the workload.

    Sample: the depth-1 tree (about 26k vertices, cut into subdomains of the workload's
    size), one call each of FuncEval, JacEval and PCSetUp and a 30-iteration GMRES cycle;
    the per-call times are combined with the GPU run's per-step call counts and scaled by
    the vertex ratio (every phase is linear in the mesh size at fixed subdomain size).
    `bench.py --validate-cpu-baseline` checks that scaling against the oracle's phases
    timed on the workload's own mesh.
    """
    if small_mesh is not None:  # a workload small enough to time whole
        t = oracle_phase_times(small_mesh, nsub_work, ilu_level, overlap, ordering)
        return {"value": per_step(t, counts), "unit": "s/step", "cores": 1, "kind": "oracle",
                "sample": (f"oracle phases on the workload's own mesh ({small_mesh.nverts} vertices): FuncEval "
                           f"{t['funceval']:.4f}s, JacEval {t['jaceval']:.4f}s, PCSetUp {t['pcsetup']:.4f}s, GMRES iter "
                           f"{t['gmres_iter']:.5f}s (30-iteration cycle); combined with the GPU run's per-step counts "
                           f"{counts}"),
                "cpu": _cpu_model()}
    m = W.tree_mesh(depth=1, h=W.TREE_H[1])
    ns = max(1, round(nsub_work * m.nverts / V_work))
    t = oracle_phase_times(m, ns, ilu_level, overlap, ordering)
    scale = V_work / m.nverts
    corr, src = validation_factors(V_work, nsub_work, ilu_level, overlap, ordering)
    tc = {k: t[k] * scale * corr.get(k, 1.0) for k in ("funceval", "jaceval", "pcsetup", "gmres_iter")}
    return {"value": per_step(tc, counts), "unit": "s/step", "cores": 1, "kind": "oracle",
            "uncorrected_value": per_step(t, counts) * scale,
            "sample": (f"oracle phases on the depth-1 tree ({m.nverts} vertices, {ns} subdomains, ILU({ilu_level}), "
                       f"{ORDERING[ordering]} ordering): FuncEval {t['funceval']:.3f}s, JacEval {t['jaceval']:.3f}s, "
                       f"PCSetUp {t['pcsetup']:.3f}s, GMRES iter {t['gmres_iter']:.4f}s (30-iteration cycle); "
                       f"combined with the GPU run's per-step counts {counts}, extrapolated by {scale:.2f} (vertex "
                       f"ratio) and by the per-phase factors {corr} by which the oracle on the workload's own mesh "
                       f"exceeded that extrapolation ({src})"),
            "cpu": _cpu_model()}


def validation_factors(V_work, nsub, ilu_level, overlap, ordering):
    """Per-phase ratios full-mesh / extrapolated sample from the record --validate-cpu-baseline
    wrote for this configuration (profiles/cpu_baseline_validation_*.json), or none."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "cpu_baseline_validation_*.json"))):
        try:
            rec = json.load(open(path))
        except (OSError, ValueError):
            continue
        cfg = rec.get("config", {})
        if (rec.get("workload_vertices") == V_work and cfg.get("nsub") == nsub and cfg.get("ilu_level") == ilu_level
                and cfg.get("overlap") == overlap and cfg.get("ordering") == ordering):
            return rec["full_over_extrapolated"], (f"{os.path.relpath(path, ROOT)}, measured on "
                                                   f"{rec.get('cpu', 'an unnamed CPU')}")
    return {}, "no full-mesh record for this configuration: uncorrected"


def validate_cpu_baseline(args, counts: dict) -> dict:
    """The oracle's phases timed on the workload's own mesh against the depth-1 sample scaled
    by the vertex ratio (CPU only; no GPU needed)."""
    mesh = W.tree_mesh(depth=args.depth, h=W.TREE_H[args.depth])
    full = oracle_phase_times(mesh, args.nsub, args.ilu, args.overlap, args.ordering)
    log(f"[validate] full mesh ({mesh.nverts} vertices): {full}")
    m1 = W.tree_mesh(depth=1, h=W.TREE_H[1])
    ns = max(1, round(args.nsub * m1.nverts / mesh.nverts))
    samp = oracle_phase_times(m1, ns, args.ilu, args.overlap, args.ordering)
    scale = mesh.nverts / m1.nverts
    log(f"[validate] sample ({m1.nverts} vertices, {ns} subdomains) x {scale:.3f}: {samp}")
    ratio = {k: full[k] / (samp[k] * scale) for k in ("funceval", "jaceval", "pcsetup", "gmres_iter")}
    est, meas = per_step(samp, counts) * scale, per_step(full, counts)
    return {"workload_vertices": mesh.nverts, "sample_vertices": m1.nverts, "vertex_ratio": round(scale, 4),
            "sample_subdomains": ns, "config": {"nsub": args.nsub, "ilu_level": args.ilu, "overlap": args.overlap,
                                                "ordering": args.ordering},
            "full_mesh_s": {k: round(v, 4) for k, v in full.items()},
            "sample_s": {k: round(v, 4) for k, v in samp.items()},
            "full_over_extrapolated": {k: round(v, 3) for k, v in ratio.items()},
            "counts_per_step": counts, "per_step_extrapolated_s": round(est, 2), "per_step_full_mesh_s": round(meas, 2),
            "extrapolation_error": round(est / meas - 1.0, 4), "cpu": _cpu_model(), "cores": 1}


def _cpu_model() -> str:
    """Model name of the host CPU with its family/model/stepping numbers (a virtual machine
    may report only a generic name)."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k = k.strip()
            if k in ("model name", "cpu family", "model", "stepping", "cpu MHz") and k not in info:
                info[k] = v.strip()
            if not line.strip() and info:
                break
    except OSError:
        return "unknown"
    return (f"{info.get('model name', 'unknown')} (family {info.get('cpu family', '?')}, model {info.get('model', '?')}, "
            f"stepping {info.get('stepping', '?')}, {info.get('cpu MHz', '?')} MHz; {os.cpu_count()} logical CPUs)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=("tree", "tube"), default="tree",
                    help="tree: the bifurcating compliant tree (default); tube: the straight compliant tube, one "
                         "backward-Euler step from the Poiseuille state, repeated")
    ap.add_argument("--depth", type=int, default=3)
    ap.add_argument("--nsub", type=int, default=0, help="Schwarz subdomains (default: 256 tree, 4 tube)")
    ap.add_argument("--ilu", type=int, default=-1, help="ILU fill level (default: 3 tree, 0 tube)")
    ap.add_argument("--dt", type=float, default=1e-3)
    ap.add_argument("--overlap", type=int, default=1)
    ap.add_argument("--ordering", type=int, default=0, help="subdomain ordering: 0 RCM, 1 one-way dissection")
    ap.add_argument("--jac-lag", type=int, default=1, help="Newton iterations per Jacobian and Schwarz setup")
    ap.add_argument("--precision", type=int, default=0,
                    help="Schwarz precision: 0 FP64, 1 FP32 sweeps from rounded FP64 factors, 2 BF16 factors "
                         "with FP32 sweeps, 3 FP32 factorization and sweeps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the row-length rule's sweep schedule")
    ap.add_argument("--sweep-mb", type=int, default=0,
                    help="use this sweep schedule (blocks per task) instead of tuning, e.g. to take "
                         "counters on the schedule a tuned run chose")
    ap.add_argument("--graphs", action="store_true", help="GMRES Arnoldi steps as captured graphs")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before timing, run a plain elementwise copy of this many MiB three times "
                         "(reference dispatch for scaling rocprofv3 byte counters)")
    ap.add_argument("--validate-cpu-baseline", action="store_true",
                    help="CPU only: time the oracle's phases on the workload's own mesh and compare them with "
                         "the extrapolated depth-1 sample; prints one JSON line")
    ap.add_argument("--newton-progress", action="store_true",
                    help="the FP64 reference path reports every Newton iteration as it ends")
    ap.add_argument("--allow-divergence", action="store_true",
                    help="a step that fails ends the run with a JSON line (value null) that records every step's "
                         "Newton and GMRES iterations, instead of an exception")
    ap.add_argument("--counts", default="4,3,3,185",
                    help="per-step FuncEval, JacEval, PCSetUp and GMRES-iteration counts for --validate-cpu-baseline")
    args = ap.parse_args()
    tube = args.workload == "tube"
    if args.nsub <= 0:
        args.nsub = 4 if tube else 256
    if args.ilu < 0:
        args.ilu = 0 if tube else 3
    if args.validate_cpu_baseline:
        c = [float(x) for x in args.counts.split(",")]
        counts = dict(funceval=c[0], jaceval=c[1], pcsetup=c[2], gmres_iters=c[3])
        print(json.dumps(validate_cpu_baseline(args, counts)), flush=True)
        return
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
    mesh = W.tube_mesh() if tube else W.tree_mesh(depth=args.depth, h=W.TREE_H[args.depth])
    ph = W.physics_config1()
    opts = dict(nsub=args.nsub, overlap=args.overlap, ilu_level=args.ilu, ordering=args.ordering, jac_lag=args.jac_lag,
                gmres_restart=30,
                gmres_maxit=600,
                gmres_rtol=1e-3, newton_rtol=1e-6, newton_maxit=20, precision=args.precision)
    ref = None
    if args.precision != 0 and not tube:
        # the FP64 path first, with its own solver, which is freed before the rounded one is
        # built (at the largest sizes the two would not fit side by side)
        ref, ref_sec = fp64_path(fsi, mesh, ph, opts, args.dt, 2 + args.warmup + args.steps, dev, 2 + args.warmup,
                                 reported=args.newton_progress)
    s = fsi.Solver(mesh, ph, opts)
    if args.graphs:
        s.set_graphs(True)
    log(f"[bench] mesh V={mesh.nverts} E={mesh.ntets} n={s.n} nnzb={s.nnzb} setup {time.perf_counter() - t0:.1f}s")

    dt = args.dt
    # tree: two rigid-wall steps from rest start the flow, then warmup and timed steps of the
    # pulsatile inflow; tube: every step is the same backward-Euler step from the Poiseuille
    # state with the peak inflow 30 cm/s
    nstart = 0 if tube else 2
    nsteps = nstart + args.warmup + args.steps
    if tube:
        y_start = torch.as_tensor(W.poiseuille_state(mesh, 30.0, ph["mu_f"], 5.0)).to(dev)
        G = [torch.as_tensor(W.dirichlet_values(mesh, 30.0)).to(dev)] * (nsteps + 1)
    else:
        G = [torch.as_tensor(W.dirichlet_values(mesh, W.inflow_peak((k + 1) * dt))).to(dev) for k in range(nsteps + 1)]
    rigid = W.rigid_wall_mask(mesh)
    y_old = torch.zeros(s.n, dtype=torch.float64, device=dev)
    y = torch.empty_like(y_old)
    step_log = []

    class StepFailed(Exception):
        pass

    def step(k, mask=None, phase="timed"):
        if tube:
            y_old.copy_(y_start)
        elif ref is not None:  # every step from the FP64 path's state at the same time
            y_old.copy_(ref[k])
        s.set_step(dt if tube else (k + 1) * dt, dt, y_old, G[k], None, mask)
        y.copy_(y_old)
        st, rc = s.newton_solve(y, check=False)
        ni = st["newton_iters"]
        step_log.append({"step": k, "phase": phase, "rc": rc, "converged": st["converged"], "NI": ni,
                         "LI": st["lin_hist"][:max(ni, 1)], "cap_hits": sum(1 for x in st["lin_hist"][:max(ni, 1)]
                                                                         if x >= opts["gmres_maxit"]),
                         "fnorm_ratio": st["fnorm"] / st["fnorm0"] if st["fnorm0"] else 0.0})
        if rc != 0:
            if args.allow_divergence:
                raise StepFailed()
            raise RuntimeError(f"step {k} failed with status {rc}: {st}")
        y_old.copy_(y)
        return st

    def failed_record():
        return {"metric": METRIC, "value": None, "unit": "s/step", "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "higher_is_better": False, "dtype": "f64", "data": "synthetic",
                "config": {"workload": workload_name(), "nverts": mesh.nverts, "n": s.n, "nsub": args.nsub,
                           "ilu_level": args.ilu, "overlap": args.overlap, "ordering": args.ordering},
                "failed_step": step_log[-1], "step_log": step_log}

    def workload_name():
        sch = (f"{args.nsub} RAS subdomains overlap {args.overlap}, ILU({args.ilu}), {ORDERING[args.ordering]} ordering, "
               f"GMRES(30) rtol 1e-3, Newton rtol 1e-6"
               + {0: "", 1: ", FP32 sweeps", 2: ", BF16 factors with FP32 sweeps",
                  3: ", FP32 factorization and sweeps"}[args.precision])
        if tube:
            return (f"straight compliant tube, {mesh.nverts} vertices, {mesh.ntets} tets, {s.n} unknowns, one "
                    f"backward-Euler step dt {dt} from the Poiseuille state (peak 30 cm/s), {sch}")
        return (f"bifurcating compliant tree depth {args.depth}, {mesh.nverts} vertices, {mesh.ntets} tets, {s.n} "
                f"unknowns, dt {dt}, {sch}")

    try:
        # with an FP64 reference the start steps are its own: the steps below begin from its
        # states
        for k in range(nstart if ref is None else 0):
            st = step(k, rigid, "rigid start")
            log(f"[bench] rigid start step {k}: NI {st['newton_iters']} LI {st['lin_hist'][:st['newton_iters']]}")
        for k in range(nstart, nstart + args.warmup):
            st = step(k, None, "warmup")
            log(f"[bench] warmup step {k}: NI {st['newton_iters']} LI {st['lin_hist'][:st['newton_iters']]}")
    except StepFailed:
        log(f"[bench] step failed: {step_log[-1]}")
        print(json.dumps(failed_record()), flush=True)
        s.close()
        return

    tune = None
    if args.sweep_mb:
        s.pc_select(args.sweep_mb)
        tune = {"best_blocks_per_task": args.sweep_mb, "selected": True}
        log(f"[bench] sweep schedule selected: {args.sweep_mb} blocks per task")
    elif not args.no_tune and (nstart if ref is None else 0) + args.warmup > 0:  # sweep schedule timed on the last step's factors,
        # outside the timed steps
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
    stats, outs = [], []
    t_start = time.perf_counter()
    try:
        for k in range(nstart + args.warmup, nsteps):
            stats.append(step(k))
            if ref is not None:
                outs.append(y.clone())
            log(f"[bench] step {k}: NI {stats[-1]['newton_iters']} LI {stats[-1]['lin_hist'][:stats[-1]['newton_iters']]} "
                f"cuts {stats[-1]['line_search_cuts']}")
    except StepFailed:
        log(f"[bench] step failed: {step_log[-1]}")
        print(json.dumps(failed_record()), flush=True)
        s.close()
        return
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    sec_per_step = elapsed / args.steps
    if args.graphs:
        s.prof_enable(True)
        step(nsteps)
        torch.cuda.synchronize()

    kernels = {}
    for name in ("ilu_fwd", "ilu_bwd", "ilu_factor", "spmv", "elem_jac_fluid", "elem_jac_solid", "jac_init",
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
        "dtype": {0: "f64", 1: "f64 (f32 Schwarz sweeps)", 2: "f64 (bf16 factors, f32 Schwarz sweeps)",
                  3: "f64 (f32 Schwarz factorization and sweeps)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": workload_name(),
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
        "step_log": step_log,
    }
    if tube:
        out["roofline"]["note"] = ("the tube's matrix and factors (about 20 MB) stay in the caches: an in-cache "
                                   "rate, not an HBM figure")
    if ref is not None:
        rel = [float(torch.linalg.vector_norm(yk - ref[k + 1]) / torch.linalg.vector_norm(ref[k + 1]))
               for k, yk in zip(range(nstart + args.warmup, nsteps), outs)]
        out["error_vs_fp64"] = {"per_step_rel_2norm": [float(f"{r:.3e}") for r in rel], "max": float(f"{max(rel):.3e}"),
                                "newton_rtol": opts["newton_rtol"],
                                "note": "each timed step starts from the FP64 path's state y_k and is compared with "
                                        "its y_k+1; both meet the same Newton tolerance"}
        out["fp64_path"] = {"s_per_step": round(ref_sec, 5), "speedup": round(ref_sec / sec_per_step, 3),
                            "note": "the plain FP64 path on the same timed steps from the same states"}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(counts, args.ilu, mesh.nverts, args.nsub, args.overlap, args.ordering,
                                           small_mesh=mesh if tube else None)
    print(json.dumps(out), flush=True)
    s.close()


def newton_reported(s, y, maxit, k):
    """One step's Newton solve, one library iteration per call (the solver was created with
    newton_maxit 1), each reported as it ends.  The first call's target, 1e-6 of its
    ||F_0||, is kept as an absolute one for the later calls, so the iterates are those of a
    single call; each call evaluates the residual once more at its start."""
    s.set_newton_tol(1e-6, 0.0)
    tot = {"newton_iters": 0, "linear_iters": 0, "lin_hist": []}
    target = None
    for _ in range(maxit):
        st, rc = s.newton_solve(y, check=False)
        if target is None:
            target = 1e-6 * st["fnorm0"]
            s.set_newton_tol(0.0, target)
        ni = st["newton_iters"]
        tot["newton_iters"] += ni
        tot["linear_iters"] += st["linear_iters"]
        tot["lin_hist"] += list(st["lin_hist"][:ni])
        log(f"[bench] FP64 reference step {k}, Newton iteration {tot['newton_iters']}: ||F|| {st['fnorm']:.3e} "
            f"(target {target:.3e}), GMRES {list(st['lin_hist'][:ni])}")
        if st["converged"]:
            return tot, 0
        if ni == 0:  # a failure other than the one-iteration limit
            return tot, rc
    return tot, 7


def fp64_path(fsi, mesh, ph, opts, dt, nsteps, dev, timed_from, reported=False):
    """The FP64 path's states y_0 .. y_nsteps of the run (two rigid-wall steps from rest, then
    the pulsatile steps), from an FP64 solver that is closed afterwards, and its seconds per
    step over steps timed_from .. nsteps-1 (the run's timed steps).  reported: every Newton
    iteration is reported as it ends (for meshes whose start-up steps run for minutes)."""
    import torch
    s64 = fsi.Solver(mesh, ph, dict(opts, precision=0, newton_maxit=1) if reported else dict(opts, precision=0))
    rigid = W.rigid_wall_mask(mesh)
    ys = [torch.zeros(s64.n, dtype=torch.float64, device=dev)]
    secs = []
    for k in range(nsteps):
        g = torch.as_tensor(W.dirichlet_values(mesh, W.inflow_peak((k + 1) * dt))).to(dev)
        s64.set_step((k + 1) * dt, dt, ys[-1], g, None, rigid if k < 2 else None)
        y = ys[-1].clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, rc = newton_reported(s64, y, opts["newton_maxit"], k) if reported else s64.newton_solve(y, check=False)
        torch.cuda.synchronize()
        if k >= timed_from:
            secs.append(time.perf_counter() - t0)
        if rc != 0:
            raise RuntimeError(f"FP64 reference step {k} failed with status {rc}")
        ys.append(y)
        log(f"[bench] FP64 reference step {k}: NI {st['newton_iters']} LI {st['lin_hist'][:st['newton_iters']]} "
            f"{time.perf_counter() - t0:.2f}s")
    s64.close()
    torch.cuda.synchronize()
    return ys, float(np.mean(secs)) if secs else None


if __name__ == "__main__":
    main()
