"""Summarise rocprofv3 output of the benchmark into short text records.

Reads a kernel-trace run (``--kernel-trace --stats``, CSV) and two counter runs
(``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``, CSV) of ``bench.py --calib-copy-mib N``
and writes:

* a Markdown summary (per-kernel call counts and durations, HBM bytes per launch of the
  triangular sweeps, the commands that produced them);
* a JSON record of the sweeps' HBM bytes per launch, tagged with the SHA-256 of the sweep
  source it was measured with (``bench.py`` reports it only while the source is unchanged).

FETCH_SIZE and WRITE_SIZE are scaled by what they read for the calibration dispatch, a
plain elementwise copy of known size (N MiB read, N MiB written).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
# sweep kernels by their template arguments: k_ilu_sweep<scalar, 0|1 (direction), MB, D>;
# sweep_patterns(mb) keeps only the schedule with mb blocks per task (None: any)


def sweep_patterns(mb=None):
    m = r"\d+" if mb is None else str(int(mb))
    return {"ilu_fwd": re.compile(r"k_ilu_sweep<(?:[^,<>]+, )?0, " + m + ","),
            "ilu_bwd": re.compile(r"k_ilu_sweep<(?:[^,<>]+, )?1, " + m + ",")}


SWEEPS = sweep_patterns()


def _one(d: str, pattern: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no {pattern} under {d}")
    return hits[0]


def counter_values(d: str, counter: str) -> list[tuple[str, float]]:
    """(kernel name, counter value) per dispatch, in dispatch order."""
    rows = []
    with open(_one(d, "*counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") == counter:
                rows.append((int(r.get("Dispatch_Id", 0)), r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort()
    return [(k, v) for _, k, v in rows]


def calib_factor(vals: list[tuple[str, float]], nbytes: int) -> float:
    """Counter bytes per algorithmic byte on the calibration copy: the three largest
    dispatches of kernels outside the library."""
    other = sorted((v for k, v in vals if "fsi::" not in k), reverse=True)[:3]
    if len(other) < 3:
        raise RuntimeError("calibration copy dispatches not found")
    return statistics.median(other) * 1024.0 / nbytes


def sweep_bytes(vals: list[tuple[str, float]], factor: float, pats=None) -> dict:
    out = {}
    for name, tag in (pats or SWEEPS).items():
        v = [x for k, x in vals if tag.search(k)]
        if v:
            out[name] = dict(dispatches=len(v), mean_kib=statistics.mean(v),
                             bytes_per_launch=statistics.mean(v) * 1024.0 / factor)
    return out


def kernel_stats(d: str, top: int = 14) -> list[dict]:
    rows = []
    with open(_one(d, "*kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            rows.append(dict(name=r["Name"], calls=int(r["Calls"]), total_ms=float(r["TotalDurationNs"]) / 1e6,
                             avg_us=float(r["AverageNs"]) / 1e3, pct=float(r["Percentage"])))
    rows.sort(key=lambda x: -x["total_ms"])
    return rows[:top]


def short(name: str) -> str:
    n = name.split("(")[0]
    return n if len(n) <= 70 else n[:67] + "..."


def factor_summary(dirs: list[str], cmds: list[str], copy_mib: int, nblocks: int, out_md: str,
                   pattern: str = "k_ilu_factor"):
    """Counters of the factorization kernel, mean per dispatch, from counter runs that each
    hold some of them (FETCH_SIZE and WRITE_SIZE scaled by the calibration copy), with the
    shares of wave-cycles spent waiting and issuing VALU and LDS instructions."""
    vals, scale = {}, {}
    for d in dirs:
        with open(_one(d, "*counter_collection.csv")) as f:
            rows = list(csv.DictReader(f))
        for c in sorted({r["Counter_Name"] for r in rows}):
            per = [(r["Kernel_Name"], float(r["Counter_Value"])) for r in rows if r["Counter_Name"] == c]
            v = [x for k, x in per if pattern in k]
            if v:
                vals[c] = statistics.mean(v)
            if c in ("FETCH_SIZE", "WRITE_SIZE"):
                scale[c] = calib_factor(per, copy_mib << 20)
    L = [f"# Block ILU factorization (`{pattern}`): rocprofv3 counters", "",
         "Mean per dispatch over the run's factorizations. One counter group per run:", ""]
    L += [f"    {c}" for c in cmds]
    L += ["", "| counter | mean per dispatch |", "|---|---:|"]
    L += [f"| {c} | {v:,.0f} |" for c, v in sorted(vals.items())]
    wc = vals.get("SQ_WAVE_CYCLES")
    if wc:
        L += ["", "| share of wave-cycles | value |", "|---|---:|"]
        for c in ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS"):
            if c in vals:
                L.append(f"| {c} | {vals[c] / wc:.3f} |")
    if "SQ_LDS_BANK_CONFLICT" in vals and "SQ_ACTIVE_INST_LDS" in vals:
        L += ["", f"LDS bank-conflict cycles per LDS-active cycle: "
                  f"{vals['SQ_LDS_BANK_CONFLICT'] / max(vals['SQ_ACTIVE_INST_LDS'], 1):.2f}"]
    if "FETCH_SIZE" in vals and "WRITE_SIZE" in vals:
        fb = vals["FETCH_SIZE"] * 1024.0 / scale["FETCH_SIZE"]
        wb = vals["WRITE_SIZE"] * 1024.0 / scale["WRITE_SIZE"]
        algo = 2.0 * nblocks * 392
        L += ["", f"HBM bytes per factorization (FETCH_SIZE and WRITE_SIZE scaled by a {copy_mib} MiB copy: "
                  f"fetch scale {scale['FETCH_SIZE']:.4f}, write scale {scale['WRITE_SIZE']:.4f}): "
                  f"fetch {fb / 1e9:.2f} GB, write {wb / 1e9:.2f} GB; algorithmic 2 x {nblocks:,} blocks x 392 B "
                  f"= {algo / 1e9:.2f} GB; ratio {(fb + wb) / algo:.2f}"]
    src = open(os.path.join(HERE, "csrc", "ilu.hip"), "rb").read()
    L += ["", f"`ilu.hip` SHA-256: `{hashlib.sha256(src).hexdigest()}`", ""]
    with open(out_md, "w") as f:
        f.write("\n".join(L))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--factor-dirs", nargs="*", default=None,
                    help="counter runs of the factorization (then only its summary is written)")
    ap.add_argument("--factor-cmds", nargs="*", default=None)
    ap.add_argument("--factor-blocks", type=int, default=0, help="local blocks NB of the run's configuration")
    ap.add_argument("--trace-dir")
    ap.add_argument("--fetch-dir")
    ap.add_argument("--write-dir")
    ap.add_argument("--copy-mib", type=int, required=True)
    ap.add_argument("--trace-cmd")
    ap.add_argument("--fetch-cmd")
    ap.add_argument("--write-cmd")
    ap.add_argument("--algo-bytes", default="", help="JSON of the bench line with the algorithmic bytes")
    ap.add_argument("--out-md", required=True)
    ap.add_argument("--out-json")
    a = ap.parse_args()
    if a.factor_dirs:
        factor_summary(a.factor_dirs, a.factor_cmds or [], a.copy_mib, a.factor_blocks, a.out_md)
        return

    nbytes = a.copy_mib << 20
    fv = counter_values(a.fetch_dir, "FETCH_SIZE")
    wv = counter_values(a.write_dir, "WRITE_SIZE")
    ff, wf = calib_factor(fv, nbytes), calib_factor(wv, nbytes)
    algo, config, mb = {}, {}, None
    if a.algo_bytes:
        line = json.load(open(a.algo_bytes))
        config = {k: line["config"].get(k) for k in ("nsub", "ilu_level", "overlap", "ordering")}
        # the schedule the timed steps ran: the tuner's choice (the tuner's trial launches of
        # the other schedules are left out)
        mb = (line.get("sweep_schedule") or {}).get("best_blocks_per_task")
        config["sweep_mb"] = mb
        rl = line["roofline"]
        algo[rl["kernel"]] = rl["bytes_per_launch"]
        algo[rl["other_sweep"]["kernel"]] = rl["other_sweep"]["bytes_per_launch"]
    pats = sweep_patterns(mb)
    fb, wb = sweep_bytes(fv, ff, pats), sweep_bytes(wv, wf, pats)
    kern = {}
    for k in pats:
        if k in fb and k in wb:
            kern[k] = dict(fetch_bytes_per_launch=round(fb[k]["bytes_per_launch"]),
                           write_bytes_per_launch=round(wb[k]["bytes_per_launch"]),
                           hbm_bytes_per_launch=round(fb[k]["bytes_per_launch"] + wb[k]["bytes_per_launch"]),
                           dispatches=fb[k]["dispatches"])
            if k in algo:
                kern[k]["algorithmic_bytes_per_launch"] = algo[k]
                kern[k]["traffic_over_algorithmic"] = round(kern[k]["hbm_bytes_per_launch"] / algo[k], 3)
    src = open(os.path.join(HERE, "csrc", "ilu.hip"), "rb").read()
    rec = dict(ilu_hip_sha256=hashlib.sha256(src).hexdigest(), copy_mib=a.copy_mib,
               fetch_scale=round(ff, 4), write_scale=round(wf, 4), kernels=kern,
               commands=dict(fetch=a.fetch_cmd, write=a.write_cmd))
    if config:
        rec["config"] = config  # the Schwarz configuration the counters were taken on
    with open(a.out_json, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")

    ks = kernel_stats(a.trace_dir)
    L = ["# Triangular sweeps and the NKS step on the depth-3 tree: rocprofv3 summary", "",
         "Kernel trace (`--kernel-trace --stats`), command:", "", f"    {a.trace_cmd}", "",
         "| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    L += [f"| `{short(r['name'])}` | {r['calls']} | {r['total_ms']:.1f} | {r['avg_us']:.1f} | {r['pct']:.1f} |"
          for r in ks]
    L += ["", "HBM bytes per launch from `FETCH_SIZE` and `WRITE_SIZE` (KiB per dispatch), each scaled by "
          f"what it reads for a plain elementwise copy of {a.copy_mib} MiB (fetch scale {ff:.4f}, write "
          f"scale {wf:.4f} counter bytes per copied byte). Commands:", "", f"    {a.fetch_cmd}",
          f"    {a.write_cmd}", "",
          "| kernel | dispatches | fetch MB | write MB | HBM MB | algorithmic MB | ratio |",
          "|---|---:|---:|---:|---:|---:|---:|"]
    for k, v in kern.items():
        al = v.get("algorithmic_bytes_per_launch")
        L.append(f"| {k} | {v['dispatches']} | {v['fetch_bytes_per_launch'] / 1e6:.1f} | "
                 f"{v['write_bytes_per_launch'] / 1e6:.1f} | {v['hbm_bytes_per_launch'] / 1e6:.1f} | "
                 f"{al / 1e6 if al else float('nan'):.1f} | {v.get('traffic_over_algorithmic', float('nan'))} |")
    L += ["", f"Sweep source SHA-256: `{rec['ilu_hip_sha256']}`", ""]
    with open(a.out_md, "w") as f:
        f.write("\n".join(L))


if __name__ == "__main__":
    main()
