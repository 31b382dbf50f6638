"""FP64 vector arithmetic of the assembly kernels from rocprofv3 counters, as a short record.

Reads two counter runs of the benchmark (CSV):

* ``--pmc SQ_INSTS_VALU_FLOPS_FP64 SQ_INSTS_VALU_FLOPS_FP64_TRANS SQ_INSTS_VALU SQ_WAVES``
* ``--pmc SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_TRANS_F64``

and a kernel-trace run (``--kernel-trace --stats``) for the kernels' durations, and writes
a Markdown table per kernel: FP64 flops per dispatch, flops per element, the achieved rate
and its fraction of the FP64 vector peak (78.6 TFLOP/s), plus a JSON record of the mean
counter values per dispatch.

On this GPU the FLOPS counters count flops per wavefront instruction, not per lane: they
agree with ADD + MUL + TRANS + 2 FMA instructions to within 2% (they include a few more
FP64 operation kinds).  The flops reported are therefore 64 times the counter, with the
instruction count times 64 beside it; both count every lane of an issued instruction.

    python -m paper_1810_04289_amd.valu_summary --flops-dir D1 --inst-dir D2 --trace-dir D3 \
        --cmd-flops "..." --cmd-inst "..." --cmd-trace "..." --out-md OUT.md --out-json OUT.json
    python -m paper_1810_04289_amd.valu_summary --from-json OUT.json --cmd-flops ... --out-md OUT.md
"""
from __future__ import annotations

import argparse
import csv
import statistics

from .pmc_summary import _one

PEAK_FP64_VECTOR = 78.6e12  # FLOP/s
KERNELS = {  # short name: (kernel-name fragment, element kind)
    "k_elem_jac<0> (fluid Jacobian)": ("k_elem_jac<0>", "fluid"),
    "k_elem_jac<1> (wall Jacobian)": ("k_elem_jac<1>", "wall"),
    "k_elem_res<0> (fluid residual)": ("k_elem_res<0>", "fluid"),
    "k_elem_res<1> (wall residual)": ("k_elem_res<1>", "wall"),
}


def per_kernel(d: str) -> dict[str, dict[str, float]]:
    """kernel name -> counter -> mean value per dispatch (counters summed over dimensions)."""
    acc: dict[tuple[str, int], dict[str, float]] = {}
    with open(_one(d, "*counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            key = (r["Kernel_Name"], int(r.get("Dispatch_Id", 0)))
            c = acc.setdefault(key, {})
            c[r["Counter_Name"]] = c.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    out: dict[str, dict[str, list[float]]] = {}
    for (name, _), cs in acc.items():
        for k, v in cs.items():
            out.setdefault(name, {}).setdefault(k, []).append(v)
    return {n: {k: statistics.mean(v) for k, v in cs.items()} for n, cs in out.items()}


def durations(d: str) -> dict[str, float]:
    """kernel name -> average duration in seconds (kernel trace)."""
    out = {}
    with open(_one(d, "*kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            out[r["Name"]] = float(r["AverageNs"]) * 1e-9
    return out


def _find(table: dict, frag: str):
    hits = [k for k in table if frag in k]
    return table[hits[0]] if hits else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--flops-dir")
    ap.add_argument("--inst-dir")
    ap.add_argument("--trace-dir")
    ap.add_argument("--from-json", default="", help="a JSON record written by --out-json, instead of the runs")
    ap.add_argument("--cmd-flops", required=True)
    ap.add_argument("--cmd-inst", required=True)
    ap.add_argument("--cmd-trace", required=True)
    ap.add_argument("--tree-depth", type=int, default=3, help="element counts from the generator's tree")
    ap.add_argument("--out-md", required=True)
    ap.add_argument("--out-json", default="")
    a = ap.parse_args()
    import json
    if a.from_json:
        raw = json.load(open(a.from_json))
    else:
        from . import workload as W
        mesh = W.tree_mesh(depth=a.tree_depth, h=W.TREE_H[a.tree_depth])
        nel = {"fluid": int((mesh.tet_domain == 0).sum()), "wall": int((mesh.tet_domain == 1).sum())}
        fl, ins, dur = per_kernel(a.flops_dir), per_kernel(a.inst_dir), durations(a.trace_dir)
        raw = {}
        for label, (frag, kind) in KERNELS.items():
            f, i, t = _find(fl, frag), _find(ins, frag), _find(dur, frag)
            if f is not None and i is not None and t is not None:
                raw[label] = dict(elements=nel[kind], avg_s=t, **f, **i)
    rows = []
    for label, r in raw.items():
        flops = 64.0 * (r.get("SQ_INSTS_VALU_FLOPS_FP64", 0.0) + r.get("SQ_INSTS_VALU_FLOPS_FP64_TRANS", 0.0))
        by_inst = 64.0 * (r.get("SQ_INSTS_VALU_ADD_F64", 0.0) + r.get("SQ_INSTS_VALU_MUL_F64", 0.0)
                          + r.get("SQ_INSTS_VALU_TRANS_F64", 0.0) + 2.0 * r.get("SQ_INSTS_VALU_FMA_F64", 0.0))
        rows.append((label, r["elements"], flops, by_inst, r.get("SQ_INSTS_VALU", 0.0), r["avg_s"]))
    with open(a.out_md, "w") as o:
        o.write(f"# FP64 vector arithmetic of the assembly kernels, depth-{a.tree_depth} tree: rocprofv3 counters\n\n")
        o.write("FP64 flops per dispatch: 64 x `SQ_INSTS_VALU_FLOPS_FP64` (+ `_TRANS`), which on this GPU counts "
                "flops per wavefront instruction; beside it 64 x (ADD + MUL + TRANS + 2 FMA) FP64 instructions. "
                "Both count every lane of an issued instruction. Durations from the kernel trace. "
                "Peak: FP64 vector 78.6 TFLOP/s.\n\n")
        o.write("Commands:\n\n")
        for c in (a.cmd_flops, a.cmd_inst, a.cmd_trace):
            o.write(f"    {c}\n")
        o.write("\n| kernel | elements | FP64 flops / dispatch | 64·(ADD+MUL+TRANS+2FMA) | flops / element "
                "| VALU instr / dispatch | avg us | TFLOP/s | of peak |\n|---|---:|---:|---:|---:|---:|---:|---:|---:|\n")
        for label, ne, flops, by_inst, valu, t in rows:
            rate = flops / t
            o.write(f"| `{label}` | {ne} | {flops:.4g} | {by_inst:.4g} | {flops / ne:.4g} | {valu:.4g} "
                    f"| {1e6 * t:.1f} | {rate / 1e12:.2f} | {rate / PEAK_FP64_VECTOR:.1%} |\n")
    if a.out_json:
        with open(a.out_json, "w") as o:
            json.dump(raw, o, indent=1)
    print(open(a.out_md).read())


if __name__ == "__main__":
    main()
