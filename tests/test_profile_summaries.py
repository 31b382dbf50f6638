"""Host logic of the measurement tools (CPU): the rocprofv3 summarizers on small synthetic
counter files in rocprofv3's CSV layout.

pmc_summary: the calibration copy fixes the counter scale (FETCH_SIZE counts half the copied
bytes here, WRITE_SIZE all of them), sweep dispatches of other schedules are left out, and
bytes per launch, the traffic ratio and the source hash come out as stated.
valu_summary: counters split over hardware dimensions are summed per dispatch, and the FP64
flops are 64 times the per-instruction FLOPS counter.
"""
import csv
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1810_04289_amd")
COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
        "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
        "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
FWD8 = "void fsi::k_ilu_sweep<double, 0, 8, 6>(int const*, int const*)"
BWD8 = "void fsi::k_ilu_sweep<double, 1, 8, 6>(int const*, int const*)"
FWD16 = "void fsi::k_ilu_sweep<double, 0, 16, 4>(int const*, int const*)"


def write_counters(path, rows):
    """rows: (dispatch id, kernel name, counter, value in KiB or counts)."""
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(COLS)
        for d, k, c, v in rows:
            w.writerow([d, d, "Agent 1", 1, 1, 1, 64, 1, k, 64, 0, 0, 8, 0, 16, c, v, 0, 1])


def write_stats(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_kernel_stats.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        for name, calls, avg_ns in rows:
            w.writerow([name, calls, calls * avg_ns, avg_ns, 50.0, avg_ns, avg_ns, 0.0])


def run(mod, *args):
    r = subprocess.run([sys.executable, "-m", f"paper_1810_04289_amd.{mod}", *args], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return r.stdout


def test_pmc_summary_scales_filters_and_hashes(tmp_path):
    mib = 4
    copy = "__amd_rocclr_copyBuffer"
    # calibration: three copies of 4 MiB; FETCH_SIZE reads half the bytes, WRITE_SIZE all
    fetch = [(i, copy, "FETCH_SIZE", 0.5 * mib * 1024) for i in range(3)]
    write = [(i, copy, "WRITE_SIZE", 1.0 * mib * 1024) for i in range(3)]
    # two launches of each timed sweep (8-block schedule), one of another schedule (left out)
    fetch += [(3, FWD8, "FETCH_SIZE", 1000.0), (4, FWD8, "FETCH_SIZE", 1200.0), (5, BWD8, "FETCH_SIZE", 2000.0),
              (6, BWD8, "FETCH_SIZE", 2000.0), (7, FWD16, "FETCH_SIZE", 9999.0)]
    write += [(3, FWD8, "WRITE_SIZE", 10.0), (4, FWD8, "WRITE_SIZE", 10.0), (5, BWD8, "WRITE_SIZE", 20.0),
              (6, BWD8, "WRITE_SIZE", 20.0), (7, FWD16, "WRITE_SIZE", 999.0)]
    write_counters(tmp_path / "fetch", fetch)
    write_counters(tmp_path / "write", write)
    write_stats(tmp_path / "trace", [(BWD8, 10, 1_000_000), (FWD8, 10, 900_000)])
    line = {"config": {"nsub": 256, "ilu_level": 3, "overlap": 1, "ordering": 0},
            "sweep_schedule": {"best_blocks_per_task": 8},
            "roofline": {"kernel": "ilu_bwd", "bytes_per_launch": 4_000_000,
                         "other_sweep": {"kernel": "ilu_fwd", "bytes_per_launch": 2_000_000}}}
    (tmp_path / "line.json").write_text(json.dumps(line))
    md, js = tmp_path / "out.md", tmp_path / "out.json"
    run("pmc_summary", "--trace-dir", str(tmp_path / "trace"), "--fetch-dir", str(tmp_path / "fetch"),
        "--write-dir", str(tmp_path / "write"), "--copy-mib", str(mib), "--trace-cmd", "T", "--fetch-cmd", "F",
        "--write-cmd", "W", "--algo-bytes", str(tmp_path / "line.json"), "--out-md", str(md), "--out-json", str(js))
    rec = json.loads(js.read_text())
    assert rec["fetch_scale"] == 0.5 and rec["write_scale"] == 1.0
    fwd, bwd = rec["kernels"]["ilu_fwd"], rec["kernels"]["ilu_bwd"]
    assert fwd["dispatches"] == 2 and bwd["dispatches"] == 2           # the 16-block launch is left out
    assert fwd["fetch_bytes_per_launch"] == round(1100.0 * 1024 / 0.5)  # mean KiB, unscaled by 0.5
    assert fwd["write_bytes_per_launch"] == round(10.0 * 1024)
    assert bwd["hbm_bytes_per_launch"] == round(2000.0 * 1024 / 0.5 + 20.0 * 1024)
    assert bwd["traffic_over_algorithmic"] == round(bwd["hbm_bytes_per_launch"] / 4_000_000, 3)
    assert rec["config"]["sweep_mb"] == 8
    src = open(os.path.join(PKG, "csrc", "ilu.hip"), "rb").read()
    assert rec["ilu_hip_sha256"] == hashlib.sha256(src).hexdigest()
    text = md.read_text()
    assert "fsi::k_ilu_sweep<double, 1, 8, 6>" in text and "| 1000.0 |" in text


def test_valu_summary_sums_dimensions_and_scales_flops(tmp_path):
    jac, res = "void fsi::k_elem_jac<0>(PhysDev, int)", "void fsi::k_elem_res<0>(PhysDev, int)"
    flops, inst = [], []
    for d, k, f in ((0, jac, 1000.0), (1, jac, 3000.0), (2, res, 50.0)):
        # each counter arrives as two rows (two hardware dimensions) per dispatch
        flops += [(d, k, "SQ_INSTS_VALU_FLOPS_FP64", f / 2), (d, k, "SQ_INSTS_VALU_FLOPS_FP64", f / 2),
                  (d, k, "SQ_INSTS_VALU_FLOPS_FP64_TRANS", 0.0), (d, k, "SQ_INSTS_VALU", 10 * f)]
        inst += [(d, k, "SQ_INSTS_VALU_FMA_F64", f / 2), (d, k, "SQ_INSTS_VALU_ADD_F64", 0.0),
                 (d, k, "SQ_INSTS_VALU_MUL_F64", 0.0), (d, k, "SQ_INSTS_VALU_TRANS_F64", 0.0)]
    write_counters(tmp_path / "flops", flops)
    write_counters(tmp_path / "inst", inst)
    write_stats(tmp_path / "trace", [(jac, 2, 2000), (res, 1, 100)])
    raw = tmp_path / "raw.json"
    # element counts come from the generator's tree; this test gives them through the JSON record
    rec = {}
    sys.path.insert(0, ROOT)
    from paper_1810_04289_amd import valu_summary as V
    fl, ins, dur = V.per_kernel(str(tmp_path / "flops")), V.per_kernel(str(tmp_path / "inst")), \
        V.durations(str(tmp_path / "trace"))
    f = V._find(fl, "k_elem_jac<0>")
    assert f["SQ_INSTS_VALU_FLOPS_FP64"] == 2000.0       # mean over dispatches of the summed rows
    assert V._find(ins, "k_elem_jac<0>")["SQ_INSTS_VALU_FMA_F64"] == 1000.0
    assert abs(V._find(dur, "k_elem_jac<0>") - 2e-6) < 1e-15
    for label, frag, ne in (("k_elem_jac<0> (fluid Jacobian)", "k_elem_jac<0>", 100),
                            ("k_elem_res<0> (fluid residual)", "k_elem_res<0>", 100)):
        rec[label] = dict(elements=ne, avg_s=V._find(dur, frag), **V._find(fl, frag), **V._find(ins, frag))
    raw.write_text(json.dumps(rec))
    md = tmp_path / "out.md"
    out = run("valu_summary", "--from-json", str(raw), "--cmd-flops", "F", "--cmd-inst", "I", "--cmd-trace", "T",
              "--out-md", str(md))
    row = [l for l in out.splitlines() if "fluid Jacobian" in l][0].split("|")
    # 64 x 2000 flops per dispatch = 1.28e5; the instruction count gives 64 x 2 x 1000 alike;
    # 1.28e5 flops in 2 us = 0.064 TFLOP/s
    assert row[3].strip() == "1.28e+05" and row[4].strip() == "1.28e+05"
    assert row[5].strip() == "1280" and row[8].strip() == "0.06"
