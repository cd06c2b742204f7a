"""rocprofv3 passes over a bench.py workload, summarised into profiles/.

Runs, each as a child process with its own time limit (the profiler is the
program that starts bench.py, so nothing here touches the GPU itself):

* one kernel-trace pass (``--kernel-trace --stats``): per-kernel launch counts
  and durations -> ``kernels_<workload>.txt``;
* counter passes, one counter group per run (rocprofv3 does not split
  counters over passes): FETCH_SIZE; WRITE_SIZE; VALU instructions, waves and
  the GRBM clock; L2 hits and misses; wave residency and waiting; LDS
  instructions and bank conflicts -> ``counters_<workload>.txt`` and one
  ``traffic_<kernel>_<workload>.json`` per kernel that bench.py reads back.

HBM bytes are FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by what the
same counters read for the bandwidth probe's copy of known size
(``bench.py --workload copy``: 1 GiB read + 1 GiB written per launch), the
factors written to ``traffic_calibration.txt``.

Usage (from the repository root, on the GPU machine):

    python -m paper_2608_13696_amd.profiling --workload large --out profiles

The clock: GRBM_GUI_ACTIVE counts GPU-busy cycles of each XCD's graphics block
over a dispatch, summed over the 8 XCDs, so GRBM_GUI_ACTIVE / 8 / duration is
the clock the kernel ran at (the paper measures its clock the same way,
Section 2.2) and 256 CUs x that clock is the VALU issue ceiling.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# counter groups, one rocprofv3 run each (within the per-block limits: 8 SQ,
# 4 TCC, 2 GRBM counters per run)
PASSES = {
    "fetch": ["FETCH_SIZE"],
    "write": ["WRITE_SIZE"],
    "valu": ["SQ_INSTS_VALU", "SQ_WAVES", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR", "SQ_INSTS_LDS", "SQ_INSTS_SALU",
             "GRBM_GUI_ACTIVE", "GRBM_COUNT"],
    "tcc": ["TCC_HIT_sum", "TCC_MISS_sum"],
    # derived: OccupancyPercent = 400 SQ_WAVE_CYCLES / GRBM_GUI_ACTIVE(max over XCDs) / CUs / 32 waves
    "occ": ["OccupancyPercent", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY", "SQ_BUSY_CYCLES"],
    # derived: LdsBankConflict = conflict cycles / (LDS index-active cycles - conflict cycles)
    "lds": ["LdsBankConflict", "LdsUtil"],
}

# rocprofv3 kernel names -> the library's per-kernel timer names (bench.py)
def timer_name(kernel: str) -> str:
    k = kernel.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0].strip()
    side = "fact" if "<true>" in k else "dim" if "<false>" in k else None
    base = k.split("<")[0]
    table = {"k_p1_hist": "p1_hist", "k_p1_colscan": "p1_colscan", "k_p1_scatter": "p1_scatter",
             "k_p2_hist": "p2_hist", "k_p2_scan": "p2_scan", "k_p2_scatter": "p2_scatter"}
    if base in table and side:
        return f"{side}_{table[base]}"
    names = {"k_part_groupjoin": "part_groupjoin", "k_part_join_agg": "part_join_agg",
             "k_part_join_eager": "part_join_agg", "k_unit_count": "unit_count", "k_unit_emit": "unit_emit",
             "k_fused": "probe_agg", "k_finalize": "finalize", "k_join_build": "join_build",
             "k_join_probe": "join_probe", "k_join_gather": "join_gather", "k_filter_compact": "filter_compact",
             "k_pred_compiled": "pred_compiled", "k_pred_interpreted": "pred_interpreted", "k_bw_copy": "bw_copy",
             "k_bw_read": "bw_read", "k_bw_write": "bw_write", "k_key_minmax": "key_minmax", "k_keymap": "keymap",
             "k_index_clear": "join_table_init", "k_index_build": "join_build", "k_group_merge": "group_merge",
             "k_init_groups": "group_table_init", "k_index_verify": "join_index_verify"}
    return names.get(base, base)


def source_sha() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2608_13696_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg: str):
    print(f"[profiling] {msg}", flush=True)


def run_pass(outdir: str, args: list[str], bench_args: list[str], limit: int) -> str:
    d = os.path.join(outdir, f"pass_{int(time.time() * 1000)}")
    os.makedirs(d, exist_ok=True)
    cmd = ["rocprofv3", *args, "--output-format", "csv", "-d", d, "-o", "run", "--", sys.executable, "bench.py",
           *bench_args]
    log("$ " + " ".join(cmd))
    r = subprocess.run(cmd, cwd=ROOT, timeout=limit, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    with open(os.path.join(d, "stdout.txt"), "w") as f:
        f.write(r.stdout)
    if r.returncode != 0:
        # the profiler can end with a segmentation fault after a complete run: accept it when results exist
        if not glob.glob(os.path.join(d, "**", "*.csv"), recursive=True):
            raise RuntimeError(f"rocprofv3 failed ({r.returncode}):\n{r.stdout[-3000:]}")
        log(f"rocprofv3 exit {r.returncode}, results present")
    return d


def read_csv(d: str, suffix: str) -> list[dict]:
    rows = []
    for p in glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True):
        with open(p, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


# Kernels that one library call launches several times under one name: their
# counters and durations are summed per call, as the library's own timer spans
# all the launches. (None at present; the table keeps the summaries honest if
# a kernel is ever split into instances again.)
LAUNCHES_PER_CALL: dict = {}


def counter_means(d: str) -> dict:
    """{kernel name: {counter: mean value per call}} from a counter pass."""
    acc: dict = {}
    for r in read_csv(d, "counter_collection.csv"):
        k = timer_name(r["Kernel_Name"])
        c = r["Counter_Name"]
        v = float(r["Counter_Value"])
        disp = r.get("Dispatch_Id") or r.get("Correlation_Id")
        e = acc.setdefault(k, {}).setdefault(c, {})
        e[disp] = e.get(disp, 0.0) + v  # a counter can come as several rows (per XCD / instance) of one dispatch
    return {k: {c: sum(v.values()) / max(len(v) / LAUNCHES_PER_CALL.get(k, 1), 1) for c, v in cs.items()}
            for k, cs in acc.items()}


def kernel_stats(d: str) -> dict:
    out = {}
    for r in read_csv(d, "kernel_stats.csv"):
        k = timer_name(r["Name"])
        calls = int(r["Calls"])
        avg_ns = float(r["AverageNs"])
        e = out.setdefault(k, {"calls": 0, "total_ns": 0.0, "min_ns": float("inf"), "max_ns": 0.0})
        e["calls"] += calls / LAUNCHES_PER_CALL.get(k, 1)
        e["total_ns"] += avg_ns * calls
        e["min_ns"] = min(e["min_ns"], float(r.get("MinNs", avg_ns)))
        e["max_ns"] = max(e["max_ns"], float(r.get("MaxNs", avg_ns)))
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    ap.add_argument("--raw", default=os.path.join(ROOT, "gpurun_out", "prof"))
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--trace-steps", type=int, default=20)
    ap.add_argument("--passes", default="trace,fetch,write,valu,tcc,occ,lds")
    ap.add_argument("--calibrate", action="store_true", help="also profile the copy probe and write the factors")
    ap.add_argument("--limit", type=int, default=240, help="seconds per rocprofv3 run")
    args = ap.parse_args()
    os.makedirs(args.raw, exist_ok=True)
    os.makedirs(args.out, exist_ok=True)
    wl = args.workload
    bench = ["--workload", wl, "--steps", str(args.steps), "--warmup", "0", "--no-cpu-baseline"]
    passes = args.passes.split(",")
    cmd_lines = {}

    cal_path = os.path.join(args.out, "traffic_calibration.json")
    if args.calibrate:
        copy_args = ["--workload", "copy", "--steps", "2", "--warmup", "1"]
        f = counter_means(run_pass(args.raw, ["--pmc", "FETCH_SIZE"], copy_args, args.limit))["bw_copy"]["FETCH_SIZE"]
        w = counter_means(run_pass(args.raw, ["--pmc", "WRITE_SIZE"], copy_args, args.limit))["bw_copy"]["WRITE_SIZE"]
        gib_kib = float(1 << 20)
        cal = {"fetch_factor": gib_kib / f, "write_factor": gib_kib / w, "fetch_kib_per_launch": f,
               "write_kib_per_launch": w, "bytes_per_launch": 1 << 30,
               "commands": [f"rocprofv3 --pmc {c} --output-format csv -d <dir> -o run -- python3 bench.py "
                            + " ".join(copy_args) for c in ("FETCH_SIZE", "WRITE_SIZE")]}
        json.dump(cal, open(cal_path, "w"), indent=1)
        with open(os.path.join(args.out, "traffic_calibration.txt"), "w") as fh:
            fh.write("Counter calibration: the bandwidth probe's copy (rel_bw_probe, 1 GiB read + 1 GiB written "
                     "per launch)\n\nCommands (from the repository root, on the MI355X):\n")
            for c in cal["commands"]:
                fh.write(f"  {c}\n")
            fh.write(f"\nFETCH_SIZE per launch: {f:.1f} KiB for {gib_kib:.0f} KiB read   -> fetch factor "
                     f"{cal['fetch_factor']:.4f}\nWRITE_SIZE per launch: {w:.1f} KiB for {gib_kib:.0f} KiB written "
                     f"-> write factor {cal['write_factor']:.4f}\n\nHBM bytes of a kernel = FETCH_SIZE x 1024 x fetch "
                     "factor + WRITE_SIZE x 1024 x write factor.\n")
        log(f"calibration: fetch x{cal['fetch_factor']:.4f}, write x{cal['write_factor']:.4f}")
    cal = json.load(open(cal_path)) if os.path.exists(cal_path) else {"fetch_factor": 1.0, "write_factor": 1.0}

    stats = {}
    if "trace" in passes:
        targs = ["--workload", wl, "--steps", str(args.trace_steps), "--warmup", "3", "--no-cpu-baseline"]
        d = run_pass(args.raw, ["--kernel-trace", "--stats"], targs, args.limit)
        stats = kernel_stats(d)
        cmd_lines["trace"] = ("rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o run -- python3 bench.py "
                              + " ".join(targs))
        with open(os.path.join(args.out, f"kernels_{wl}.txt"), "w") as fh:
            fh.write(f"rocprofv3 kernel-trace statistics, workload '{wl}' (bench.py)\n\nCommand (from the repository "
                     f"root, on the MI355X), via python -m paper_2608_13696_amd.profiling --workload {wl}:\n  "
                     f"{cmd_lines['trace']}\n\n")
            for k, c in LAUNCHES_PER_CALL.items():
                if k in stats:
                    fh.write(f"{k}: {c} launches per call (calls and avg us per call; min and max per launch)\n")
            tot = sum(e["total_ns"] for e in stats.values()) or 1.0
            fh.write(f"{'kernel':34s} {'calls':>6s} {'avg us':>9s} {'min us':>9s} {'max us':>9s} {'% time':>7s}\n")
            for k, e in sorted(stats.items(), key=lambda kv: -kv[1]["total_ns"]):
                fh.write(f"{k[:34]:34s} {int(e['calls']):6d} {e['total_ns'] / e['calls'] / 1e3:9.1f} {e['min_ns'] / 1e3:9.1f} "
                         f"{e['max_ns'] / 1e3:9.1f} {100 * e['total_ns'] / tot:7.2f}\n")
        log(f"kernel trace written ({len(stats)} kernels)")

    per = {}  # kernel -> counter -> mean per dispatch
    for p in passes:
        if p == "trace":
            continue
        ctrs = PASSES[p]
        d = run_pass(args.raw, ["--pmc", *ctrs], bench, args.limit)
        cmd_lines[p] = f"rocprofv3 --pmc {' '.join(ctrs)} --output-format csv -d <dir> -o run -- python3 bench.py " + " ".join(bench)
        for k, cs in counter_means(d).items():
            per.setdefault(k, {}).update(cs)
        log(f"pass {p} done")

    sha = source_sha()
    lines = [f"Counters per dispatch (mean), workload '{wl}', from python -m paper_2608_13696_amd.profiling "
             f"--workload {wl}; one rocprofv3 run per counter group:"]
    for p in passes:
        if p in cmd_lines and p != "trace":
            lines.append(f"  {cmd_lines[p]}")
    lines.append(f"HBM bytes = FETCH_SIZE x 1024 x {cal['fetch_factor']:.4f} + WRITE_SIZE x 1024 x "
                 f"{cal['write_factor']:.4f} (traffic_calibration.txt). GHz = GRBM_GUI_ACTIVE / 8 XCDs / duration "
                 "(duration from the kernel trace). L2 hit = TCC_HIT / (TCC_HIT + TCC_MISS). waves/CU = "
                 "OccupancyPercent x 32 / 100 (resident waves per CU, 32 at most). wait = SQ_WAIT_ANY / "
                 "(SQ_WAVE_CYCLES), from OccupancyPercent's wave cycles. LDS conf = LdsBankConflict (conflict "
                 "cycles per conflict-free LDS cycle). VALU/B = SQ_INSTS_VALU per HBM byte (ridge 0.077 at 2.4 GHz).")
    lines.append("")
    hdr = (f"{'kernel':24s} {'us':>7s} {'read MB':>9s} {'write MB':>9s} {'GB/s':>6s} {'VALU M':>8s} {'VALU/B':>6s} "
           f"{'VMEM M':>7s} {'LDS M':>7s} {'GHz':>5s} {'L2 hit':>6s} {'waves/CU':>8s} {'wait':>5s} {'LDSconf':>7s}")
    lines.append(hdr)
    for k, cs in sorted(per.items(), key=lambda kv: -kv[1].get("FETCH_SIZE", 0.0)):
        rd = cs.get("FETCH_SIZE", 0.0) * 1024 * cal["fetch_factor"]
        wr = cs.get("WRITE_SIZE", 0.0) * 1024 * cal["write_factor"]
        dur = stats.get(k, {}).get("total_ns", 0.0) / max(stats.get(k, {}).get("calls", 1), 1)
        ghz = cs["GRBM_GUI_ACTIVE"] / 8 / dur if dur and cs.get("GRBM_GUI_ACTIVE") else None
        hit = (cs["TCC_HIT_sum"] / (cs["TCC_HIT_sum"] + cs["TCC_MISS_sum"])
               if cs.get("TCC_HIT_sum", 0) + cs.get("TCC_MISS_sum", 0) > 0 else None)
        occ = cs["OccupancyPercent"] * 32 / 100 if "OccupancyPercent" in cs else None
        wave_cycles = (cs["OccupancyPercent"] / 400 * 32 * 256 * cs["GRBM_GUI_ACTIVE"] / 8
                       if "OccupancyPercent" in cs and cs.get("GRBM_GUI_ACTIVE") else None)
        wait = cs["SQ_WAIT_ANY"] / wave_cycles if wave_cycles and "SQ_WAIT_ANY" in cs else None
        ldsc = cs.get("LdsBankConflict")
        vmem = (cs.get("SQ_INSTS_VMEM_RD", 0.0) + cs.get("SQ_INSTS_VMEM_WR", 0.0)) / 1e6
        gbs = (rd + wr) / dur if dur else None
        vpb = cs.get("SQ_INSTS_VALU", 0.0) / (rd + wr) if rd + wr > 0 else None
        f = lambda v, fmt: (fmt % v) if v is not None else "-"
        lines.append(f"{k[:24]:24s} {f(dur / 1e3 if dur else None, '%7.1f')} {rd / 1e6:9.1f} {wr / 1e6:9.1f} "
                     f"{f(gbs, '%6.0f')} {cs.get('SQ_INSTS_VALU', 0) / 1e6:8.2f} {f(vpb, '%6.3f')} {vmem:7.2f} "
                     f"{cs.get('SQ_INSTS_LDS', 0) / 1e6:7.2f} {f(ghz, '%5.2f')} {f(hit, '%6.3f')} {f(occ, '%8.2f')} "
                     f"{f(wait, '%5.2f')} {f(ldsc, '%7.3f')}")
        rec = {"kernel": k, "workload": wl, "src_sha": sha, "counters_per_dispatch": cs,
               "fetch_factor": cal["fetch_factor"], "write_factor": cal["write_factor"],
               "read_bytes_per_launch": rd, "write_bytes_per_launch": wr, "traffic_bytes_per_launch": rd + wr,
               "valu_insts_per_launch": cs.get("SQ_INSTS_VALU"), "clock_ghz": ghz, "l2_hit_rate": hit,
               "waves_per_cu": occ, "wait_frac": wait, "lds_bank_conflict": ldsc,
               "trace_avg_us": dur / 1e3 if dur else None,
               "commands": [cmd_lines[p] for p in passes if p in cmd_lines]}
        json.dump(rec, open(os.path.join(args.out, f"traffic_{k}_{wl}.json"), "w"), indent=1)
    with open(os.path.join(args.out, f"counters_{wl}.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    log(f"wrote counters_{wl}.txt and {len(per)} traffic json files")
    return 0


if __name__ == "__main__":
    sys.exit(main())
