"""rocprofv3 profiling of the benchmark and text summaries for ``profiles/``.

Usage on a GPU machine (from the repository root)::

    python -m paper_2507_20461_amd.profiling run       # kernel trace + counter passes,
                                                       # summaries into <OUT>/profiles
    python -m paper_2507_20461_amd.profiling summarize # summaries into profiles/

Each counter pass is its own rocprofv3 run (FETCH_SIZE, WRITE_SIZE, VALU
activity). Summaries record the commands, the per-kernel averages and a hash of
the kernel sources, so that the benchmark reports HBM traffic only for the
kernels the counters were taken on.

HBM traffic calibration: the benchmark runs one plain device-to-device copy of
256 MiB (the runtime's copy kernel: 256 MiB read, 256 MiB written) before
anything else; the ratio of its counted FETCH_SIZE / WRITE_SIZE to that size
scales the counts of the method's kernels.
"""
from __future__ import annotations

import collections
import csv
import glob
import hashlib
import json
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
OUT = os.path.join(ROOT, "gpurun_out")   # raw output folder of the runs (not committed)
PROFILES = os.path.join(ROOT, "profiles")
CAL_BYTES = 256 * 1024 * 1024
CAL_ELEMS = CAL_BYTES // 8

BENCH_FULL = ["python3", os.path.join(ROOT, "bench.py")]
BENCH_SHORT = ["python3", os.path.join(ROOT, "bench.py"), "--steps", "5", "--warmup", "1",
               "--no-cpu-baseline", "--no-kernel-timing", "--no-forms", "--no-batched", "--noncompact-steps", "2",
               "--no-paper-problems", "--tri-reps", "3"]
OWN = ("k_", "kb_", "k6_")   # prefixes of the library's kernels
PASSES = {
    "ktrace": (["--kernel-trace", "--stats"], BENCH_FULL),
    "fetch": (["--pmc", "FETCH_SIZE"], BENCH_SHORT),
    "write": (["--pmc", "WRITE_SIZE"], BENCH_SHORT),
    "valu": (["--pmc", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_WAVES", "GRBM_GUI_ACTIVE"], BENCH_SHORT),
    "stall": (["--pmc", "SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY",
               "SQ_ACTIVE_INST_VMEM", "SQ_LEVEL_WAVES", "SQ_INSTS_VALU_TRANS_F64", "SQ_INSTS_VMEM_RD"],
              BENCH_SHORT),
}
XCDS = 8          # GRBM_GUI_ACTIVE is summed over the XCDs of the device
SIMDS = 256 * 4   # 256 CUs x 4 SIMDs


def source_hash() -> str:
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(PKG, "csrc", "*"))):
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def command(name, extra=()):
    opts, bench = PASSES[name]
    return (["rocprofv3", *opts, "--output-format", "csv", "-d", os.path.join(OUT, "prof_" + name), "-o", "run",
             "--", *bench, *extra])


def run(extra=()):
    """One rocprofv3 run per pass. Stops at the first pass that fails, except
    for a segmentation fault of the profiler after the program has finished
    and the result file is complete."""
    os.makedirs(OUT, exist_ok=True)
    env = dict(os.environ, TMPDIR="/tmp")
    dest = os.path.join(OUT, "profiles")
    for name in PASSES:
        cmd = command(name, extra)
        print("==", " ".join(cmd), flush=True)
        with open(os.path.join(OUT, "prof_%s.log" % name), "w") as log:
            rc = subprocess.run(["timeout", "-s", "KILL", "420" if name == "ktrace" else "120", *cmd], stdout=log, stderr=log, env=env).returncode
        res = os.path.join(OUT, "prof_" + name, "run_kernel_stats.csv" if name == "ktrace"
                           else "run_counter_collection.csv")
        print("   exit %d, results %s" % (rc, "present" if os.path.exists(res) else "missing"), flush=True)
        if name == "ktrace" and os.path.exists(os.path.join(OUT, "prof_ktrace", "run_kernel_trace.csv")):
            # summarised next to the raw output at once; the per-dispatch
            # trace (tens of MB for the default benchmark) is then dropped
            summarize_ktrace(dest=dest)
            os.remove(os.path.join(OUT, "prof_ktrace", "run_kernel_trace.csv"))
        if rc != 0 and not (rc in (139, -11) and os.path.exists(res)):
            sys.exit(rc if rc > 0 else 1)
    summarize(dest=dest)


def _short(name):
    n = name.replace("void (anonymous namespace)::", "").replace("(anonymous namespace)::", "")
    return n.split("(")[0].strip()


def _counters(path, counter):
    """Per kernel name, the counter values of its dispatches on the largest
    grid it ran on (the benchmark's workload; a kernel also launched on
    smaller grids, as the non-compact stage on the paper's 1800-cell test,
    is summarised at the large size only)."""
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            d[_short(r["Kernel_Name"])].append((int(r["Grid_Size"]), float(r["Counter_Value"])))
    out = {}
    for k, v in d.items():
        g = max(x[0] for x in v)
        out[k] = [x[1] for x in v if x[0] == g]
    return out


def _cal_scale(path, counter):
    """The calibration copy is the first dispatch of the run (a device copy
    of CAL_BYTES made before any of the method's kernels)."""
    rows = sorted((r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter),
                  key=lambda r: int(r["Dispatch_Id"]))
    for r in rows:
        if _short(r["Kernel_Name"]).startswith(OWN):
            break
        v = float(r["Counter_Value"]) * 1024
        if abs(v - CAL_BYTES) <= 0.75 * CAL_BYTES:
            return v / CAL_BYTES
    return None


def summarize_ktrace(tag="stage_fp64_2048", dest=PROFILES):
    """Per-workload kernel averages from the kernel trace into
    <tag>_kernel_stats.txt, and the averages of the benchmark's two
    workloads into <tag>_ktrace_avg.json (read by the counter summary)."""
    os.makedirs(dest, exist_ok=True)
    sh = source_hash()
    lines = []
    # kernel trace, per workload: every gks_step call starts with k_init, so
    # the dispatches from one k_init to the next belong to one call; calls
    # are labelled by the element type and grid of their k_init
    trace = sorted(csv.DictReader(open(os.path.join(OUT, "prof_ktrace", "run_kernel_trace.csv"))),
                   key=lambda r: int(r["Dispatch_Id"]))
    label, per = None, collections.OrderedDict()
    for r in trace:
        k = _short(r["Kernel_Name"])
        cells = int(r["Grid_Size_X"])
        if k.startswith("k_init<2"):
            n = int(round(cells ** 0.5))
            label = "%s %dx%d" % ("mixed" if "float" in k else "fp64", n, n)
        if k.startswith("k6_init"):
            # one geno6_step call: 255 cells per work-group of 256 lanes
            label = "noncompact fp64 %d tiles of 255 cells" % (cells // 256)
        if k.startswith("k6_faces"):
            # a geno6_faces call (no k6_init before it)
            label = "noncompact faces fp64 %d lanes" % cells
        if k.startswith("k_tri"):
            # one lane per cell and variable (four variables)
            label = "triangles fp64 %d cells" % (cells // 4)
        if k.startswith("kb_"):
            lab = "batched (mixed)"
        elif label is None or not k.startswith(("k_", "k6_")):
            continue
        else:
            lab = label
        per.setdefault(lab, collections.OrderedDict()).setdefault(k, []).append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines.append("# rocprofv3 kernel trace of bench.py (default run), per workload")
    lines.append("# command: " + " ".join(command("ktrace")).replace(ROOT + "/", ""))
    lines.append("# kernel sources sha256[:16]: " + sh)
    lines.append("# workload labels: element type and grid of the gks_step call (k_init grid size = cells,")
    lines.append("# rounded to the next work-group); the bench's 2048x2048 workload is 'fp64 2048x2048', its")
    lines.append("# 2^24-cell non-compact workload 'noncompact fp64 65794 tiles of 255 cells', its")
    lines.append("# triangle mesh of 2 x 512^2 cells 'triangles fp64 524288 cells'")
    ktrace = {}
    for lab, ks in per.items():
        lines.append("")
        lines.append("[%s]" % lab)
        lines.append("%-28s %7s %10s %10s" % ("kernel", "calls", "avg_us", "total_ms"))
        for k, v in sorted(ks.items(), key=lambda kv: -sum(kv[1])):
            lines.append("%-28s %7d %10.2f %10.3f" % (k[:28], len(v), sum(v) / len(v), sum(v) / 1e3))
            if lab.startswith(("fp64 2048x2048", "noncompact fp64 65794 ", "triangles fp64 524288 ")):
                ktrace.setdefault(k, []).extend(v)
    ktrace = {k: sum(v) / len(v) for k, v in ktrace.items()}
    open(os.path.join(dest, "%s_kernel_stats.txt" % tag), "w").write("\n".join(lines) + "\n")
    open(os.path.join(dest, "%s_ktrace_avg.json" % tag), "w").write(json.dumps(ktrace, indent=1) + "\n")


def summarize(tag="stage_fp64_2048", dest=PROFILES):
    os.makedirs(dest, exist_ok=True)
    sh = source_hash()
    trace_csv = os.path.join(OUT, "prof_ktrace", "run_kernel_trace.csv")
    if os.path.exists(trace_csv):
        summarize_ktrace(tag, dest)
    ktrace = json.load(open(os.path.join(dest, "%s_ktrace_avg.json" % tag)))
    # counters
    F = _counters(os.path.join(OUT, "prof_fetch", "run_counter_collection.csv"), "FETCH_SIZE")
    Wr = _counters(os.path.join(OUT, "prof_write", "run_counter_collection.csv"), "WRITE_SIZE")
    V = {c: _counters(os.path.join(OUT, "prof_valu", "run_counter_collection.csv"), c)
         for c in ("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_WAVES", "GRBM_GUI_ACTIVE")}
    # the calibration copy is the largest dispatch that is not one of the method's kernels
    fcal = _cal_scale(os.path.join(OUT, "prof_fetch", "run_counter_collection.csv"), "FETCH_SIZE")
    wcal = _cal_scale(os.path.join(OUT, "prof_write", "run_counter_collection.csv"), "WRITE_SIZE")
    avg = lambda v: sum(v) / len(v)
    rows = {}
    for k in sorted(F):
        if not k.startswith(("k_", "k6_")):
            continue
        f, w = avg(F[k]) * 1024, avg(Wr.get(k, [0.0])) * 1024
        insts = avg(V["SQ_INSTS_VALU"].get(k, [0.0]))
        active = avg(V["SQ_ACTIVE_INST_VALU"].get(k, [0.0]))
        waves = avg(V["SQ_WAVES"].get(k, [0.0]))
        gui = avg(V["GRBM_GUI_ACTIVE"].get(k, [1.0])) / XCDS
        rows[k] = {"fetch_bytes": f, "write_bytes": w,
                   "fetch_bytes_cal": f / fcal if fcal else None, "write_bytes_cal": w / wcal if wcal else None,
                   "valu_insts_per_wave": insts / waves if waves else None,
                   "valu_busy": 4.0 * active / SIMDS / gui if gui else None}
    lines = ["# rocprofv3 counters per dispatch (separate --pmc passes), 2-D Euler 2048x2048 FP64 (k_*),",
             "# the 1-D non-compact workload of 2^24 cells (k6_*) and the triangle mesh of 2 x 512^2 cells",
             "# (k_tri)",
             "# commands:"]
    for name in ("fetch", "write", "valu"):
        lines.append("#   " + " ".join(command(name)).replace(ROOT + "/", ""))
    lines.append("# kernel sources sha256[:16]: " + sh)
    lines.append("# calibration: device copy of 256 MiB: FETCH scale %s, WRITE scale %s"
                 % ("%.4f" % fcal if fcal else "n/a", "%.4f" % wcal if wcal else "n/a"))
    lines.append("# valu_busy = 4 * SQ_ACTIVE_INST_VALU / (1024 SIMDs * GRBM_GUI_ACTIVE / 8 XCDs)")
    lines.append("%-28s %12s %12s %12s %12s %10s %9s" % ("kernel", "FETCH_MB", "WRITE_MB", "FETCH_cal", "WRITE_cal",
                                                        "valu/wave", "valu_busy"))
    for k, r in rows.items():
        lines.append("%-28s %12.2f %12.2f %12s %12s %10.0f %9.3f" % (
            k[:28], r["fetch_bytes"] / 1e6, r["write_bytes"] / 1e6,
            "%.2f" % (r["fetch_bytes_cal"] / 1e6) if r["fetch_bytes_cal"] else "n/a",
            "%.2f" % (r["write_bytes_cal"] / 1e6) if r["write_bytes_cal"] else "n/a",
            r["valu_insts_per_wave"] or 0, r["valu_busy"] or 0))
    spath = os.path.join(OUT, "prof_stall", "run_counter_collection.csv")
    if os.path.exists(spath):
        S = {c: _counters(spath, c) for c in ("SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY",
                                               "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VMEM", "SQ_LEVEL_WAVES",
                                               "SQ_INSTS_VALU_TRANS_F64", "SQ_INSTS_VMEM_RD")}
        lines.append("")
        lines.append("# per-wave shares of wave-cycles (one more --pmc pass):")
        lines.append("#   " + " ".join(command("stall")).replace(ROOT + "/", ""))
        lines.append("%-28s %9s %9s %9s %9s %11s %9s" % ("kernel", "wait_any", "wait_inst", "active", "vmem_act",
                                                       "trans64/wv", "vmemrd/wv"))
        for k in sorted(S["SQ_WAVE_CYCLES"]):
            if not k.startswith(("k_", "k6_")):
                continue
            wc = avg(S["SQ_WAVE_CYCLES"][k]) or 1.0
            nw = avg(V["SQ_WAVES"].get(k, [1.0])) or 1.0
            lines.append("%-28s %9.3f %9.3f %9.3f %9.3f %11.1f %9.1f" % (
                k[:28], avg(S["SQ_WAIT_ANY"][k]) / wc, avg(S["SQ_WAIT_INST_ANY"][k]) / wc,
                avg(S["SQ_ACTIVE_INST_ANY"][k]) / wc, avg(S["SQ_ACTIVE_INST_VMEM"][k]) / wc,
                avg(S["SQ_INSTS_VALU_TRANS_F64"][k]) / nw, avg(S["SQ_INSTS_VMEM_RD"][k]) / nw))
    open(os.path.join(dest, "%s_counters.txt" % tag), "w").write("\n".join(lines) + "\n")
    meta = {"source_hash": sh, "calibration": {"fetch": fcal, "write": wcal}, "kernels": rows,
            "ktrace_avg_us": ktrace}
    open(os.path.join(dest, "%s_counters.json" % tag), "w").write(json.dumps(meta, indent=1) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "summarize"
    if what == "run":
        run(sys.argv[2:])
    else:
        summarize()
