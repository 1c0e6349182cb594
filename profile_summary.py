"""Reduces raw rocprofv3 output into the short text summaries under profiles/.

Two kinds of input, both CSV files written by rocprofv3 with
``--output-format csv``:

  kernel trace   ``rocprofv3 --kernel-trace --stats ... -o kt`` writes
                 kt_kernel_stats.csv (name, calls, total / average / min /
                 max duration in ns); ``trace`` turns it into a markdown
                 table of the kernels by share of GPU time.
  counters       one ``rocprofv3 --pmc <counters> ... -o p`` run per counter
                 group writes p_counter_collection.csv (one row per dispatch
                 and counter); ``pmc`` takes the median per dispatch of each
                 counter for the sweep kernels and writes, per kernel class,
                 HBM bytes per launch and VALU instructions per launch in the
                 key: value form bench.py reads.

HBM bytes: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what
the same counters read for the plain copy kernel of the streaming benchmark
(claw_stream_bench's k_copy, 1 GiB read and 1 GiB written per dispatch) in
the same run, so the summary states bytes in the copy's calibration: on
MI355X FETCH_SIZE reads half the copy's 1 GiB (factor 2.000) and WRITE_SIZE
all of it (factor 1.000).

VALU issue: SQ_INSTS_VALU counts wave instructions.  Without packed FP32 a
wave64 VALU instruction occupies a SIMD for 4 clocks, so a launch of N
instructions needs at least 4 N / (1024 SIMDs x 2.4 GHz) seconds; the
summary divides that by the kernel's average traced duration to give the
fraction of the VALU issue peak (transcendental instructions take longer, so
this understates how busy the VALU is).

Usage:
  python profile_summary.py trace <kernel_stats.csv> <title> <command> > profiles/kernels_X.md
  python profile_summary.py pmc --title T --commands-file F --ncell N --real-bytes B \
      --trace <kernel_stats.csv> <counter_collection.csv> ... > profiles/pmc_sweeps_X.txt
"""
import argparse
import csv
import hashlib
import os
import statistics
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.abspath(__file__))
VALU_PEAK_SIMD_CLOCKS = 1024 * 2.4e9  # SIMDs x clock (Hz)
# kernel name patterns of each class (the whole-row x sweep is an x sweep; the
# fused x and y step of 3D acoustics moves as many bytes per launch as a sweep)
SWEEP_CLASSES = ((("k_sweep_row<", "k_sweep_row_whole<"), "x_sweep"), (("k_sweep_col<",), "y_sweep"),
                 (("k_sweep_col<",), "z_sweep"), (("k_step2d<",), "step2d"), (("k_step_xy3<",), "xy_step"))
FUSED_CLASSES = ("step2d", "xy_step")


def _col_normal(name):
    """Normal component (2: y sweep, 3: z sweep) of a k_sweep_col<R, SYS, MEQN, NRM, ...> name."""
    args = name.split("<", 1)[1].split(">", 1)[0].split(",")
    return args[3].strip() if len(args) > 3 else None


SOURCE_FILES = {"step2d": ("fused.hip", "step2d_body.inc", "sweep_body.h", "claw_device.h", "plugins.h"),
                "sweeps": ("sweeps.hip", "sweep_body.h", "claw_device.h", "plugins.h")}


def kernel_source_hash(kernel_class):
    """Hash of a kernel class's sources without comments and blank lines
    (the same function bench.py uses to accept a summary)."""
    h = hashlib.sha256()
    for f in SOURCE_FILES["step2d" if kernel_class in FUSED_CLASSES else "sweeps"]:
        with open(os.path.join(ROOT, "paper_1805_08846_amd", "csrc", f)) as fh:
            for line in fh:
                code = line.split("//", 1)[0].strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def read_stats(path):
    """kernel name -> (calls, average ns, min ns, max ns, total ns)."""
    out = {}
    with open(path) as fh:
        for row in csv.DictReader(fh):
            name = row.get("Name") or row.get("KernelName") or row.get("Kernel_Name")
            out[name] = (int(float(row["Calls"])), float(row["AverageNs"]), float(row["MinNs"]),
                         float(row["MaxNs"]), float(row["TotalDurationNs"]))
    return out


def trace(path, title, command):
    st = read_stats(path)
    total = sum(v[4] for v in st.values()) or 1.0
    lines = [f"# rocprofv3 kernel trace summary: {title}", "",
             f"command (from the repository root): {command}", "",
             "| kernel | calls | average (us) | min (us) | max (us) | share of GPU time |",
             "|---|---|---|---|---|---|"]
    for name, (calls, avg, mn, mx, tot) in sorted(st.items(), key=lambda kv: -kv[1][4]):
        short = name if len(name) <= 100 else name[:100]
        lines.append(f"| {short} | {calls} | {avg / 1e3:.2f} | {mn / 1e3:.2f} | {mx / 1e3:.2f} | "
                     f"{100 * tot / total:.1f} % |")
    return "\n".join(lines) + "\n"


def read_counters(paths):
    """(kernel name, counter) -> list of per-dispatch values in dispatch order."""
    vals = defaultdict(dict)
    for p in paths:
        with open(p) as fh:
            for row in csv.DictReader(fh):
                key = (row["Kernel_Name"], row["Counter_Name"])
                d = int(row["Dispatch_Id"])
                vals[key][d] = vals[key].get(d, 0.0) + float(row["Counter_Value"])
    return {k: [v[d] for d in sorted(v)] for k, v in vals.items()}


def _median(v):
    return statistics.median(v) if v else None


def pmc(args):
    c = read_counters(args.csv)
    kernels = sorted({k for k, _ in c})
    # the copy calibration comes from these runs, or from --calib runs (the
    # same counters for a workload whose command runs no copy kernel)
    cal = read_counters(args.calib) if args.calib else c
    copy = [k for k, _ in cal if "k_copy<false>" in k][:1]
    # one sweep reads and writes every field and reads the coefficient fields;
    # the fused step carries two sweeps
    alg = (2 * args.meqn + args.maux) * args.real_bytes * args.ncell
    out = [f"# rocprofv3 counters: {args.title}", ""]
    if args.commands_file:
        with open(args.commands_file) as fh:
            out += [ln.rstrip() for ln in fh if ln.strip()]
        out.append("")
    scale = {"FETCH_SIZE": 1.0, "WRITE_SIZE": 1.0}
    if copy:
        # the benchmark's first copy dispatches (warm-up and repetitions of the
        # achievable-bandwidth run) move 1 GiB each way (2^20 KiB read and written)
        for cn in scale:
            v = cal.get((copy[0], cn), [])[:3]
            if v and statistics.median(v) > 0.25 * 2 ** 20:
                scale[cn] = 2 ** 20 / statistics.median(v)
        src = ("runs " + " ".join(os.path.relpath(x, ROOT) for x in args.calib)) if args.calib else "same runs"
        out.append("calibration: plain copy kernel k_copy<false> (claw_stream_bench), 1 GiB read + 1 GiB "
                   f"written per dispatch (the run's first copy dispatches), {src}")
        for cn in scale:
            v = cal.get((copy[0], cn), [])[:3]
            if v and statistics.median(v) > 0.25 * 2 ** 20:
                out.append(f"- {cn} per copy dispatch (KiB): {statistics.median(v):.1f} -> scale {scale[cn]:.4f}")
        out.append("")
    out.append(f"algorithmic bytes per sweep launch: {alg}")
    stats = read_stats(args.trace) if args.trace else {}
    classes = []
    for pats, cls in SWEEP_CLASSES:
        # the MC-specialised kernels: sweeps <..., false (no speed pass), 0>, fused steps <..., 0>
        names = [k for k in kernels if any(p in k for p in pats) and
                 (", false, 0>" in k or (cls in FUSED_CLASSES and ", 0>" in k))]
        if cls in ("y_sweep", "z_sweep"):
            names = [k for k in names if _col_normal(k) == ("2" if cls == "y_sweep" else "3")]
        if not names:
            continue
        name = names[0]
        classes.append(cls)
        out.append("")
        n = len(c.get((name, "SQ_WAVES"), []) or c.get((name, "FETCH_SIZE"), []))
        out.append(f"{cls} kernel {name}: {n} dispatches (medians per dispatch)")
        fs, ws = _median(c.get((name, "FETCH_SIZE"), [])), _median(c.get((name, "WRITE_SIZE"), []))
        alg_k = alg * (2 if cls == "step2d" else 1)
        if fs is not None and ws is not None:
            rb, wb = fs * scale["FETCH_SIZE"] * 1024, ws * scale["WRITE_SIZE"] * 1024
            out.append(f"- algorithmic bytes per launch: {alg_k}")
            out.append(f"- FETCH_SIZE KiB: {fs:.1f} (scaled {rb / 1024:.1f})")
            out.append(f"- WRITE_SIZE KiB: {ws:.1f} (scaled {wb / 1024:.1f})")
            out.append(f"- {cls}_hbm_bytes_per_launch: {rb + wb:.0f}")
            k = 2 if cls == "step2d" else 1
            alg_r = k * (args.meqn + args.maux) * args.real_bytes * args.ncell
            alg_w = k * args.meqn * args.real_bytes * args.ncell
            out.append(f"- ratio to algorithmic bytes: {(rb + wb) / alg_k:.3f} (read {rb / alg_r:.3f}, "
                       f"written {wb / alg_w:.3f})")
        waves = _median(c.get((name, "SQ_WAVES"), []))
        valu = _median(c.get((name, "SQ_INSTS_VALU"), []))
        if waves:
            out.append(f"- SQ_WAVES: {waves:.0f}")
        if valu:
            out.append(f"- {cls}_valu_insts_per_launch: {valu:.0f}")
            if waves:
                out.append(f"- VALU instructions per wave: {valu / waves:.1f}; per cell (x 64 lanes / cells): "
                           f"{valu * 64 / args.ncell:.1f}")
            salu = _median(c.get((name, "SQ_INSTS_SALU"), []))
            if salu and waves:
                out.append(f"- SQ_INSTS_SALU: {salu:.0f} ({salu / waves:.1f} per wave)")
            tr = [v for k, v in stats.items() if k.startswith(name.split("(")[0])]
            if tr:
                avg_s = tr[0][1] * 1e-9
                frac = 4 * valu / (VALU_PEAK_SIMD_CLOCKS * avg_s)
                out.append(f"- traced average duration: {tr[0][1] / 1e3:.2f} us -> VALU issue fraction = "
                           f"4 x SQ_INSTS_VALU / (1024 SIMDs x 2.4 GHz x duration) = {frac:.3f}")
                out.append(f"- {cls}_valu_issue_frac_per_launch: {frac:.4f}")
    out.append("")
    for cls in classes:
        out.append(f"{cls}_source_hash: {kernel_source_hash(cls)}")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("stats")
    t.add_argument("title")
    t.add_argument("command")
    p = sub.add_parser("pmc")
    p.add_argument("csv", nargs="+")
    p.add_argument("--title", required=True)
    p.add_argument("--commands-file")
    p.add_argument("--ncell", type=int, required=True)
    p.add_argument("--real-bytes", type=int, default=4)
    p.add_argument("--meqn", type=int, default=3, help="fields per cell (3 shallow water, 4 3D acoustics)")
    p.add_argument("--maux", type=int, default=0, help="coefficient fields a sweep reads per cell")
    p.add_argument("--calib", nargs="+", help="counter CSVs of runs with the copy kernel, for the calibration")
    p.add_argument("--trace")
    a = ap.parse_args()
    if a.cmd == "trace":
        sys.stdout.write(trace(a.stats, a.title, a.command))
    else:
        sys.stdout.write(pmc(a))


if __name__ == "__main__":
    main()
