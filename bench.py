"""Throughput benchmark of the split wave-propagation step on one MI355X.

Workload (default): 2D shallow water, Roe solver with entropy fix, MC limiter,
8192 x 8192 cells on [-2.5, 2.5]^2 (768 MiB per state, beyond the 256 MB
MALL, so the bandwidth figure is an HBM figure), radial dam break with seeded
+-1e-3 noise on h, reflecting walls, CFL 0.9, FP32.  The 2048 x 2048
configuration (whose working set stays in the MALL) runs next and is reported
under "mall_resident_2048".  A step is one adaptive time step of
the whole path: x sweep, y sweep (Riemann solve, limiter, correction flux,
update, fused speed maximum) and the device CFL control.  The timed region is
K steps run from captured HIP graphs (claw_advance) with the state resident
in HBM; value = cells * K / T in Gcell-updates/s.

The roofline object reports the dominant sweep kernel: algorithmic bytes per
launch (each sweep reads and writes every field of every cell once:
2 * meqn * sizeof(real) * cells) divided by its average duration, measured
with HIP events around every kernel launch on the solver's stream over a
second run of the same steps.  cpu_baseline times the CPU oracle (FP64, all
host threads) on the first steps of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f32|f64]
"""
import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E


# the sources each kernel class is built from (the shared headers and its own file)
SOURCE_FILES = {"step2d": ("fused.hip", "step2d_body.inc", "sweep_body.h", "claw_device.h", "plugins.h"),
                "sweeps": ("sweeps.hip", "sweep_body.h", "claw_device.h", "plugins.h")}


def kernel_source_hash(kernel_class):
    """Hash of the sources of a kernel class (step2d, xy_step: the fused 2D step
    and the fused x and y step of 3D acoustics; x_sweep, y_sweep, z_sweep: the
    sweeps) with comments and blank lines removed (a
    PMC summary stays valid across comment edits, not across code edits)."""
    h = hashlib.sha256()
    for f in SOURCE_FILES["step2d" if kernel_class in ("step2d", "xy_step") else "sweeps"]:
        with open(os.path.join(ROOT, "paper_1805_08846_amd", "csrc", f)) as fh:
            for line in fh:
                code = line.split("//", 1)[0].strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def load_pmc(path, kernel_class, quantity):
    """A per-launch figure (quantity: "hbm_bytes", "valu_insts") of a kernel
    class from a committed rocprofv3 PMC summary, or None if missing or taken
    on other sources of that kernel class."""
    if not path or not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip().lstrip("-* ")
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get(f"{kernel_class}_source_hash") != kernel_source_hash(kernel_class):
        return None
    key = f"{kernel_class}_{quantity}_per_launch"
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def load_traffic(path, kernel_class):
    """HBM bytes per launch of a kernel class (calibrated FETCH_SIZE + WRITE_SIZE)."""
    return load_pmc(path, kernel_class, "hbm_bytes")


# VALU issue peak of MI355X without packed FP32: 256 CUs x 4 SIMDs x 16 lanes
# per clock x 2.4 GHz (a wave64 instruction occupies a SIMD for 4 clocks).
VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9


def host_cpu():
    """Model name and clock of the host CPU (from /proc/cpuinfo and sysfs)."""
    model, mhz = None, []
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name") and model is None:
                    model = line.split(":", 1)[1].strip()
                elif line.startswith("cpu MHz"):
                    mhz.append(float(line.split(":", 1)[1]))
    except OSError:
        pass
    max_mhz = None
    try:
        with open("/sys/devices/system/cpu/cpu0/cpufreq/cpuinfo_max_freq") as fh:
            max_mhz = int(fh.read().strip()) / 1000.0
    except (OSError, ValueError):
        pass
    return {"cpu_model": model, "cpu_mhz_now_mean": (sum(mhz) / len(mhz)) if mhz else None,
            "cpu_mhz_max": max_mhz, "logical_cpus": os.cpu_count()}


def cpu_baseline(prob, q0, steps, aux=None):
    import oracle
    t0 = time.perf_counter()
    res = oracle.advance(prob, q0, aux, steps)
    dt = time.perf_counter() - t0
    ncell = prob["n"][0] * prob["n"][1] * prob["n"][2]
    out = {
        "value": ncell * steps / dt / 1e9,
        "unit": "Gcell-updates/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"first {steps} adaptive steps ({steps + res['nreject']} trials) of the same "
                  f"{'x'.join(str(v) for v in prob['n'][:prob['ndim']])} workload, FP64 oracle, {dt:.2f} s",
    }
    out.update(host_cpu())
    return out


def achievable_bandwidth(torch, claw, nbytes=1 << 30, reps=10):
    """GB/s of the library's streaming microbenchmark kernels (copy, copy with
    non-temporal stores, read, write, write non-temporal) over two buffers."""
    a = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    res = claw.claw_stream_bench(a, b, reps, torch.cuda.current_stream().cuda_stream)
    del a, b
    return res


def bench_ensemble(args, torch, claw, inputs):
    """Batched ensemble of 256 shallow-water instances (sides U{128..1024},
    Gaussian humps, walls, FP32) for `steps` accepted steps each.  The batch
    runs the fused 2D step (one opening and one fused launch per trial for all
    instances; --split-step: the batched x and y sweeps); it is compared with
    the batch on the other step and with the same instances advanced one
    after another through the single-grid path on the library's default step
    (the x and y sweeps at these sizes).  A batch equals its single grids on
    the same step bit for bit (tested); the fused and the split step agree to
    FP32 rounding, so the L1 error is the same and the speedups are ratios of
    times."""
    steps = args.steps if args.steps_given else 500
    members = inputs.sw_ensemble(count=args.count, seed=0, dtype="f32", nsteps=steps)
    cells = sum(p["n"][0] * p["n"][1] for p, _ in members)
    warm = args.warmup if args.warmup_given else 1

    def run_batch(fused):
        probs = [dict(p, fused_step=fused) for p, _ in members]
        qs = [torch.tensor(q0, dtype=torch.float32, device="cuda").contiguous() for _, q0 in members]
        b = claw.BatchSolver(probs, qs)
        tuned = b.tune(os.environ.get("CLAW_AUTOTUNE_CACHE"))
        print(f"# ensemble ({'fused' if fused else 'split'}): {len(members)} instances, {cells} cells; "
              f"tuned {tuned}", file=sys.stderr, flush=True)
        # untimed steps, as for the single-grid runs below: all time steps
        # warm+1 .. warm+steps (the autotuning above has warmed the GPU)
        b.advance(warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rej = b.advance(steps)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        b.close()
        return t, tuned, int(sum(rej))

    fused = args.fused_step is not False
    t_batch, tuned, nrej = run_batch(fused)
    t_other, tuned_other, _ = run_batch(not fused)
    # the same instances one after another through the single-grid path
    t_single = 0.0
    for p, q0 in members:
        q = torch.tensor(q0, dtype=torch.float32, device="cuda").contiguous()
        s = claw.Solver(p, q)
        s.advance(warm)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.advance(steps)
        torch.cuda.synchronize()
        t_single += time.perf_counter() - t1
        s.close()
    value = cells * steps / t_batch / 1e9
    return {
        "metric": "ensemble Gcell-updates/s",
        "value": value,
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": t_batch / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Gaussian humps, sides U{128..1024})",
        "config": {"workload": "batched 2D shallow-water ensemble, walls, MC, CFL 0.9, adaptive dt per "
                               "instance", "instances": len(members), "cells": cells,
                   "parallelism": "single GPU"},
        "step": "fused 2D step" if fused else "x and y sweeps",
        "tuned": tuned,
        "rejected_trials": nrej,
        "batch_seconds": t_batch,
        ("split" if fused else "fused") + "_batch": {"value": cells * steps / t_other / 1e9, "seconds": t_other,
                                                     "tuned": tuned_other},
        "single_grid_seconds": t_single,
        "single_grid_value": cells * steps / t_single / 1e9,
        "speedup_vs_single_grid": t_single / t_batch,
    }


def bench_learned(args, torch, claw, inputs):
    """Learned coarse correction: train the two direction networks on the GPU
    (200 seeded Gaussian-hump runs at 1024^2, 500 fine steps each, samples
    every 2 fine steps coarse-grained to 512^2), then on held-out seeds compare
    the corrected 512^2 run with plain 512^2 and 1024^2 runs against the plain
    2048^2 run coarse-grained (L1 of depth over T = 250 coarse steps).  The
    value is the speedup at equal L1: T_plain(n_eq) / T_learned."""
    from paper_1805_08846_amd import learned
    runs = args.train_runs
    t0 = time.perf_counter()
    tr = learned.Trainer(n_fine=1024, total_samples=runs * 250)
    for k in range(runs):
        tr.run(seed=1000 + k)
        if (k + 1) % 25 == 0:
            print(f"# learned: {k + 1} of {runs} training runs", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    print(f"# learned: trained on {runs} runs ({tr.samples} Adam steps) in {t_train:.1f} s", file=sys.stderr,
          flush=True)
    seeds = list(range(1, 1 + args.eval_seeds))
    one_plain, one_learned = learned.one_step_gain(tr.lc, seeds=seeds[:2])
    res = learned.evaluate(tr.lc, seeds=seeds, steps_coarse=250)
    rows = res.pop("rows")
    tr.close()
    fields = {
        "plain_512": np.mean([r["plain"][512]["l1_fields"] for r in rows], axis=0).tolist(),
        "plain_1024": np.mean([r["plain"][1024]["l1_fields"] for r in rows], axis=0).tolist(),
        "learned_512": np.mean([r["learned"]["l1_fields"] for r in rows], axis=0).tolist(),
    }
    return {
        "metric": "speedup at equal L1 error vs plain fine grid (learned 512^2)",
        "value": res["speedup_equal_l1"],
        "unit": "x",
        "n_gpus": 1,
        "steps": 250,
        "warmup": 0,
        "ms_per_step": res["seconds_learned"] / 250 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 state, bf16 network (fp32 accumulation)",
        "data": "synthetic (seeded Gaussian humps; held-out seeds for evaluation)",
        "config": {"workload": "learned coarse flux correction, shallow water 512^2 (trained at 1024^2, "
                               "reference 2048^2)", "train_runs": runs, "eval_seeds": seeds,
                   "parallelism": "single GPU"},
        "l1_depth": {"plain_512": res["l1_plain"][0], "plain_1024": res["l1_plain"][-1],
                     "learned_512": res["l1_learned"]},
        "l1_fields_h_hu_hv": fields,
        "seconds_per_run": {"plain_512": res["seconds_plain"][0], "plain_1024": res["seconds_plain"][-1],
                            "learned_512": res["seconds_learned"]},
        "n_equal": res["n_equal"],
        "note": res.get("note"),
        "one_step_l1_h_hu_hv": {"plain": one_plain, "learned": one_learned},
        "mass_drift_max": res["mass_drift_max"],
        "train_seconds": t_train,
    }


def restart_after_warmup(torch, solver, q, warmup):
    """Runs `warmup` untimed steps (clocks, caches, the captured step graph),
    then puts the initial state back and restarts the clock at t = 0, so the
    timed steps are the workload's first steps."""
    if warmup <= 0:
        torch.cuda.synchronize()
        return
    q_init = q.clone()
    solver.advance(warmup)
    q.copy_(q_init)
    solver.set_control(0.0, 0.0)
    torch.cuda.synchronize()


def _timed_run(torch, claw, prob, q0, steps, warmup, timed_steps):
    """Throughput (Gcell-updates/s) of claw_advance on one grid and per-kernel
    average durations (us) from the event-timed path."""
    ncell = prob["n"][0] * prob["n"][1] * prob["n"][2]
    tdt = torch.float32 if prob["dtype"] == "f32" else torch.float64
    q = torch.tensor(q0, dtype=tdt, device="cuda").contiguous()
    solver = claw.Solver(prob, q, None)
    restart_after_warmup(torch, solver, q, warmup)
    t0 = time.perf_counter()
    _, nrej = solver.advance(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms, cnt = solver.advance_timed(timed_steps)
    avg_us = {n: (ms[k] / cnt[k] * 1e3 if cnt[k] else None)
              for k, n in enumerate(["x_sweep", "y_sweep", "z_sweep", "control"])}
    solver.close()
    del q
    return {"value": ncell * steps / elapsed / 1e9, "ms_per_step": elapsed / steps * 1e3,
            "kernel_avg_us": avg_us, "rejected_trials": nrej}


def bench_plugin(args, torch, claw, inputs):
    """Point-wise solver plug-ins at 2048^2 FP32: the scalar Burgers-type law
    (one field, one wave), and shallow water through the plug-in path next to
    the specialised shallow-water sweep on the same dam break."""
    n = args.n if args.n_given else 2048
    steps = args.steps if args.steps_given else 1000
    warmup = args.warmup if args.warmup_given else 3000
    prob, q0, _ = inputs.burgers2d(n=n, seed=0, dtype=args.dtype, nsteps=steps)
    print(f"# burgers {n}^2 {args.dtype}", file=sys.stderr, flush=True)
    bur = _timed_run(torch, claw, prob, q0, steps, warmup, args.timed_steps)
    real_bytes = 4 if args.dtype == "f32" else 8
    ncell = n * n
    alg_bytes = 2 * 1 * real_bytes * ncell  # one field read and written per sweep
    dom = max(("x_sweep", "y_sweep"), key=lambda k: bur["kernel_avg_us"][k])
    achieved = alg_bytes / (bur["kernel_avg_us"][dom] * 1e-6) / 1e9
    swp, swq0, _ = inputs.sw_radial_dam(n=n, dtype=args.dtype, nsteps=steps)
    print(f"# shallow water {n}^2 {args.dtype}: specialised, then plug-in", file=sys.stderr, flush=True)
    spec = _timed_run(torch, claw, swp, swq0, steps, warmup, args.timed_steps)
    gen = _timed_run(torch, claw, dict(swp, solver="generic"), swq0, steps, warmup, args.timed_steps)
    line = {
        "metric": "Gcell-updates/s", "value": bur["value"], "unit": "Gcell-updates/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": bur["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
        "data": "synthetic (seeded signed Gaussian bumps on 0.1; seeded radial dam break)",
        "config": {"workload": "plug-in Riemann solvers: 2D Burgers-type law (c = (1, 0.5)), MC, "
                               "periodic, CFL 0.9; shallow water as a plug-in vs specialised",
                   "grid": [n, n], "cells": ncell, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": None, "kernel": "burgers_" + dom,
                     "alg_bytes_per_launch": alg_bytes, "avg_launch_us": bur["kernel_avg_us"][dom]},
        "burgers": bur,
        "shallow_water_specialised": spec,
        "shallow_water_plugin": gen,
        "plugin_over_specialised": gen["value"] / spec["value"],
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob, q0, args.cpu_steps or max(2, int(round(1e9 / ncell))))
    return line


def bench_ac3d(args, torch, claw, inputs):
    """3D linear acoustics in a two-layer medium, 256^3 FP32 (per-cell rho, K):
    throughput of the adaptive graph path and the slowest sweep against HBM."""
    n = args.n if args.n_given else 256
    steps = args.steps if args.steps_given else 200
    warmup = args.warmup if args.warmup_given else 200
    prob, q0, aux = inputs.acoustics3d_layers(n=n, dtype=args.dtype, nsteps=steps)
    prob["fused_step"] = args.fused_step  # None: the library's choice (the fused x and y step at 256^3 FP32)
    ncell = n ** 3
    tdt = torch.float32 if args.dtype == "f32" else torch.float64
    q = torch.tensor(q0, dtype=tdt, device="cuda").contiguous()
    qa = torch.tensor(aux, dtype=tdt, device="cuda").contiguous()
    solver = claw.Solver(prob, q, qa)
    print(f"# acoustics3d_layers {n}^3 {args.dtype}: warmup {warmup}", file=sys.stderr, flush=True)
    restart_after_warmup(torch, solver, q, warmup)
    t0 = time.perf_counter()
    _, nrej = solver.advance(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms, cnt = solver.advance_timed(args.timed_steps)
    solver.close()
    fused = cnt[0] > 0 and cnt[1] == 0  # slot 0 holds the fused x and y step
    names = ["xy_step" if fused else "x_sweep", "y_sweep", "z_sweep", "control"]
    avg_us = {names[k]: (ms[k] / cnt[k] * 1e3 if cnt[k] else None) for k in range(4) if cnt[k] or k != 1}
    dom = max(range(3), key=lambda k: ms[k] / cnt[k] if cnt[k] else 0.0)
    real_bytes = 4 if args.dtype == "f32" else 8
    # per launch, a sweep and the fused x and y step alike: p, u, v, w read and
    # written, Z and c read
    alg_bytes = (2 * 4 + 2) * real_bytes * ncell
    dom_s = ms[dom] / cnt[dom] * 1e-3
    achieved = alg_bytes / dom_s / 1e9
    pmc_file = os.path.join(ROOT, "profiles", f"pmc_sweeps_ac3d{n}_{args.dtype}.txt")
    line = {
        "metric": "Gcell-updates/s + % HBM roofline", "value": ncell * steps / elapsed / 1e9,
        "unit": "Gcell-updates/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": elapsed / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.dtype,
        "data": "synthetic (two-layer medium, Gaussian pulse at a seeded centre)",
        "config": {"workload": "3D linear acoustics, two-layer medium (rho 1 / 4, K 1), extrapolation, "
                               "MC, CFL 0.9", "grid": [n, n, n], "cells": ncell, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": load_traffic(pmc_file, names[dom]),
                     "kernel": names[dom], "alg_bytes_per_launch": alg_bytes, "avg_launch_us": dom_s * 1e6},
        "kernel_avg_us": avg_us, "rejected_trials": nrej,
        "path": "fused x and y step, then the z sweep" if fused else "x, y and z sweeps",
        # the metric's whole-step figure: the method's bytes per cell-update
        # (three sweeps of 40 B in FP32) at the measured rate, against 8 TB/s;
        # the fused path moves two sweeps' worth, so this can exceed what its
        # kernels move (the roofline above charges each launch its own bytes)
        "hbm_frac_whole_step": (ncell * steps / elapsed) * 3 * alg_bytes / ncell / (HBM_PEAK_GBPS * 1e9),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob, q0, args.cpu_steps or 10, aux)
    return line


def bench_sizes(args, torch, claw, inputs):
    """The radial dam break scaled from 256^2 to 16384^2 (FP32, plus FP64 at
    4096^2): throughput and the slower sweep against HBM at each size, from the
    MALL-resident sizes to the HBM-bound ones."""
    steps = args.steps if args.steps_given else 200
    rows = []
    cases = [(n, "f32") for n in (256, 512, 1024, 2048, 4096, 8192, 16384)] + [(4096, "f64")]
    for n, dt in cases:
        prob, q0, _ = inputs.sw_radial_dam(n=n, dtype=dt, nsteps=steps)
        warm = max(200, min(3000, int(2e9 // (n * n))))
        print(f"# sizes {n}^2 {dt}: warmup {warm}", file=sys.stderr, flush=True)
        r = _timed_run(torch, claw, prob, q0, steps, warm, min(args.timed_steps, 20))
        us = r["kernel_avg_us"]
        dom = max(("x_sweep", "y_sweep"), key=lambda k: us[k])
        alg = 2 * 3 * (4 if dt == "f32" else 8) * n * n
        frac = alg / (us[dom] * 1e-6) / 1e9 / HBM_PEAK_GBPS
        whole = r["value"] * 1e9 * 2 * alg / (n * n) / (HBM_PEAK_GBPS * 1e9)
        rows.append({"n": n, "dtype": dt, "Gcell_per_s": r["value"], "x_us": us["x_sweep"],
                     "y_us": us["y_sweep"], "sweep_frac_hbm": frac, "step_frac_hbm": whole})
        del q0
        torch.cuda.empty_cache()
    big = [r for r in rows if r["n"] == 8192 and r["dtype"] == "f32"][0]
    return {
        "metric": "Gcell-updates/s + % HBM roofline (size sweep)", "value": big["Gcell_per_s"],
        "unit": "Gcell-updates/s (8192^2 FP32)", "n_gpus": 1, "steps": steps, "warmup": None,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (and f64 at 4096^2)",
        "data": "synthetic (seeded radial dam break + U(-1e-3,1e-3) noise on h)",
        "config": {"workload": "2D shallow water radial dam break, walls, MC, CFL 0.9, sides 256..16384",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": big["sweep_frac_hbm"] * HBM_PEAK_GBPS,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": big["sweep_frac_hbm"],
                     "traffic": None, "kernel": "slower sweep at 8192^2"},
        "sizes": rows,
    }


def bench_dpsp(args, torch, claw, inputs):
    """Double and single precision at 1024^2 (the radial dam break): the GPU
    path against the oracle on the host cores, each precision (the oracle's
    FP32 instantiation is the same source with real = float)."""
    import oracle
    n = 1024
    steps = args.steps if args.steps_given else 500
    warmup = args.warmup if args.warmup_given else 1500
    cpu_steps = args.cpu_steps or 150
    out = {}
    for dt in ("f64", "f32"):
        prob, q0, _ = inputs.sw_radial_dam(n=n, dtype=dt, nsteps=steps)
        print(f"# dpsp {n}^2 {dt}: gpu", file=sys.stderr, flush=True)
        g = _timed_run(torch, claw, prob, q0, steps, warmup, args.timed_steps)
        print(f"# dpsp {n}^2 {dt}: oracle {cpu_steps} steps", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        oracle.advance(prob, q0, None, cpu_steps, precision=dt)
        el = time.perf_counter() - t0
        cpu = n * n * cpu_steps / el / 1e9
        out[dt] = {"gpu_Gcell_per_s": g["value"], "gpu_kernel_avg_us": g["kernel_avg_us"],
                   "oracle_Gcell_per_s": cpu, "oracle_seconds": el, "gpu_over_oracle": g["value"] / cpu}
    return {
        "metric": "GPU over CPU oracle, FP64 and FP32 (1024^2 shallow water)",
        "value": out["f64"]["gpu_over_oracle"], "unit": "x (FP64)", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 and f32",
        "data": "synthetic (seeded radial dam break + U(-1e-3,1e-3) noise on h)",
        "config": {"workload": "2D shallow water radial dam break at 1024^2, walls, MC, CFL 0.9",
                   "grid": [n, n], "parallelism": "single GPU; oracle on the host cores"},
        "results": out,
        "fp32_over_fp64_gpu": out["f32"]["gpu_Gcell_per_s"] / out["f64"]["gpu_Gcell_per_s"],
        "cpu_cores": oracle.num_threads(),
        "cpu_sample": f"first {cpu_steps} adaptive steps of each precision",
    }


def run_record(torch):
    """Provenance of a run for the JSONL record: time, command, sources (git
    commit where a checkout is present, and the kernel classes' source
    hashes), host CPU, GPU and software versions."""
    sha = None
    try:
        sha = subprocess.run(["git", "rev-parse", "HEAD"], cwd=ROOT, capture_output=True, text=True,
                             timeout=10).stdout.strip() or None
    except (OSError, subprocess.SubprocessError):
        pass
    return {"time_utc": time.strftime("%Y-%m-%dT%H:%M:%SZ", time.gmtime()), "argv": sys.argv[1:],
            "git_sha": sha, "source_hashes": {k: kernel_source_hash(k) for k in ("step2d", "x_sweep")},
            "host": host_cpu(), "gpu": torch.cuda.get_device_name(0), "torch": torch.__version__,
            "hip": getattr(torch.version, "hip", None)}


def emit(line, args, torch):
    """Prints the result line; with --record (or CLAW_RECORD) also appends it,
    with the run's provenance, to a JSONL file."""
    print(json.dumps(line), flush=True)
    path = args.record or os.environ.get("CLAW_RECORD")
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps(dict(line, record=run_record(torch))) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 100 at 8192^2, the 2048^2 configuration's 1000)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (also lets the GPU clocks ramp up); default 300 / 3000")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--n", type=int, default=8192,
                    help="grid side of the headline run (8192: beyond the MALL; 2048 also runs, as extra keys)")
    ap.add_argument("--timed-steps", type=int, default=200,
                    help="steps of the per-kernel event timing run")
    ap.add_argument("--reps", type=int, default=5,
                    help="timed repetitions of the steps from the initial state (median reported)")
    ap.add_argument("--cpu-steps", type=int, default=None,
                    help="oracle steps of the CPU baseline sample (default: about 1e9 cell-updates, "
                         "10-20 s on 16 threads)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-bw", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="skip the 2048^2 run that follows the headline size (profiling runs)")
    ap.add_argument("--traffic-file", default=None)
    ap.add_argument("--record", default=None,
                    help="append the result line with its provenance to this JSONL file (default: $CLAW_RECORD)")
    ap.add_argument("--workload", default="sw2048", choices=["sw2048", "ensemble", "learned", "plugin", "dpsp", "ac3d", "sizes"])
    ap.add_argument("--fused-step", dest="fused_step", action="store_const", const=True, default=None,
                    help="one fused kernel per 2D step (CLAW_FLAG_FUSED_STEP) at every size")
    ap.add_argument("--split-step", dest="fused_step", action="store_const", const=False,
                    help="x and y sweep kernels at every size (CLAW_FLAG_SPLIT_STEP); by default the "
                         "library fuses FP32 steps for states of 96 MiB and more")
    ap.add_argument("--count", type=int, default=256, help="ensemble instances")
    ap.add_argument("--train-runs", type=int, default=200, help="learned: training runs")
    ap.add_argument("--eval-seeds", type=int, default=5, help="learned: held-out evaluation seeds")
    args = ap.parse_args()
    args.steps_given = args.steps is not None
    args.warmup_given = args.warmup is not None
    args.n_given = "--n" in sys.argv

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the "
              "multi-GPU decomposition is a design note, not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1805_08846_amd import claw, inputs

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.workload == "ensemble":
        emit(bench_ensemble(args, torch, claw, inputs), args, torch)
        return
    if args.workload == "learned":
        emit(bench_learned(args, torch, claw, inputs), args, torch)
        return
    if args.workload == "plugin":
        emit(bench_plugin(args, torch, claw, inputs), args, torch)
        return
    if args.workload == "sizes":
        emit(bench_sizes(args, torch, claw, inputs), args, torch)
        return
    if args.workload == "ac3d":
        emit(bench_ac3d(args, torch, claw, inputs), args, torch)
        return
    if args.workload == "dpsp":
        emit(bench_dpsp(args, torch, claw, inputs), args, torch)
        return

    n = args.n
    steps = args.steps if args.steps_given else (100 if n >= 4096 else 1000)
    warmup = args.warmup if args.warmup_given else (300 if n >= 4096 else 3000)
    line = bench_grid(args, torch, claw, inputs, n, steps, warmup, headline=True)
    if n != 2048 and not args.headline_only:
        # the 2048^2 configuration itself (its 3 x 48 MiB working set stays in
        # the 256 MB MALL, so its bandwidth figure is not an HBM figure)
        st2 = args.steps if args.steps_given else 1000
        wu2 = args.warmup if args.warmup_given else 3000
        line["mall_resident_2048"] = bench_grid(args, torch, claw, inputs, 2048, st2, wu2, headline=False)
    if not args.no_copy_bw:
        bw = achievable_bandwidth(torch, claw)
        line["achievable_GBps"] = bw
        best_rw = max(bw["copy"], bw["copy_nt"])
        # a sweep and the fused step both read the state once and write it once:
        # that copy rate of the dominant kernel against the copy kernels
        rf = line["roofline"]
        state_rate = 2 * rf["state_bytes"] / (rf["avg_launch_us"] * 1e-6) / 1e9
        rf["state_copy_GBps"] = state_rate
        rf["frac_of_achievable_copy"] = state_rate / best_rw
        # the same copy kernels at the state's size, back to back like the
        # sweeps: launch gaps and ramp included
        bw_s = achievable_bandwidth(torch, claw, nbytes=rf["state_bytes"], reps=50 if n >= 4096 else 200)
        line["achievable_GBps_sweep_size"] = bw_s
        rf["frac_of_copy_at_sweep_size"] = state_rate / max(bw_s["copy"], bw_s["copy_nt"])
    if not args.no_cpu_baseline:
        prob, q0, _ = inputs.sw_radial_dam(n=n, dtype=args.dtype, nsteps=steps)
        csteps = args.cpu_steps if args.cpu_steps else max(2, int(round(1e9 / (n * n))))
        print(f"# cpu baseline: oracle on {csteps} steps of {n}^2", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(prob, q0, csteps)
    emit(line, args, torch)


def bench_grid(args, torch, claw, inputs, n, steps, warmup, headline):
    """The radial dam break at n^2: `steps` adaptive steps from t = 0 timed
    (median of the repetitions), per-kernel event times over a second run,
    the dominant sweep against HBM.  headline: the full bench line, else the
    figures only."""
    prob, q0, _ = inputs.sw_radial_dam(n=n, dtype=args.dtype, nsteps=steps)
    prob["fused_step"] = args.fused_step
    ncell = prob["n"][0] * prob["n"][1]
    real_bytes = 4 if args.dtype == "f32" else 8
    tdt = torch.float32 if args.dtype == "f32" else torch.float64
    q = torch.tensor(q0, dtype=tdt, device="cuda").contiguous()
    solver = claw.Solver(prob, q, None)

    print(f"# workload sw_radial_dam {n}^2 {args.dtype}: warmup {warmup} steps, then "
          f"{steps} timed steps from t = 0", file=sys.stderr, flush=True)
    # each repetition times the configuration's steps from the initial state;
    # the reported time is the median repetition
    q_init = q.clone()
    restart_after_warmup(torch, solver, q, warmup)
    times = []
    for rep in range(args.reps):
        if rep > 0:
            q.copy_(q_init)
            solver.set_control(0.0, 0.0)
            torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, nrej = solver.advance(steps)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    elapsed = sorted(times)[len(times) // 2]
    value = ncell * steps / elapsed / 1e9
    print(f"# timed {steps} steps from t = 0, {args.reps} repetitions: median {elapsed:.4f} s, "
          f"min {min(times):.4f} s, max {max(times):.4f} s ({nrej} rejected trials)",
          file=sys.stderr, flush=True)

    # per-kernel durations with HIP events on the solver's stream
    timed = args.timed_steps if n < 4096 else min(args.timed_steps, 100)
    ms, cnt = solver.advance_timed(timed)
    names = ["x_sweep", "y_sweep", "z_sweep", "control"]
    fused = cnt[0] > 0 and cnt[1] == 0  # the library ran one fused kernel per step
    if fused:
        names[0] = "step2d"
    avg_us = {names[k]: (ms[k] / cnt[k] * 1e3 if cnt[k] else None) for k in range(4)}
    sweeps = [k for k in range(2) if cnt[k]]
    dom = max(sweeps, key=lambda k: ms[k] / cnt[k])
    # algorithmic bytes of the method per launch: each sweep reads and writes
    # every field of every cell once (2 meqn sizeof(real) per cell per sweep);
    # a fused launch carries both sweeps of a step
    alg_bytes = (2 if fused else 1) * 2 * 3 * real_bytes * ncell
    dom_s = ms[dom] / cnt[dom] * 1e-3
    achieved = alg_bytes / dom_s / 1e9
    pmc_file = args.traffic_file or os.path.join(ROOT, "profiles", f"pmc_sweeps_sw{n}_{args.dtype}.txt")
    traffic = load_traffic(pmc_file, names[dom])
    valu = load_pmc(pmc_file, names[dom], "valu_insts")
    valu_frac = load_pmc(pmc_file, names[dom], "valu_issue_frac")
    print(f"# kernel averages (us): {avg_us}", file=sys.stderr, flush=True)
    solver.close()
    del q, q_init
    torch.cuda.empty_cache()

    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                "kernel": names[dom], "alg_bytes_per_launch": alg_bytes,
                "state_bytes": 3 * real_bytes * ncell, "avg_launch_us": dom_s * 1e6}
    if fused:
        roofline["note"] = ("one fused kernel per step: it carries both sweeps' algorithmic bytes and "
                            "moves about half of them (the intermediate state stays in LDS); "
                            "traffic gives the measured HBM bytes")
    figures = {
        "value": value,
        "ms_per_step": elapsed / steps * 1e3,
        "steps": steps,
        "warmup": warmup,
        "roofline": roofline,
        "kernel_avg_us": avg_us,
        # the same kernel against the VALU issue rate, from the committed PMC
        # summary: SQ_INSTS_VALU per launch and its fraction of the issue peak
        # over the profiled run's own traced durations (its steps are the run's
        # first ones, not the event-timed window above)
        "valu_issue": None if valu is None else {
            "wave_insts_per_launch": valu, "peak_lane_ops_per_s": VALU_LANE_OPS_PEAK,
            "frac_in_profiled_run": valu_frac, "source": os.path.relpath(pmc_file, ROOT)},
        "hbm_frac_whole_step": value * 1e9 * sum(1 for k in range(4) if cnt[k]) * alg_bytes / ncell /
        (HBM_PEAK_GBPS * 1e9),
        "rejected_trials": nrej,
        "repetitions": {"count": args.reps, "seconds": times},
    }
    if not headline:
        figures["grid"] = [n, n]
        return figures
    line = {
        "metric": "Gcell-updates/s + % HBM roofline",
        "value": value,
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded radial dam break + U(-1e-3,1e-3) noise on h)",
        "config": {"workload": f"2D shallow water Roe+entropy fix, MC limiter, radial dam break, "
                               f"reflecting walls, CFL 0.9, {n}x{n}"
                               + (" (working set beyond the 256 MB MALL)" if n >= 4096 else ""),
                   "grid": [n, n], "cells": ncell, "parallelism": "single GPU"},
    }
    line.update({k: v for k, v in figures.items() if k not in ("value", "ms_per_step", "steps", "warmup")})
    return line


if __name__ == "__main__":
    main()
