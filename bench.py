"""Benchmark of the superlattice BTE time-stepping hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision fp64|fp32]

One "step" is a whole leap-frog step of the solver over the workload: the
whole-grid half-step, the fractional-grid half-step and the per-step
drift-velocity/absorption accumulation, as ``bte_step(1)`` queues it.  The
default workload is the large low-temperature instance (512 harmonics x 8193
phi_y points, mu = 10, E_dc = 4, E_w = 0.5, omega = 3, B = 6, dt = 2e-5),
whose FP64 state (four planes, 134 MB per ping-pong set) is far larger than
the L2 caches.  The state is resident in device memory before timing starts.

Prints ONE JSON line.  ``value`` is grid-point updates per second
(N_x * N_y * steps / s, whole steps, the paper's MLUPS convention x 1e6).
``roofline`` compares the step kernel's algorithmic bytes per launch over its
average launch duration (HIP events on the solver's stream) with the 8 TB/s
HBM peak.  ``cpu_baseline`` times the FP64 CPU oracle on a bounded sample of
the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
# FP64 vector FMA rate of the MI355X (256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz)
FP64_PEAK_TFLOPS = 78.6

# Algorithmic bytes per cell and launch: the fused kernels read and write the
# four state values of both grids once per launch (8 values; the two-step
# kernel covers two steps with them); a single half-step reads its own two
# values and the other grid's two and writes two (6 values).
VALUES_PER_CELL = {0: 8, 1: 6, 2: 8, 3: 8}   # kernel form -> state values moved per launch
KERNEL_NAMES = {0: "k_fused_step", 1: "k_half_step", 2: "k_fused_step2", 3: "k_fused_step3"}
FORM_NAMES = {"fused": 0, "two_pass": 1, "fused2": 2, "fused3": 3, "auto": -1}
# passes over the warm-start network's training states in the sweep leg
WARM_EPOCHS = 60


def launches_for(kernel, steps):
    if kernel == 1:
        return 2 * steps
    if kernel == 2:
        return steps // 2 + steps % 2
    if kernel == 3:
        return steps // 3 + (1 if steps % 3 else 0)
    return steps


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="large_512x8193")
    ap.add_argument("--precision", choices=("fp64", "fp32"), default="fp64")
    ap.add_argument("--kernel", choices=tuple(FORM_NAMES), default="auto",
                    help="kernel form; auto = whichever the autotuner finds fastest")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=0)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--rows-per-wave", type=int, default=0,
                    help="fix the launch shape instead of autotuning (with --waves-per-block)")
    ap.add_argument("--waves-per-block", type=int, default=0)
    ap.add_argument("--sweep", type=int, default=192,
                    help="instances of the batched-sweep measurement (0: skip)")
    ap.add_argument("--sweep-fp64", type=int, default=12,
                    help="draws the plain FP64 solver also runs (split evenly over the mu classes)")
    ap.add_argument("--warm-train", type=int, default=16384,
                    help="coarse-grid training states for the warm-started sweep (0: no warm run)")
    ap.add_argument("--reconstruct", type=int, default=512,
                    help="phi_x samples of the timed f(phi_x, phi_y) reconstruction (0: skip; "
                         "powers of two from 8 to 1024 run the FFT kernel)")
    ap.add_argument("--reconstruct-direct", type=int, default=500,
                    help="also time the direct-sum kernel at this many samples (0: skip)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--batch-probe", type=int, default=0,
                    help="instead of timing the solver: run a fixed-work batch of this many "
                         "sweep-grid instances (two periods of 400 steps each, wide schedule, "
                         "FP32 bulk) twice and report the second run; for profiling the "
                         "batch kernels")
    ap.add_argument("--probe-rows", type=int, default=43)
    ap.add_argument("--probe-waves", type=int, default=4)
    ap.add_argument("--full-run", choices=("fp64", "fp32"), default=None,
                    help="instead of timing: integrate the workload from f0 over "
                         "--full-periods ac periods in this precision and report the "
                         "observables over the last --full-avg periods")
    ap.add_argument("--full-periods", type=int, default=500)
    ap.add_argument("--full-avg", type=int, default=10)
    ap.add_argument("--full-until", type=int, default=0,
                    help="stop after this many periods and write --full-ckpt (0: run to the end)")
    ap.add_argument("--full-ckpt", default="", help="checkpoint (.npz) written when stopping early")
    ap.add_argument("--full-resume", default="", help="checkpoint (.npz) to resume from")
    return ap.parse_args()


def full_run(bte, torch, w, precision, args):
    """One long trajectory of the workload (e.g. 500 ac periods of the large
    instance), with the averaging window over its last periods (R14: n_end =
    round(P T/dt), lo = n_end - round(K T/dt)).  It can stop at a period
    boundary and write the whole state (both grids, exact in the solver's
    storage precision) to a checkpoint, and resume from one, so that a run
    longer than one job can be split; a resumed run is bitwise the
    uninterrupted one.  Prints progress to stderr about once a minute."""
    import numpy as np
    L = 2.0 * math.pi / (w.omega * w.dt)
    n_end = round(args.full_periods * L)
    lo = n_end - round(args.full_avg * L)
    target = round(args.full_until * L) if args.full_until else n_end
    if target > lo and target != n_end:
        raise SystemExit("--full-until must end before the averaging window starts")
    s = bte.Solver.from_workload(w, precision=precision)
    if args.full_resume:
        ck = np.load(args.full_resume)
        k0 = int(ck["step"])
        norm0 = float(ck["norm0"])
        assert int(ck["precision"]) == precision and str(ck["workload"]) == w.name
        # the launch shape of the first segment (in FP32 bulk the rounding
        # bits depend on how steps are grouped into launches)
        kt, kr, kw, kg = (int(x) for x in ck["tuning"])
        s.set_tuning(kernel=kt, rows_per_wave=kr, waves_per_block=kw, graph_steps=kg)
        s.set_state(*(ck[x].astype(np.float64) for x in ("a_h", "b_h", "a_f", "b_f")), step=k0)
    else:
        s.autotune()
        k0 = 0
        norm0 = s.observables().norm
    t = s.tuning()
    s.set_window(lo, n_end)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    log(f"full run {w.name} {args.full_run}: steps {k0} -> {target} of {n_end} "
        f"(window {lo} < k <= {n_end}), kernel {t.kernel} R{t.rows_per_wave} W{t.waves_per_block}")
    period = max(1, round(L))
    t0 = time.perf_counter()
    last = t0
    k = k0
    status = "ok"
    try:
        while k < target:
            n = min(period, target - k)
            s.step(n)
            k += n
            # one period in flight at a time (the step calls only queue work)
            torch.cuda.synchronize()
            now = time.perf_counter()
            if now - last >= 45.0:
                log(f"  step {k} of {target} ({k / L:.1f} periods), {now - t0:.0f} s, "
                    f"{(now - t0) * 1e6 / (k - k0):.2f} us/step")
                last = now
        torch.cuda.synchronize()
    except bte.BteError as e:
        status = f"stopped: {e}"
    wall = time.perf_counter() - t0
    out = {"workload": w.name, "precision": args.full_run, "kernel": KERNEL_NAMES[t.kernel],
           "tuning": {"kernel": t.kernel, "rows_per_wave": t.rows_per_wave,
                      "waves_per_block": t.waves_per_block, "graph_steps": t.graph_steps},
           "periods": args.full_periods, "avg_periods": args.full_avg, "n_end": n_end,
           "window": [lo, n_end], "from_step": k0, "to_step": k, "wall_s": wall,
           "us_per_step": wall * 1e6 / max(1, k - k0), "status": status}
    o = s.observables()
    out.update(norm=o.norm, norm0=norm0, norm_dev=abs(o.norm - norm0) / abs(norm0),
               v_dr=o.v_dr, edge_mass=o.edge_mass, top_harm_mass=o.top_harm_mass,
               obs_status=int(o.status))
    if k < n_end and status == "ok" and args.full_ckpt:
        st = s.state()
        dt = np.float32 if precision == 1 else np.float64
        np.savez_compressed(args.full_ckpt, step=k, norm0=norm0, precision=precision,
                            workload=w.name,
                            tuning=np.array([t.kernel, t.rows_per_wave, t.waves_per_block,
                                             t.graph_steps]),
                            **{x: a.astype(dt) for x, a in zip(("a_h", "b_h", "a_f", "b_f"), st)})
        out["checkpoint"] = args.full_ckpt
        out["checkpoint_bytes"] = os.path.getsize(args.full_ckpt)
    elif k == n_end:
        out.update(n_avg=int(o.n_avg), v_avg=o.v_avg, absorption=o.absorption,
                   absorption_cov=o.absorption_cov)
    s.close()
    print(json.dumps({"full_run": out}), flush=True)


def time_solver(bte, torch, w, precision, kernel, steps, warmup, autotune=True, shape=None):
    s = bte.Solver.from_workload(w, precision=precision)
    tuned_us = None
    if shape:
        s.set_tuning(kernel=max(kernel, 0), rows_per_wave=shape[0], waves_per_block=shape[1])
    elif autotune:
        # outside the timed region: pick the launch shape (and, for kernel -1,
        # the kernel form) by measurement
        _, tuned_us = s.autotune(kernel_form=kernel)
    else:
        s.set_tuning(kernel=max(kernel, 0))
    s.step(warmup)
    # the timed steps are the averaging window: every one of them takes the
    # drift-velocity and absorption accumulation (outside the window the
    # kernels skip it)
    s.set_window(warmup, warmup + steps)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    stream = s.stream
    t0 = time.perf_counter()
    start.record(stream)
    s.step(steps)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop)
    obs = s.observables()
    if obs.n_avg != steps:
        raise RuntimeError(f"window holds {obs.n_avg} steps, expected {steps}")
    tune = s.tuning()
    elem = 4 if precision == 1 else 8
    form = tune.kernel
    bytes_per_launch = VALUES_PER_CELL[form] * elem * w.nx * w.ny
    avg_launch_s = ms * 1e-3 / launches_for(form, steps)
    out = {
        "ms": ms, "wall_s": wall, "steps": steps,
        "cell_steps_per_s": w.nx * w.ny * steps / (ms * 1e-3),
        "us_per_step": ms * 1e3 / steps,
        "avg_launch_us": avg_launch_s * 1e6,
        "bytes_per_launch": bytes_per_launch,
        "kernel": KERNEL_NAMES[form], "steps_per_launch": {2: 2, 3: 3}.get(form, 1),
        "achieved_GBs": bytes_per_launch / avg_launch_s / 1e9,
        "status": int(obs.status), "v_dr": obs.v_dr, "norm": obs.norm,
        "window_steps": int(obs.n_avg), "v_avg": obs.v_avg, "absorption": obs.absorption,
        "autotune_best_us_per_step": tuned_us,
        "tuning": {"kernel": tune.kernel, "rows_per_wave": tune.rows_per_wave,
                   "waves_per_block": tune.waves_per_block, "graph_steps": tune.graph_steps},
    }
    s.close()
    return out


def stream_copy_rate(bte, torch, mib=2048, reps=10):
    """Read+write streaming rate of the library's plain copy kernel over two
    buffers of `mib` MiB (HIP events on the current stream): the practical
    HBM ceiling for a kernel that reads and writes its data once."""
    n = mib << 20
    src = torch.ones(n // 8, dtype=torch.float64, device="cuda")
    dst = torch.zeros_like(src)
    st = torch.cuda.current_stream()
    for _ in range(2):
        bte.bte_stream_copy(src.data_ptr(), dst.data_ptr(), n, st.cuda_stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        bte.bte_stream_copy(src.data_ptr(), dst.data_ptr(), n, st.cuda_stream)
    e1.record(st)
    torch.cuda.synchronize()
    if not torch.equal(src[-1024:], dst[-1024:]):
        raise RuntimeError("stream copy produced wrong data")
    rate = 2.0 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return rate


def reconstruct_bench(bte, torch, w, n_phix=512, launches=20):
    """f(phi_x, phi_y) reconstruction (Eq. f_fourier) of the workload's state
    on n_phix phi_x samples: average launch time by HIP events on the
    solver's stream, against the FP64 vector FMA rate (the direct sum does
    two FMAs per sample, phi_y point and harmonic n >= 1)."""
    s = bte.Solver.from_workload(w)
    out = torch.empty((n_phix, w.ny), dtype=torch.float64, device="cuda")
    for _ in range(3):
        s.reconstruct(n_phix, out)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(s.stream)
    for _ in range(launches):
        s.reconstruct(n_phix, out)
    stop.record(s.stream)
    torch.cuda.synchronize()
    s.close()
    us = start.elapsed_time(stop) * 1e3 / launches
    if 8 <= n_phix <= 1024 and n_phix & (n_phix - 1) == 0:
        # one FFT per phi_y column: bound by reading the coefficients once
        # (a_n for n < N_x, b_n for 1 <= n < N_x) and writing the samples
        nbytes = (2 * w.nx - 1) * w.ny * 8 + n_phix * w.ny * 8
        gbs = nbytes / (us * 1e-6) / 1e9
        return {"workload": f"{w.name} state, {n_phix} phi_x samples",
                "kernel": "k_reconstruct_fft", "avg_launch_us": us, "bytes_per_launch": nbytes,
                "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}}
    flops = 4.0 * (w.nx - 1) * n_phix * w.ny
    tf = flops / (us * 1e-6) / 1e12
    return {"workload": f"{w.name} state, {n_phix} phi_x samples", "kernel": "k_reconstruct",
            "avg_launch_us": us, "flops_per_launch": flops,
            "roofline": {"bound": "alu", "achieved": tf, "peak": FP64_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": tf / FP64_PEAK_TFLOPS}}


def main_run_form(run):
    return run["tuning"]["kernel"]


KERNEL_SOURCES = ("bte_device.h", "bte_internal.h", "bte_kernels.hip")


def kernel_source_hash():
    """sha256 over the sources of the single-instance step kernels."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(HERE, "paper_1401_6047_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_traffic(kernel, precision, tuning):
    """HBM bytes per launch from a committed counter summary
    (profiles/*_counters.txt: rocprofv3 FETCH_SIZE and WRITE_SIZE per dispatch,
    scaled by what the same counters read for a plain copy of known size),
    or None when no summary matches this kernel, precision and launch shape
    or the kernel sources changed since the counters were taken."""
    import glob
    want = kernel_source_hash()
    for path in sorted(glob.glob(os.path.join(HERE, "profiles", "*_counters.txt"))):
        kv = {}
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        try:
            if (kv.get("kernel") == kernel and kv.get("precision") == precision
                    and int(kv.get("rows_per_wave", -1)) == tuning["rows_per_wave"]
                    and int(kv.get("waves_per_block", -1)) == tuning["waves_per_block"]
                    and kv.get("source_sha256") == want):
                return float(kv["traffic_bytes_per_launch"])
        except (KeyError, ValueError):
            continue
    return None


def counter_valu_busy(kernel, precision, tuning):
    """VALU busy fraction of the step kernel from a committed SQ-counter
    summary (profiles/*_sq_counters.txt: SQ_ACTIVE_INST_VALU over the CUs'
    cycles), or None when none matches this kernel, precision, launch shape
    and kernel sources."""
    import glob
    want = kernel_source_hash()
    for path in sorted(glob.glob(os.path.join(HERE, "profiles", "*_sq_counters.txt"))):
        kv = {}
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        try:
            if (kv.get("kernel") == kernel and kv.get("precision") == precision
                    and int(kv.get("rows_per_wave", -1)) == tuning["rows_per_wave"]
                    and int(kv.get("waves_per_block", -1)) == tuning["waves_per_block"]
                    and kv.get("source_sha256") == want):
                return float(kv["valu_busy"])
        except (KeyError, ValueError):
            continue
    return None


def cpu_model():
    """The host CPU's model name (first 'model name' line of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(w, sample_steps):
    """The FP64 oracle on a bounded sample of the workload, with all host
    threads and with one thread (the paper's single-thread baseline style)."""
    import oracle
    pb = oracle.Problem(nx=w.nx, ny=w.ny, phiy_min=w.phiy_min, phiy_max=w.phiy_max,
                        E_dc=w.E_dc, E_w=w.E_w, omega=w.omega, B=w.B, mu=w.mu, dt=w.dt,
                        alpha=w.alpha)
    threads = oracle.max_threads()
    if sample_steps <= 0:
        # about 10-15 s of oracle work at ~2.5e7 cell-steps/s per thread
        sample_steps = max(4, int(12 * 2.5e7 * threads / (w.nx * w.ny)))
    oracle.run(pb, 1)                 # build/load, first touch
    t0 = time.perf_counter()
    oracle.run(pb, sample_steps)
    secs = time.perf_counter() - t0
    one_steps = max(2, sample_steps // max(threads, 1))
    t0 = time.perf_counter()
    oracle.run(pb, one_steps, n_threads=1)
    secs1 = time.perf_counter() - t0
    return {"value": w.nx * w.ny * sample_steps / secs, "unit": "grid-point updates/s",
            "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{w.name}: {sample_steps} whole steps from f0 (incl. start-up), "
                      f"FP64, {secs:.1f} s, OpenMP threads={threads}",
            "one_thread": {"value": w.nx * w.ny * one_steps / secs1, "cores": 1,
                           "sample": f"{w.name}: {one_steps} whole steps from f0, FP64, "
                                     f"{secs1:.1f} s, 1 thread"}}


def variant_report(main_run, variants, workload, precision):
    """The bench line's `variants`: each timed run's rate and launch shape,
    the observables of its timed window, and its difference from the FP64
    run of the same workload and window (`vs_fp64`; the main run when it is
    FP64, else the variant named <workload>_fp64).  Variant names are
    <workload>_<rest>."""
    fp64_ref = {workload: main_run} if precision == 0 else {}
    for k, v in variants.items():
        if k.endswith("_fp64"):
            fp64_ref.setdefault(k[:-len("_fp64")], v)
    out = {}
    for k, v in variants.items():
        e = {kk: v[kk] for kk in ("cell_steps_per_s", "us_per_step", "achieved_GBs",
                                  "avg_launch_us", "kernel", "tuning")}
        e["window"] = {"steps": v["window_steps"], "v_avg": v["v_avg"],
                       "absorption": v["absorption"]}
        ref = next((r for name, r in fp64_ref.items() if k.startswith(name + "_")), None)
        if ref is not None and ref is not v and ref["window_steps"] == v["window_steps"]:
            e["vs_fp64"] = {"rel_v_avg": abs(v["v_avg"] - ref["v_avg"]) / abs(ref["v_avg"]),
                            "abs_absorption": abs(v["absorption"] - ref["absorption"])}
        out[k] = e
    return out


def calibration_copy(torch, mib):
    """A plain device copy of known size (torch's copy: temporal 128-byte reads
    like the step kernels' row loads), five times, for scaling the HBM
    traffic counters of the kernels profiled in the same run; the FETCH_SIZE
    formula counts such reads at half their size on this chip."""
    n = mib << 20
    src = torch.ones(n // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def batch_probe(bte, torch, n, rows, waves):
    """A fixed amount of batched work: n instances of the sweep's grids (N_y
    classes in proportion to their cells, as the sweep autotuner samples
    them) with omega set for periods of 400 steps, each run for exactly two
    periods in the wide schedule with the two-step FP32-bulk kernel.  The
    first run captures the graphs; the second is timed.  Every pass advances
    every instance two steps, so a pass moves 32 B per cell (four FP32
    planes read and written once)."""
    from dataclasses import replace
    from paper_1401_6047_amd import workloads as W
    draws = W.sweep_draws(4096)
    nx, phi, dt = draws[0].nx, draws[0].phiy_max, draws[0].dt
    cells = {}
    for w in draws:
        cells[w.ny] = cells.get(w.ny, 0) + w.ny * nx
    total = sum(cells.values())
    rep = {w.ny: w for w in draws}
    sample = []
    for ny, c in sorted(cells.items()):
        sample += [replace(rep[ny], omega=2.0 * math.pi / (400 * dt))] * max(1, round(n * c / total))
    cfg = bte.make_batch_config(nx, -phi, phi, dt, precision=bte.BTE_FP32_BULK, tol=1e-6,
                                min_periods=2, max_periods=2, confirm=1)
    t = bte.bte_batch_tuning(bte.BTE_KERNEL_FUSED2, rows, waves, 0, bte.BTE_BATCH_WIDE)
    b = bte.Batch(cfg, sample, tuning=t)
    b.run(log=None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(log=None)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    res = b.results()
    b.close()
    cell_count = sum(w.ny * nx for w in sample)
    return {"instances": len(sample), "cells": cell_count, "passes": 400,
            "bytes_per_pass": 32 * cell_count, "wall_s": secs,
            "cell_steps_per_s": cell_count * 800 / secs,
            "tile": {"kernel": 2, "rows_per_wave": rows, "waves_per_group": waves},
            "all_ran_two_periods": all(r["periods"] == 2 for r in res)}


def stratified(draws, per_class):
    """Indices of the first `per_class` draws of each temperature class."""
    idx = []
    for mu in sorted({w.mu for w in draws}):
        idx += [i for i, w in enumerate(draws) if w.mu == mu][:per_class]
    return sorted(idx)


def sweep_bench(bte, torch, n, n_fp64, n_train, log):
    """Instances per hour of the parameter sweep.  The plain FP64 solver runs
    one instance after another (per-period host check) on a temperature-
    stratified subset of the draws, with its launch shape tuned once per N_y
    class before the clock starts; the batched FP32-bulk sweep (the library's
    default schedule: wide) runs the same subset, for a like-for-like ratio,
    and then all n draws, cold and warm-started from the trained network.
    Every run stops once |A_p - A_{p-1}| < 1e-6 holds for two consecutive
    periods (a single test can stop on a rotating transient); the absorption
    of the batched runs is compared with the FP64 solver's on the subset."""
    from paper_1401_6047_amd import workloads as W
    from paper_1401_6047_amd import warmstart
    draws = W.sweep_draws(n)
    nx, phi, dt = draws[0].nx, draws[0].phiy_max, draws[0].dt
    out = {"workload": f"sweep of {n} seeded draws: E_dc, B ~ U[0,8], omega ~ U[0.5,4], "
                       f"E_w = 0.1, mu in {{0.25,1,4}} -> N_y 401/801/1601, N_x {nx}, "
                       f"phi_y in [-{phi:g},{phi:g}], dt {dt:g}, tol 1e-6 over 2 periods",
           "unit": "instances/hour"}
    sub_idx = stratified(draws, max(1, n_fp64 // 3))
    sub = [draws[i] for i in sub_idx]
    # plain FP64 solver: one launch shape per N_y class, tuned before timing
    tunings = {}
    for w in sub:
        if w.ny not in tunings:
            s = bte.Solver.from_workload(w)
            tunings[w.ny], _ = s.autotune(target_ms=0.5)
            s.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref, sub_times = [], []
    for w in sub:
        t1 = time.perf_counter()
        s = bte.Solver.from_workload(w)
        bte.bte_set_tuning(s.handle, tunings[w.ny])
        ref.append(s.run_periods(tol=1e-6, max_periods=400, confirm=2))
        s.close()
        sub_times.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    t_fp64 = time.perf_counter() - t0
    log(f"  fp64 solver: {len(sub)} instances in {t_fp64:.1f} s")
    # the batch's tile from the sweep autotuner (a sample of these draws, timed
    # per candidate shape before any sweep clock starts; cached per N_y set)
    t0 = time.perf_counter()
    tile = {}
    cfg = bte.make_batch_config(nx, -phi, phi, dt, precision=bte.BTE_FP32_BULK, tol=1e-6,
                                min_periods=2, max_periods=400, confirm=2)
    bt, rate = bte.bte_batch_tune(cfg, draws)
    t_tune = time.perf_counter() - t0
    log(f"  sweep tuner: kernel {bt.kernel}, {bt.rows_per_wave} harmonics per wave, "
        f"{bt.waves_per_group} waves per group ({rate / 1e9:.0f} G cell-steps/s on its sample, "
        f"{t_tune:.1f} s)")
    sub_res, t_sub = warmstart.sweep(sub, nx, phi, dt, log=log, confirm=2, autotune=True)
    log(f"  batched fp32 on the same {len(sub)} instances: {t_sub:.1f} s")
    cold, t_cold = warmstart.sweep(draws, nx, phi, dt, log=log, confirm=2, autotune=True,
                                   info=tile)
    log(f"  batched fp32 cold: {n} instances in {t_cold:.1f} s")

    def max_dA(res):
        return max(abs(a["absorption"] - b["absorption"]) for a, b in zip(ref, res))

    out["fp64_solver"] = {"instances": len(sub), "wall_s": t_fp64,
                          "value": len(sub) / t_fp64 * 3600,
                          "periods_mean": sum(r["periods"] for r in ref) / len(sub),
                          "draws": "first %d of each mu class" % max(1, n_fp64 // 3),
                          "tunings": {str(k): [t.kernel, t.rows_per_wave, t.waves_per_block]
                                      for k, t in tunings.items()}}
    out["batched_fp32_same_draws"] = {"instances": len(sub), "wall_s": t_sub,
                                      "value": len(sub) / t_sub * 3600,
                                      "abs_dA_vs_fp64_max": max_dA(sub_res)}
    out["batched_fp32"] = {"instances": n, "wall_s": t_cold, "value": n / t_cold * 3600,
                           "periods_mean": sum(r["periods"] for r in cold) / n,
                           "converged": sum(r["converged"] for r in cold),
                           "abs_dA_vs_fp64_max": max_dA([cold[i] for i in sub_idx]),
                           "tile": tile, "tune_s": t_tune}
    # The plain FP64 solver on all n draws, projected from its measured rate:
    # per N_y class, the subset's wall time per cell-step, times the cell-steps
    # each draw needs (the periods its batched run took, L = round(T/dt) steps
    # each).  A projection from the measured subset, not a measurement.
    def cell_steps(w, periods):
        return w.nx * w.ny * periods * round(2 * math.pi / (w.omega * w.dt))
    per_class = {}
    for w, r, secs in zip(sub, ref, sub_times):
        c = per_class.setdefault(w.ny, [0.0, 0.0])
        c[0] += secs
        c[1] += cell_steps(w, r["periods"])
    proj = sum(cell_steps(w, r["periods"]) * per_class[w.ny][0] / per_class[w.ny][1]
               for w, r in zip(draws, cold))
    out["fp64_solver_projected_all_draws"] = {
        "instances": n, "wall_s": proj, "value": n / proj * 3600,
        "how": "per-N_y-class seconds per cell-step of the measured fp64 subset x the "
               "cell-steps each draw's batched run took"}
    if n_train > 0:
        train = warmstart.coarse_draws(n_train, W.SWEEP_SEED + 101)
        t0 = time.perf_counter()
        tres, states, _ = warmstart.sweep_states(train, train[0].nx, phi, train[0].dt, log=log)
        keep = torch.as_tensor([i for i, r in enumerate(tres) if r["converged"] == 1],
                               device="cuda")
        from paper_1401_6047_amd import mlp as M
        feats = M.features_of([train[i] for i in keep.tolist()])
        net, hist, _ = warmstart.train_network(feats, states.index_select(0, keep).contiguous(),
                                               epochs=WARM_EPOCHS, seed=W.SWEEP_SEED + 102)
        torch.cuda.synchronize()
        t_prep = time.perf_counter() - t0
        t0 = time.perf_counter()
        pred = net.predict(M.features_of(draws))
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t0
        net.close()
        warm, t_warm = warmstart.sweep(draws, nx, phi, dt, warm=pred, log=log, confirm=2,
                                       autotune=True)
        log(f"  batched fp32 warm: {n} instances in {t_warm:.1f} s "
            f"(+{t_inf * 1e3:.0f} ms inference; training data + training {t_prep:.1f} s)")
        pc = sum(r["periods"] for r in cold)
        pw = sum(r["periods"] for r in warm)
        out["batched_fp32_warm"] = {
            "instances": n, "wall_s": t_warm + t_inf, "value": n / (t_warm + t_inf) * 3600,
            "periods_mean": pw / n, "periods_saved_frac": 1.0 - pw / pc,
            "wall_saved_frac": 1.0 - (t_warm + t_inf) / t_cold,
            "converged": sum(r["converged"] for r in warm),
            "abs_dA_vs_fp64_max": max_dA([warm[i] for i in sub_idx]),
            "abs_dA_vs_cold_max": max(abs(a["absorption"] - b["absorption"])
                                      for a, b in zip(cold, warm)),
            "network": {"train_states": len(keep), "train_grid": "N_x 48, N_y 101/201/401, dt 1e-3",
                        "epochs": WARM_EPOCHS, "final_loss": hist[-1], "prep_s": t_prep}}
    best = out.get("batched_fp32_warm", out["batched_fp32"])
    out["value"] = best["value"]
    out["vs_fp64_solver_same_draws"] = (out["batched_fp32_same_draws"]["value"]
                                        / out["fp64_solver"]["value"])
    out["vs_fp64_solver_projected"] = best["value"] / out["fp64_solver_projected_all_draws"]["value"]
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the solver runs one instance per GPU, with no cross-GPU exchange).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_1401_6047_amd import bte
    from paper_1401_6047_amd import workloads as W

    w = W.WORKLOADS[args.workload]
    if args.batch_probe > 0:
        line = {"batch_probe": batch_probe(bte, torch, args.batch_probe, args.probe_rows,
                                           args.probe_waves)}
        if args.copy_mib > 0:
            calibration_copy(torch, args.copy_mib)
            line["copy_probe_mib"] = args.copy_mib
        print(json.dumps(line), flush=True)
        return
    if args.full_run:
        full_run(bte, torch, w, 1 if args.full_run == "fp32" else 0, args)
        return
    precision = 1 if args.precision == "fp32" else 0
    kernel = FORM_NAMES[args.kernel]
    at = not args.no_autotune
    shape = (args.rows_per_wave, args.waves_per_block) if args.rows_per_wave > 0 else None
    main_run = time_solver(bte, torch, w, precision, kernel, args.steps, args.warmup, at, shape)

    variants = {}
    if not args.no_variants:
        other = 1 - precision
        variants[f"{w.name}_{'fp32' if other else 'fp64'}"] = time_solver(
            bte, torch, w, other, kernel, args.steps, args.warmup, at)
        for name, form in (("fused", 0), ("two_pass", 1), ("fused2", 2), ("fused3", 3)):
            if form != main_run_form(main_run):
                variants[f"{w.name}_{args.precision}_{name}"] = time_solver(
                    bte, torch, w, precision, form, args.steps, args.warmup, at)
        c = W.CROSSED
        variants[f"{c.name}_fp64"] = time_solver(bte, torch, c, 0, -1, 20000, 2000, at)
        variants[f"{c.name}_fp32"] = time_solver(bte, torch, c, 1, -1, 20000, 2000, at)
        # the paper's own timing run (Table 1: 1094 MLUPS in float on its GPU)
        t1 = W.TABLE1
        variants[f"{t1.name}_fp32"] = time_solver(bte, torch, t1, 1, -1, 10000, 1000, at)
        variants[f"{t1.name}_fp64"] = time_solver(bte, torch, t1, 0, -1, 10000, 1000, at)

    ms = main_run["ms"]
    line = {
        "metric": "grid-point updates/s (N_x*N_y*steps/s) + % HBM peak; "
                  "sweep instances/hr at 1e-5 absorption err vs FP64",
        "value": main_run["cell_steps_per_s"],
        "unit": "grid-point updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if precision == 0 else "f32-storage/f64-compute",
        "data": "synthetic (seeded parameters; state from the Boltzmann equilibrium)",
        "config": {"workload": w.name, "n_x": w.nx, "n_y": w.ny, "dt": w.dt, "mu": w.mu,
                   "E_dc": w.E_dc, "E_w": w.E_w, "omega": w.omega, "B": w.B,
                   "precision": args.precision, "kernel": main_run["kernel"],
                   "tuning": main_run["tuning"]},
        "roofline": {"bound": "hbm", "achieved": main_run["achieved_GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": main_run["achieved_GBs"] / HBM_PEAK_GBS,
                     "traffic": counter_traffic(main_run["kernel"], args.precision,
                                                main_run["tuning"]),
                     "kernel": main_run["kernel"],
                     "valu_busy": counter_valu_busy(main_run["kernel"], args.precision,
                                                    main_run["tuning"]),
                     "limiter": "VALU instruction issue of two wavefronts per SIMD "
                                "(SQ counters, wavefront timeline); the HBM traffic is "
                                "hidden under it",
                     "steps_per_launch": main_run["steps_per_launch"],
                     "bytes_per_launch": main_run["bytes_per_launch"],
                     "avg_launch_us": main_run["avg_launch_us"]},
        "status": main_run["status"],
    }
    # observables over each run's timed window (the averaging window), and
    # for every variant its difference from the FP64 run of the same workload
    # and window: the error of each reported result against FP64
    line["window"] = {"steps": main_run["window_steps"], "v_avg": main_run["v_avg"],
                      "absorption": main_run["absorption"]}
    if variants:
        line["variants"] = variant_report(main_run, variants, w.name, precision)
    if args.reconstruct > 0:
        line["reconstruct"] = reconstruct_bench(bte, torch, w, n_phix=args.reconstruct)
    if args.reconstruct_direct > 0:
        line["reconstruct_direct"] = reconstruct_bench(bte, torch, w,
                                                       n_phix=args.reconstruct_direct)
    # the practical ceiling: the library's own streaming copy (reads and
    # writes every byte once, as the step kernels do)
    practical = stream_copy_rate(bte, torch)
    line["roofline"]["practical_peak_GBs"] = practical
    line["roofline"]["frac_of_practical"] = main_run["achieved_GBs"] / practical
    if args.copy_mib > 0:
        calibration_copy(torch, args.copy_mib)
        line["copy_probe_mib"] = args.copy_mib
    if args.sweep > 0:
        line["sweep"] = sweep_bench(bte, torch, args.sweep, min(args.sweep_fp64, args.sweep),
                                    args.warm_train,
                                    lambda *a, **k: print(*a, file=sys.stderr, flush=True))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
