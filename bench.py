#!/usr/bin/env python3
"""Benchmark of the batched shared-matrix solve on one MI355X.

Default workload: implicit-Euler diffusion, tridiagonal shared LHS (-r, 1+2r, -r),
r = 1.0, n = 512 unknowns, m = 2^20 interleaved right-hand sides drawn
uniform[-1, 1) from a fixed seed; one "step" is one batched FP64 solve of all
m systems (factorisation on the host, once, outside the timed region, as in
Carroll et al. arXiv:2107.05395, Section 3).  The FP32-sweep + FP64-residual
refinement form (double and FP32 right-hand sides), the paper's
thread-per-system design, a same-size device copy and the FP64 oracle on the
host cores are measured alongside and reported in the same JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, published
PEAK_FP64_TFLOPS = 78.6        # MI355X FP64 vector, published
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


KERNEL_SOURCES = ("sweep_core.h", "sweep_kernel.h", "sweep.hip", "sweep_f32.hip", "refine_kernel.h",
                  "refine.hip", "refine_f32rhs.hip", "stepper.h", "ch.hip", "ch_forced.hip",
                  "cn_stencil.h", "cn_tri.hip", "cn_penta.hip", "long_core.h", "long_sweep.hip",
                  "long_f32in.hip", "sweep_f32in.hip",
                  "adjoint_grad_kernel.h", "adjoint_grad_tri.hip", "adjoint_grad_penta.hip",
                  "internal.h")
# the device sources behind each kernel whose HBM traffic is recorded
KERNEL_FAMILIES = {
    "sweep": ("sweep_core.h", "sweep_kernel.h", "sweep.hip", "internal.h"),
    "refine": ("sweep_core.h", "refine_kernel.h", "refine.hip", "internal.h"),
    "stepper_cn": ("sweep_core.h", "stepper.h", "cn_stencil.h", "cn_tri.hip", "internal.h"),
    "stepper_ch": ("sweep_core.h", "stepper.h", "ch.hip", "internal.h"),
    "stepper_forced": ("sweep_core.h", "stepper.h", "ch_forced.hip", "internal.h"),
    "long": ("sweep_core.h", "long_core.h", "long_sweep.hip", "internal.h"),
    "adjoint_grad": ("sweep_core.h", "adjoint_grad_kernel.h", "adjoint_grad_tri.hip", "internal.h"),
}


def kernel_source_hash(family: str | None = None) -> str:
    h = hashlib.sha256()
    for name in (KERNEL_FAMILIES[family] if family else KERNEL_SOURCES):
        with open(os.path.join(ROOT, "paper_2107_05395_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, precision: str, family: str):
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None
    when they were taken on a different source of that kernel family."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    entry = rec.get("%s/%s" % (workload, precision))
    if not entry or entry.get("source_hash") != kernel_source_hash(family):
        return None
    return entry.get("bytes_per_launch")


def rel_err_cols(x, ref):
    num = np.linalg.norm(x - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    return float(np.max(num / np.where(den == 0, 1.0, den)))


def time_launches(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / 1e3, wall


def launch_stats(fn, reps, torch):
    """Median, minimum and maximum of `reps` single launches, each bracketed
    by its own pair of events on the current stream (ms)."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    torch.cuda.synchronize()
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in evs)
    return {"median": ms[len(ms) // 2], "min": ms[0], "max": ms[-1], "launches": reps}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_tri(bands, n, seed, budget_s):
    """The oracle as it stands on the host cores, on a bounded sample."""
    import oracle
    from paper_2107_05395_amd import inputs
    m_s = 1 << 15
    rhs = inputs.uniform_batch(n, m_s, seed=seed)
    calls, t0 = 0, time.perf_counter()
    while True:
        oracle.tri_solve(*bands, rhs)
        calls += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return {"value": calls * m_s / el, "unit": "systems/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d x oracle.tri_solve on %d systems of the same workload (n=%d), %.1f s"
                      % (calls, m_s, n, el)}


def bench_tri(args, torch):
    from paper_2107_05395_amd import Factor, inputs
    spec = dict(inputs.WORKLOADS[args.workload])
    n, m, r, seed = spec["n"], spec["m"], spec["r"], spec["seed"]
    bands = inputs.diffusion_tri_bands(n, r)
    f = Factor.tri(*bands)
    f.upload()
    rhs_host = inputs.uniform_batch(n, m, seed=seed)
    rhs = torch.from_numpy(rhs_host).cuda()
    x = torch.empty_like(rhs)
    algo_bytes = 16.0 * n * m          # read b, write x (double)

    results = {}
    for prec in ("f64", "f32r"):
        t, wall = time_launches(lambda: f.solve(rhs, out=x, precision=prec), args.steps,
                                args.warmup, torch)
        cols = np.unique(np.r_[np.linspace(0, m - 1, 254).astype(np.int64), 0, m - 1])
        import oracle
        ref = oracle.tri_solve(*bands, rhs_host[:, cols])
        err = rel_err_cols(x[:, torch.from_numpy(cols).cuda()].cpu().numpy(), ref)
        results[prec] = dict(seconds=t, wall=wall, err=err)
    # FP32 right-hand-side data (the same draws rounded), refined to double:
    # 4 B read + 8 B written per row
    rhs32 = rhs.float()
    t32, _ = time_launches(lambda: f.solve(rhs32, out=x, precision="f32rhs"), args.steps,
                           args.warmup, torch)
    import oracle
    cols32 = np.unique(np.r_[np.linspace(0, m - 1, 254).astype(np.int64), 0, m - 1])
    ref32 = oracle.tri_solve(*bands, rhs_host[:, cols32].astype(np.float32).astype(np.float64))
    err32 = rel_err_cols(x[:, torch.from_numpy(cols32).cuda()].cpu().numpy(), ref32)
    # the same FP32 data solved with the FP64 sweeps (no refinement needed)
    t32d, _ = time_launches(lambda: f.solve(rhs32, out=x, precision="f32rhs_f64"), args.steps,
                            args.warmup, torch)
    err32d = rel_err_cols(x[:, torch.from_numpy(cols32).cuda()].cpu().numpy(), ref32)
    del rhs32
    # torch's device-to-device copy of the same array, one read + one write
    # stream (context for the roofline; not the fastest copy on this part)
    ct, _ = time_launches(lambda: x.copy_(rhs), 10, 2, torch)
    copy_gbs = algo_bytes * 10 / ct / 1e9
    # the fastest plain copy found on this part: one contiguous 16 KB tile per
    # workgroup (bb_copy_tiles), the sweep's HBM reference
    from paper_2107_05395_amd.solver import copy_tiles
    tt, _ = time_launches(lambda: copy_tiles(rhs, x), 10, 2, torch)
    assert torch.equal(x, rhs)
    tile_gbs = algo_bytes * 10 / tt / 1e9
    # the same bytes moved with the sweep's own access pattern (bb_copy_rows:
    # 64 rows of two 256-byte segments per wave, loads before stores): the
    # ceiling of that pattern on this part
    from paper_2107_05395_amd.solver import copy_rows
    x.zero_()
    rt, _ = time_launches(lambda: copy_rows(rhs, x), 10, 2, torch)
    assert torch.equal(x, rhs)
    rows_gbs = algo_bytes * 10 / rt / 1e9
    # small batches are bound by launch latency: the same solves replayed
    # from a HIP graph (captured after the eager calls uploaded the tables)
    graph = None
    if m * n < (1 << 24):
        reps = 100
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                for _ in range(reps):
                    f.solve(rhs, out=x)
        torch.cuda.current_stream().wait_stream(side)
        gt, _ = time_launches(g.replay, 10, 2, torch)
        graph = {"ms_per_step": 1e3 * gt / (10 * reps), "value": m * 10 * reps / gt,
                 "note": "%d FP64 solves per graph replay" % reps}
        del g
    # the paper's own mapping: one thread per system, intermediate through HBM
    pt, _ = time_launches(lambda: f.solve_thread_per_system(rhs, out=x), max(3, args.steps // 10),
                          1, torch)
    pt /= max(3, args.steps // 10)

    k = args.steps
    t64 = results["f64"]["seconds"]
    per_launch = t64 / k
    traffic = measured_traffic(args.workload, "f64", "sweep")
    # the same solve launch by launch: median and minimum over the repeats
    stats = launch_stats(lambda: f.solve(rhs, out=x), k, torch)
    line = {
        "metric": "systems solved/s", "value": m * k / t64, "unit": "systems/s",
        "n_gpus": 1, "steps": k, "warmup": args.warmup, "ms_per_step": 1e3 * per_launch,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded uniform[-1,1) right-hand sides)",
        "config": {"workload": args.workload, "n": n, "m": m, "r": r,
                   "matrix": "tridiagonal (-r, 1+2r, -r), zero Dirichlet", "parallelism": "none"},
        "rel_err_vs_oracle": results["f64"]["err"],
        "hbm_gbs_algorithmic": algo_bytes / per_launch / 1e9,
        "launch_ms": stats,
        "f32r": {"value": m * k / results["f32r"]["seconds"], "unit": "systems/s",
                 "ms_per_step": 1e3 * results["f32r"]["seconds"] / k,
                 "rel_err_vs_oracle": results["f32r"]["err"],
                 "hbm_gbs_algorithmic": algo_bytes * k / results["f32r"]["seconds"] / 1e9},
        "f32rhs": {"value": m * k / t32, "unit": "systems/s", "ms_per_step": 1e3 * t32 / k,
                   "rel_err_vs_oracle": err32, "hbm_gbs_algorithmic": 12.0 * n * m * k / t32 / 1e9,
                   "note": "FP32 right-hand sides (the same draws rounded), double solution; "
                           "oracle on the rounded values"},
        "f32rhs_f64": {"value": m * k / t32d, "unit": "systems/s", "ms_per_step": 1e3 * t32d / k,
                       "rel_err_vs_oracle": err32d,
                       "hbm_gbs_algorithmic": 12.0 * n * m * k / t32d / 1e9,
                       "note": "the same FP32 right-hand sides solved with the FP64 sweeps and "
                               "factor (promoted exactly on load), double solution"},
        "copy_gbs": copy_gbs, "tile_copy_gbs": tile_gbs,
        "hip_graph": graph,
        "thread_per_system_design": {"ms_per_step": 1e3 * pt, "value": m / pt,
                                     "hbm_gbs_algorithmic": algo_bytes / pt / 1e9},
        "roofline": {"bound": "hbm", "achieved": algo_bytes / per_launch / 1e9,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": algo_bytes / per_launch / 1e9 / PEAK_HBM_GBS,
                     "traffic": traffic,
                     "counter_gbs": traffic / per_launch / 1e9 if traffic else None,
                     "kernel": "sweep_kernel<double,1,%d,false,full>" % f.chunk(),
                     "algorithmic_bytes_per_launch": algo_bytes,
                     "torch_copy_gbs": copy_gbs,
                     "tile_copy_gbs": tile_gbs,
                     "frac_of_tile_copy": algo_bytes / per_launch / 1e9 / tile_gbs,
                     "pattern_copy_gbs": rows_gbs,
                     "frac_of_pattern_copy": algo_bytes / per_launch / 1e9 / rows_gbs,
                     "pattern_copy_frac_of_peak": rows_gbs / PEAK_HBM_GBS},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_tri(bands, n, seed + 100, args.cpu_seconds)
    return line


def bench_penta(args, torch):
    from paper_2107_05395_amd import Factor, inputs
    spec = dict(inputs.WORKLOADS[args.workload])
    n, m, r, seed = spec["n"], spec["m"], spec["r"], spec["seed"]
    bands = inputs.hyperdiffusion_penta_bands(n, r)
    f = Factor.penta(*bands)
    f.upload()
    rhs_host = inputs.sine_mode_batch(n, m, seed=seed)
    rhs = torch.from_numpy(rhs_host).cuda()
    x = torch.empty_like(rhs)
    algo_bytes = 16.0 * n * m
    out = {}
    import oracle
    cols = np.unique(np.r_[np.linspace(0, m - 1, 254).astype(np.int64), 0, m - 1])
    ref = oracle.penta_solve(*bands, rhs_host[:, cols])
    for prec in ("f64", "f32r"):
        t, _ = time_launches(lambda: f.solve(rhs, out=x, precision=prec), args.steps, args.warmup, torch)
        err = rel_err_cols(x[:, torch.from_numpy(cols).cuda()].cpu().numpy(), ref)
        out[prec] = (t, err)
    rhs32 = rhs.float()
    t, _ = time_launches(lambda: f.solve(rhs32, out=x, precision="f32rhs"), args.steps, args.warmup,
                         torch)
    ref32 = oracle.penta_solve(*bands, rhs_host[:, cols].astype(np.float32).astype(np.float64))
    out["f32rhs"] = (t, rel_err_cols(x[:, torch.from_numpy(cols).cuda()].cpu().numpy(), ref32))
    t, _ = time_launches(lambda: f.solve(rhs32, out=x, precision="f32rhs_f64"), args.steps,
                         args.warmup, torch)
    out["f32rhs_f64"] = (t, rel_err_cols(x[:, torch.from_numpy(cols).cuda()].cpu().numpy(), ref32))
    del rhs32
    # the same batch in arrays with a leading dimension of m + 32 (rows no
    # longer a power of two apart; the library takes any ld >= m)
    from paper_2107_05395_amd import empty_batch
    rp, xp = empty_batch(n, m), empty_batch(n, m)
    pad = rp.stride(0) - m
    rp.copy_(rhs)
    tpad, _ = time_launches(lambda: f.solve(rp, out=xp), args.steps, args.warmup, torch)
    err_pad = rel_err_cols(xp[:, torch.from_numpy(cols).cuda()].cpu().numpy(), ref)
    del rp, xp
    from paper_2107_05395_amd.solver import copy_rows
    rt, _ = time_launches(lambda: copy_rows(rhs, x), 10, 2, torch)
    rows_gbs = algo_bytes * 10 / rt / 1e9
    k = args.steps
    per = out["f64"][0] / k
    stats = launch_stats(lambda: f.solve(rhs, out=x), k, torch)
    line = {
        "metric": "systems solved/s", "value": m * k / out["f64"][0], "unit": "systems/s",
        "n_gpus": 1, "steps": k, "warmup": args.warmup, "ms_per_step": 1e3 * per,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (random-phase sums of 8 sine modes)",
        "config": {"workload": args.workload, "n": n, "m": m, "r": r},
        "rel_err_vs_oracle": out["f64"][1],
        "launch_ms": stats,
        "f32r": {"value": m * k / out["f32r"][0], "rel_err_vs_oracle": out["f32r"][1],
                 "ms_per_step": 1e3 * out["f32r"][0] / k},
        "f32rhs": {"value": m * k / out["f32rhs"][0], "rel_err_vs_oracle": out["f32rhs"][1],
                   "ms_per_step": 1e3 * out["f32rhs"][0] / k,
                   "hbm_gbs_algorithmic": 12.0 * n * m * k / out["f32rhs"][0] / 1e9},
        "f32rhs_f64": {"value": m * k / out["f32rhs_f64"][0], "rel_err_vs_oracle": out["f32rhs_f64"][1],
                       "ms_per_step": 1e3 * out["f32rhs_f64"][0] / k,
                       "hbm_gbs_algorithmic": 12.0 * n * m * k / out["f32rhs_f64"][0] / 1e9},
        "padded_ld": {"ld": m + pad, "ms_per_step": 1e3 * tpad / k, "value": m * k / tpad,
                      "hbm_gbs_algorithmic": algo_bytes * k / tpad / 1e9,
                      "rel_err_vs_oracle": err_pad},
        "roofline": {"bound": "hbm", "achieved": algo_bytes / per / 1e9, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": algo_bytes / per / 1e9 / PEAK_HBM_GBS,
                     "traffic": measured_traffic(args.workload, "f64", "sweep"),
                     "counter_gbs": (measured_traffic(args.workload, "f64", "sweep") / per / 1e9
                                     if measured_traffic(args.workload, "f64", "sweep") else None),
                     "pattern_copy_gbs": rows_gbs,
                     "frac_of_pattern_copy": algo_bytes / per / 1e9 / rows_gbs},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_penta(bands, n, seed + 100, args.cpu_seconds)
    return line


def cpu_baseline_penta(bands, n, seed, budget_s):
    """The oracle on the host cores on bounded blocks of the same workload."""
    import oracle
    from paper_2107_05395_amd import inputs
    m_s = 1 << 14
    rhs = inputs.sine_mode_batch(n, m_s, seed=seed)
    calls, t0 = 0, time.perf_counter()
    while True:
        oracle.penta_solve(*bands, rhs)
        calls += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return {"value": calls * m_s / el, "unit": "systems/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d x oracle.penta_solve on %d systems of the same workload (n=%d), %.1f s"
                      % (calls, m_s, n, el)}


def bench_ch(args, torch):
    """The configured Cahn-Hilliard ensemble: all of its steps (5000) from the
    seeded start, in launches of --ch-fuse fused steps (state on chip), then
    the same start in one launch per step for a sample of steps (the state
    through HBM each step).  The final state of at least 2^12 runs, sampled
    evenly over the batch, is compared with the oracle run over the same 5000
    steps; that oracle run on the host cores is also the cpu_baseline."""
    from paper_2107_05395_amd import Factor, inputs
    import oracle
    spec = dict(inputs.WORKLOADS[args.workload])
    n, m, seed, T = spec["n"], spec["m"], spec["seed"], spec["steps"]
    L, gamma, dt = 2.0 * np.pi, spec["gamma"], spec["dt"]
    f = Factor.cahn_hilliard(n, L, gamma, dt)
    f.upload()
    c_host = inputs.uniform_batch(n, m, seed=seed, lo=-0.1, hi=0.1)
    c0 = torch.from_numpy(c_host).cuda()
    bufs = [c0.clone(), torch.empty_like(c0)]
    fuse = max(1, min(args.ch_fuse, T))

    def run_all():
        bufs[0].copy_(c0)
        done, cur = 0, 0
        while done < T:
            k = min(fuse, T - done)
            f.ch_step(bufs[cur], f.alpha, steps=k, out=bufs[1 - cur])
            cur, done = 1 - cur, done + k
        return bufs[cur]

    f.ch_step(c0, f.alpha, steps=2, out=bufs[1])        # warm-up (tables, code)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    final = run_all()
    stop.record()
    torch.cuda.synchronize()
    secs = start.elapsed_time(stop) / 1e3
    per_step = secs / T
    # one launch per step: 200 steps from the same start (HBM-bound)
    single = 200
    tp, _ = time_launches(lambda: f.ch_step(bufs[0], f.alpha, steps=1, out=bufs[1]), single, 3,
                          torch)
    final = run_all()                                    # the timed trajectory's result again
    torch.cuda.synchronize()
    # parity over the full trajectory on >= 2^12 sampled runs
    samp = max(1 << 12, args.ch_sample)
    cols = np.unique(np.r_[np.linspace(0, m - 1, samp).astype(np.int64), m - 1])
    sigma, alpha = oracle.ch_coefficients(gamma, L / n, dt)
    t0 = time.perf_counter()
    ref = oracle.ch_step(c_host[:, cols], sigma, alpha, steps=T)
    cpu_s = time.perf_counter() - t0
    got = final[:, torch.from_numpy(cols).cuda()].cpu().numpy()
    num = np.linalg.norm(got - ref, axis=0)
    errs = num / np.linalg.norm(ref, axis=0)
    flag = 1e-10
    outliers = [{"run": int(cols[j]), "rel_err": float(errs[j])}
                for j in np.argsort(-errs)[:8] if errs[j] > flag]
    # Roofline of the fused launches: FP64 arithmetic.  Algorithmic
    # operations per row and step of the scheme (Section 5.1): N = C^3 - C
    # (3), the stencil f = C + a(N_{i-1} - 2N_i + N_{i+1}) (5), the LR forward
    # step with stored reciprocal (5), the back substitution (4) and the
    # periodic rank-2 correction (4).
    flops_row_step = 21.0
    ach = flops_row_step * n * m / per_step / 1e12
    line = {
        "metric": "system-steps/s", "value": m * T / secs, "unit": "system-steps/s",
        "n_gpus": 1, "steps": T, "warmup": 1, "ms_per_step": 1e3 * per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded uniform[-0.1,0.1) initial states)",
        "config": {"workload": args.workload, "n": n, "m": m, "L": L, "gamma": gamma, "dt": dt,
                   "steps": T, "steps_per_launch": fuse},
        "trajectory_check": {"runs": int(len(cols)), "steps": T,
                             "max_rel_err_vs_oracle": float(errs.max()),
                             "median_rel_err_vs_oracle": float(np.median(errs)),
                             "flag_above": flag, "outliers": outliers},
        "one_step_per_launch": {"ms_per_step": 1e3 * tp / single,
                                "hbm_gbs_algorithmic": 16.0 * n * m * single / tp / 1e9,
                                "frac_of_hbm_peak": 16.0 * n * m * single / tp / 1e9 / PEAK_HBM_GBS},
        "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach / PEAK_FP64_TFLOPS, "traffic": None,
                     "note": "fused launches; algorithmic FP64 operations of the scheme, "
                             "21 per row and step"},
        "cpu_baseline": {"value": len(cols) * T / cpu_s, "unit": "system-steps/s",
                         "cores": oracle.num_threads(), "kind": "oracle",
                         "sample": "oracle.ch_step over all %d steps on the %d sampled runs "
                                   "(n=%d) of the trajectory check, %.1f s"
                                   % (T, len(cols), n, cpu_s)},
    }
    return line


# The paper's own times for 1000 steps on the same grid (Tesla V100; Section
# 3 and Section 4 benchmark tables, cuThomasConstantBatch and
# cuPentConstantBatch columns), keyed by (M, N), as printed.  Context only:
# other hardware, and the printed unit is not certain.
PAPER_CN_TABLE = {
    "diffusion": {(64, 64): 0.097, (64, 256): 0.161, (64, 1024): 0.510,
                  (4096, 64): 0.101, (4096, 256): 0.255, (4096, 1024): 1.020,
                  (65536, 64): 1.278, (65536, 256): 5.015, (65536, 1024): 20.268},
    "hyperdiffusion": {(64, 64): 369.902, (64, 256): 461.727, (64, 1024): 658.475,
                       (4096, 64): 460.857, (4096, 256): 429.127, (4096, 1024): 1344.377,
                       (65536, 64): 1786.018, (65536, 256): 6535.750, (65536, 1024): 25893.904},
}

# Algorithmic FP64 operations per row and Crank-Nicolson step: the explicit
# stencil (3 points: 5; 5 points: 9), the forward sweep with stored
# reciprocal (tri 3, penta 5), the back substitution (tri 2, penta 4) and the
# periodic correction (rank 1: 2, rank 2: 4).
CN_FLOPS_ROW_STEP = {"diffusion": 12.0, "hyperdiffusion": 22.0}


def cpu_baseline_cn(bands, w, n, seed, budget_s):
    import oracle
    from paper_2107_05395_amd import inputs
    m_s = 1 << 12
    c = inputs.uniform_batch(n, m_s, seed=seed)
    steps, t0 = 0, time.perf_counter()
    while True:
        c = oracle.cn_step(bands, w, c, steps=5)
        steps += 5
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return {"value": steps * m_s / el, "unit": "system-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d x oracle.cn_step on %d systems of n=%d (the largest grid point's n), %.1f s"
                      % (steps, m_s, n, el)}


def bench_cn(args, torch):
    """Crank-Nicolson time stepping over the paper's benchmark grid: every
    (n, m) point runs the workload's step count three ways: all steps in one
    fused launch (state on chip), one launch per step (state through HBM),
    and those single-step launches replayed from a HIP graph."""
    from paper_2107_05395_amd import Factor, inputs
    import oracle
    spec = dict(inputs.WORKLOADS[args.workload])
    prob, sigma, T, seed = spec["problem"], spec["sigma"], spec["steps"], spec["seed"]
    build = inputs.cn_diffusion_problem if prob == "diffusion" else inputs.cn_hyperdiffusion_problem
    grid = []
    last = None
    for n in spec["ns"]:
        bands, w = build(n, sigma)
        f = Factor.tri(*bands, cyclic=True) if prob == "diffusion" else Factor.penta(*bands, cyclic=True)
        f.upload()
        for m in spec["ms"]:
            c_host = inputs.uniform_batch(n, m, seed=seed + n + m)
            c = torch.from_numpy(c_host).cuda()
            out = torch.empty_like(c)
            tf, _ = time_launches(lambda: f.cn_step(c, w, steps=T, out=out), 1, 1, torch)
            cols = np.unique(np.r_[np.linspace(0, m - 1, 16).astype(np.int64), m - 1])
            ref = oracle.cn_step(bands, w, c_host[:, cols], steps=T)
            err = rel_err_cols(out[:, torch.from_numpy(cols).cuda()].cpu().numpy(), ref)
            bufs = [c.clone(), out]

            def per_step():
                for i in range(T):
                    f.cn_step(bufs[i & 1], w, out=bufs[(i + 1) & 1])
            tp, _ = time_launches(per_step, 1, 1, torch)
            # the same T single-step launches replayed from a HIP graph
            g = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                with torch.cuda.graph(g, stream=side):
                    per_step()
            torch.cuda.current_stream().wait_stream(side)
            tg, _ = time_launches(g.replay, 1, 1, torch)
            del g
            grid.append({"n": n, "m": m, "fused_ms": 1e3 * tf, "per_step_launch_ms": 1e3 * tp,
                         "per_step_graph_ms": 1e3 * tg,
                         "fused_system_steps_per_s": m * T / tf,
                         "per_step_hbm_gbs": 16.0 * n * m * T / tp / 1e9,
                         "rel_err_vs_oracle": err,
                         "paper_v100_cuconstant_time": PAPER_CN_TABLE[prob][(m, n)]})
            last = (n, m, tf, tp, bands, w)
            del c, out, bufs
    n, m, tf, tp, bands, w = last
    flops = CN_FLOPS_ROW_STEP[prob] * n * m * T
    line = {
        "metric": "system-steps/s", "value": m * T / tf, "unit": "system-steps/s",
        "n_gpus": 1, "steps": T, "warmup": 1, "ms_per_step": 1e3 * tf / T,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded uniform[-1,1) initial states)",
        "config": {"workload": args.workload, "n": n, "m": m, "sigma": sigma, "periodic": True,
                   "steps_per_launch": T},
        "grid": grid,
        "roofline": {"bound": "alu", "achieved": flops / tf / 1e12, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": flops / tf / 1e12 / PEAK_FP64_TFLOPS,
                     "traffic": None,
                     "note": "fused launch; algorithmic FP64 operations %d per row and step"
                             % CN_FLOPS_ROW_STEP[prob]},
        "per_step_roofline": {"bound": "hbm", "achieved": 16.0 * n * m * T / tp / 1e9,
                              "peak": PEAK_HBM_GBS, "unit": "GB/s",
                              "frac": 16.0 * n * m * T / tp / 1e9 / PEAK_HBM_GBS,
                              "traffic": measured_traffic(args.workload,
                                                          "per_step_n%d_m%d" % (n, m), "stepper_cn")},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_cn(bands, w, n, seed + 1, args.cpu_seconds)
    return line


def bench_ch_coarsening(args, torch):
    """The coarsening campaign: m runs of the Cahn-Hilliard scheme to t = T
    with the ensemble-mean typical domain size lbar(t) = mean 1/(1 - <C^2>)
    taken at every step inside the stepping kernel, then a straight-line fit
    of lbar against log t (the paper fits lbar against log t and reports the
    correlation coefficient)."""
    from paper_2107_05395_amd import Factor, inputs
    import oracle
    spec = dict(inputs.WORKLOADS[args.workload])
    n, L, m, gamma, T, seed = (spec[k] for k in ("n", "length", "m", "gamma", "T", "seed"))
    dx = L / n
    dt = 0.1 * dx
    steps = int(round(T / dt))
    f = Factor.cahn_hilliard(n, L, gamma, dt)
    f.upload()
    alpha = f.alpha
    sigma_o, alpha_o = oracle.ch_coefficients(gamma, dx, dt)
    # parity first: 256 runs, 20 steps, lbar at every step against the oracle
    c_small = inputs.uniform_batch(n, 256, seed=seed + 1, lo=-0.1, hi=0.1)
    _, lb_small = f.ch_step_stats(torch.from_numpy(c_small).cuda(), alpha, steps=20, every=1)
    ref_small, _ = oracle.ch_coarsening(c_small, sigma_o, alpha_o, 20, 1)
    err = float(np.max(np.abs(lb_small.cpu().numpy() - ref_small) / ref_small))

    c = torch.from_numpy(inputs.uniform_batch(n, m, seed=seed, lo=-0.1, hi=0.1)).cuda()
    nxt = torch.empty_like(c)
    f.ch_step_stats(c, alpha, steps=4, every=1, out=nxt)          # warm-up (tables, code)
    chunk = 2000
    lbars = []
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        nxt, lb = f.ch_step_stats(c, alpha, steps=k, every=1, out=nxt)
        lbars.append(lb)
        c, nxt = nxt, c
        done += k
    stop.record()
    torch.cuda.synchronize()
    secs = start.elapsed_time(stop) / 1e3
    lbar = torch.cat(lbars).cpu().numpy()
    t = dt * np.arange(1, steps + 1)

    def fit(t0):
        # samples evenly spaced in log t between t0 and T
        idx = np.unique(np.searchsorted(t, np.exp(np.linspace(np.log(t0), np.log(t[-1]), 400))))
        idx = idx[idx < steps]
        x, y = np.log(t[idx]), lbar[idx]
        slope, icpt = np.polyfit(x, y, 1)
        return {"t_from": t0, "r": float(np.corrcoef(x, y)[0, 1]), "slope": float(slope),
                "intercept": float(icpt), "points": int(len(idx))}

    flops = 21.0 * n * m * steps
    line = {
        "metric": "system-steps/s", "value": m * steps / secs, "unit": "system-steps/s",
        "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": 1e3 * secs / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded uniform[-0.1,0.1) initial states)",
        "config": {"workload": args.workload, "n": n, "L": L, "m": m, "gamma": gamma, "dt": dt,
                   "T": steps * dt, "statistic_every": 1, "steps_per_launch": chunk},
        "lbar_rel_err_vs_oracle_256_runs_20_steps": err,
        "coarsening": {"fit_log_t": [fit(1.0), fit(10.0)],
                       "lbar_at": {"%g" % tt: float(lbar[min(steps - 1, int(round(tt / dt)) - 1)])
                                   for tt in (0.1, 1.0, 10.0, 50.0, 100.0)},
                       "paper_r": 0.9989 if abs(L - 2 * np.pi) < 1e-9 else 0.9996},
        "roofline": {"bound": "alu", "achieved": flops / secs / 1e12, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": flops / secs / 1e12 / PEAK_FP64_TFLOPS,
                     "traffic": None,
                     "note": "algorithmic FP64 operations of the scheme, 21 per row and step "
                             "(the statistic adds 2 per row at each sample)"},
    }
    if not args.no_cpu_baseline:
        m_s = 1 << 12
        cs = inputs.uniform_batch(n, m_s, seed=seed + 2, lo=-0.1, hi=0.1)
        done_s, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < args.cpu_seconds:
            cs = oracle.ch_step(cs, sigma_o, alpha_o, steps=10)
            oracle.ch_domain_size(cs)
            done_s += 10
        el = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": done_s * m_s / el, "unit": "system-steps/s",
                                "cores": oracle.num_threads(), "kind": "oracle",
                                "sample": "%d steps of %d runs (n=%d) with oracle.ch_step, "
                                          "domain sizes every 10 steps, %.1f s"
                                          % (done_s, m_s, n, el)}
    return line


FORCED_FLOPS_ROW_STEP = 112


def bench_ch_forced(args, torch):
    """A flow-pattern batch of the forced Cahn-Hilliard equation: every run of
    a grid over (f0, <C>) stepped to t = T in launches of many fused steps."""
    from paper_2107_05395_amd import Factor, inputs
    import oracle
    spec = dict(inputs.WORKLOADS[args.workload])
    n, L, G, gamma, T, seed = (spec[k] for k in ("n", "length", "grid", "gamma", "T", "seed"))
    m = G * G
    dx = L / n
    dt = 0.1 * dx
    steps = int(round(T / dt))
    f0 = np.repeat(np.linspace(spec["f0"][0], spec["f0"][1], G), G)
    mean = np.tile(np.linspace(spec["mean"][0], spec["mean"][1], G), G)
    v, kw = np.full(m, spec["v"]), np.full(m, spec["k"])
    f = Factor.cahn_hilliard(n, L, gamma, dt)
    f.upload()
    c_host = mean + inputs.uniform_batch(n, m, seed=seed, lo=-0.1, hi=0.1)
    # parity first: 64 sampled runs, 20 steps, against the oracle (its own
    # coefficients and mapping of v, f0, k)
    sigma_o, alpha_o = oracle.ch_coefficients(gamma, dx, dt)
    beta, amp, kdx = oracle.ch_forced_parameters(dt, dx, v, f0, kw)
    cols = np.unique(np.r_[np.linspace(0, m - 1, 64).astype(np.int64), m - 1])
    ref = oracle.ch_forced_step(c_host[:, cols], sigma_o, alpha_o, beta[cols], amp[cols],
                                kdx[cols], steps=20)
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    pv, pf, pk = dv(v), dv(f0), dv(kw)
    c = dv(c_host)
    nxt = torch.empty_like(c)
    f.ch_forced_step(c, dt, dx, pv, pf, pk, steps=20, out=nxt)
    err = rel_err_cols(nxt[:, torch.from_numpy(cols).cuda()].cpu().numpy(), ref)
    chunk = 2000
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        f.ch_forced_step(c, dt, dx, pv, pf, pk, steps=k, out=nxt)
        c, nxt = nxt, c
        done += k
    stop.record()
    torch.cuda.synchronize()
    secs = start.elapsed_time(stop) / 1e3
    final = c
    flops = FORCED_FLOPS_ROW_STEP * n * m * steps
    # per-run summaries of the final state (what a classifier would start from)
    cmin = final.min(dim=0).values.cpu().numpy()
    cmax = final.max(dim=0).values.cpu().numpy()
    domains = float(np.mean((cmin < -0.5) & (cmax > 0.5)))
    line = {
        "metric": "system-steps/s", "value": m * steps / secs, "unit": "system-steps/s",
        "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": 1e3 * secs / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded <C> + uniform[-0.1,0.1) initial states on a parameter grid)",
        "config": {"workload": args.workload, "n": n, "L": L, "m": m, "grid": [G, G],
                   "v": spec["v"], "k": spec["k"], "f0": spec["f0"], "mean": spec["mean"],
                   "gamma": gamma, "dt": dt, "T": steps * dt, "steps_per_launch": chunk},
        "rel_err_vs_oracle_64_runs_20_steps": err,
        "fraction_of_runs_with_both_phases": domains,
        "roofline": {"bound": "alu", "achieved": flops / secs / 1e12, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": flops / secs / 1e12 / PEAK_FP64_TFLOPS,
                     "traffic": None,
                     "note": "algorithmic FP64 operations, %d per row and step: the Cahn-Hilliard "
                             "step 21, the WENO5 derivative 81 (differences 5, candidates 15, "
                             "smoothness 33, eps 11, weights 9, blend 8), the advection and "
                             "forcing terms with the cosine rotation 10" % FORCED_FLOPS_ROW_STEP},
    }
    if not args.no_cpu_baseline:
        m_s = 1 << 10
        cs = c_host[:, :m_s].copy()
        done_s, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < args.cpu_seconds:
            cs = oracle.ch_forced_step(cs, sigma_o, alpha_o, beta[:m_s], amp[:m_s], kdx[:m_s],
                                       steps=5)
            done_s += 5
        el = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": done_s * m_s / el, "unit": "system-steps/s",
                                "cores": oracle.num_threads(), "kind": "oracle",
                                "sample": "%d steps of %d runs (n=%d) with oracle.ch_forced_step, "
                                          "%.1f s" % (done_s, m_s, n, el)}
    return line


def bench_adjoint(args, torch):
    """One step = forward rollout of T implicit steps (checkpoint every c), the
    mean-squared-error loss, and the backward pass: adjoint solves with the
    same factor, band-gradient reductions and recomputation between
    checkpoints, through torch.autograd."""
    from paper_2107_05395_amd import banded_rollout, mse_loss, inputs
    spec = dict(inputs.WORKLOADS[args.workload])
    n, m, r, T, every, seed = (spec[k] for k in ("n", "m", "r", "steps", "checkpoint", "seed"))
    D0 = inputs.rng(seed).uniform(0.5, 1.5, n)
    u0_host = inputs.uniform_batch(n, m, seed=seed + 1)
    y_host = inputs.uniform_batch(n, m, seed=seed + 2)
    u0, y = torch.from_numpy(u0_host).cuda(), torch.from_numpy(y_host).cuda()
    grads = {}

    def step(prec):
        D = torch.tensor(D0, requires_grad=True)
        u = u0.detach().requires_grad_(True)
        uT = banded_rollout(u, (-r * D, 1 + 2 * r * D, -r * D), steps=T, checkpoint_every=every,
                            precision=prec)
        mse_loss(uT, y).backward()
        grads[prec] = u.grad

    out = {}
    import oracle
    cols = np.unique(np.r_[np.linspace(0, m - 1, 254).astype(np.int64), 0, m - 1])
    t_cpu = time.perf_counter()
    _, _, du0_ref = oracle.diffusion_loss_and_grads(D0, r, u0_host[:, cols], y_host[:, cols], T)
    t_cpu = time.perf_counter() - t_cpu
    du0_ref *= len(cols) / m          # the loss is a mean over all n*m entries
    for prec in ("f64", "f32r"):
        t, _ = time_launches(lambda: step(prec), args.steps, args.warmup, torch)
        du0 = grads[prec][:, torch.from_numpy(cols).cuda()].cpu().numpy()
        out[prec] = (t, rel_err_cols(du0, du0_ref))
    k = args.steps
    t64 = out["f64"][0]
    # algorithmic HBM bytes of one FP64 training step: the forward pass in
    # ceil(T/c) fused launches (read the checkpoint, write the next one or
    # u_T: 16 B per row each); per segment one trajectory launch recomputing
    # the states (read the checkpoint, write every state: 8 B per row and
    # step) and one stepping the adjoints on A^T with the band gradients
    # reduced as it goes (read the incoming adjoint and every state, write
    # the outgoing adjoint); the loss (read u and target, write the
    # gradient: 24 B per row).  The groups' partial sums of the band
    # gradients (about 1.5 B per row and segment here) are not counted.
    segments = -(-T // every)
    step_bytes = (40.0 * segments + 16.0 * T + 24.0) * n * m
    return {
        "roofline": {"bound": "hbm", "achieved": step_bytes * k / t64 / 1e9, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": step_bytes * k / t64 / 1e9 / PEAK_HBM_GBS,
                     "traffic": None,
                     "note": "whole training step, %.0f GB of algorithmic traffic" % (step_bytes / 1e9)},
        "metric": "system-steps/s (forward + backward)", "value": m * T * k / t64,
        "unit": "system-steps/s", "n_gpus": 1, "steps": k, "warmup": args.warmup,
        "ms_per_step": 1e3 * t64 / k, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded uniform[-1,1) initial states and targets, D ~ U[0.5,1.5))",
        "config": {"workload": args.workload, "n": n, "m": m, "r": r, "T": T,
                   "checkpoint_every": every},
        "du0_rel_err_vs_oracle": out["f64"][1],
        "f32r": {"value": m * T * k / out["f32r"][0], "ms_per_step": 1e3 * out["f32r"][0] / k,
                 "du0_rel_err_vs_oracle": out["f32r"][1]},
        "cpu_baseline": {"value": len(cols) * T / t_cpu, "unit": "system-steps/s (forward + backward)",
                         "cores": oracle.num_threads(), "kind": "oracle",
                         "sample": "oracle.diffusion_loss_and_grads (T=%d forward solves, T adjoint "
                                   "solves and band gradients) on %d of the m systems (n=%d), "
                                   "%.1f s" % (T, len(cols), n, t_cpu)},
    }


def probe(torch):
    """One dispatch of each kernel of interest, for rocprofv3 counter runs:
    a plain copy of known size (4 GiB read + 4 GiB written), the library's
    16 KB-tile copy of the same array, the FP64 and FP32+refine sweeps, the
    FP64 sweep of FP32 right-hand sides, the
    thread-per-system design and the sweep-pattern copy on the bench
    workload, the FP64 and FP32+refine pentadiagonal sweeps on the
    hyperdiffusion workload, the three launches of a long tridiagonal solve
    (n = 8192, m = 2^16), one launch
    of 10 fused Cahn-Hilliard steps on the n=256, m=2^20 ensemble, one
    Crank-Nicolson diffusion step (n=1024, m=2^16, periodic), and one fused
    adjoint + band-gradient launch of 10 steps (n=1024, m=2^16)."""
    from paper_2107_05395_amd import Factor, inputs
    n, m = 512, 1 << 20
    rhs = torch.rand(n, m, dtype=torch.float64, device="cuda")
    x = torch.empty_like(rhs)
    x.copy_(rhs)
    torch.cuda.synchronize()
    from paper_2107_05395_amd.solver import copy_tiles
    copy_tiles(rhs, x)
    torch.cuda.synchronize()
    f = Factor.tri(*inputs.diffusion_tri_bands(n, 1.0))
    for prec in ("f64", "f32r"):
        f.solve(rhs, out=x, precision=prec)
        torch.cuda.synchronize()
    rhs32 = rhs.float()
    f.solve(rhs32, out=x, precision="f32rhs_f64")
    torch.cuda.synchronize()
    del rhs32
    f.solve_thread_per_system(rhs, out=x)
    torch.cuda.synchronize()
    from paper_2107_05395_amd.solver import copy_rows
    copy_rows(rhs, x)
    torch.cuda.synchronize()
    del rhs, x
    n, m = 1024, 1 << 18
    rhs = torch.rand(n, m, dtype=torch.float64, device="cuda")
    x = torch.empty_like(rhs)
    g = Factor.penta(*inputs.hyperdiffusion_penta_bands(n, 0.25))
    for prec in ("f64", "f32r"):
        g.solve(rhs, out=x, precision=prec)
        torch.cuda.synchronize()
    del rhs, x
    # a long system: tri n = 8192, m = 2^16 (reduce, scan, solve)
    n, m = 8192, 1 << 16
    rhs = torch.rand(n, m, dtype=torch.float64, device="cuda")
    x = torch.empty_like(rhs)
    Factor.tri(*inputs.diffusion_tri_bands(n, 1.0)).solve(rhs, out=x)
    torch.cuda.synchronize()
    del rhs, x
    n, m = 256, 1 << 20
    c = torch.rand(n, m, dtype=torch.float64, device="cuda").mul_(0.2).sub_(0.1)
    h = Factor.cahn_hilliard(n, 2.0 * np.pi, 0.01, 1e-3)
    h.ch_step(c, h.alpha, steps=10)
    torch.cuda.synchronize()
    del c
    n, m = 1024, 1 << 16
    bands, w = inputs.cn_diffusion_problem(n, 1.0)
    cn = Factor.tri(*bands, cyclic=True)
    c = torch.rand(n, m, dtype=torch.float64, device="cuda")
    cn.cn_step(c, w, steps=1, out=torch.empty_like(c))
    torch.cuda.synchronize()
    # one segment of the differentiated rollout's backward: 10 transposed
    # steps with the band gradients reduced as they go (tri n=1024, m=2^16)
    D = inputs.rng(5).uniform(0.5, 1.5, n)
    fa = Factor.tri(-0.5 * D, 1 + D, -0.5 * D)
    traj = torch.rand(10, n, m, dtype=torch.float64, device="cuda")
    fa.adjoint_band_grad(c, traj)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "done"}), flush=True)


# Table 3 of the paper (Section 5.2, N_x, E_N, log2(E_N / E_2N)), as printed;
# context only: the paper does not define E_N or give the end time.
PAPER_TABLE3 = [(128, 0.0310, 3.7932), (256, 0.0022, 2.0376), (512, 5.45e-4, 2.0089),
                (1024, 1.35e-4, 2.0022), (2048, 3.38e-5, 2.0005), (4096, 8.45e-6, 0.8947),
                (8192, 4.54e-6, None)]
# the forced scheme's study (k = 1, v = 0.5, f0 = 1), as printed
PAPER_TABLE4 = [(256, 0.0013, 2.8363), (512, 1.8e-4, 1.9869), (1024, 4.54e-5, 2.0086),
                (2048, 1.13e-5, 1.9673), (4096, 2.88e-5, None)]


def bench_ch_convergence(args, torch):
    """The Section 5.2 convergence study of the Cahn-Hilliard scheme, or the
    same study of the forced scheme in the travelling frame: one run per N
    from eps cos(5x) to the same end time T with dt = 0.1 dx, and the
    self-convergence error E_N = max_i |C_N(x_i, T) - C_2N(x_i, T)| over the
    N points the two grids share, with the observed order log2(E_N / E_2N).
    N <= 1024 run fused on chip, longer systems one three-launch step per
    call.  The oracle repeats the runs up to N = 2048 (or the workload's
    limit) on the host; its E_N and final states are compared with the
    GPU's."""
    from paper_2107_05395_amd import Factor, inputs
    import oracle
    spec = dict(inputs.WORKLOADS[args.workload])
    L, gamma, eps, mode, s128 = (spec["length"], spec["gamma"], spec["eps"], spec["mode"],
                                 spec["steps128"])
    forced = spec.get("forced")
    ns = list(spec["ns"]) + [2 * spec["ns"][-1]]
    finals, times, steps_of = {}, {}, {}
    total_steps = 0
    for n in ns:
        dx = L / n
        dt = 0.1 * dx
        steps = s128 * n // 128
        f = Factor.cahn_hilliard(n, L, gamma, dt)
        x = np.arange(n) * dx
        c0 = torch.from_numpy((eps * np.cos(mode * x))[:, None].copy()).cuda()
        if forced:
            par = [torch.full((1,), forced[key], dtype=torch.float64, device="cuda")
                   for key in ("v", "f0", "k")]
            run = lambda s: f.ch_forced_run(c0, dt, dx, *par, s)
        else:
            run = lambda s: f.ch_run(c0, f.alpha, s)
        run(2)                                   # warm-up (tables, code)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = run(steps)
        torch.cuda.synchronize()
        times[n] = time.perf_counter() - t0
        finals[n] = out[:, 0].cpu().numpy()
        steps_of[n] = steps
        total_steps += steps
        print("N = %d: %d steps in %.2f s" % (n, steps, times[n]), file=sys.stderr, flush=True)
    table = []
    for n in spec["ns"]:
        e = float(np.max(np.abs(finals[n] - finals[2 * n][::2])))
        table.append({"N": n, "E_N": e, "steps": steps_of[n], "gpu_s": times[n]})
    for i in range(len(table) - 1):
        table[i]["order"] = float(np.log2(table[i]["E_N"] / table[i + 1]["E_N"]))
    # the oracle on the same runs up to N = 2048 (or the workload's limit)
    t0 = time.perf_counter()
    ref_finals = {}
    for n in [n for n in ns if n <= spec.get("oracle_max_n", 2048)]:
        dx = L / n
        sigma, alpha = oracle.ch_coefficients(gamma, dx, 0.1 * dx)
        c = (eps * np.cos(mode * np.arange(n) * dx))[:, None]
        if forced:
            beta, amp, kdx = oracle.ch_forced_parameters(
                0.1 * dx, dx, np.array([forced["v"]]), np.array([forced["f0"]]),
                np.array([forced["k"]]))
            ref_finals[n] = oracle.ch_forced_step(c, sigma, alpha, beta, amp, kdx,
                                                  steps=steps_of[n])[:, 0]
        else:
            ref_finals[n] = oracle.ch_step(c, sigma, alpha, steps=steps_of[n])[:, 0]
    cpu_s = time.perf_counter() - t0
    cpu_steps = sum(steps_of[n] for n in ref_finals)
    checks = []
    for row in table:
        n = row["N"]
        if n in ref_finals and 2 * n in ref_finals:
            e_ref = float(np.max(np.abs(ref_finals[n] - ref_finals[2 * n][::2])))
            row["E_N_oracle"] = e_ref
        if n in ref_finals:
            checks.append({"N": n, "max_abs_diff_vs_oracle":
                           float(np.max(np.abs(finals[n] - ref_finals[n])))})
    gpu_total = sum(times.values())
    paper = PAPER_TABLE4 if forced else PAPER_TABLE3
    return {
        "metric": "system-steps/s", "value": total_steps / gpu_total, "unit": "system-steps/s",
        "n_gpus": 1, "steps": total_steps, "warmup": 1, "ms_per_step": 1e3 * gpu_total / total_steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (the cosine initial state of Section 5.2)",
        "config": {"workload": args.workload, "ns": ns, "L": L, "gamma": gamma, "eps": eps,
                   "mode": mode, "dt": "0.1 dx", "T": s128 * 0.1 * L / 128,
                   "forced": forced},
        "table": table, "state_checks": checks,
        "paper_table": [{"N": a, "E_N": b, "order": c} for a, b, c in paper],
        "roofline": None,
        "cpu_baseline": {"value": cpu_steps / cpu_s, "unit": "system-steps/s", "cores": 1,
                         "kind": "oracle",
                         "sample": "the oracle's steps over the runs N = %s (one system each, one "
                                   "thread), %.1f s" % (sorted(ref_finals), cpu_s)},
    }


def bench_long(args, torch):
    """Long systems (tri and penta beyond one launch's on-chip limit), FP64:
    every (n, m) point times eager solves and solves replayed from a HIP graph
    (small batches are bound by latency), periodic penta as well; the oracle
    solves the same batch on the host cores (sampled systems for large m)."""
    from paper_2107_05395_amd import Factor, inputs
    import oracle
    spec = dict(inputs.WORKLOADS[args.workload])
    points = []
    for n in spec["ns"]:
        for m in spec["ms"]:
            for kind, cyclic in (("tri", False), ("penta", True)):
                bands = (inputs.diffusion_tri_bands(n, 1.0) if kind == "tri"
                         else inputs.hyperdiffusion_penta_bands(n, 0.25))
                f = Factor.tri(*bands) if kind == "tri" else Factor.penta(*bands, cyclic=cyclic)
                rhs_host = inputs.uniform_batch(n, m, seed=spec["seed"] + n + m)
                rhs = torch.from_numpy(rhs_host).cuda()
                x = torch.empty_like(rhs)
                reps = args.steps
                t, _ = time_launches(lambda: f.solve(rhs, out=x), reps, args.warmup, torch)
                graph_ms = None
                if m * n <= (1 << 22):
                    g = torch.cuda.CUDAGraph()
                    side = torch.cuda.Stream()
                    side.wait_stream(torch.cuda.current_stream())
                    with torch.cuda.stream(side):
                        with torch.cuda.graph(g, stream=side):
                            for _ in range(20):
                                f.solve(rhs, out=x)
                    torch.cuda.current_stream().wait_stream(side)
                    gt, _ = time_launches(g.replay, 5, 1, torch)
                    graph_ms = 1e3 * gt / (5 * 20)
                    del g
                cols = np.unique(np.linspace(0, m - 1, min(m, 64)).astype(np.int64))
                solve = oracle.tri_solve if kind == "tri" else oracle.penta_solve
                t0 = time.perf_counter()
                ref = solve(*bands, rhs_host[:, cols], cyclic=cyclic)
                cpu_s = (time.perf_counter() - t0) / len(cols) * m
                got = x[:, torch.from_numpy(cols).cuda()].cpu().numpy()
                err = rel_err_cols(got, ref)
                # the same draws as FP32 data, solved in FP64 (12 B per row)
                r32 = rhs.float()
                t32, _ = time_launches(lambda: f.solve(r32, out=x, precision="f32rhs_f64"), reps,
                                       args.warmup, torch)
                del r32
                pl = f.plan(m)
                points.append({"kind": kind + ("_cyclic" if cyclic else ""), "n": n, "m": m,
                               "chunk": pl["chunk"], "chunks": pl["lanes"],
                               "ms_per_solve": 1e3 * t / reps, "graph_ms_per_solve": graph_ms,
                               "hbm_gbs_algorithmic": 16.0 * n * m * reps / t / 1e9,
                               "f32rhs_f64_ms_per_solve": 1e3 * t32 / reps,
                               "oracle_ms_per_solve": 1e3 * cpu_s,
                               "rel_err_vs_oracle": err})
                del rhs, x
    # the largest tridiagonal point (the one whose counters are recorded)
    big = max(points, key=lambda p: (p["n"] * p["m"], p["kind"] == "tri"))
    ach = big["hbm_gbs_algorithmic"]
    return {
        "metric": "systems solved/s", "value": big["m"] / (big["ms_per_solve"] / 1e3),
        "unit": "systems/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": big["ms_per_solve"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded uniform[-1,1) right-hand sides)",
        "config": {"workload": args.workload, "ns": list(spec["ns"]), "ms": list(spec["ms"]),
                   "matrices": "tri (-1, 3, -1); periodic penta (0.25, -1, 2.5, -1, 0.25)"},
        "points": points,
        "roofline": {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": ach / PEAK_HBM_GBS,
                     "traffic": measured_traffic(args.workload, "f64", "long"),
                     "note": "largest point (%s n=%d m=%d), algorithmic 16 B per row; the three "
                             "launches move 24 B per row (traffic: bytes of all three)"
                             % (big["kind"], big["n"], big["m"])},
        "cpu_baseline": {"value": big["m"] / (big["oracle_ms_per_solve"] / 1e3),
                         "unit": "systems/s", "cores": oracle.num_threads(), "kind": "oracle",
                         "sample": "oracle solves of %d sampled systems per point, scaled to m"
                                   % 64},
    }


def bench_batch_sweep(args, torch):
    """The FP64 tridiagonal sweep of one matrix over batch sizes (the row
    stride of the interleaved layout is 8 m bytes), each point beside the
    sweep-pattern copy and the 16 KB-tile copy of the same n x m array: how
    the streaming rate of the sweep and of its access pattern depend on the
    stride.  With --steps 1 --warmup 0 every kernel runs once per point (for
    counter runs)."""
    from paper_2107_05395_amd import Factor, inputs
    from paper_2107_05395_amd.solver import copy_rows, copy_tiles
    import oracle
    spec = dict(inputs.WORKLOADS[args.workload])
    n = spec["n"]
    bands = inputs.diffusion_tri_bands(n, spec["r"])
    f = Factor.tri(*bands)
    points = []
    for m in spec["ms"]:
        rhs_host = inputs.uniform_batch(n, m, seed=spec["seed"] + m)
        rhs = torch.from_numpy(rhs_host).cuda()
        x = torch.empty_like(rhs)
        gb = 16.0 * n * m / 1e9
        t_sweep, _ = time_launches(lambda: f.solve(rhs, out=x), args.steps, args.warmup, torch)
        cols = np.unique(np.linspace(0, m - 1, 64).astype(np.int64))
        err = rel_err_cols(x[:, torch.from_numpy(cols).cuda()].cpu().numpy(),
                           oracle.tri_solve(*bands, rhs_host[:, cols]))
        t_rows, _ = time_launches(lambda: copy_rows(rhs, x), args.steps, args.warmup, torch)
        t_tiles, _ = time_launches(lambda: copy_tiles(rhs, x), args.steps, args.warmup, torch)
        points.append({"m": m, "row_stride_kib": 8 * m // 1024,
                       "sweep_ms": 1e3 * t_sweep / args.steps,
                       "sweep_gbs": gb * args.steps / t_sweep,
                       "pattern_copy_gbs": gb * args.steps / t_rows,
                       "tile_copy_gbs": gb * args.steps / t_tiles,
                       "rel_err_vs_oracle": err})
        del rhs, x
    big = max(points, key=lambda p: p["m"])
    return {
        "metric": "systems solved/s", "value": big["m"] / (big["sweep_ms"] / 1e3),
        "unit": "systems/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": big["sweep_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded uniform[-1,1) right-hand sides)",
        "config": {"workload": args.workload, "n": n, "ms": list(spec["ms"]),
                   "matrix": "tridiagonal (-r, 1+2r, -r), r = %g" % spec["r"]},
        "points": points,
        "roofline": {"bound": "hbm", "achieved": big["sweep_gbs"], "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": big["sweep_gbs"] / PEAK_HBM_GBS, "traffic": None,
                     "note": "largest batch; algorithmic 16 B per row"},
        "cpu_baseline": None,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="diffusion_n512_m1048576")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--ch-fuse", type=int, default=1000, help="CH steps per kernel launch")
    ap.add_argument("--ch-sample", type=int, default=1 << 12,
                    help="runs of the CH ensemble checked against the oracle after all steps")
    ap.add_argument("--probe", action="store_true",
                    help="one dispatch of each kernel (for rocprofv3 counter runs); no timing")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs every system of a batch on a "
              "single MI355X and has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        print(json.dumps({"error": "single-GPU benchmark; --gpus %d not supported" % args.gpus}))
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        sys.exit("bench.py needs a GPU")
    if args.probe:
        probe(torch)
        return
    from paper_2107_05395_amd import inputs
    kind = inputs.WORKLOADS[args.workload]["kind"]
    if kind == "tri":
        line = bench_tri(args, torch)
    elif kind == "penta":
        line = bench_penta(args, torch)
    elif kind == "ch":
        line = bench_ch(args, torch)
    elif kind == "adjoint":
        line = bench_adjoint(args, torch)
    elif kind == "cn":
        line = bench_cn(args, torch)
    elif kind == "ch_coarsening":
        line = bench_ch_coarsening(args, torch)
    elif kind == "ch_forced":
        line = bench_ch_forced(args, torch)
    elif kind == "ch_convergence":
        line = bench_ch_convergence(args, torch)
    elif kind == "long":
        line = bench_long(args, torch)
    elif kind == "batch_sweep":
        line = bench_batch_sweep(args, torch)
    else:
        sys.exit("workload %s is not a bench workload" % args.workload)
    line["device"] = torch.cuda.get_device_name(0)
    if isinstance(line.get("cpu_baseline"), dict):
        line["cpu_baseline"]["cpu_model"] = cpu_model()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
