#!/usr/bin/env python3
"""Benchmark of the temporally blocked stencil sweep on one MI355X.

Workload (one "step" = one whole sweep): 2D 5-point star (radius 1), float32,
16384 x 16384 interior plus a 1-cell fixed boundary, 1000 time steps, random
coefficients normalised to sum 1 and a U[0,1) grid from seed 1473+1, with the
library's tuned temporal blocking degree b_T.  Inputs are resident in HBM
before the timed region; timing uses HIP events on the stream the kernels run
on.  Reported:

* value: effective GCell-updates/s = interior cells * T / seconds (redundant
  halo work is not credited) and its fraction of the b_T = 1 HBM bound;
* roofline: the dominant kernel (one b_T round) timed per launch, against the
  HBM roofline (algorithmic bytes 2*w per cell per launch) and the vector-ALU
  roofline (algorithmic FLOP (2n-1)*b_T per cell per launch), whichever the
  kernel is closer to; HBM traffic from rocprofv3 counters when the counter
  record matches the current kernel source;
* sweep: the other stencils and dtypes of the same workload family (star
  r = 1..4, box r = 1..2, float32 and float64, T = 1000) at their tuned b_T,
  and the b_T = 1..10 curve of the 5-point star;
* cpu_baseline: the CPU oracle (naive loop, OpenMP) on a bounded sample of the
  same grid.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-sweep]
       python bench.py --probe      (a few launches of the dominant kernel and a
                                     copy of known size, for rocprofv3 counters)
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
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import stencil_inputs as si  # noqa: E402

N = 16384
T_STEPS = 1000
HBM_PEAK_GBS = 8000.0
# Published MI355X vector peaks (256 CUs at 2.4 GHz): float32 157.3 TFLOP/s,
# float64 78.6 TFLOP/s.  The float32 figure counts packed operations; built
# without them, float32 FMAs issue at 64 lanes per clock per CU like float64,
# so the ceiling of these kernels is 78.6 TFLOP/s in both types (reported
# beside the published figure).
ALU_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
ALU_PEAK_UNPACKED_TFLOPS = 78.6
STENCILS = [(1, False), (2, False), (3, False), (4, False), (1, True), (2, True)]
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_sweep2d_star_r1_f32_16384.json")
# kernel kinds of the library: (storage dtype, accumulation)
KINDS = {0: ("f32", "plain"), 1: ("f64", "plain"), 2: ("f32", "compensated")}
KIND_NAMES = {0: "f32", 1: "f64", 2: "f32c"}


def npts(r, box):
    return si.n_points(2, r, box)


def flop_per_cell(r, box):
    return 2 * npts(r, box) - 1  # AN5D Table 3 (FMA counted as 2)


def stencil_name(r, box):
    return "%s2d%dr" % ("box" if box else "star", r)


def kernel_source_hash():
    h = hashlib.sha1()
    for p in ("paper_2001_01473_amd/csrc/sweep2d.h", "paper_2001_01473_amd/csrc/s5d_internal.h",
              "paper_2001_01473_amd/csrc/kcommon.h"):
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


class Problem:
    """Device buffers and a plan for one (stencil, dtype, tuning)."""

    def __init__(self, r, box, dtype, steps=T_STEPS, interior=(N, N), seed=None, accum="plain",
                 **tuning):
        import torch
        import paper_2001_01473_amd as s5d
        self.r, self.box, self.dtype, self.steps = r, box, dtype, steps
        seed = si.workload_seed(1) if seed is None else seed
        rng = np.random.default_rng(seed)
        c = si.random_coeffs(rng, si.n_points(len(interior), r, box))
        self.coeffs = c
        shape = si.padded_shape(interior, r)
        td = torch.float32 if dtype == "f32" else torch.float64
        gen = torch.Generator(device="cuda:0").manual_seed(seed)
        # U[0,1) grid generated on the device (same distribution as the host
        # generator; the benchmark never compares values)
        self.buf0 = torch.rand(shape, dtype=td, device="cuda:0", generator=gen)
        self.buf1 = torch.empty_like(self.buf0)
        self.init = self.buf0.clone()
        self.plan = s5d.Plan(ndim=len(interior), radius=r, box=box, dtype=dtype, interior=interior,
                             steps=steps, coeffs=c, accum=accum, **tuning)
        self.info = self.plan.query()
        self.cells = int(np.prod(interior))

    def reset(self):
        self.buf0.copy_(self.init)

    def run(self):
        return self.plan.run(self.buf0, self.buf1)

    def close(self):
        self.plan.close()
        del self.buf0, self.buf1, self.init


def time_steps(prob, steps, warmup):
    """Mean seconds per whole sweep over `steps` timed sweeps (HIP events)."""
    import torch
    for _ in range(warmup):
        prob.reset()
        prob.run()
    torch.cuda.synchronize()
    total = 0.0
    for _ in range(steps):
        prob.reset()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        prob.run()
        b.record()
        b.synchronize()
        total += a.elapsed_time(b) / 1e3
    return total / steps


def time_one_round(r, box, dtype, bt, launches=20, **tuning):
    """Average duration of one launch of the b_T kernel (one round), HIP events.

    A plan of 2*b_T steps is exactly two full rounds (an even round count, as
    the result parity requires), so each run is one tiny boundary copy plus
    two launches of the b_T kernel."""
    import torch
    prob = Problem(r, box, dtype, steps=2 * bt, bt=bt, **tuning)
    for _ in range(3):
        prob.run()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(launches):
        prob.run()
    b.record()
    b.synchronize()
    dt = a.elapsed_time(b) / 1e3 / (2 * launches)
    info = prob.info
    prob.close()
    return dt, info


def roofline(r, box, dtype, bt, tuning):
    w = 4 if dtype == "f32" else 8
    dt, info = time_one_round(r, box, dtype, bt, **tuning)
    cells = N * N
    bytes_alg = 2.0 * w * cells
    flop_alg = float(flop_per_cell(r, box)) * cells * bt
    hbm = bytes_alg / dt / 1e9
    alu = flop_alg / dt / 1e12
    hbm_frac = hbm / HBM_PEAK_GBS
    alu_frac = alu / ALU_PEAK_TFLOPS[dtype]
    traffic = None
    if os.path.exists(TRAFFIC_RECORD):
        with open(TRAFFIC_RECORD) as f:
            rec = json.load(f)
        if rec.get("kernel_hash") == kernel_source_hash() and rec.get("bt") == bt:
            traffic = rec.get("hbm_bytes_per_launch")
    family = "stream2d" if info.get("kernel") == 2 else "sweep2d"  # direct row streaming at b_T = 1
    common = {"kernel": "%s %s r=%d %s bt=%d" % (family, "box" if box else "star", r, dtype, bt),
              "alu_unpacked": {"peak": ALU_PEAK_UNPACKED_TFLOPS, "unit": "TFLOP/s",
                               "frac": alu / ALU_PEAK_UNPACKED_TFLOPS},
              "launch_ms": dt * 1e3, "traffic": traffic,
              "bytes_per_launch": bytes_alg, "flop_per_launch": flop_alg}
    if alu_frac >= hbm_frac:
        out = {"bound": "alu", "achieved": alu, "peak": ALU_PEAK_TFLOPS[dtype], "unit": "TFLOP/s",
               "frac": alu_frac, "alt": {"bound": "hbm", "achieved": hbm, "peak": HBM_PEAK_GBS,
                                         "unit": "GB/s", "frac": hbm_frac}}
    else:
        out = {"bound": "hbm", "achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": hbm_frac, "alt": {"bound": "alu", "achieved": alu,
                                         "peak": ALU_PEAK_TFLOPS[dtype], "unit": "TFLOP/s",
                                         "frac": alu_frac}}
    out.update(common)
    return out


def cpu_baseline(r, box, dtype, target_s=12.0):
    """The CPU oracle on a bounded sample: the full grid for a few steps, on
    all the threads OpenMP gives the process (os.cpu_count() unless
    OMP_NUM_THREADS says otherwise)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    rng = np.random.default_rng(si.workload_seed(1))
    c = si.random_coeffs(rng, npts(r, box))
    g = rng.random(si.padded_shape((N, N), r)).astype(np.float32 if dtype == "f32" else np.float64)
    oracle.sweep(g, radius=r, box=box, coeffs=c, steps=1, threads=threads)  # warm-up: first touch of the pages
    # grow the sample until one run takes at least target_s (each call also
    # copies the grid into its own two buffers, as the oracle always does)
    steps = 8
    while True:
        t0 = time.perf_counter()
        oracle.sweep(g, radius=r, box=box, coeffs=c, steps=steps, threads=threads)
        dt = time.perf_counter() - t0
        if dt >= target_s or steps >= T_STEPS:
            break
        steps = min(T_STEPS, int(steps * 1.15 * target_s / max(dt, 1e-3)) + 1)
    cpu = _host_cpu()
    return {"value": N * N * steps / dt / 1e9, "unit": "GCell-updates/s",
            "cores": threads, "nproc": cpu["nproc"], "cpu_model": cpu["cpu_model"], "kind": "oracle",
            "sample": "%s %s %dx%d interior, %d steps (of %d), %.1f s" % (
                stencil_name(r, box), dtype, N, N, steps, T_STEPS, dt)}


def bench_plain512(reps=20):
    """The 512^2 float64 5-point star, T = 100, as a plain sweep (b_T = 1, one
    launch per step; a 4 MB grid stays in the caches, so launch latency
    dominates): eager launches and the same sweep replayed from a HIP graph
    (checked to give the eager bits), beside the oracle on 1 thread and on all
    threads (full grid, same steps)."""
    import torch
    import oracle
    n, T = 512, 100
    rng = np.random.default_rng(si.workload_seed(0))
    c = si.random_coeffs(rng, 5)
    g = si.random_grid(rng, si.padded_shape((n, n), 1))
    p = Problem(1, False, "f64", steps=T, interior=(n, n), bt=1)
    p.init.copy_(torch.from_numpy(g))
    p.plan.close()
    import paper_2001_01473_amd as s5d
    p.plan = s5d.Plan(ndim=2, radius=1, box=False, dtype="f64", interior=(n, n), steps=T, coeffs=c, bt=1)
    eager = time_steps(p, reps, 2)
    p.reset()
    idx = p.run()
    torch.cuda.synchronize()
    want = (p.buf0 if idx == 0 else p.buf1).clone()
    # capture the whole sweep (boundary copy + 100 launches) into a graph
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    p.reset()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=side):
        p.plan.run(p.buf0, p.buf1, stream=side)
    for _ in range(3):
        p.reset()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        if not torch.equal((p.buf0 if idx == 0 else p.buf1), want):
            raise AssertionError("graph replay of the 512^2 sweep differs from the eager run")
    total = 0.0
    for _ in range(reps):
        p.reset()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        graph.replay()
        b.record()
        b.synchronize()
        total += a.elapsed_time(b) / 1e3
    graphed = total / reps
    n_all = oracle.max_threads()  # before the 1-thread run below changes OpenMP's default
    want_host = oracle.sweep(g, radius=1, box=False, coeffs=c, steps=T, threads=n_all)
    got = want.cpu().numpy()
    from oracle import norms as onorms
    nm = onorms.error_norms(got, want_host)
    t1 = time.perf_counter()
    oracle.sweep(g, radius=1, box=False, coeffs=c, steps=T, threads=1)
    one = time.perf_counter() - t1
    t1 = time.perf_counter()
    oracle.sweep(g, radius=1, box=False, coeffs=c, steps=T, threads=n_all)
    allc = time.perf_counter() - t1
    p.close()
    upd = n * n * T
    cpu = _host_cpu()
    return {"workload": "star2d1r 512x512 f64 T=100, plain sweep (b_T = 1)",
            "eager_gcells": upd / eager / 1e9, "graph_gcells": upd / graphed / 1e9,
            "eager_ms": eager * 1e3, "graph_ms": graphed * 1e3,
            "vs_oracle_normwise": float(nm[0] / nm[1]), "vs_oracle_elementwise": float(nm[2]),
            "oracle_1thread_gcells": upd / one / 1e9, "oracle_all_gcells": upd / allc / 1e9,
            "oracle_threads": n_all, "nproc": cpu["nproc"], "cpu_model": cpu["cpu_model"]}


N3 = 512


def full_sweep3d(only=None, direct=True):
    """Every compiled 3D variant at 512^3, T = 1000 (one warm-up, one timed run);
    `only`: a regular expression on "<stencil> <kind>" (e.g. "star3d1r f32$")."""
    import re
    import torch
    from paper_2001_01473_amd import build as lib_build
    for kind, box, r, cpl, m, nw, bt, nr in lib_build.linear_variants_3d():
        dtype, accum = KINDS[kind]
        name = "%s3d%dr" % ("box" if box else "star", r)
        if only and not re.search(only, "%s %s" % (name, KIND_NAMES[kind])):
            continue
        try:
            p = Problem(r, bool(box), dtype, interior=(N3, N3, N3), bt=bt, cells_per_lane=cpl,
                        rows_per_wave=m, tile0=m * nw, accum=accum)
        except Exception as e:  # noqa: BLE001 - reported, not fatal
            print(json.dumps({"stencil": name, "kind": KIND_NAMES[kind], "bt": bt,
                              "tile": [nw * m, 64 * cpl], "error": str(e)[:120]}), flush=True)
            continue
        s = time_steps(p, 1, 1)
        g = N3 ** 3 * T_STEPS / s / 1e9
        print(json.dumps({"stencil": name, "kind": KIND_NAMES[kind], "bt": bt,
                          "tile": [nw * m, 64 * cpl], "kernel": "blocked",
                          "stream_chunk": p.info["stream_chunk"], "gcells": round(g, 1)}), flush=True)
        p.close()
        torch.cuda.empty_cache()
    # the direct kernels (one step per launch) for every 3D stencil and kind
    for kind in ((0, 1, 2) if direct else ()):
        dtype, accum = KINDS[kind]
        for r in (1, 2, 3, 4):
            for box in (False, True):
                name = "%s3d%dr" % ("box" if box else "star", r)
                p = Problem(r, box, dtype, interior=(N3, N3, N3), accum=accum, kernel="direct",
                            steps=100 if (box and r >= 3) else T_STEPS)
                s = time_steps(p, 1, 1)
                g = N3 ** 3 * p.steps / s / 1e9
                print(json.dumps({"stencil": name, "kind": KIND_NAMES[kind], "bt": 1,
                                  "kernel": "direct", "steps": p.steps, "gcells": round(g, 1)}),
                      flush=True)
                p.close()
                torch.cuda.empty_cache()


def sweep3d_default():
    """Every 3D stencil of the synthetic suite at 512^3, T = 1000, default plan;
    the 7-point star and the 27-point box also with compensated float32; the
    radius-3 and radius-4 stars and boxes (one step per launch), the boxes over
    100 steps."""
    import torch
    out = []
    cases = [(dt, r, box) for dt in ("f32", "f64") for r, box in ((1, False), (2, False), (1, True), (2, True))]
    cases += [("f32c", 1, False), ("f32c", 1, True)]
    cases += [(dt, r, box) for dt in ("f32", "f64") for box in (False, True) for r in (3, 4)]
    for kind, r, box in cases:
        dtype = "f64" if kind == "f64" else "f32"
        steps = 100 if (box and r >= 3) else T_STEPS
        p = Problem(r, box, dtype, interior=(N3, N3, N3), steps=steps,
                    accum="compensated" if kind == "f32c" else "plain")
        s = time_steps(p, 1, 1)
        g = N3 ** 3 * steps / s / 1e9
        w = 4 if dtype == "f32" else 8
        out.append({"stencil": "%s3d%dr" % ("box" if box else "star", r), "dtype": kind,
                    "bt": p.info["bt"], "kernel": ("auto", "blocked", "direct")[p.info["kernel"]],
                    "tile": [p.info["tile0"], p.info["tile1"]], "steps": steps, "gcells": g,
                    "pct_hbm_bound": 100.0 * g * 2 * w / HBM_PEAK_GBS})
        print("sweep3d %s %s bt=%d: %.1f GCell/s" % (out[-1]["stencil"], kind, p.info["bt"], g),
              file=sys.stderr, flush=True)
        p.close()
        torch.cuda.empty_cache()
    return out


def full_sweep():
    """Every compiled 2D variant at 16384^2, T = 1000 (one warm-up, one timed run)."""
    import torch
    from paper_2001_01473_amd import build as lib_build
    for kind, box, r, cpl, bt, nr in lib_build.linear_variants_2d():
        dtype, accum = KINDS[kind]
        try:
            p = Problem(r, bool(box), dtype, bt=bt, cells_per_lane=cpl, accum=accum)
        except Exception as e:  # noqa: BLE001 - reported, not fatal
            print(json.dumps({"stencil": stencil_name(r, box), "kind": KIND_NAMES[kind], "bt": bt,
                              "cpl": cpl, "error": str(e)[:120]}), flush=True)
            continue
        s = time_steps(p, 1, 1)
        g = N * N * T_STEPS / s / 1e9
        print(json.dumps({"stencil": stencil_name(r, box), "kind": KIND_NAMES[kind], "bt": bt,
                          "cpl": cpl,
                          "stream_chunk": p.info["stream_chunk"], "gcells": round(g, 1)}),
              flush=True)
        p.close()
        torch.cuda.empty_cache()


# The general benchmarks of AN5D Table 3 (FLOP per cell as printed there) and
# the variable-coefficient stencils.  V100 "Tuned" GCell/s of Table 5 (its
# GFLOP/s divided by the FLOP count) are context for the reader, not targets.
EXPR_CASES = [
    # name, ndim, radius, box, expr, FLOP/cell, V100 f32, V100 f64 GCell/s
    ("j2d5pt", 2, 1, False, "div", 10, 616.0, 125.8),
    ("j2d9pt", 2, 2, False, "div", 18, 355.4, 153.9),
    ("j2d9pt-gol", 2, 1, True, "div", 18, 381.4, 77.4),
    ("gradient2d", 2, 1, False, "gradient", 19, 419.2, 123.3),
    ("j3d27pt", 3, 1, True, "div", 54, 115.8, 36.2),
    ("varcoef2d1r", 2, 1, False, "varcoef", 9, None, None),
    ("varcoef2d2r", 2, 2, False, "varcoef", 17, None, None),
    ("varcoefbox2d1r", 2, 1, True, "varcoef", 17, None, None),
]


def sweep_expr(dtypes=("f32", "f64")):
    """The expression stencils at the paper's sizes (16384^2, 512^3), T = 1000,
    default plans.  Algorithmic bytes: 2w per cell per launch, plus n*w for
    the per-cell weights (read once per launch)."""
    import torch
    import paper_2001_01473_amd as s5d
    out = []
    for name, nd, r, box, expr, flop, v100_32, v100_64 in EXPR_CASES:
        for dtype in dtypes:
            interior = (N3,) * 3 if nd == 3 else (N, N)
            rng = np.random.default_rng(si.workload_seed(1 if nd == 2 else 2))
            n = si.n_points(nd, r, box)
            if expr == "div":
                u = rng.random(n)
                coeffs = list(u) + [float(u.sum())]
            elif expr == "gradient":
                coeffs = [0.3, 1.5]
            else:
                coeffs = None
            td = torch.float32 if dtype == "f32" else torch.float64
            shape = si.padded_shape(interior, r)
            gen = torch.Generator(device="cuda:0").manual_seed(si.workload_seed(1))
            x = torch.rand(shape, dtype=td, device="cuda:0", generator=gen)
            y = torch.empty_like(x)
            init = x.clone()
            fields = None
            if expr == "varcoef":
                fields = torch.rand((n,) + interior, dtype=td, device="cuda:0", generator=gen)
                fields /= fields.sum(dim=0, keepdim=True)
            plan = s5d.Plan(ndim=nd, radius=r, box=box, dtype=dtype, interior=interior, steps=T_STEPS,
                            coeffs=coeffs, expr=expr)
            info = plan.query()
            secs = []
            for rep in range(2):
                x.copy_(init)
                torch.cuda.synchronize()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                plan.run(x, y, fields=fields)
                b.record()
                b.synchronize()
                secs.append(a.elapsed_time(b) / 1e3)
            sec = secs[-1]
            cells = float(np.prod(interior))
            g = cells * T_STEPS / sec / 1e9
            w = 4 if dtype == "f32" else 8
            rec = {"stencil": name, "dtype": dtype, "bt": info["bt"], "gcells": g,
                   "gflops_table3": g * flop, "pct_hbm_bound": 100.0 * g * 2 * w / HBM_PEAK_GBS,
                   "v100_tuned_gcells": v100_32 if dtype == "f32" else v100_64}
            out.append(rec)
            print("expr %s %s bt=%d: %.1f GCell/s" % (name, dtype, info["bt"], g), file=sys.stderr, flush=True)
            plan.close()
            del x, y, init, fields
            torch.cuda.empty_cache()
    return out


def _device_grid(shape, dtype, seed):
    """U[0,1) grid generated on the device from `seed` (values are not compared
    here, only timed)."""
    import torch
    td = torch.float32 if dtype == "f32" else torch.float64
    gen = torch.Generator(device="cuda:0").manual_seed(int(seed) % (1 << 63))
    return torch.rand(shape, dtype=td, device="cuda:0", generator=gen)


def _plan_for(spec, dtype):
    import paper_2001_01473_amd as s5d
    rng = np.random.default_rng(spec["seed"])
    c = si.random_coeffs(rng, si.n_points(spec["ndim"], spec["radius"], spec["box"]))
    return s5d.Plan(ndim=spec["ndim"], radius=spec["radius"], box=spec["box"], dtype=dtype,
                    interior=spec["interior"], steps=spec["steps"], coeffs=c)


def _timed(fn, reset, reps):
    """Mean seconds of fn() over reps runs (HIP events on the current stream)."""
    import torch
    reset()
    fn()
    torch.cuda.synchronize()
    total = 0.0
    for _ in range(reps):
        reset()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        total += a.elapsed_time(b) / 1e3
    return total / reps


def bench_batch(reps=2):
    """Many-grid workload: 64 independent 2D star grids (sides U{256..4096} per
    axis, radius 1 or 2, float32, 200 steps).  Batched (one HIP graph) against
    the same grids run one after the other with s5d_run."""
    import torch
    import paper_2001_01473_amd as s5d
    specs = si.batch_mix(si.workload_seed(3))
    updates = sum(int(np.prod(s["interior"])) * s["steps"] for s in specs)
    out = {"workload": "64 2D star grids, sides U{256..4096}, r in {1,2}, f32, T=200",
           "updates": updates}
    for dtype in ("f32", "f64"):
        plans = [_plan_for(s, dtype) for s in specs]
        b0 = [_device_grid(si.padded_shape(s["interior"], s["radius"]), dtype, s["seed"])
              for s in specs]
        b1 = [torch.empty_like(x) for x in b0]
        init = [x.clone() for x in b0]

        def reset():
            for x, i in zip(b0, init):
                x.copy_(i)

        def sequential():
            for p, x, y in zip(plans, b0, b1):
                p.run(x, y)

        def sequential_sync():
            for p, x, y in zip(plans, b0, b1):
                p.run(x, y)
                torch.cuda.synchronize()

        res = {"sequential": _timed(sequential, reset, reps),
               "sequential_sync": _timed(sequential_sync, reset, reps)}
        if dtype == "f32":
            for graph in (False, True):
                batch = s5d.Batch(plans, b0, b1, graph=graph)
                res["batched_graph" if graph else "batched_eager"] = _timed(batch.run, reset, reps)
                out["launches_batched"] = batch.query()["launches"]
                batch.close()
            for graph in (False, True):
                batch = s5d.Batch(plans, b0, b1, graph=graph, persistent=True)
                res["persistent_graph" if graph else "persistent_eager"] = _timed(batch.run, reset, reps)
                batch.status()
                out["launches_persistent"] = batch.query()["launches"]
                batch.close()
            # b_T, tile and h_SN from the autotuner, once per (radius, extent
            # bucket) key; plans made afterwards take the cached choices
            import math

            def bucket(x):
                return 0 if x <= 1 else int(math.ceil(math.log2(x)))
            keys = {}
            t0 = time.perf_counter()
            for spec in specs:
                key = (spec["radius"],) + tuple(bucket(x) for x in spec["interior"])
                if key not in keys:
                    rng = np.random.default_rng(spec["seed"])
                    c = si.random_coeffs(rng, si.n_points(2, spec["radius"], False))
                    keys[key] = s5d.autotune(ndim=2, radius=spec["radius"], box=False, dtype=dtype,
                                             interior=spec["interior"], steps=spec["steps"], coeffs=c,
                                             top_k=4)[0]["bt"]
            out["autotune_keys"] = len(keys)
            out["autotune_seconds"] = time.perf_counter() - t0
            tuned = [_plan_for(s, dtype) for s in specs]
            out["autotuned_bt_histogram"] = {str(b): sum(1 for p in tuned if p.query()["bt"] == b)
                                             for b in sorted({p.query()["bt"] for p in tuned})}
            batch = s5d.Batch(tuned, b0, b1, graph=True)
            res["batched_autotuned_graph"] = _timed(batch.run, reset, reps)
            batch.close()
            for p in tuned:
                p.close()
            # leave the process's cache as it was: the shipped choices only
            s5d.tune_cache_clear()
            shipped = os.path.join(ROOT, "paper_2001_01473_amd", "tuning_gfx950.txt")
            if os.path.exists(shipped) and os.environ.get("S5D_TUNING_FILE") is None:
                s5d.tune_cache_load(shipped)
            out["launches_sequential"] = sum(
                1 + -(-p.steps // p.query()["bt"]) for p in plans)
        for k, sec in res.items():
            out["%s_%s_gcells" % (k, dtype)] = updates / sec / 1e9
            print("batch %s %s: %.1f GCell/s (%.1f ms)" % (dtype, k, updates / sec / 1e9, sec * 1e3),
                  file=sys.stderr, flush=True)
        for p in plans:
            p.close()
        del b0, b1, init
        torch.cuda.empty_cache()
    # against the faster of the two one-grid-at-a-time modes
    seq32 = max(out["sequential_f32_gcells"], out["sequential_sync_f32_gcells"])
    seq64 = max(out["sequential_f64_gcells"], out["sequential_sync_f64_gcells"])
    out["speedup_vs_sequential_f32"] = out["batched_graph_f32_gcells"] / seq32
    out["persistent_speedup_vs_sequential_f32"] = out["persistent_graph_f32_gcells"] / seq32
    out["batched_vs_plain_f64"] = out["batched_graph_f32_gcells"] / seq64
    out["persistent_vs_plain_f64"] = out["persistent_graph_f32_gcells"] / seq64
    return out


def bench_serve(n_requests=32, loads=(0.5, 0.9), budgets=(64 << 30,)):
    """Serving mix: Poisson arrivals of mixed 2D/3D, star/box, r in {1,2}
    requests with 10..1000 steps, float32/float64 50/50 as drawn ("mixed"),
    and the same requests all in float32 ("f32").  For each: the closed-loop
    capacity (all requests queued at once), then open-loop runs at the given
    fractions of that capacity; p50/p99 latency = completion - arrival.  The
    plain baselines run the same requests one at a time with s5d_run: in
    their own dtypes, and all in float64 (the plain per-grid float64 path)."""
    import torch
    import paper_2001_01473_amd as s5d
    base = si.serve_mix(si.workload_seed(4), n_requests, rate_per_s=1.0)
    updates = [int(np.prod(s["interior"])) * s["steps"] for s in base]
    out = {"workload": "%d requests: 50%% 2D U{512..8192}^2 / 50%% 3D U{64..256}^3, star/box, "
                       "r in {1,2}, f32/f64, T U{10..1000}" % n_requests,
           "updates": sum(updates), "streams": 4}

    def make(dtype_of):
        plans = [_plan_for(s, dtype_of(s)) for s in base]
        inits = [_device_grid(si.padded_shape(s["interior"], s["radius"]), dtype_of(s), s["seed"])
                 for s in base]
        return plans, inits

    def serve(plans, inits, arrivals, budget):
        srv = s5d.Server(hbm_budget_bytes=budget)
        t0 = srv.now()
        order = sorted(range(len(plans)), key=lambda i: arrivals[i])
        k = 0
        reported = ticks = 0
        while True:
            now = srv.now() - t0
            while k < len(order) and arrivals[order[k]] <= now:
                i = order[k]
                srv.submit(plans[i], inits[i], arrival=t0 + arrivals[i])
                k += 1
            running, queued = srv.tick()
            ticks += 1
            if ticks % 64 == 0:
                done = srv.stats()["done"]
                if done >= reported + max(4, len(order) // 8):
                    reported = done
                    print("serve: %d of %d requests done" % (done, len(order)), file=sys.stderr,
                          flush=True)
            if running == 0 and queued == 0:
                if k == len(order):
                    break
                time.sleep(max(0.0, min(0.01, arrivals[order[k]] - (srv.now() - t0))))
        srv.sync()
        st = srv.stats()
        srv.close()
        return st

    def one_by_one(plans, inits, label):
        t = time.perf_counter()
        for p, x in zip(plans, inits):
            y = torch.empty_like(x)
            p.run(x.clone(), y)
            torch.cuda.synchronize()
        sec = time.perf_counter() - t
        print("plain %s one by one: %.1f GCell/s" % (label, sum(updates) / sec / 1e9), file=sys.stderr,
              flush=True)
        return sum(updates) / sec / 1e9

    mean_upd = float(np.mean(updates))
    plans64, inits64 = make(lambda s: "f64")
    out["plain_f64_one_by_one_gcells"] = one_by_one(plans64, inits64, "f64")
    for p in plans64:
        p.close()
    del inits64
    for label, dtype_of in (("mixed", lambda s: s["dtype"]), ("f32", lambda s: "f32")):
        plans, inits = make(dtype_of)
        rec = {"plain_one_by_one_gcells": one_by_one(plans, inits, label)}
        cap = serve(plans, inits, [0.0] * len(plans), budgets[0])
        capacity = cap["updates_done"] / cap["makespan"]
        rec.update(capacity_gcells=capacity / 1e9, capacity_p50_s=cap["latency_p50"],
                   capacity_p99_s=cap["latency_p99"])
        print("serve %s capacity %.1f GCell/s" % (label, capacity / 1e9), file=sys.stderr, flush=True)
        points = []
        for budget in budgets:
            for load in loads:
                rate = load * capacity / mean_upd
                arrivals = [s["arrival"] / rate for s in base]  # unit-rate arrivals rescaled
                st = serve(plans, inits, arrivals, budget)
                points.append({"offered_load": load, "budget_gib": budget / (1 << 30),
                               "rate_per_s": rate, "throughput_gcells": st["updates_done"] /
                               st["makespan"] / 1e9, "p50_s": st["latency_p50"],
                               "p99_s": st["latency_p99"], "ticks": st["ticks"],
                               "launches": st["launches"], "peak_gib": st["bytes_peak"] / (1 << 30),
                               "failed": st["failed"]})
                print("serve %s load %.2f budget %.0f GiB: p50 %.3f s p99 %.3f s, %.1f GCell/s" % (
                    label, load, budget / (1 << 30), st["latency_p50"], st["latency_p99"],
                    points[-1]["throughput_gcells"]), file=sys.stderr, flush=True)
        rec["points"] = points
        out[label] = rec
        for p in plans:
            p.close()
        del inits
        torch.cuda.empty_cache()
    out["f32_capacity_vs_plain_f64"] = out["f32"]["capacity_gcells"] / out["plain_f64_one_by_one_gcells"]
    return out


def bench_accuracy():
    """Error after T = 1000 steps of float64, float32 and compensated float32
    against the CPU oracle over every cell, at sizes the oracle finishes in
    seconds: star2d1r at 2048^2, star3d1r and box3d1r at 128^3 (the same
    comparison at the benchmark sizes is `--accuracy-full`)."""
    rows = accuracy_full("all", None, n2=2048, n3=128, stencils2d=[(1, False)])
    for row in rows:
        print("accuracy %s %s: normwise %.3g, max abs %.3g (bar %.3g)" % (
            row["stencil"], row["kind"], row["normwise"], row["max_abs_err"], row["bound"]),
            file=sys.stderr, flush=True)
    return rows


def _host_cpu():
    """Threads the oracle uses, the host's logical CPU count and its model name."""
    import oracle
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cores": oracle.max_threads(), "nproc": os.cpu_count(), "cpu_model": model}


def _accuracy_row(name, kind, got, ref, steps, n, max_a0, bound_kind):
    """Error of a whole GPU grid against the whole oracle grid (numpy norms)."""
    from oracle import norms as onorms
    nm = onorms.error_norms(got, ref)
    u32 = 2.0 ** -24
    gamma = n * u32 / (1 - n * u32)
    if bound_kind == "f64":
        bound, ok = 1e-12, nm[0] / nm[1] <= 1e-12 and nm[2] <= 1e-12
    elif bound_kind == "plain":
        bound = steps * (gamma + u32) * max_a0
        ok = nm[0] <= bound
    else:
        bound = steps * (u32 + gamma * gamma) * max_a0
        ok = nm[0] <= bound
    return {"stencil": name, "kind": kind, "max_abs_err": float(nm[0]), "normwise": float(nm[0] / nm[1]),
            "elementwise": float(nm[2]), "rms_err": float(nm[3]), "bound": float(bound),
            "bound_on": "normwise and elementwise relative" if bound_kind == "f64" else "max abs",
            "ok": bool(ok)}


def accuracy_full(which="all", md=None, n2=N, n3=N3, stencils2d=STENCILS, kinds=("f64", "f32", "f32c")):
    """Whole-grid comparison with the CPU oracle at the benchmark sizes and
    T = 1000: the six 2D stencils at 16384^2 and the 7-point star and 27-point
    box at 512^3.  Float64 runs on float64 inputs against the oracle on the same
    inputs (bar: normwise and elementwise relative error <= 1e-12); float32 and
    compensated float32 on float32-rounded grid and coefficients against the
    float64 oracle run on those rounded inputs (bars: T*(gamma_n + u)*max|A0|
    plain, T*(u + gamma_n^2)*max|A0| compensated).  Every cell is compared.
    `kinds`: the subset of f64, f32, f32c to run."""
    import torch
    import oracle
    import paper_2001_01473_amd as s5d
    cases = []
    if which in ("all", "2d"):
        cases += [(2, r, box, (n2, n2)) for r, box in stencils2d]
    if which in ("all", "3d"):
        cases += [(3, 1, False, (n3,) * 3), (3, 1, True, (n3,) * 3)]
    rows = []

    def gpu_run(g, ndim, r, box, c, dtype, accum):
        x = torch.from_numpy(g).to("cuda:0")
        y = torch.empty_like(x)
        p = s5d.Plan(ndim=ndim, radius=r, box=box, dtype=dtype, interior=tuple(s - 2 * r for s in g.shape),
                     steps=T_STEPS, coeffs=c, accum=accum)
        info = p.query()
        idx = p.run(x, y)
        torch.cuda.synchronize()
        p.close()
        out = (x if idx == 0 else y).cpu().numpy()
        del x, y
        torch.cuda.empty_cache()
        return out, info

    for ndim, r, box, interior in cases:
        name = "%s%dd%dr %s" % ("box" if box else "star", ndim, r, "x".join(str(i) for i in interior))
        rng = np.random.default_rng(si.workload_seed(1 if ndim == 2 else 2))
        n = si.n_points(ndim, r, box)
        c = si.random_coeffs(rng, n)
        grid = si.random_grid(rng, si.padded_shape(interior, r))
        if "f64" in kinds:
            t0 = time.perf_counter()
            ref = oracle.sweep(grid, radius=r, box=box, coeffs=c, steps=T_STEPS)
            t_or = time.perf_counter() - t0
            print("accuracy-full %s: float64 oracle %.0f s" % (name, t_or), file=sys.stderr, flush=True)
            got, info = gpu_run(grid, ndim, r, box, c, "f64", "plain")
            row = _accuracy_row(name, "f64", got, ref, T_STEPS, n, float(grid.max()), "f64")
            row.update(bt=info["bt"], kernel=("auto", "blocked", "direct")[info["kernel"]], oracle_s=t_or)
            rows.append(row)
            print(json.dumps(row), flush=True)
            del got, ref
        g32, c32 = grid.astype(np.float32), c.astype(np.float32)
        del grid
        if "f32" not in kinds and "f32c" not in kinds:
            continue
        t0 = time.perf_counter()
        ref = oracle.sweep(g32.astype(np.float64), radius=r, box=box, coeffs=c32.astype(np.float64),
                           steps=T_STEPS)
        t_or = time.perf_counter() - t0
        print("accuracy-full %s: float64 oracle on float32 inputs %.0f s" % (name, t_or), file=sys.stderr,
              flush=True)
        for kind, accum in (("f32", "plain"), ("f32c", "compensated")):
            if kind not in kinds:
                continue
            got, info = gpu_run(g32, ndim, r, box, c32.astype(np.float64), "f32", accum)
            row = _accuracy_row(name, kind, got, ref, T_STEPS, n, float(g32.max()),
                                "plain" if accum == "plain" else "comp")
            row.update(bt=info["bt"], kernel=("auto", "blocked", "direct")[info["kernel"]], oracle_s=t_or)
            rows.append(row)
            print(json.dumps(row), flush=True)
            del got
        del ref, g32
    if md:
        cpu = _host_cpu()
        with open(md, "w") as f:
            f.write("# Whole-grid accuracy against the CPU oracle, T = 1000\n\n")
            f.write("Command (from the repository root): `python bench.py --accuracy-full %s --acc-kinds %s "
                    "--md <this file>`\n\n" % (which, ",".join(kinds)))
            f.write("Oracle: the naive double-buffered loop in C (no FMA), OpenMP over axis 0, %d threads on "
                    "%s.  Every cell of the GPU result is compared with the oracle's.  float64 rows: "
                    "float64 inputs, bar 1e-12 on the normwise (max|g-o|/max|o|) and elementwise "
                    "(max |g-o|/|o|) relative error.  float32 rows: float32-rounded grid and coefficients, "
                    "compared with the float64 oracle run on those rounded inputs; bar on max|g-o|: "
                    "T(gamma_n + u)max|A0| (plain), T(u + gamma_n^2)max|A0| (compensated), u = 2^-24.\n\n"
                    % (cpu["cores"], cpu["cpu_model"] or "the host"))
            f.write("| stencil | kind | b_T | kernel | max abs err | normwise rel | elementwise rel | "
                    "bar | ok |\n|---|---|---|---|---|---|---|---|---|\n")
            for row in rows:
                f.write("| %s | %s | %d | %s | %.3e | %.3e | %.3e | %.3e | %s |\n" % (
                    row["stencil"], row["kind"], row["bt"], row["kernel"], row["max_abs_err"],
                    row["normwise"], row["elementwise"], row["bound"], "yes" if row["ok"] else "NO"))
    return rows


def model_accuracy(md=None, kinds=(0, 1), top=5):
    """Performance model against measurement (AN5D "Model Accuracy"): every
    compiled blocked variant of the six 2D stencils at 16384^2 and of the
    7-point star and 27-point box at 512^3, T = 1000, library-chosen stream
    blocks.  For each stencil: the model's predicted and the measured time of
    every variant, whether the model's top `top` holds the measured best, and
    Tuned / Model = (model-predicted time of the model's best) / (measured
    time of the best of the model's top `top`)."""
    import torch
    import paper_2001_01473_amd as s5d
    from paper_2001_01473_amd import build as lib_build
    groups = {}
    for kind, box, r, cpl, bt, nr in lib_build.linear_variants_2d():
        if kind in kinds and (r, bool(box)) in STENCILS:
            groups.setdefault((2, kind, r, bool(box)), []).append(dict(bt=bt, cells_per_lane=cpl))
    for kind, box, r, cpl, m, nw, bt, nr in lib_build.linear_variants_3d():
        if kind in kinds and r == 1:
            groups.setdefault((3, kind, r, bool(box)), []).append(
                dict(bt=bt, cells_per_lane=cpl, rows_per_wave=m, tile0=m * nw))
    summary, rows = [], []
    for (nd, kind, r, box), tunings in sorted(groups.items()):
        dtype, accum = KINDS[kind]
        interior = (N, N) if nd == 2 else (N3, N3, N3)
        name = "%s%dd%dr" % ("box" if box else "star", nd, r)
        base = Problem(r, box, dtype, interior=interior, accum=accum)
        cand = []
        for tun in tunings:
            try:
                plan = s5d.Plan(ndim=nd, radius=r, box=box, dtype=dtype, interior=interior, steps=T_STEPS,
                                coeffs=base.coeffs, accum=accum, **tun)
            except Exception as e:  # noqa: BLE001 - reported, not fatal
                print(json.dumps({"stencil": name, "kind": KIND_NAMES[kind], "tuning": tun,
                                  "error": str(e)[:120]}), flush=True)
                continue
            base.plan.close()
            base.plan, base.info = plan, plan.query()
            pred = plan.model()["seconds"]
            meas = time_steps(base, 1, 1)
            row = {"stencil": name, "kind": KIND_NAMES[kind], "bt": base.info["bt"],
                   "tile": [base.info["tile0"], base.info["tile1"]] if nd == 3 else [base.info["tile0"]],
                   "stream_chunk": base.info["stream_chunk"], "model_s": pred, "measured_s": meas,
                   "measured_over_model": meas / pred}
            rows.append(row)
            cand.append(row)
            print(json.dumps(row), flush=True)
        base.close()
        torch.cuda.empty_cache()
        if not cand:
            continue
        by_model = sorted(cand, key=lambda x: x["model_s"])
        best = min(cand, key=lambda x: x["measured_s"])
        tuned = min(by_model[:top], key=lambda x: x["measured_s"])
        cells = float(np.prod(interior)) * T_STEPS
        summary.append({"stencil": name, "kind": KIND_NAMES[kind], "variants": len(cand),
                        "model_best_bt": by_model[0]["bt"], "model_best_gcells": cells / by_model[0]["model_s"] / 1e9,
                        "tuned_bt": tuned["bt"], "tuned_gcells": cells / tuned["measured_s"] / 1e9,
                        "measured_best_bt": best["bt"], "measured_best_gcells": cells / best["measured_s"] / 1e9,
                        "best_in_top": best in by_model[:top],
                        "tuned_over_model": by_model[0]["model_s"] / tuned["measured_s"]})
        print(json.dumps(summary[-1]), flush=True)
    if md:
        with open(md, "w") as f:
            f.write("# Performance model against measurement\n\n")
            f.write("Command (from the repository root): `python bench.py --model-accuracy --md <this file>`\n\n")
            f.write("Every compiled blocked variant of each stencil (2D at 16384^2, 3D at 512^3, T = 1000, "
                    "stream blocks chosen by the library), predicted by `s5d_plan_model` and timed once after "
                    "one warm-up sweep (HIP events).  *Tuned* is the best measured of the model's top %d; "
                    "Tuned / Model is the model's predicted rate for its best over Tuned's measured rate "
                    "(AN5D \"Model Accuracy\").\n\n" % top)
            f.write("| stencil | kind | variants | model best b_T | model GCell/s | tuned b_T | tuned GCell/s | "
                    "measured best b_T | measured best GCell/s | best in model top %d | Tuned / Model |\n"
                    "|---|---|---|---|---|---|---|---|---|---|---|\n" % top)
            for x in summary:
                f.write("| %s | %s | %d | %d | %.0f | %d | %.0f | %d | %.0f | %s | %.2f |\n" % (
                    x["stencil"], x["kind"], x["variants"], x["model_best_bt"], x["model_best_gcells"],
                    x["tuned_bt"], x["tuned_gcells"], x["measured_best_bt"], x["measured_best_gcells"],
                    "yes" if x["best_in_top"] else "no", x["tuned_over_model"]))
            f.write("\n## Every variant\n\n| stencil | kind | b_T | tile | h_SN | model ms | measured ms | "
                    "measured / model |\n|---|---|---|---|---|---|---|---|\n")
            for x in rows:
                f.write("| %s | %s | %d | %s | %d | %.2f | %.2f | %.2f |\n" % (
                    x["stencil"], x["kind"], x["bt"], "x".join(str(t) for t in x["tile"]), x["stream_chunk"],
                    x["model_s"] * 1e3, x["measured_s"] * 1e3, x["measured_over_model"]))
    return summary


def write_tuning(path, top_k=5, steps=200):
    """Autotune (s5d_autotune, model-ranked, top_k measured) every stencil of
    the benchmark suite at the benchmark sizes -- the six 2D stencils at
    16384^2 and the 3D stars and boxes of radius 1 and 2 at 512^3, in float32,
    float64 and compensated float32, and the expression stencils of Table 3 --
    and save the winners as the library's shipped tuning file."""
    import paper_2001_01473_amd as s5d
    s5d.tune_cache_clear()
    cases = []
    for kind in (0, 1, 2):
        for r, box in STENCILS:
            cases.append((2, r, box, kind, "linear", (N, N)))
        for r in (1, 2):
            for box in (False, True):
                cases.append((3, r, box, kind, "linear", (N3, N3, N3)))
    for name, nd, r, box, expr, _, _, _ in EXPR_CASES:
        for kind in (0, 1):
            cases.append((nd, r, box, kind, expr, (N, N) if nd == 2 else (N3, N3, N3)))
    for nd, r, box, kind, expr, interior in cases:
        dtype, accum = KINDS[kind]
        n = si.n_points(nd, r, box)
        c = si.random_coeffs(np.random.default_rng(si.workload_seed(1)), n)
        if expr == "div":
            c = np.append(c, 1.0)
        elif expr == "gradient":
            c = np.array([0.5, 1.0])
        elif expr == "varcoef":
            c = None
        try:
            tun, rep = s5d.autotune(ndim=nd, radius=r, box=box, dtype=dtype, interior=interior, steps=steps,
                                    coeffs=c, accum=accum, expr=expr, top_k=top_k)
        except Exception as e:  # noqa: BLE001 - reported, not fatal
            print(json.dumps({"ndim": nd, "r": r, "box": box, "kind": KIND_NAMES[kind], "expr": expr,
                              "error": str(e)[:120]}), flush=True)
            continue
        print(json.dumps({"ndim": nd, "r": r, "box": box, "kind": KIND_NAMES[kind], "expr": expr,
                          "bt": tun["bt"], "stream_chunk": tun["stream_chunk"],
                          "best_s_per_step": rep["best_seconds_per_step"],
                          "default_s_per_step": rep["default_seconds_per_step"]}), flush=True)
    s5d.tune_cache_save(path)
    text = open(path).read()
    with open(path, "w") as f:
        f.write("# written by: python bench.py --write-tuning <this file>  (s5d_autotune, top %d measured, "
                "T = %d, on MI355X)\n" % (top_k, steps))
        f.write(text)


def summarize_trace(d, top=12):
    """Markdown table of per-kernel dispatch durations from a rocprofv3
    --kernel-trace run (its *kernel_trace.csv): calls, total, mean, median,
    min, max, share of all kernel time; kernel names shortened to their
    template arguments."""
    import csv
    import glob
    import re
    dur = {}
    for f in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            name = r["Kernel_Name"]
            m = re.match(r"(?:void )?(?:s5d::)?([A-Za-z0-9_]+)(<[^()]*>)?", name)
            short = (m.group(1) + (m.group(2) or "")) if m else name[:60]
            dur.setdefault(short, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in dur.values())
    rows = sorted(dur.items(), key=lambda kv: -sum(kv[1]))[:top]
    print("| kernel | calls | total (ms) | mean (us) | median (us) | min (us) | max (us) | share |")
    print("|---|---|---|---|---|---|---|---|")
    for k, v in rows:
        v = sorted(v)
        print("| `%s` | %d | %.2f | %.1f | %.1f | %.1f | %.1f | %.1f%% |" % (
            k, len(v), sum(v) / 1e3, sum(v) / len(v), v[len(v) // 2], v[0], v[-1], 100.0 * sum(v) / total))
    return rows


def summarize_pmc(d, kernel):
    """Markdown table of per-dispatch counter averages (rocprofv3 --pmc CSV)."""
    import csv
    import glob
    vals = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if kernel in r["Kernel_Name"]:
                vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    print("| counter | dispatches | average per dispatch |")
    print("|---|---|---|")
    for k in sorted(vals):
        v = vals[k]
        print("| %s | %d | %.6g |" % (k, len(v), sum(v) / len(v)))


def ingest_counters(fetch_dir, write_dir, out_json, out_md, command):
    """Per-launch HBM traffic of the headline kernel from two rocprofv3 --pmc
    runs of `bench.py --probe` (FETCH_SIZE, then WRITE_SIZE), each scaled by what
    the same counter reads for the probe's copy of known size."""
    import csv
    import glob

    def load(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            rows += [r for r in csv.DictReader(open(f)) if r["Counter_Name"] == counter]
        kern = [float(r["Counter_Value"]) for r in rows if "sweep2d_kernel" in r["Kernel_Name"]]
        # the copy of known size is torch's elementwise add kernel
        copy = [float(r["Counter_Value"]) for r in rows if "add" in r["Kernel_Name"].lower()
                and "sweep2d" not in r["Kernel_Name"]]
        if not kern or not copy:
            raise SystemExit("no %s records in %s" % (counter, d))
        return sum(kern) / len(kern), max(copy), len(kern)

    copy_bytes = float(PROBE_COPY_BYTES)
    kf, cf, nk = load(fetch_dir, "FETCH_SIZE")
    kw, cw, _ = load(write_dir, "WRITE_SIZE")
    f_scale = copy_bytes / (cf * 1024.0)
    w_scale = copy_bytes / (cw * 1024.0)
    read_b = kf * 1024.0 * f_scale
    write_b = kw * 1024.0 * w_scale
    rec = {"kernel": "sweep2d star r=1 f32 bt=%d 16384^2" % PROBE_BT, "bt": PROBE_BT,
           "kernel_hash": kernel_source_hash(),
           "fetch_size_kib_per_launch": kf, "write_size_kib_per_launch": kw,
           "copy_fetch_kib": cf, "copy_write_kib": cw, "copy_bytes_each_way": copy_bytes,
           "fetch_scale": f_scale, "write_scale": w_scale, "launches": nk,
           "hbm_read_bytes_per_launch": read_b, "hbm_write_bytes_per_launch": write_b,
           "hbm_bytes_per_launch": read_b + write_b,
           "algorithmic_bytes_per_launch": 2.0 * 4 * N * N, "command": command}
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1)
    with open(out_md, "w") as f:
        f.write("# HBM traffic: sweep2d star r=1 float32 b_T=%d, 16384^2 interior\n\n" % PROBE_BT)
        f.write("Commands (run from the repository root):\n\n```\n%s\n```\n\n" % command)
        f.write("| counter | kernel (KiB/launch) | copy of %.0f MiB (KiB) | scale | bytes/launch |\n"
                % (copy_bytes / 2**20))
        f.write("|---|---|---|---|---|\n")
        f.write("| FETCH_SIZE | %.0f | %.0f | %.3f | %.3e |\n" % (kf, cf, f_scale, read_b))
        f.write("| WRITE_SIZE | %.0f | %.0f | %.3f | %.3e |\n" % (kw, cw, w_scale, write_b))
        f.write("\nAlgorithmic bytes per launch (one read + one write of the 16386^2 "
                "float32 grid, interior only counted): %.3e.  Measured / algorithmic = %.2f.\n"
                % (2.0 * 4 * N * N, (read_b + write_b) / (2.0 * 4 * N * N)))
    print(json.dumps(rec))


PROBE_BT = 10
PROBE_COPY_BYTES = 1 << 30


def bt_traffic(d, out_md, command):
    """HBM traffic of the star2d1r float32 16384^2 launch for every b_T, from
    rocprofv3 --pmc runs of `bench.py --probe --bt k` in d/FETCH_SIZE_bt<k> and
    d/WRITE_SIZE_bt<k>; each counter is scaled by what it reads for the probe's
    copy of known size.  The kernel of a run is the one other than the copy
    with the most dispatches (the row-streaming kernel at b_T = 1)."""
    import csv
    import glob

    def is_copy(k):
        return "add" in k.lower() and "s5d" not in k

    def load(path, counter):
        per = {}
        for f in glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] == counter:
                    per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        copy = [max(v) for k, v in per.items() if is_copy(k)]
        kern = sorted(((len(v), k) for k, v in per.items() if not is_copy(k)), reverse=True)
        if not copy or not kern:
            raise SystemExit("no %s records in %s" % (counter, path))
        name = kern[0][1]
        return sum(per[name]) / len(per[name]), max(copy), name

    rows = []
    algo = 2.0 * 4 * N * N
    for bt in range(1, 11):
        try:
            kf, cf, name = load(os.path.join(d, "FETCH_SIZE_bt%d" % bt), "FETCH_SIZE")
            kw, cw, _ = load(os.path.join(d, "WRITE_SIZE_bt%d" % bt), "WRITE_SIZE")
        except SystemExit as e:
            print(e, file=sys.stderr)
            continue
        rd = kf * PROBE_COPY_BYTES / cf
        wr = kw * PROBE_COPY_BYTES / cw
        rows.append((bt, name.split("(")[0][:60], rd, wr, (rd + wr) / algo))
    with open(out_md, "w") as f:
        f.write("# HBM traffic per launch against b_T: star2d1r float32, 16384^2 interior\n\n")
        f.write("Commands (from the repository root):\n\n```\n%s\n```\n\n" % command)
        f.write("Each counter is scaled by what it reads for a copy of %d MiB each way.  Algorithmic bytes "
                "per launch: one read and one write of the interior, %.3e.\n\n" % (PROBE_COPY_BYTES >> 20, algo))
        f.write("| b_T | kernel | read bytes | write bytes | (read + write) / algorithmic |\n"
                "|---|---|---|---|---|\n")
        for bt, name, rd, wr, ratio in rows:
            f.write("| %d | `%s` | %.3e | %.3e | %.2f |\n" % (bt, name, rd, wr, ratio))
    return rows


def probe(args):
    """Launches for rocprofv3 counter runs: a copy of known size, then the kernel."""
    import torch
    nbytes = PROBE_COPY_BYTES
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").uniform_()
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    # the copy of known size: y = x + x reads x once and writes y once
    torch.add(x, x, out=y)
    torch.cuda.synchronize()
    print("probe copy bytes_read=%d bytes_written=%d" % (nbytes, nbytes), flush=True)
    del x, y
    import paper_2001_01473_amd as s5d
    nd = 3 if args.probe3d else 2
    interior = (N3,) * 3 if nd == 3 else (N, N)
    shape = si.padded_shape(interior, 1)
    b0 = torch.full(shape, 0.5, dtype=torch.float32, device="cuda:0")
    b1 = torch.empty_like(b0)
    # 2*b_T steps = two launches of the b_T kernel per run
    if nd == 2 and args.bt:
        tuning, bt = {"bt": args.bt}, args.bt
    else:
        # the launch of the default plan of the 1000-step sweep (the headline's)
        ref = s5d.Plan(ndim=nd, radius=1, box=False, dtype="f32", interior=interior, steps=T_STEPS,
                       coeffs=np.full(si.n_points(nd, 1, False), 1.0 / si.n_points(nd, 1, False)))
        q = ref.query()
        ref.close()
        bt = q["bt"]
        tuning = {k: q[k] for k in ("bt", "cells_per_lane", "stream_chunk")} if nd == 2 else {}
    plan = s5d.Plan(ndim=nd, radius=1, box=False, dtype="f32", interior=interior, steps=2 * bt,
                    coeffs=si.random_coeffs(np.random.default_rng(si.workload_seed(nd - 1)),
                                            si.n_points(nd, 1, False)), **tuning)
    for _ in range(args.launches):
        plan.run(b0, b1)
    torch.cuda.synchronize()
    print("probe kernel %s runs=%d" % (json.dumps(plan.query()), args.launches), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--bt", type=int, default=0, help="force b_T for the headline run")
    ap.add_argument("--probe", action="store_true")
    ap.add_argument("--probe3d", action="store_true",
                    help="with --probe: the 7-point star at 512^3 (default plan) instead")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("DIR", "KERNEL"),
                    help="print per-dispatch averages of every counter in a rocprofv3 --pmc "
                         "output directory for kernels whose name contains KERNEL")
    ap.add_argument("--full-sweep3d", action="store_true",
                    help="time every compiled 3D variant at 512^3, T = 1000")
    ap.add_argument("--full-sweep", action="store_true",
                    help="time every compiled (stencil, dtype, b_T, cells per lane) at the "
                         "benchmark size and print one JSON line per variant")
    ap.add_argument("--launches", type=int, default=3)
    ap.add_argument("--only", default=None, help="with --full-sweep3d: regex on '<stencil> <kind>'")
    ap.add_argument("--batch", action="store_true",
                    help="also measure the 64-grid batched workload")
    ap.add_argument("--serve", action="store_true", help="also measure the serving loop")
    ap.add_argument("--accuracy", action="store_true",
                    help="also report float32 and compensated errors against float64 after T steps")
    ap.add_argument("--accuracy-full", nargs="?", const="all", choices=("all", "2d", "3d"),
                    help="compare whole T = 1000 grids at the benchmark sizes with the CPU oracle")
    ap.add_argument("--expr", action="store_true", help="time only the expression stencils")
    ap.add_argument("--write-tuning", default=None, metavar="PATH",
                    help="autotune the benchmark suite and save the library's tuning file")
    ap.add_argument("--model-accuracy", action="store_true",
                    help="predicted against measured time of every blocked variant (with --md: a table)")
    ap.add_argument("--model-kinds", default="0,1", help="with --model-accuracy: kinds (0 f32, 1 f64, 2 f32c)")
    ap.add_argument("--md", default=None, help="with --accuracy-full: write a markdown table here")
    ap.add_argument("--acc-stencils", default=None,
                    help="with --accuracy-full: comma-separated 2D stencils (e.g. star2d1r,box2d2r)")
    ap.add_argument("--acc-kinds", default=None,
                    help="with --accuracy-full: comma-separated subset of f64,f32,f32c")
    ap.add_argument("--serve-requests", type=int, default=32)
    ap.add_argument("--serve-loads", default="0.5,0.9")
    ap.add_argument("--serve-budgets-gib", default="64")
    ap.add_argument("--only-extras", action="store_true",
                    help="skip the headline sweep; print only the --batch/--serve records")
    ap.add_argument("--no-extras", action="store_true",
                    help="leave the batched, serving (32 requests) and accuracy records out of "
                         "the default run")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc runs of --probe into the traffic record")
    ap.add_argument("--command", default="", help="command line recorded with --ingest-counters")
    ap.add_argument("--summarize-trace", default=None, metavar="DIR",
                    help="per-kernel duration table of a rocprofv3 --kernel-trace run")
    ap.add_argument("--bt-traffic", nargs=2, metavar=("DIR", "OUT_MD"),
                    help="per-b_T HBM traffic table from rocprofv3 --pmc runs of --probe --bt k")
    args = ap.parse_args(argv)
    if args.summarize_trace:
        summarize_trace(args.summarize_trace)
        return 0
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return 0
    if args.bt_traffic:
        bt_traffic(args.bt_traffic[0], args.bt_traffic[1], args.command)
        return 0
    if args.ingest_counters:
        ingest_counters(args.ingest_counters[0], args.ingest_counters[1], TRAFFIC_RECORD,
                        TRAFFIC_RECORD.replace(".json", ".md"), args.command)
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the stencil sweep here runs on a single MI355X "
              "(multi-GPU sharding is described, not built); use --gpus 1", file=sys.stderr)
        return 2
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    if args.probe:
        probe(args)
        return 0
    if args.full_sweep:
        full_sweep()
        return 0
    if args.full_sweep3d:
        full_sweep3d(args.only, direct=not args.only)
        return 0
    if args.expr:
        print(json.dumps(sweep_expr()))
        return 0
    if args.accuracy_full:
        sel = STENCILS
        if args.acc_stencils:
            names = args.acc_stencils.split(",")
            sel = [(r, box) for r, box in STENCILS if stencil_name(r, box) in names]
        kinds = tuple(args.acc_kinds.split(",")) if args.acc_kinds else ("f64", "f32", "f32c")
        rows = accuracy_full(args.accuracy_full, args.md, stencils2d=sel, kinds=kinds)
        return 0 if all(r["ok"] for r in rows) else 1
    if args.write_tuning:
        os.environ["S5D_TUNING_FILE"] = ""  # measure against the built-in defaults
        write_tuning(args.write_tuning)
        return 0
    if args.model_accuracy:
        model_accuracy(args.md, kinds=tuple(int(k) for k in args.model_kinds.split(",")))
        return 0

    extras = {}
    if args.accuracy:
        extras["accuracy"] = bench_accuracy()
    if args.batch:
        extras["batched"] = bench_batch()
    if args.serve:
        extras["serving"] = bench_serve(
            args.serve_requests, tuple(float(x) for x in args.serve_loads.split(",")),
            tuple(int(float(x) * (1 << 30)) for x in args.serve_budgets_gib.split(",")))
    if args.only_extras:
        print(json.dumps(extras))
        return 0

    tuning = {"bt": args.bt} if args.bt else {}
    prob = Problem(1, False, "f32", **tuning)
    info = prob.info
    sec = time_steps(prob, args.steps, args.warmup)
    prob.close()
    gcells = N * N * T_STEPS / sec / 1e9
    rec = {
        "metric": "GCell-updates/s & % HBM roofline; batched/served vs plain, p50/p99",
        "value": gcells, "unit": "GCell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "star2d1r 16384x16384 f32 T=1000", "stencil": "star2d1r",
                   "interior": [N, N], "time_steps": T_STEPS, "bt": info["bt"],
                   "tile": info["tile0"], "stream_chunk": info["stream_chunk"],
                   "cells_per_lane": info["cells_per_lane"]},
        "pct_hbm_bound": 100.0 * gcells * 2 * 4 / HBM_PEAK_GBS,
    }
    print("headline: %.1f GCell/s (%.0f%% of the b_T=1 HBM bound)" %
          (gcells, rec["pct_hbm_bound"]), file=sys.stderr, flush=True)
    rec["roofline"] = roofline(1, False, "f32", info["bt"],
                               {k: info[k] for k in ("stream_chunk", "cells_per_lane")})
    if not args.no_sweep:
        sweep = []
        for dtype in ("f32", "f64"):
            for r, box in STENCILS + [(3, True), (4, True)]:
                p = Problem(r, box, dtype)
                s = time_steps(p, 1, 1)
                w = 4 if dtype == "f32" else 8
                g = N * N * T_STEPS / s / 1e9
                sweep.append({"stencil": stencil_name(r, box), "dtype": dtype, "bt": p.info["bt"],
                              "cells_per_lane": p.info["cells_per_lane"],
                              "stream_chunk": p.info["stream_chunk"], "gcells": g,
                              "pct_hbm_bound": 100.0 * g * 2 * w / HBM_PEAK_GBS})
                p.close()
                print("sweep %s %s bt=%d: %.1f GCell/s" % (stencil_name(r, box), dtype,
                                                           sweep[-1]["bt"], g),
                      file=sys.stderr, flush=True)
        rec["sweep"] = sweep
        curve = []
        for dtype in ("f32", "f64"):
            for bt in range(1, 11):
                try:
                    p = Problem(1, False, dtype, bt=bt)
                except Exception as e:  # a depth without a compiled kernel
                    curve.append({"dtype": dtype, "bt": bt, "gcells": None, "note": str(e)[:80]})
                    continue
                s = time_steps(p, 1, 1)
                g = N * N * T_STEPS / s / 1e9
                curve.append({"dtype": dtype, "bt": bt, "cells_per_lane": p.info["cells_per_lane"],
                              "stream_chunk": p.info["stream_chunk"],
                              "kernel": ("auto", "blocked", "direct")[p.info["kernel"]], "gcells": g,
                              "pct_of_bt_hbm_roofline": 100.0 * g * 2 * (4 if dtype == "f32" else 8) /
                              HBM_PEAK_GBS / bt})
                p.close()
                print("bt-curve star2d1r %s bt=%d: %.1f GCell/s" % (dtype, bt, g),
                      file=sys.stderr, flush=True)
        rec["bt_curve_star2d1r"] = curve
        rec["sweep3d_512"] = sweep3d_default()
        rec["expression_stencils"] = sweep_expr()
    if not args.no_extras:
        # the metric's batched/served-vs-plain and p50/p99 parts, at their
        # default (short) sizes; --batch / --serve / --accuracy alone give
        # the larger runs recorded under profiles/
        if "batched" not in extras:
            extras["batched"] = bench_batch()
        if "serving" not in extras:
            extras["serving"] = bench_serve()
        if "accuracy" not in extras:
            extras["accuracy"] = bench_accuracy()
        extras["plain_512_f64"] = bench_plain512()
    rec.update(extras)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(1, False, "f32")
    torch.cuda.synchronize()
    print(json.dumps(rec))
    return 0


if __name__ == "__main__":
    sys.exit(main())
