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
    """The CPU oracle on a bounded sample: the full grid for a few steps."""
    import oracle
    rng = np.random.default_rng(si.workload_seed(1))
    c = si.random_coeffs(rng, npts(r, box))
    g = rng.random(si.padded_shape((N, N), r)).astype(np.float32 if dtype == "f32" else np.float64)
    oracle.sweep(g, radius=r, box=box, coeffs=c, steps=1)  # warm-up: first touch of the pages
    # grow the sample until one run takes at least target_s (each call also
    # copies the grid into its own two buffers, as the oracle always does)
    steps = 8
    while True:
        t0 = time.perf_counter()
        oracle.sweep(g, radius=r, box=box, coeffs=c, steps=steps)
        dt = time.perf_counter() - t0
        if dt >= target_s or steps >= T_STEPS:
            break
        steps = min(T_STEPS, int(steps * 1.15 * target_s / max(dt, 1e-3)) + 1)
    return {"value": N * N * steps / dt / 1e9, "unit": "GCell-updates/s",
            "cores": oracle.max_threads(), "kind": "oracle",
            "sample": "%s %s %dx%d interior, %d steps (of %d), %.1f s" % (
                stencil_name(r, box), dtype, N, N, steps, T_STEPS, dt)}


N3 = 512


def full_sweep3d():
    """Every compiled 3D variant at 512^3, T = 1000 (one warm-up, one timed run)."""
    import torch
    from paper_2001_01473_amd import build as lib_build
    for kind, box, r, cpl, m, nw, bt, nr in lib_build.variants_3d():
        dtype, accum = KINDS[kind]
        name = "%s3d%dr" % ("box" if box else "star", r)
        try:
            p = Problem(r, bool(box), dtype, interior=(N3, N3, N3), bt=bt, cells_per_lane=cpl,
                        rows_per_wave=m, accum=accum)
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
    for kind in (0, 1, 2):
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
    the 7-point star and the 27-point box also with compensated float32."""
    import torch
    out = []
    cases = [(dt, r, box) for dt in ("f32", "f64") for r, box in ((1, False), (2, False), (1, True), (2, True))]
    cases += [("f32c", 1, False), ("f32c", 1, True)]
    for kind, r, box in cases:
        dtype = "f64" if kind == "f64" else "f32"
        p = Problem(r, box, dtype, interior=(N3, N3, N3), accum="compensated" if kind == "f32c" else "plain")
        s = time_steps(p, 1, 1)
        g = N3 ** 3 * T_STEPS / s / 1e9
        w = 4 if dtype == "f32" else 8
        out.append({"stencil": "%s3d%dr" % ("box" if box else "star", r), "dtype": kind,
                    "bt": p.info["bt"], "kernel": ("auto", "blocked", "direct")[p.info["kernel"]],
                    "tile": [p.info["tile0"], p.info["tile1"]], "gcells": g,
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
    for kind, box, r, cpl, bt, nr in lib_build.variants_2d():
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
    out["speedup_vs_sequential_f32"] = (out["batched_graph_f32_gcells"] /
                                        out["sequential_f32_gcells"])
    return out


def bench_serve(n_requests=32, loads=(0.8,), budgets=(64 << 30,)):
    """Serving mix: Poisson arrivals of mixed 2D/3D, star/box, r in {1,2},
    float32/float64 requests with 10..1000 steps.  First the closed-loop
    capacity (all requests queued at once), then open-loop runs at the given
    fractions of that capacity; p50/p99 latency = completion - arrival."""
    import torch
    import paper_2001_01473_amd as s5d
    base = si.serve_mix(si.workload_seed(4), n_requests, rate_per_s=1.0)
    plans = [_plan_for(s, s["dtype"]) for s in base]
    inits = [_device_grid(si.padded_shape(s["interior"], s["radius"]), s["dtype"], s["seed"])
             for s in base]
    updates = [int(np.prod(s["interior"])) * s["steps"] for s in base]
    out = {"workload": "%d requests: 50%% 2D U{512..8192}^2 / 50%% 3D U{64..256}^3, star/box, "
                       "r in {1,2}, f32/f64, T U{10..1000}" % n_requests,
           "updates": sum(updates)}

    def serve(arrivals, budget):
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

    # plain: every request alone, one after the other
    t = time.perf_counter()
    for j, (p, x) in enumerate(zip(plans, inits)):
        y = torch.empty_like(x)
        p.run(x.clone(), y)
        torch.cuda.synchronize()
        print("plain: request %d done" % j, file=sys.stderr, flush=True)
    plain = time.perf_counter() - t
    out["plain_sequential_gcells"] = sum(updates) / plain / 1e9
    cap = serve([0.0] * len(plans), budgets[0])
    capacity = cap["updates_done"] / cap["makespan"]
    out["capacity_gcells"] = capacity / 1e9
    out["capacity_p50_s"], out["capacity_p99_s"] = cap["latency_p50"], cap["latency_p99"]
    print("serve capacity %.1f GCell/s, plain %.1f GCell/s" % (capacity / 1e9,
                                                                 out["plain_sequential_gcells"]),
          file=sys.stderr, flush=True)
    mean_upd = float(np.mean(updates))
    points = []
    for budget in budgets:
        for load in loads:
            rate = load * capacity / mean_upd
            arrivals = [s["arrival"] / rate for s in base]  # unit-rate arrivals rescaled
            st = serve(arrivals, budget)
            points.append({"offered_load": load, "budget_gib": budget / (1 << 30),
                           "rate_per_s": rate, "throughput_gcells": st["updates_done"] /
                           st["makespan"] / 1e9, "p50_s": st["latency_p50"],
                           "p99_s": st["latency_p99"], "ticks": st["ticks"],
                           "launches": st["launches"], "peak_gib": st["bytes_peak"] / (1 << 30)})
            print("serve load %.2f budget %.0f GiB: p50 %.3f s p99 %.3f s, %.1f GCell/s" % (
                load, budget / (1 << 30), st["latency_p50"], st["latency_p99"],
                points[-1]["throughput_gcells"]), file=sys.stderr, flush=True)
    out["points"] = points
    return out


def bench_accuracy():
    """Error after T steps of float32 (plain and compensated accumulation)
    against float64, all three started from the same float32-rounded grid and
    coefficients and run on the GPU; the norms are the library's float64
    reductions.  The float64 result is tied to the CPU oracle on sampled 2D
    cells (the oracle run on the window of the initial grid that a cell's T-step
    result depends on).  Workloads: 512^3 star3d1r and box3d1r, 16384^2
    star2d1r, T = 1000."""
    import torch
    import oracle
    import paper_2001_01473_amd as s5d
    out = []
    for ndim, r, box, interior in ((3, 1, False, (N3, N3, N3)), (3, 1, True, (N3, N3, N3)),
                                   (2, 1, False, (N, N))):
        rng = np.random.default_rng(si.workload_seed(2 if ndim == 3 else 1))
        c32 = si.random_coeffs(rng, si.n_points(ndim, r, box)).astype(np.float32)
        c = c32.astype(np.float64)
        shape = si.padded_shape(interior, r)
        g32 = _device_grid(shape, "f32", si.workload_seed(5))
        results = {}
        for kind, dt, accum in (("f64", torch.float64, "plain"), ("f32", torch.float32, "plain"),
                                ("f32c", torch.float32, "compensated")):
            x = g32.to(dt, copy=True)  # each run starts from its own copy of the grid
            y = torch.empty_like(x)
            p = s5d.Plan(ndim=ndim, radius=r, box=box, dtype="f64" if kind == "f64" else "f32",
                         interior=interior, steps=T_STEPS, coeffs=c, accum=accum)
            idx = p.run(x, y)
            torch.cuda.synchronize()
            p.close()
            results[kind] = x if idx == 0 else y
            del x, y
        assert not any(v.data_ptr() == g32.data_ptr() for v in results.values())
        ref = results["f64"]
        rec = {"stencil": stencil_name(r, box).replace("2d", "%dd" % ndim),
               "interior": list(interior), "steps": T_STEPS}
        for kind in ("f32", "f32c"):
            nm = s5d.error_norms(results[kind], ref).cpu().numpy()
            rec[kind] = {"max_abs_err": float(nm[0]), "max_rel_err": float(nm[2]),
                         "rms_err": float(nm[3]), "normwise": float(nm[0] / nm[1])}
        rec["f64_vs_oracle_sampled_rel"] = None
        if ndim == 2:
            g_host = g32.cpu().numpy().astype(np.float64)
            prng = np.random.default_rng(7)
            H = T_STEPS * r + r
            worst = 0.0
            for _ in range(3):
                pt = tuple(int(v) for v in prng.integers(r, np.array(shape) - r))
                lo = [max(0, pt[a] - H) for a in range(ndim)]
                hi = [min(shape[a], pt[a] + H + 1) for a in range(ndim)]
                win = g_host[tuple(slice(lo[a], hi[a]) for a in range(ndim))]
                want = oracle.sweep(win, radius=r, box=box, coeffs=c, steps=T_STEPS)[
                    tuple(pt[a] - lo[a] for a in range(ndim))]
                worst = max(worst, abs(float(ref[pt].item()) - want) / abs(want))
            rec["f64_vs_oracle_sampled_rel"] = worst
        out.append(rec)
        print("accuracy %s: f32 normwise %.3g, compensated %.3g" % (
            rec["stencil"], rec["f32"]["normwise"], rec["f32c"]["normwise"]), file=sys.stderr,
            flush=True)
        del results, ref, g32
        torch.cuda.empty_cache()
    return out


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
    tuning = {"bt": args.bt} if nd == 2 else {}
    bt = args.bt if nd == 2 else s5d.Plan(ndim=3, radius=1, box=False, dtype="f32", interior=interior,
                                          steps=1000, coeffs=np.full(7, 1 / 7)).query()["bt"]
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
    ap.add_argument("--batch", action="store_true",
                    help="also measure the 64-grid batched workload")
    ap.add_argument("--serve", action="store_true", help="also measure the serving loop")
    ap.add_argument("--accuracy", action="store_true",
                    help="also report float32 and compensated errors against float64 after T steps")
    ap.add_argument("--serve-requests", type=int, default=32)
    ap.add_argument("--serve-loads", default="0.8")
    ap.add_argument("--serve-budgets-gib", default="64")
    ap.add_argument("--only-extras", action="store_true",
                    help="skip the headline sweep; print only the --batch/--serve records")
    ap.add_argument("--no-extras", action="store_true",
                    help="leave the batched, serving (32 requests) and accuracy records out of "
                         "the default run")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc runs of --probe into the traffic record")
    ap.add_argument("--command", default="", help="command line recorded with --ingest-counters")
    args = ap.parse_args(argv)
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
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
        if args.bt == 0:
            args.bt = PROBE_BT
        probe(args)
        return 0
    if args.full_sweep:
        full_sweep()
        return 0
    if args.full_sweep3d:
        full_sweep3d()
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
            for r, box in STENCILS:
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
    rec.update(extras)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(1, False, "f32")
    torch.cuda.synchronize()
    print(json.dumps(rec))
    return 0


if __name__ == "__main__":
    sys.exit(main())
