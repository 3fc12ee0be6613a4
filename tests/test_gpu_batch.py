"""GPU tests of batched execution (s5d_batch_*).

Bars: every grid of a batch is bit-identical to the same grid run alone with
s5d_run (same plan), eager and graph-replayed alike; grids of the float64
kinds are also within 1e-12 of the oracle, float32 grids within the a-priori
bound.  The many-grid workload (64 2D star grids, sides U{256..4096}, radius
1 or 2, float32, 200 steps) is checked in full against single runs and, for
its eight smallest grids, against the oracle.
"""
import numpy as np
import pytest

import oracle
import paper_2001_01473_amd as s5d
import pins
import stencil_inputs as si
from gpu_util import rel_errors, say, torch

pytestmark = pytest.mark.gpu

DT = {"f32": np.float32, "f64": np.float64}


def _plan(spec, dtype, accum="plain", **tuning):
    case = si.make_case(spec["seed"], spec["ndim"], spec["radius"], spec["box"],
                        spec["interior"], spec["steps"])
    c_in, g_in = case.as_dtype(dtype)
    plan = s5d.Plan(ndim=spec["ndim"], radius=spec["radius"], box=spec["box"], dtype=dtype,
                    interior=spec["interior"], steps=spec["steps"], coeffs=case.coeffs,
                    accum=accum, **tuning)
    return plan, g_in, c_in


def _alone(plan, g_in):
    t = torch()
    x = t.from_numpy(g_in).to("cuda:0")
    y = t.empty_like(x)
    idx = plan.run(x, y)
    t.cuda.synchronize()
    return (x if idx == 0 else y).cpu().numpy()


def _run_batch(plans, grids, graph, repeats=1):
    t = torch()
    b0 = [t.from_numpy(g).to("cuda:0") for g in grids]
    b1 = [t.empty_like(x) for x in b0]
    batch = s5d.Batch(plans, b0, b1, graph=graph)
    outs = []
    for rep in range(repeats):
        if rep:
            for x, g in zip(b0, grids):  # eager work between replays
                x.copy_(t.from_numpy(g))
            t.cuda.synchronize()
        idx = batch.run()
        t.cuda.synchronize()
        outs.append([(b0[i] if idx[i] == 0 else b1[i]).cpu().numpy() for i in range(len(plans))])
    info = batch.query()
    batch.close()
    return outs, info


def _mixed_specs():
    specs = []
    shapes = [(2, 1, False, (300, 517)), (2, 2, False, (77, 1030)), (2, 1, True, (129, 65)),
              (2, 2, True, (260, 300)), (3, 1, False, (40, 37, 150)), (3, 1, True, (21, 19, 70)),
              (2, 1, False, (5, 3)), (2, 3, False, (200, 211))]
    for j, (nd, r, box, interior) in enumerate(shapes):
        for T in (0, 1, 6, 13):
            specs.append(dict(ndim=nd, radius=r, box=box, interior=interior, steps=T,
                              seed=si.item_seed(77, 10 * j + T)))
    return specs


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("kind", ["f32", "f64", "f32c"])
def test_mixed_batch_equals_alone(kind, graph):
    dtype = np.float32 if kind != "f64" else np.float64
    accum = "compensated" if kind == "f32c" else "plain"
    specs = _mixed_specs()
    made = [_plan(s, dtype, accum) for s in specs]
    plans = [m[0] for m in made]
    grids = [m[1] for m in made]
    say("batch mixed", kind, "graph" if graph else "eager", len(specs), "grids")
    outs, info = _run_batch(plans, grids, graph, repeats=3 if graph else 1)
    lo = max(-(-p.steps // p.query()["bt"]) for p in plans)
    assert lo <= info["round_steps"] <= lo + 2
    for i, (p, g) in enumerate(zip(plans, grids)):
        alone = _alone(p, g)
        for rep, out in enumerate(outs):
            np.testing.assert_array_equal(out[i], alone, err_msg="grid %d replay %d" % (i, rep))
    for i, ((p, g, c), s) in enumerate(zip(made, specs)):
        ref_kw = dict(radius=s["radius"], box=s["box"], steps=s["steps"])
        if kind == "f64":
            ref = oracle.sweep(g, coeffs=c, **ref_kw)
            assert max(rel_errors(outs[0][i], ref)) <= 1e-12
        elif kind == "f32c":
            ref = oracle.sweep(g, coeffs=c, accum="compensated", **ref_kw)
            np.testing.assert_array_equal(outs[0][i], ref)


def test_batch_launch_count_and_empty():
    specs = [dict(ndim=2, radius=1, box=False, interior=(600, 700), steps=40,
                  seed=si.item_seed(5, j)) for j in range(16)]
    made = [_plan(s, np.float32) for s in specs]
    t = torch()
    b0 = [t.from_numpy(m[1]).to("cuda:0") for m in made]
    b1 = [t.empty_like(x) for x in b0]
    batch = s5d.Batch([m[0] for m in made], b0, b1)
    q = batch.query()
    # one boundary-copy launch for all grids plus one launch per round index (one variant)
    assert q["launches"] == 1 + q["round_steps"]
    batch.close()
    empty = s5d.Batch([], [], [])
    assert empty.run() == [] and empty.query() == {"launches": 0, "round_steps": 0}
    empty.close()


def test_batch_rejects_shared_buffers():
    spec = dict(ndim=2, radius=1, box=False, interior=(64, 64), steps=3, seed=1)
    p, g, _ = _plan(spec, np.float64)
    t = torch()
    a, b = t.from_numpy(g).to("cuda:0"), t.empty(g.shape, dtype=t.float64, device="cuda:0")
    with pytest.raises(s5d.Stencil5DError) as err:
        s5d.Batch([p, p], [a, a], [b, t.empty_like(b)])
    assert err.value.status == 1


def test_many_grid_workload_bitwise_and_oracle():
    """64 2D star grids, sides U{256..4096}, radius 1 or 2, float32, T = 200,
    default tuning, one graph: all 64 bit-identical to single runs, the eight
    smallest within the float32 bound of the float64 oracle."""
    specs = si.batch_mix(si.workload_seed(3))
    made = [_plan(s, np.float32) for s in specs]
    plans, grids = [m[0] for m in made], [m[1] for m in made]
    say("batch 64 grids, graph")
    outs, info = _run_batch(plans, grids, graph=True, repeats=2)
    say("batch launches", info)
    for i in range(len(plans)):
        alone = _alone(plans[i], grids[i])
        np.testing.assert_array_equal(outs[0][i], alone, err_msg="grid %d" % i)
        np.testing.assert_array_equal(outs[1][i], alone, err_msg="grid %d replay" % i)
    order = sorted(range(len(specs)), key=lambda i: np.prod(specs[i]["interior"]))[:8]
    for i in order:
        s, (p, g, c) = specs[i], made[i]
        ref = oracle.sweep(g.astype(np.float64), radius=s["radius"], box=False,
                           coeffs=c.astype(np.float64), steps=s["steps"])
        n = len(c)
        bound = s["steps"] * (pins.gamma(n, pins.U32) + pins.U32) * float(g.max()) * 1.01
        assert float(np.max(np.abs(outs[0][i].astype(np.float64) - ref))) <= bound, i


def test_autotuned_plan_same_bits():
    """The autotuner's choice (cached, then taken by a plan without tuning)
    gives the same bits as the library's default choice."""
    s5d.tune_cache_clear()
    spec = dict(ndim=2, radius=1, box=False, interior=(900, 1400), steps=37, seed=si.item_seed(9, 1))
    p0, g, _ = _plan(spec, np.float32)
    base = _alone(p0, g)
    case = si.make_case(spec["seed"], 2, 1, False, spec["interior"], spec["steps"])
    tun, rep = s5d.autotune(ndim=2, radius=1, box=False, dtype="f32", interior=spec["interior"],
                            steps=spec["steps"], coeffs=case.coeffs, top_k=3)
    assert rep["n_measured"] == 3 and rep["best_seconds_per_step"] > 0
    p1, _, c = _plan(spec, np.float32)
    got = p1.query()
    assert (got["bt"], got["stream_chunk"]) == (min(tun["bt"], spec["steps"]), tun["stream_chunk"])
    tuned = _alone(p1, g)
    np.testing.assert_array_equal(tuned, base)
    # and both agree with the float64 oracle on the same rounded inputs
    ref = oracle.sweep(g.astype(np.float64), radius=1, box=False, coeffs=c.astype(np.float64),
                       steps=spec["steps"])
    bound = spec["steps"] * (pins.gamma(5, pins.U32) + pins.U32) * float(g.max()) * 1.01
    assert float(np.max(np.abs(tuned.astype(np.float64) - ref))) <= bound
    s5d.tune_cache_clear()


@pytest.mark.parametrize("kind", ["f64", "f32c"])
def test_autotuned_plans_match_oracle(kind):
    """Autotuned plans (model-ranked, GPU-timed, cached) for a 2D box and a 3D
    star: float64 within 1e-12 of the oracle, compensated float32 bit-exact
    against the compensated oracle."""
    dtype = np.float64 if kind == "f64" else np.float32
    accum = "compensated" if kind == "f32c" else "plain"
    for spec in (dict(ndim=2, radius=2, box=True, interior=(333, 517), steps=23,
                      seed=si.item_seed(9, 2)),
                 dict(ndim=3, radius=1, box=False, interior=(41, 66, 130), steps=11,
                      seed=si.item_seed(9, 3))):
        s5d.tune_cache_clear()
        case = si.make_case(spec["seed"], spec["ndim"], spec["radius"], spec["box"],
                            spec["interior"], spec["steps"])
        c_in, g_in = case.as_dtype(dtype)
        say("autotune", kind, spec)
        tun, rep = s5d.autotune(ndim=spec["ndim"], radius=spec["radius"], box=spec["box"],
                                dtype=dtype, interior=spec["interior"], steps=spec["steps"],
                                coeffs=case.coeffs, accum=accum, top_k=3)
        p, _, _ = _plan(spec, dtype, accum)
        got = p.query()
        if rep["n_measured"]:
            assert got["bt"] == min(tun["bt"], spec["steps"])
        out = _alone(p, g_in)
        kw = dict(radius=spec["radius"], box=spec["box"], steps=spec["steps"])
        if kind == "f64":
            ref = oracle.sweep(g_in, coeffs=c_in, **kw)
            assert max(rel_errors(out, ref)) <= 1e-12
        else:
            ref = oracle.sweep(g_in, coeffs=c_in, accum="compensated", **kw)
            np.testing.assert_array_equal(out, ref)
        p.close()
    s5d.tune_cache_clear()


def test_batch_outlives_its_plans():
    """Plans may be destroyed once the batch is built: the batch keeps the
    device state its launches read (the coefficient table of a direct b_T = 1
    plan among them).  Results are the same bits as single runs with fresh
    plans, and within 1e-12 of the oracle."""
    specs = [dict(ndim=2, radius=1, box=False, interior=(300, 517), steps=9, seed=si.item_seed(6, 0)),
             dict(ndim=2, radius=2, box=True, interior=(140, 260), steps=7, seed=si.item_seed(6, 1)),
             dict(ndim=3, radius=1, box=True, interior=(30, 41, 70), steps=5, seed=si.item_seed(6, 2)),
             dict(ndim=2, radius=3, box=True, interior=(90, 120), steps=4, seed=si.item_seed(6, 3))]
    tunings = [dict(bt=1), {}, dict(kernel="direct"), {}]
    made = [_plan(s, np.float64, **t) for s, t in zip(specs, tunings)]
    assert made[0][0].query()["kernel"] == 2  # b_T = 1: the direct row-streaming kernel
    t = torch()
    b0 = [t.from_numpy(m[1]).to("cuda:0") for m in made]
    b1 = [t.empty_like(x) for x in b0]
    batch = s5d.Batch([m[0] for m in made], b0, b1, graph=True)
    for m in made:
        m[0].close()
    batch._plans = []
    say("batch after its plans were destroyed")
    idx = batch.run()
    t.cuda.synchronize()
    outs = [(b0[i] if idx[i] == 0 else b1[i]).cpu().numpy() for i in range(len(made))]
    batch.close()
    for i, (s, tu) in enumerate(zip(specs, tunings)):
        p, g, c = _plan(s, np.float64, **tu)
        np.testing.assert_array_equal(outs[i], _alone(p, g), err_msg="grid %d" % i)
        ref = oracle.sweep(g, radius=s["radius"], box=s["box"], coeffs=c, steps=s["steps"])
        assert max(rel_errors(outs[i], ref)) <= 1e-12
