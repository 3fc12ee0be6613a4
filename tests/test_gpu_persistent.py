"""GPU tests of the persistent batched launch (S5D_BATCH_PERSISTENT).

Bars: every grid bit-identical to the same plan run alone with s5d_run
(eager and graph-replayed, three replays with eager work between them);
float64 grids within 1e-12 of the oracle; the 64-grid workload (2D stars,
sides U{256..4096}, r in {1,2}, float32, T = 200) bit-identical to single runs
for all 64 grids and within the float32 bound of the float64 oracle for its
eight smallest.  A wait limit of zero polls, forced from the host, makes the
run stop with S5D_ETIMEDOUT (every kernel still exits normally), and the same
batch then runs correctly with the default limit.
"""
import numpy as np
import pytest

import oracle
import paper_2001_01473_amd as s5d
import pins
import stencil_inputs as si
from gpu_util import rel_errors, say, torch

pytestmark = pytest.mark.gpu


NP = {"f32": np.float32, "f64": np.float64}


def _plan(spec, dtype, **tuning):
    case = si.make_case(spec["seed"], 2, spec["radius"], spec["box"], spec["interior"], spec["steps"])
    c_in, g_in = case.as_dtype(NP[dtype])
    plan = s5d.Plan(ndim=2, radius=spec["radius"], box=spec["box"], dtype=dtype, interior=spec["interior"],
                    steps=spec["steps"], coeffs=case.coeffs, **tuning)
    return plan, g_in, c_in


def _alone(plan, g_in):
    t = torch()
    x = t.from_numpy(g_in).to("cuda:0")
    y = t.empty_like(x)
    idx = plan.run(x, y)
    t.cuda.synchronize()
    return (x if idx == 0 else y).cpu().numpy()


def _run(plans, grids, graph, repeats=1, wait_limit=None):
    t = torch()
    b0 = [t.from_numpy(g).to("cuda:0") for g in grids]
    b1 = [t.empty_like(x) for x in b0]
    batch = s5d.Batch(plans, b0, b1, graph=graph, persistent=True)
    if wait_limit is not None:
        batch.set_wait_limit(wait_limit)
    outs = []
    for rep in range(repeats):
        if rep:
            for x, g in zip(b0, grids):  # eager work between replays
                x.copy_(t.from_numpy(g))
            t.cuda.synchronize()
        idx = batch.run()
        batch.status()
        outs.append([(b0[i] if idx[i] == 0 else b1[i]).cpu().numpy() for i in range(len(plans))])
    info = batch.query()
    batch.close()
    return outs, info


def _specs(dtype):
    """Stars of radius 1 and 2 (and, in float32, the 9-point box) with step
    counts that leave tail rounds, several stream blocks, ragged tiles."""
    shapes = [(1, False, (300, 517)), (2, False, (77, 1030)), (1, False, (5, 3)), (2, False, (260, 300)),
              (1, False, (1000, 240))]
    if dtype == "f32":
        shapes += [(1, True, (129, 650)), (1, True, (400, 90))]
    specs = []
    for j, (r, box, interior) in enumerate(shapes):
        for T in (0, 1, 6, 13, 37):
            specs.append(dict(radius=r, box=box, interior=interior, steps=T, seed=si.item_seed(91, 10 * j + T)))
    return specs


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_persistent_batch_equals_alone(dtype, graph):
    specs = _specs(dtype)
    made = [_plan(s, dtype) for s in specs]
    # explicit depths and short stream blocks too (tails of other lengths)
    made += [_plan(dict(radius=1, box=False, interior=(333, 700), steps=23, seed=si.item_seed(92, bt)), dtype,
                   bt=bt, stream_chunk=40) for bt in (2, 3, 5, 7)]
    plans, grids = [m[0] for m in made], [m[1] for m in made]
    say("persistent batch", dtype, "graph" if graph else "eager", len(plans), "grids")
    outs, info = _run(plans, grids, graph, repeats=3 if graph else 1)
    say("persistent launches", info)
    for i, (p, g) in enumerate(zip(plans, grids)):
        alone = _alone(p, g)
        for rep, out in enumerate(outs):
            np.testing.assert_array_equal(out[i], alone, err_msg="grid %d replay %d" % (i, rep))
    if dtype == "f64":
        for i, (p, g, c) in enumerate(made):
            ref = oracle.sweep(g, radius=p.radius, box=p.box, coeffs=c, steps=p.steps)
            assert max(rel_errors(outs[0][i], ref)) <= 1e-12, i


def test_persistent_many_grid_workload():
    specs = si.batch_mix(si.workload_seed(3))
    made = []
    for s in specs:
        case = si.make_case(s["seed"], s["ndim"], s["radius"], s["box"], s["interior"], s["steps"])
        c_in, g_in = case.as_dtype(np.float32)
        made.append((s5d.Plan(ndim=2, radius=s["radius"], box=s["box"], dtype="f32", interior=s["interior"],
                              steps=s["steps"], coeffs=case.coeffs), g_in, c_in))
    plans, grids = [m[0] for m in made], [m[1] for m in made]
    say("persistent batch 64 grids, graph")
    outs, info = _run(plans, grids, graph=True, repeats=2)
    say("persistent launches", info)
    # clear + boundary copy + one launch per family (radius 1 and radius 2)
    assert info["launches"] == 4 and info["persistent_launches"] == 2
    assert 0 < info["persistent_workgroups"] <= info["persistent_items"]
    for i in range(len(plans)):
        alone = _alone(plans[i], grids[i])
        np.testing.assert_array_equal(outs[0][i], alone, err_msg="grid %d" % i)
        np.testing.assert_array_equal(outs[1][i], alone, err_msg="grid %d replay" % i)
    order = sorted(range(len(specs)), key=lambda i: np.prod(specs[i]["interior"]))[:8]
    for i in order:
        s, (p, g, c) = specs[i], made[i]
        ref = oracle.sweep(g.astype(np.float64), radius=s["radius"], box=False, coeffs=c.astype(np.float64),
                           steps=s["steps"])
        bound = s["steps"] * (pins.gamma(len(c), pins.U32) + pins.U32) * float(g.max()) * 1.01
        assert float(np.max(np.abs(outs[0][i].astype(np.float64) - ref))) <= bound, i


def test_persistent_wait_limit_reports_and_recovers():
    specs = [dict(radius=1 + j % 2, box=False, interior=(2048, 1500 + 37 * j), steps=30 + j,
                  seed=si.item_seed(93, j)) for j in range(12)]
    made = [_plan(s, "f32") for s in specs]
    plans, grids = [m[0] for m in made], [m[1] for m in made]
    t = torch()
    b0 = [t.from_numpy(g).to("cuda:0") for g in grids]
    b1 = [t.empty_like(x) for x in b0]
    batch = s5d.Batch(plans, b0, b1, persistent=True)
    batch.set_wait_limit(0)
    say("persistent batch, wait limit 0")
    batch.run()
    with pytest.raises(s5d.Stencil5DError) as err:
        batch.status()
    assert err.value.status == 7  # S5D_ETIMEDOUT
    batch.set_wait_limit(1 << 24)
    for x, g in zip(b0, grids):
        x.copy_(t.from_numpy(g))
    say("persistent batch, default wait limit")
    idx = batch.run()
    batch.status()
    for i, (p, g) in enumerate(zip(plans, grids)):
        np.testing.assert_array_equal((b0[i] if idx[i] == 0 else b1[i]).cpu().numpy(), _alone(p, g),
                                      err_msg="grid %d" % i)
    batch.close()
    with pytest.raises(s5d.Stencil5DError):
        batch_bad = s5d.Batch(plans[:1], b0[:1], b1[:1], persistent=True)
        batch_bad.set_wait_limit(-1)


@pytest.mark.parametrize("kw", [
    dict(ndim=3, interior=(20, 30, 40), radius=1, box=False, dtype="f32"),
    dict(ndim=2, interior=(64, 300), radius=1, box=False, dtype="f32", accum="compensated"),
    dict(ndim=2, interior=(64, 300), radius=2, box=False, dtype="f32", bt=9),
    dict(ndim=2, interior=(64, 300), radius=1, box=True, dtype="f64"),
    dict(ndim=2, interior=(64, 300), radius=1, box=False, dtype="f32", bt=1),
])
def test_persistent_rejects_plans_outside_the_families(kw):
    nd = kw["ndim"]
    n = si.n_points(nd, kw["radius"], kw["box"])
    plan = s5d.Plan(steps=12, coeffs=np.full(n, 1.0 / n), **kw)
    t = torch()
    shape = tuple(i + 2 * kw["radius"] for i in kw["interior"])
    td = t.float32 if kw["dtype"] == "f32" else t.float64
    x = t.zeros(shape, dtype=td, device="cuda:0")
    y = t.empty_like(x)
    with pytest.raises(s5d.Stencil5DError) as err:
        s5d.Batch([plan], [x], [y], persistent=True)
    assert err.value.status == 2  # S5D_EUNSUPPORTED
