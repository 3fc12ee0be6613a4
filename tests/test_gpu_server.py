"""GPU tests of the serving loop (s5d_server_*).

Bars: every served result is bit-identical to the same request run alone
with s5d_run; the HBM budget is never exceeded (peak of held grid memory);
timestamps are ordered (arrival <= admission <= completion); all memory is
returned once results are fetched.
"""
import numpy as np
import pytest

import paper_2001_01473_amd as s5d
import stencil_inputs as si
from gpu_util import say, torch

pytestmark = pytest.mark.gpu


def _request(spec):
    dt = np.float32 if spec["dtype"] == "f32" else np.float64
    case = si.make_case(spec["seed"], spec["ndim"], spec["radius"], spec["box"],
                        spec["interior"], spec["steps"])
    _, g = case.as_dtype(dt)
    plan = s5d.Plan(ndim=spec["ndim"], radius=spec["radius"], box=spec["box"], dtype=dt,
                    interior=spec["interior"], steps=spec["steps"], coeffs=case.coeffs)
    return plan, g


def _alone(plan, g):
    t = torch()
    x = t.from_numpy(g).to("cuda:0")
    y = t.empty_like(x)
    idx = plan.run(x, y)
    t.cuda.synchronize()
    return (x if idx == 0 else y).cpu().numpy()


def _small_mix(n, seed):
    """Requests shaped like the serving mix, scaled down to test size."""
    return si.serve_mix(seed, n, rate_per_s=1.0, side2d=(40, 700), side3d=(12, 70), steps=(0, 40))


def _serve(server, made, stagger=0, fetch_each=False):
    """Submit (all at once, or `stagger` requests per tick), tick until every
    request is done; with fetch_each, fetch results as they finish (which
    returns their memory to the budget).  Returns (ids, fetched results)."""
    t = torch()
    ids, outs = [], {}

    def fetch_done():
        for rid, (plan, g) in zip(ids, made):
            if rid not in outs and server.request(rid)["state"] == 2:
                outs[rid] = server.fetch(rid, np.empty_like(g))

    pending = list(range(len(made)))
    while True:
        take = pending if stagger <= 0 else pending[:stagger]
        for i in take:
            plan, g = made[i]
            init = t.from_numpy(g).to("cuda:0") if i % 2 else g  # device and host sources
            ids.append(server.submit(plan, init, keep_result=True))
        pending = pending[len(take):]
        running, queued = server.tick()
        if fetch_each:
            fetch_done()
        if not pending and running == 0 and queued == 0:
            break
    server.sync()
    if fetch_each:
        fetch_done()
    return ids, outs


@pytest.mark.parametrize("stagger", [0, 3])
def test_served_results_equal_alone(stagger):
    specs = _small_mix(24, 91)
    made = [_request(s) for s in specs]
    server = s5d.Server(hbm_budget_bytes=1 << 30)
    say("serve", len(specs), "requests, stagger", stagger)
    ids, _ = _serve(server, made, stagger)
    st = server.stats()
    assert st["done"] == len(specs) and st["queued"] == 0 and st["running"] == 0
    for rid, (plan, g) in zip(ids, made):
        info = server.request(rid)
        assert info["state"] == 2
        assert info["t_arrival"] <= info["t_admit"] + 1e-6 and info["t_admit"] <= info["t_done"] + 1e-3
        out = np.empty_like(g)
        server.fetch(rid, out)
        np.testing.assert_array_equal(out, _alone(plan, g), err_msg="request %d" % rid)
        assert server.request(rid)["state"] == 3
    st = server.stats()
    assert st["bytes_in_use"] == 0
    assert 0 < st["latency_p50"] <= st["latency_p99"]
    assert st["makespan"] > 0 and st["updates_done"] == sum(
        s["steps"] * int(np.prod(s["interior"])) for s in specs)
    server.close()


def test_tight_budget_and_admission_order():
    specs = _small_mix(12, 92)
    made = [_request(s) for s in specs]
    biggest = max(2 * g.nbytes for _, g in made)
    budget = int(biggest * 1.5)
    server = s5d.Server(hbm_budget_bytes=budget)
    say("serve tight budget", budget)
    ids, outs = _serve(server, made, fetch_each=True)
    st = server.stats()
    assert st["bytes_peak"] <= budget and st["done"] == len(specs) and st["bytes_in_use"] == 0
    admits = [server.request(r)["t_admit"] for r in ids]
    assert admits == sorted(admits)  # FIFO admission
    for rid, (plan, g) in zip(ids, made):
        np.testing.assert_array_equal(outs[rid], _alone(plan, g))
    server.close()


def test_kept_results_hold_the_budget_until_fetched():
    """Kept results keep their memory: with a budget for one request, the
    second one waits (nothing running, one queued) until the first result is
    fetched, then runs."""
    specs = _small_mix(2, 95)
    made = [_request(s) for s in specs]
    budget = max(2 * g.nbytes for _, g in made)
    server = s5d.Server(hbm_budget_bytes=budget)
    ids = [server.submit(plan, g, keep_result=True) for plan, g in made]
    for _ in range(10000):
        running, queued = server.tick()
        if running == 0:
            break
    server.sync()
    assert server.tick() == (0, 1)  # blocked: the kept result holds the budget
    assert server.request(ids[1])["state"] == 0
    first = server.fetch(ids[0], np.empty_like(made[0][1]))
    while server.tick() != (0, 0):
        pass
    server.sync()
    second = server.fetch(ids[1], np.empty_like(made[1][1]))
    np.testing.assert_array_equal(first, _alone(*made[0]))
    np.testing.assert_array_equal(second, _alone(*made[1]))
    server.close()


def test_max_running_one_and_budget_error():
    specs = _small_mix(5, 93)
    made = [_request(s) for s in specs]
    server = s5d.Server(hbm_budget_bytes=1 << 30, max_running=1)
    ids, _ = _serve(server, made)
    for rid, (plan, g) in zip(ids, made):
        out = np.empty_like(g)
        np.testing.assert_array_equal(server.fetch(rid, out), _alone(plan, g))
    server.close()
    small = s5d.Server(hbm_budget_bytes=1024)
    with pytest.raises(s5d.Stencil5DError) as err:
        small.submit(made[0][0], made[0][1])
    assert err.value.status == 5  # S5D_EBUDGET
    small.close()


def test_dropped_results_release_memory():
    specs = _small_mix(8, 94)
    made = [_request(s) for s in specs]
    server = s5d.Server(hbm_budget_bytes=1 << 30)
    for plan, g in made:
        server.submit(plan, g)
    while server.tick() != (0, 0):
        pass
    server.sync()
    st = server.stats()
    assert st["done"] == len(specs) and st["bytes_in_use"] == 0
    server.close()
