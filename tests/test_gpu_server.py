"""GPU tests of the serving loop (s5d_server_*).

Bars: every served result is bit-identical to the same request run alone
with s5d_run, and agrees with the CPU oracle (float64: normwise and
elementwise relative error <= 1e-12; float32: within T*(gamma_n + u)*max|A0|
of the float64 oracle run on the same float32-rounded grid and
coefficients); the HBM budget is never exceeded (peak of held grid memory);
timestamps are ordered (arrival <= admission <= completion); all memory is
returned once results are fetched.  Failures (forced from the host through
the server's fault-injection knobs) and cancellations stay with the request
they hit: every other request finishes with the same bits as alone.
"""
import numpy as np
import pytest

import oracle
import paper_2001_01473_amd as s5d
import pins
import stencil_inputs as si
from gpu_util import rel_errors, say, torch

pytestmark = pytest.mark.gpu

DONE, RELEASED, FAILED = 2, 3, 4


def _request(spec):
    dt = np.float32 if spec["dtype"] == "f32" else np.float64
    case = si.make_case(spec["seed"], spec["ndim"], spec["radius"], spec["box"],
                        spec["interior"], spec["steps"])
    c, g = case.as_dtype(dt)
    plan = s5d.Plan(ndim=spec["ndim"], radius=spec["radius"], box=spec["box"], dtype=dt,
                    interior=spec["interior"], steps=spec["steps"], coeffs=case.coeffs)
    plan.spec, plan.c_in = spec, c
    return plan, g


def _alone(plan, g):
    t = torch()
    x = t.from_numpy(g).to("cuda:0")
    y = t.empty_like(x)
    idx = plan.run(x, y)
    t.cuda.synchronize()
    return (x if idx == 0 else y).cpu().numpy()


def _check_oracle(plan, g, out):
    """The served result against the CPU oracle (float64 oracle on the
    request's own, possibly float32-rounded, inputs)."""
    s = plan.spec
    ref = oracle.sweep(g.astype(np.float64), radius=s["radius"], box=s["box"],
                       coeffs=plan.c_in.astype(np.float64), steps=s["steps"])
    if g.dtype == np.float64:
        norm, elem = rel_errors(out, ref)
        assert norm <= 1e-12 and elem <= 1e-12, (s, norm, elem)
    else:
        n = si.n_points(s["ndim"], s["radius"], s["box"])
        bound = s["steps"] * (pins.gamma(n, pins.U32) + pins.U32) * float(np.abs(g).max()) * 1.01
        err = float(np.max(np.abs(out.astype(np.float64) - ref)))
        assert err <= bound, (s, err, bound)


def _small_mix(n, seed):
    """Requests shaped like the serving mix, scaled down to test size."""
    return si.serve_mix(seed, n, rate_per_s=1.0, side2d=(40, 700), side3d=(12, 70), steps=(0, 40))


def _serve(server, made, stagger=0, fetch_each=False, tolerate_tick_errors=False):
    """Submit (all at once, or `stagger` requests per tick), tick until every
    request is done or failed; with fetch_each, fetch results as they finish
    (which returns their memory to the budget).  Returns (ids, fetched
    results, number of ticks that raised)."""
    t = torch()
    ids, outs = [], {}
    raised = 0

    def fetch_done():
        for rid, (plan, g) in zip(ids, made):
            if rid not in outs and server.request(rid)["state"] == DONE:
                outs[rid] = server.fetch(rid, np.empty_like(g))

    pending = list(range(len(made)))
    while True:
        take = pending if stagger <= 0 else pending[:stagger]
        for i in take:
            plan, g = made[i]
            init = t.from_numpy(g).to("cuda:0") if i % 2 else g  # device and host sources
            ids.append(server.submit(plan, init, keep_result=True))
        pending = pending[len(take):]
        try:
            running, queued = server.tick()
        except s5d.Stencil5DError:
            if not tolerate_tick_errors:
                raise
            raised += 1
            st = server.stats()
            running, queued = st["running"], st["queued"]
        if fetch_each:
            fetch_done()
        if not pending and running == 0 and queued == 0:
            break
    server.sync()
    if fetch_each:
        fetch_done()
    return ids, outs, raised


@pytest.mark.parametrize("stagger", [0, 3])
def test_served_results_equal_alone_and_oracle(stagger):
    specs = _small_mix(24, 91)
    made = [_request(s) for s in specs]
    server = s5d.Server(hbm_budget_bytes=1 << 30)
    say("serve", len(specs), "requests, stagger", stagger)
    ids, _, _ = _serve(server, made, stagger)
    st = server.stats()
    assert st["done"] == len(specs) and st["queued"] == 0 and st["running"] == 0
    assert st["failed"] == 0
    for rid, (plan, g) in zip(ids, made):
        info = server.request(rid)
        assert info["state"] == DONE and info["status"] == 0 and info["init_in_use"] == 0
        assert info["t_arrival"] <= info["t_admit"] + 1e-6 and info["t_admit"] <= info["t_done"] + 1e-3
        out = np.empty_like(g)
        server.fetch(rid, out)
        np.testing.assert_array_equal(out, _alone(plan, g), err_msg="request %d" % rid)
        _check_oracle(plan, g, out)
        assert server.request(rid)["state"] == RELEASED
    st = server.stats()
    assert st["bytes_in_use"] == 0
    assert 0 < st["latency_p50"] <= st["latency_p99"]
    assert st["makespan"] > 0 and st["updates_done"] == sum(
        s["steps"] * int(np.prod(s["interior"])) for s in specs)
    server.close()


@pytest.mark.parametrize("n_streams", [1, 2, 4])
def test_stream_count_gives_same_bits(n_streams):
    specs = _small_mix(10, 96)
    made = [_request(s) for s in specs]
    server = s5d.Server(hbm_budget_bytes=1 << 30, n_streams=n_streams)
    say("serve on", n_streams, "streams")
    ids, outs, _ = _serve(server, made, fetch_each=True)
    for rid, (plan, g) in zip(ids, made):
        np.testing.assert_array_equal(outs[rid], _alone(plan, g), err_msg="request %d" % rid)
    server.close()


def test_tight_budget_and_admission_order():
    specs = _small_mix(12, 92)
    made = [_request(s) for s in specs]
    biggest = max(2 * g.nbytes for _, g in made)
    budget = int(biggest * 1.5)
    server = s5d.Server(hbm_budget_bytes=budget)
    say("serve tight budget", budget)
    ids, outs, _ = _serve(server, made, fetch_each=True)
    st = server.stats()
    assert st["bytes_peak"] <= budget and st["done"] == len(specs) and st["bytes_in_use"] == 0
    admits = [server.request(r)["t_admit"] for r in ids]
    assert admits == sorted(admits)  # FIFO admission
    for rid, (plan, g) in zip(ids, made):
        np.testing.assert_array_equal(outs[rid], _alone(plan, g))
        _check_oracle(plan, g, outs[rid])
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
    _check_oracle(*made[0], first)
    _check_oracle(*made[1], second)
    server.close()


def test_max_running_one_and_budget_error():
    specs = _small_mix(5, 93)
    made = [_request(s) for s in specs]
    server = s5d.Server(hbm_budget_bytes=1 << 30, max_running=1)
    ids, _, _ = _serve(server, made)
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


def test_failed_admissions_are_isolated():
    """Every third admission fails (forced from the host): those requests are
    FAILED with their memory returned; every other request finishes with the
    bits it gets alone."""
    specs = _small_mix(14, 97)
    made = [_request(s) for s in specs]
    server = s5d.Server(hbm_budget_bytes=1 << 30, fail_admit_every=3)
    say("serve with failing admissions")
    ids, outs, _ = _serve(server, made, stagger=2, fetch_each=True)
    st = server.stats()
    failed = [r for r in ids if server.request(r)["state"] == FAILED]
    assert len(failed) == len(specs) // 3 and st["failed"] == len(failed)
    assert st["done"] == len(specs) - len(failed) and st["bytes_in_use"] == 0
    for rid, (plan, g) in zip(ids, made):
        info = server.request(rid)
        if rid in failed:
            assert info["status"] == 4 and info["init_in_use"] == 0  # S5D_EDEVICE
            with pytest.raises(s5d.Stencil5DError):
                server.fetch(rid, np.empty_like(g))
        else:
            np.testing.assert_array_equal(outs[rid], _alone(plan, g), err_msg="request %d" % rid)
            _check_oracle(plan, g, outs[rid])
    server.close()


def test_failed_launch_without_progress_is_retried():
    """One round per tick, every fourth tick's launch fails before anything of
    it is enqueued: the tick raises, no request loses a round, and the
    retried ticks finish every request with the bits it gets alone."""
    specs = _small_mix(9, 98)
    made = [_request(s) for s in specs]
    server = s5d.Server(hbm_budget_bytes=1 << 30, rounds_per_tick=1, fail_tick_every=4)
    say("serve with failing tick launches, one round per tick")
    ids, outs, raised = _serve(server, made, fetch_each=True, tolerate_tick_errors=True)
    assert raised > 0
    st = server.stats()
    assert st["failed"] == 0 and st["done"] == len(specs)
    for rid, (plan, g) in zip(ids, made):
        np.testing.assert_array_equal(outs[rid], _alone(plan, g), err_msg="request %d" % rid)
    server.close()


def test_failed_launch_mid_tick_fails_only_its_requests():
    """Two rounds per tick, the second round of every third tick fails to
    launch: requests with a round in it are FAILED; requests that finished in
    the first round of such a tick, and all others, have the bits they get
    alone and agree with the oracle."""
    specs = _small_mix(16, 99)
    made = [_request(s) for s in specs]
    server = s5d.Server(hbm_budget_bytes=1 << 30, rounds_per_tick=2, fail_tick_every=3)
    say("serve with failing second rounds")
    ids, outs, raised = _serve(server, made, stagger=3, fetch_each=True,
                               tolerate_tick_errors=True)
    st = server.stats()
    states = [server.request(r)["state"] for r in ids]
    assert raised > 0 and st["failed"] == states.count(FAILED) > 0
    assert st["done"] == len(specs) - st["failed"] and st["bytes_in_use"] == 0
    for rid, (plan, g), state in zip(ids, made, states):
        if state == FAILED:
            assert server.request(rid)["status"] == 4
            continue
        np.testing.assert_array_equal(outs[rid], _alone(plan, g), err_msg="request %d" % rid)
        _check_oracle(plan, g, outs[rid])
    server.close()


def test_cancel_queued_and_running():
    specs = _small_mix(6, 100)
    for s in specs:
        s["steps"] = max(s["steps"], 20)
    made = [_request(s) for s in specs]
    server = s5d.Server(hbm_budget_bytes=1 << 30, max_running=2, rounds_per_tick=1)
    ids = [server.submit(plan, g, keep_result=True) for plan, g in made]
    server.tick()  # admits the first two, runs one round of each
    assert server.request(ids[0])["state"] == 1 and server.request(ids[5])["state"] == 0
    server.cancel(ids[5])  # queued
    server.cancel(ids[0])  # running
    assert server.request(ids[5])["state"] == FAILED
    while server.tick() != (0, 0):
        pass
    server.sync()
    for i in (0, 5):
        info = server.request(ids[i])
        assert info["state"] == FAILED and info["status"] == 6  # S5D_ECANCELED
    st = server.stats()
    assert st["failed"] == 2 and st["done"] == 4
    for i in (1, 2, 3, 4):
        plan, g = made[i]
        out = server.fetch(ids[i], np.empty_like(g))
        np.testing.assert_array_equal(out, _alone(plan, g))
    assert server.stats()["bytes_in_use"] == 0
    server.close()
