"""GPU: the serving loop (fthms_server_*, fthms_submit/poll/fetch/cancel).

Requests are exterior scattering jobs of different sizes (1-3 obstacles of 4
arcs each).  Checks: a served request equals the same problem run directly
through fthms_problem_traces (bit for bit); every request's result is the
same alone and in a mix of concurrent requests; a queued request can be
cancelled; a request larger than the server budget is refused at
submission."""
import sys
import time

import numpy as np
import pytest

from workloads import serving_requests

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch  # the HIP runtime comes up through torch first
    torch.cuda.init()
    import paper_2507_05725_amd as fth
    reqs = serving_requests(seed=5, count=6, n_range=(24, 40), nk_range=(24, 48),
                            max_steps=12)
    return fth, reqs


def test_served_equals_direct_problem(env):
    fth, reqs = env
    r = reqs[0]
    srv = fth.Server(0, workers=2)
    t = srv.submit(fth.request_from_workload(r))
    got, steps, lat = srv.wait(t)
    srv.close()
    say("served: steps", steps, "latency %.3f s" % lat)
    ctx = fth.Context(0)
    arcs = [ctx.arc_from_curve(a.curve, a.n) for a in r["arcs"]]
    iv = np.array([a.curve.interval for a in r["arcs"]])
    prob = fth.Problem(ctx, arcs, r["incident"], r["obs"], intervals=iv, M=r["max_steps"],
                       groups=[a.group for a in r["arcs"]])
    q = fth.request_from_workload(r)
    ref, ref_steps = prob.traces(q["k"], q["w"], q["t"], stop_tol=q["stop_tol"])
    assert ref_steps == steps
    assert np.array_equal(ref, got)
    prob.close()
    for a in arcs:
        a.close()
    ctx.close()


def test_alone_equals_mixed(env):
    fth, reqs = env
    srv = fth.Server(0, workers=4)
    alone = {}
    for i in (1, 2):
        alone[i] = srv.wait(srv.submit(fth.request_from_workload(reqs[i])))
    tickets = [srv.submit(fth.request_from_workload(r)) for r in reqs]
    mixed = [srv.wait(t) for t in tickets]
    srv.close()
    for i in (1, 2):
        assert alone[i][1] == mixed[i][1]
        assert np.array_equal(alone[i][0], mixed[i][0]), i
    say("mixed latencies", ["%.3f" % m[2] for m in mixed])


def test_cancel_and_refusal(env):
    fth, reqs = env
    srv = fth.Server(0, workers=1)
    t0 = srv.submit(fth.request_from_workload(reqs[3]))
    t1 = srv.submit(fth.request_from_workload(reqs[4]))
    srv.cancel(t1)
    assert srv.poll(t1) == fth.JOB_CANCELLED
    with pytest.raises(fth.FthmsError) as e:
        srv.fetch(t1)
    assert e.value.code == -8
    srv.wait(t0)
    srv.close()
    small = fth.Server(0, hbm_budget=1 << 20, workers=1)
    with pytest.raises(fth.FthmsError) as e:
        small.submit(fth.request_from_workload(reqs[0]))
    assert e.value.code == -3
    small.close()


@pytest.fixture(scope="module")
def c5():
    from workloads import serving_c5_requests
    # the serving workload's distributions at small sizes
    return serving_c5_requests(seed=11, count=6, max_obstacles=4, n_range=(64, 96),
                               nk_range=(64, 96), omega0_range=(4.0, 8.0), max_steps=40)


def _direct_closed(fth, ctx, r, precision, M=None, stop_tol=None):
    n = r["arcs"][0].n
    arcs = [ctx.closed_from_curve(a.curve, n) for a in r["arcs"]]
    prob = fth.Problem(ctx, arcs, r["incident"], r["obs"], M=M or r["max_steps"],
                       groups=list(range(len(arcs))), intervals=np.zeros((len(arcs), 2)) +
                       np.array([0.0, 2 * np.pi]), precision=precision,
                       tol=1e-12 if precision else 0.0)
    q = fth.request_from_workload(r)
    out = prob.traces(q["k"], q["w"], q["t"],
                      stop_tol=q["stop_tol"] if stop_tol is None else stop_tol)
    prob.close()
    for a in arcs:
        a.close()
    return out


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "refined"])
def test_served_closed_obstacles_equal_direct_problem(env, c5, precision):
    """Requests of closed obstacles (each one combined-field patch) in both
    precisions: the served traces and step counts equal those of the same
    problem run directly, bit for bit; and a run stopped by the
    device-decided rule (the host reading the decision one step late) equals
    the run of exactly that many steps without the rule."""
    fth, _ = env
    srv = fth.Server(0, workers=3)
    reqs = [dict(r, precision=precision) for r in c5]
    tickets = [srv.submit(fth.request_from_workload(r)) for r in reqs]
    got = [srv.wait(t) for t in tickets]
    srv.close()
    ctx = fth.Context(0)
    for r, (tr, steps, lat) in zip(reqs, got):
        say("closed request", r["name"], "obstacles", r["obstacles"], "n", r["n"], "steps",
            steps, "latency %.3f s" % lat)
        ref, ref_steps = _direct_closed(fth, ctx, r, precision)
        assert steps == ref_steps
        assert np.array_equal(ref, tr)
        if 1 < steps < r["max_steps"]:
            fixed, fixed_steps = _direct_closed(fth, ctx, r, precision, M=steps, stop_tol=0.0)
            assert fixed_steps == steps
            assert np.array_equal(fixed, tr)
    ctx.close()


def test_closed_request_refined_matches_fp64(env, c5):
    """The refined form of a served closed-obstacle request agrees with the
    FP64 one to the parity bar."""
    fth, _ = env
    srv = fth.Server(0, workers=2)
    r = c5[1]
    a = srv.wait(srv.submit(fth.request_from_workload(dict(r, precision=0))))
    b = srv.wait(srv.submit(fth.request_from_workload(dict(r, precision=1))))
    srv.close()
    assert a[1] == b[1]
    assert np.linalg.norm(b[0] - a[0]) / np.linalg.norm(a[0]) < 1e-10
