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
