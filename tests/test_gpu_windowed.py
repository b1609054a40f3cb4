"""GPU parity of the windowed, time-recentered recursion (Section 2.1,
eqs. windowing, Fourierk, TDsol; Algorithm 1 with Q windows) against the
oracle: traces of the three-arc disc with a Gaussian plane-wave pulse, and
a pulse train cut into more windows; the GPU's windowed traces also agree
with its own single-window frequency-domain traces when both are
resolved."""
import sys

import numpy as np
import pytest

from oracle import ms as oms
from oracle import transform as otr
from oracle import windowed as ow
from workloads import IncidentSpec, disc_interior_case

pytestmark = pytest.mark.gpu
TOL = 1e-10


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def fth():
    import paper_2507_05725_amd as m  # raises if the HIP library is missing
    return m


@pytest.fixture(scope="module")
def ctx(fth):
    return fth.Context(0)


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def _setup(ctx, fth, n, nf, M, om0=9.0, sig=1.0, tau0=7.0, theta=0.3):
    om = np.linspace(om0 - 6 * sig, om0 + 6 * sig, nf)
    pb = disc_interior_case(n=n, omegas=om, M=M)
    pb.incident = IncidentSpec("gplane", theta=theta, omega0=om0, sigma=sig, tau0=tau0)
    arcs = [ctx.arc_from_curve(a.curve, a.n) for a in pb.arcs]
    iv = np.array([a.curve.interval for a in pb.arcs])
    prob = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M)
    return pb, prob, om, otr.trapezoid_weights(om), arcs


@pytest.mark.parametrize("npulse,Q,H,nt", [(1, 3, 6.5, 131), (3, 5, 6.0, 201)],
                         ids=["pulse", "train"])
def test_windowed_traces_match_oracle(ctx, fth, npulse, Q, H, nt):
    pb, prob, om, w, arcs = _setup(ctx, fth, 16, 41, 2)
    inc = dict(theta=0.3, omega0=9.0, sigma=1.0, tau0=7.0, npulse=npulse, period=4.0)
    say("windowed", npulse, "pulses, Q", Q)
    u = prob.traces_windowed(om, w, 0.1, nt, Q, H, **inc)
    ref = ow.run_windowed(oms.Layout(pb), om, w, 0.1, nt, Q, H, inc)
    assert rel(u, ref) < TOL, rel(u, ref)


def test_windowed_agrees_with_single_window_traces(ctx, fth):
    pb, prob, om, w, arcs = _setup(ctx, fth, 16, 61, 2)
    t = 0.1 * np.arange(151)
    uf, steps = prob.traces(om, w, t)
    uw = prob.traces_windowed(om, w, 0.1, 151, 2, 10.0, theta=0.3, omega0=9.0, sigma=1.0,
                              tau0=7.0)
    assert rel(uw, uf) < 1e-3


def test_windowed_refined_matches_oracle(ctx, fth):
    """The windowed recursion in the refined form (FP32 factors reused by
    every window and step) against the oracle."""
    pb, _, om, w, arcs = _setup(ctx, fth, 16, 41, 2)
    iv = np.array([a.curve.interval for a in pb.arcs])
    prob = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M,
                       precision=fth.FP32_REFINED, tol=1e-12)
    inc = dict(theta=0.3, omega0=9.0, sigma=1.0, tau0=7.0, npulse=3, period=4.0)
    say("windowed refined, Q 5")
    u = prob.traces_windowed(om, w, 0.1, 201, 5, 6.0, **inc)
    ref = ow.run_windowed(oms.Layout(pb), om, w, 0.1, 201, 5, 6.0, inc)
    assert rel(u, ref) < TOL, rel(u, ref)
