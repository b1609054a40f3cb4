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


def test_windowed_real_pulses_match_oracle(ctx, fth):
    """Real pulses (u3 of Section 5, eq. planewave, two of them: eq. multi)
    through the windowed recursion, slow transforms on the frequency set of
    Section 5 and the high-frequency transform of real signals on the way
    back (Section 4.1), against the oracle.  The grid resolves the data: the
    continuation's modes reach time content pi K / (W - w_c) = 25 (K = L/4),
    beyond the window half-width, the travel times and the slowly decaying
    response of the open arcs (the least-squares fit of the windows'
    spectra leaves residuals ~1e-12).  On a grid too coarse for the data the
    least-squares continuation is ill-conditioned and two correct
    implementations differ at that condition times the rounding (1e-8 at
    (1, 6, 4, 6, 7, 80), fit residual 3e-5).  Arcs of 16 nodes: the library
    takes the geometry of near targets from the node interpolant, exact to
    rounding from about 16 Chebyshev nodes on these half circles."""
    from oracle import hftransform as hf
    grid = (1.0, 4.0, 4, 6.0, 7, 96)
    fs = hf.FreqSet(*grid)
    pb = disc_interior_case(n=16, omegas=fs.omega, M=2)
    arcs = [ctx.arc_from_curve(a.curve, a.n) for a in pb.arcs]
    iv = np.array([a.curve.interval for a in pb.arcs])
    prob = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M)
    say("windowed real pulses,", fs.omega.size, "frequencies")
    u = prob.traces_windowed_real(fth.hf_grid(*grid), 0.1, 101, 2, 6.0, theta=0.3, npulse=2,
                                  period=6.0)
    ref = ow.run_windowed_real(oms.Layout(pb), fs, 0.1, 101, 2, 6.0,
                               dict(theta=0.3, npulse=2, period=6.0))
    assert rel(u, ref) < TOL, rel(u, ref)


def test_geometry1_long_time_against_exact(ctx, fth):
    """Geometry 1 of Section 5 at the paper's long-time setting: the unit disc
    as three overlapping arcs, the five-pulse field u4 (eq. multi) at
    theta = 0, M = 40, J = 872 frequencies up to W = 20, dt = 0.1, Q = 5
    windows of H = 10, times up to 60.  Inside the disc the field is exactly
    -u4; the paper reports errors uniformly below 1e-6 at (0.5, 0).
    Composite-panel arcs of 3 x 96 nodes (2.3e-7 measured; 9e-6 at 3 x 48)."""
    from oracle import hftransform as hf
    grid = (1.0, 20.0, 10, 12.0, 15, 745)
    om = fth.hf_frequencies(fth.hf_grid(*grid))
    assert om.size == 872
    pb = disc_interior_case(n=96, omegas=om, M=40)
    obs = np.array([[0.5, 0.0]])
    iv = np.array([a.curve.interval for a in pb.arcs])
    brs = fth.tov_breaks(iv, None, pb.period)
    arcs = [ctx.panel_arc_from_curve(a.curve, 96, b) for a, b in zip(pb.arcs, brs)]
    prob = fth.Problem(ctx, arcs, pb.incident, obs, intervals=iv, M=40)
    say("geometry 1 long time, J", om.size)
    u = prob.traces_windowed_real(fth.hf_grid(*grid), 0.1, 601, 5, 10.0, theta=0.0, npulse=5,
                                  period=10.0)
    t = 0.1 * np.arange(601)
    err = np.max(np.abs(u[:, 0] + hf.u4(obs, t, 0.0)[:, 0]))
    say("geometry 1 max error %.2e" % err)
    assert err < 1e-6, err
