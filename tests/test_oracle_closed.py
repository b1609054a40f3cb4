"""Pins of the closed-patch oracle (Section 3.3, eqs. FDsolk-closed,
FDBIEk-closed; the Nystrom method the paper cites for closed curves): the
logarithmic quadrature against its defining integrals, the combined-field
solution against the exact exterior field of an interior point source
(exponential convergence), and the multiple-scattering sum over closed
patches against the exact field of two obstacles."""
import math

import numpy as np
import pytest
from scipy.special import hankel1

from oracle import closed as cl
from oracle import incident as oinc
from oracle import ms
from workloads import ClosedEllipse, ClosedKite, IncidentSpec
from workloads.configs import ArcSpec, MSProblem


def test_log_quadrature_exact_on_trigonometric_polynomials():
    """int_0^{2pi} log(4 sin^2((t - tau)/2)) cos(m tau) dtau = -(2pi/m) cos(m t)
    (m >= 1), 0 (m = 0): the weights reproduce it for m < n at every node
    and at an off-node t, and for sin(m tau) likewise."""
    n2 = 24
    n = n2 // 2
    tau = 2.0 * math.pi * np.arange(n2) / n2
    t = np.concatenate([tau, [0.37, 2.9]])
    Rt = cl.kress_weights(t, n2)
    assert np.max(np.abs(Rt @ np.ones(n2))) < 1e-13
    for m in range(1, n):
        assert np.max(np.abs(Rt @ np.cos(m * tau) + (2 * math.pi / m) * np.cos(m * t))) < 1e-13
        assert np.max(np.abs(Rt @ np.sin(m * tau) + (2 * math.pi / m) * np.sin(m * t))) < 1e-13
    # one further check by quadrature of the log integral itself (m = n - 1,
    # t off the nodes), independent of the closed form
    from scipy.integrate import quad
    f = lambda s: math.log(4.0 * math.sin(0.5 * (0.37 - s)) ** 2) * math.cos((n - 1) * s)
    ref = quad(f, 0.0, 0.37, limit=200)[0] + quad(f, 0.37, 2 * math.pi, limit=200)[0]
    assert abs(Rt[n2] @ np.cos((n - 1) * tau) - ref) < 1e-10


@pytest.mark.parametrize("curve,z0", [(ClosedEllipse(1.0, 0.6, (0.2, -0.1), 0.3), (0.3, 0.0)),
                                      (ClosedKite(1.0), (-0.2, 0.3))], ids=["ellipse", "kite"])
@pytest.mark.parametrize("k", [2.0, 7.5, 5.0 + 2.0j])
def test_exterior_point_source_exact(curve, z0, k):
    """Data -Phi(., z0) with z0 inside: the radiating solution outside is
    -Phi(x, z0) exactly; the combined-field Nystrom solution reaches it
    exponentially (1e-13 at 128 nodes on the kite, 64 on the ellipse)."""
    zt = np.array([[3.0 * math.cos(a), 3.0 * math.sin(a)] for a in np.linspace(0, 6, 8)])

    def ui(p):
        return 0.25j * hankel1(0, k * np.hypot(p[:, 0] - z0[0], p[:, 1] - z0[1]))

    errs = []
    for n2 in (32, 64, 128):
        nd = cl.nodes(curve, n2)
        psi = np.linalg.solve(cl.assemble(nd, k), -ui(nd["y"]))
        U = cl.field(k, zt, nd, psi)
        errs.append(float(np.max(np.abs(U + ui(zt))) / np.max(np.abs(ui(zt)))))
    assert errs[2] < 1e-12
    assert errs[1] < 1e-4
    assert errs[2] < 1e-3 * errs[0]


def test_ms_two_closed_patches_exact():
    """Two obstacles, each one closed patch, point source inside the first:
    at a complex wavenumber the MS sum converges geometrically and its limit
    is -U^i outside both (exact to 1e-12 at 64 nodes per obstacle)."""
    k = 5.0 + 2.0j
    obs = np.stack([2.8 * np.cos(np.linspace(0, 6, 8)), 2.8 * np.sin(np.linspace(0, 6, 8))], -1)
    errs = []
    for n2 in (32, 64):
        arcs = [ArcSpec(ClosedEllipse(0.8, 0.5, (-1.0, 0.0)), n2, group=0),
                ArcSpec(ClosedKite(0.5, (1.2, 0.3)), n2, group=1)]
        pb = MSProblem(arcs=arcs, incident=IncidentSpec("point", z0=(-1.1, 0.1), sigma=0.0),
                       omegas=np.array([k]), M=12, obs=obs, times=np.zeros(0))
        lay = ms.Layout(pb)
        assert lay.closed == [True, True] and np.all(lay.chi[0] == 1.0)
        out = ms.run_frequency(lay, k)
        ui = oinc.incident(pb.incident, k, obs)
        errs.append(float(np.max(np.abs(out["U"] + ui)) / np.max(np.abs(ui))))
    assert errs[0] < 1e-6 and errs[1] < 1e-12


def test_closed_patch_must_be_alone_on_its_curve():
    arcs = [ArcSpec(ClosedEllipse(0.8, 0.5), 16, group=0), ArcSpec(ClosedKite(0.5, (2, 0)), 16, group=0)]
    pb = MSProblem(arcs=arcs, incident=IncidentSpec("plane"), omegas=np.array([3.0]), M=2,
                   obs=np.zeros((1, 2)), times=np.zeros(0))
    with pytest.raises(ValueError):
        ms.Layout(pb)


def test_trig_interp_reproduces_trigonometric_polynomials():
    """The interpolant of 2n samples of a trigonometric polynomial of degree
    below n is that polynomial at every parameter, and equals the samples at
    the nodes for any data (degree n included: cos(n tau) is its own
    Nyquist term)."""
    n2 = 20
    tau = 2.0 * math.pi * np.arange(n2) / n2
    t = np.array([0.1, 1.234, 3.0, 5.9, -2.2])
    f = lambda s: (0.3 + 1.2j * np.cos(3 * s) - 0.7 * np.sin(9 * s) + (0.25 - 0.5j) * np.exp(4j * s))
    assert np.max(np.abs(cl.trig_interp(f(tau), t) - f(t))) < 1e-13
    rng = np.random.default_rng(5)
    g = rng.standard_normal(n2) + 1j * rng.standard_normal(n2)
    assert np.max(np.abs(cl.trig_interp(g, tau) - g)) < 1e-13
    assert np.max(np.abs(cl.trig_interp(np.cos(10 * tau), t) - np.cos(10 * t))) < 1e-13


def test_closest_param_on_an_ellipse():
    """Axis-aligned ellipse at the origin: the closest point to a target on
    the major axis beyond the tip is the tip (tau = 0), to one on the minor
    axis the co-vertex (tau = pi / 2)."""
    E = ClosedEllipse(1.0, 0.6)
    h = 2.0 * math.pi / 32
    assert abs(cl.closest_param(E, np.array([1.3, 0.0]), 0.05, h)) < 1e-8
    assert abs(cl.closest_param(E, np.array([0.0, 0.9]), math.pi / 2 - 0.04, h) - math.pi / 2) < 1e-8


def _exterior_points(curve, tt, dist):
    """Points at distance `dist` along the outward normal (x2', -x1') of
    the curve (counter-clockwise) at parameters tt."""
    y, dy = curve.x(tt), curve.dx(tt)
    nrm = np.stack([dy[:, 1], -dy[:, 0]], -1) / np.hypot(dy[:, 0], dy[:, 1])[:, None]
    return y + dist * nrm


@pytest.mark.parametrize("curve,n2", [(ClosedKite(1.0), 256),
                                      (ClosedEllipse(1.0, 0.6, (0.2, -0.1), 0.3), 128)],
                         ids=["kite256", "ellipse128"])
@pytest.mark.parametrize("k", [2.0, 7.5])
def test_field_near_exact_exterior(curve, n2, k):
    """Point source inside, resolved density: the near-target integral
    reaches the exact exterior field -Phi(x, z0) from 6 node spacings down
    to a hundredth of one, where the trapezoid rule is wrong in the first
    digit."""
    z0 = (0.05, 0.1)

    def ui(p):
        return 0.25j * hankel1(0, k * np.hypot(p[:, 0] - z0[0], p[:, 1] - z0[1]))

    nd = cl.nodes(curve, n2)
    psi = np.linalg.solve(cl.assemble(nd, k), -ui(nd["y"]))
    h = cl.near_limit(nd) / 5.0
    tt = np.array([0.31, 1.7, 2.95, 4.4, 5.9])
    for f in (0.01, 0.1, 0.5, 2.0, 6.0):
        z = _exterior_points(curve, tt, f * h)
        U = cl.field_near(k, z, curve, nd, psi)
        assert np.max(np.abs(U + ui(z)) / np.abs(ui(z))) < 1e-12, f
    z = _exterior_points(curve, tt, 0.01 * h)
    assert np.max(np.abs(cl.field(k, z, nd, psi) + ui(z)) / np.abs(ui(z))) > 0.1


def test_field_near_equals_fine_trapezoid():
    """For a density of low degree (12), given at 96 nodes, the integral of
    the interpolant is the same integral that the trapezoid rule on 384
    nodes (the same trigonometric polynomial sampled there) takes, to
    rounding at eight and sixteen node spacings off the curve; the 96-node
    rule itself is 1e-10 away (the kite's speed |x'| is not a trigonometric
    polynomial)."""
    curve = ClosedKite(1.0)
    nd, nf = cl.nodes(curve, 96), cl.nodes(curve, 384)
    rng = np.random.default_rng(9)
    m = np.arange(-12, 13)
    cm = (rng.standard_normal(m.size) + 1j * rng.standard_normal(m.size)) / (1.0 + np.abs(m))
    psi, psif = (np.exp(1j * np.outer(x["tau"], m)) @ cm for x in (nd, nf))
    for f in (8.0, 16.0):
        z = _exterior_points(curve, np.array([0.4, 2.0, 3.3, 5.0]), f * cl.near_limit(nd) / 5.0)
        a, b = cl.field_near(4.0, z, curve, nd, psi), cl.field(4.0, z, nf, psif)
        assert np.max(np.abs(a - b)) < 1e-14 * np.max(np.abs(b))


def test_ms_near_closed_patches_exact():
    """Two obstacles 0.24 apart (under five node spacings at 64 nodes each),
    point source inside the first, k = 5 + 3i: the MS sum reaches -U^i at
    far points and at points in the gap, whose fields (and the cross fields
    at the nodes facing the other obstacle) need the near-target integral;
    with the trapezoid rule alone the nearest gap point is off by more than
    1e-5."""
    E = ClosedEllipse(0.8, 0.5, (-1.0, 0.0))
    K = ClosedKite(0.5, (0.62, 0.2))
    t = np.linspace(0.0, 2.0 * math.pi, 2001)
    xe, xk = E.x(t), K.x(t)
    D = np.hypot(xe[:, None, 0] - xk[None, :, 0], xe[:, None, 1] - xk[None, :, 1])
    i, j = np.unravel_index(np.argmin(D), D.shape)
    gap = np.array([xe[i] + f * (xk[j] - xe[i]) for f in (0.3, 0.5, 0.7)])
    far = np.stack([2.8 * np.cos(np.linspace(0, 6, 4)), 2.8 * np.sin(np.linspace(0, 6, 4))], -1)
    obs = np.concatenate([far, gap])
    k = 5.0 + 3.0j
    arcs = [ArcSpec(E, 64, group=0), ArcSpec(K, 64, group=1)]
    pb = MSProblem(arcs=arcs, incident=IncidentSpec("point", z0=(-1.1, 0.1), sigma=0.0),
                   omegas=np.array([k]), M=20, obs=obs, times=np.zeros(0))
    lay = ms.Layout(pb)
    assert D.min() < cl.near_limit(lay.nodes[0])
    ui = oinc.incident(pb.incident, k, obs)
    err = np.abs(ms.run_frequency(lay, k)["U"] + ui) / np.max(np.abs(ui))
    assert np.max(err[:4]) < 1e-12 and np.max(err[4:]) < 5e-9, err
    orig = cl.near_limit
    try:
        cl.near_limit = lambda nd, factor=5.0: 0.0
        err0 = np.abs(ms.run_frequency(ms.Layout(pb), k)["U"] + ui) / np.max(np.abs(ui))
    finally:
        cl.near_limit = orig
    assert err0[4] > 1e-5
