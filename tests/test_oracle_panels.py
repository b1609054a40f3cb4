"""Pins of the composite-panel oracle (Section 4.3, eqs. cov, psi-tilde):
the changes of variables, the Fejer rule, the frequency-independent log
table against closed forms (segment, circle via Clausen's function) and
brute-force quadrature (ellipse), the single-arc solution against the
independent weighted-Chebyshev scheme, and the multiple-scattering exact
solution, where the panels restore fast convergence."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import incident as inc
from oracle import ms
from oracle import nystrom as ny
from oracle import panels as pn
from workloads import IncidentSpec, disc_interior_case
from workloads.curves import CircularArc, EllipseArc, Segment


def _coef_tail(f, n=32, m0=20):
    """max |Chebyshev coefficient| of index >= m0 of f on [-1, 1]."""
    phi, s = ny.cheb_nodes(n)
    a = ny.cheb_coeffs(f(s), phi)
    return float(np.max(np.abs(a[m0:])))


def test_cov_maps_and_singular_ends():
    """eq. cov: each map is an increasing bijection of [-1, 1] whose
    derivative vanishes exactly at the ends it treats as singular."""
    s = np.linspace(-1.0, 1.0, 2001)
    for kind, zero_at in ((pn.COV_NONE, ()), (pn.COV_BOTH, (-1, 1)),
                          (pn.COV_LEFT, (-1,)), (pn.COV_RIGHT, (1,))):
        th, d = pn.cov(kind, s)
        assert abs(th[0] + 1.0) < 1e-15 and abs(th[-1] - 1.0) < 1e-15
        assert np.all(np.diff(th) > 0.0)
        # derivative against centred differences
        h = 1e-6
        sm = np.linspace(-0.99, 0.99, 101)
        fd = (pn.cov(kind, sm + h)[0] - pn.cov(kind, sm - h)[0]) / (2 * h)
        assert np.max(np.abs(fd - pn.cov(kind, sm)[1])) < 1e-8
        for e, v in ((-1, d[0]), (1, d[-1])):
            assert (abs(v) < 1e-15) == (e in zero_at)


def test_cov_removes_square_root_end_singularities():
    """A density with inverse-square-root ends (the form of eq. sqrt_sing
    with f = 1) becomes an entire function of s once multiplied by the
    Jacobian (eq. psi-tilde); without the change of variables it is not
    even bounded.  (Near the ends 1 - theta(s) is formed with cancellation,
    which is what limits the thresholds here.)"""
    both = lambda s: pn.cov(pn.COV_BOTH, s)[1] / np.sqrt(1.0 - pn.cov(pn.COV_BOTH, s)[0] ** 2)
    assert np.max(np.abs(both(np.linspace(-0.99, 0.99, 101)) - 0.5 * math.pi)) < 1e-11
    left = lambda s: pn.cov(pn.COV_LEFT, s)[1] / np.sqrt(1.0 + pn.cov(pn.COV_LEFT, s)[0])
    right = lambda s: pn.cov(pn.COV_RIGHT, s)[1] / np.sqrt(1.0 - pn.cov(pn.COV_RIGHT, s)[0])
    assert _coef_tail(left) < 1e-9 and _coef_tail(right) < 1e-9
    # f(d^(1/2)) / d^(1/2) with a non-trivial smooth f, both ends
    g = lambda s: (pn.cov(pn.COV_BOTH, s)[1] * np.cos(np.sqrt(1.0 - pn.cov(pn.COV_BOTH, s)[0]))
                   / np.sqrt(1.0 - pn.cov(pn.COV_BOTH, s)[0] ** 2))
    assert _coef_tail(g) < 1e-9
    assert _coef_tail(lambda s: 1.0 / np.sqrt(1.0 - s * s)) > 1e-2


def test_fejer_weights_integrate_chebyshev_polynomials():
    """sum_i w_i T_m(s_i) = int T_m = 2 / (1 - m^2) (m even), 0 (m odd),
    for every m < n."""
    for n in (5, 16, 33):
        phi, s = ny.cheb_nodes(n)
        w = pn.fejer_weights(phi)
        for m in range(n):
            exact = 2.0 / (1.0 - m * m) if m % 2 == 0 else 0.0
            assert abs(np.sum(w * np.cos(m * phi)) - exact) < 1e-14


@pytest.mark.parametrize("breaks,n", [((-1.0, 1.0), 24), ((-1.0, -0.3, 0.4, 1.0), 16)])
def test_log_table_segment_closed_form(breaks, n):
    """On the segment x(t) = (t, 0):  sum_j W_ij (dt/ds)_j is the integral
    of log|t_i - t| over the arc in t (the interpolant of the entire
    function dt/ds is exact to rounding), i.e. the closed form
    (1+t) log(1+t) + (1-t) log(1-t) - 2."""
    arc = pn.PanelArc(Segment((-1.0, 0.0), (1.0, 0.0)), n, breaks)
    nd = arc.nodes()
    W = pn.log_table(arc)
    dts = np.concatenate([arc.t_of(p, arc.s)[1] for p in range(arc.P)])
    t = nd["t"]
    ref = (1 + t) * np.log(1 + t) + (1 - t) * np.log(1 - t) - 2.0
    assert np.max(np.abs(W @ dts - ref)) < 1e-12


def test_log_table_circle_clausen():
    """On the unit circle, |x(a) - x(b)| = 2 |sin((a - b)/2)|, so
    int_{a0}^{a1} log|x(tau_i) - x(tau)| dtau = Cl2(a0 - tau_i) - Cl2(a1 - tau_i)
    (Clausen's function); with the arc-length speed |dx/ds| as density the
    table must reproduce it, panel by panel summed over the arc."""
    a0, a1 = -0.7, 2.4
    arc = pn.PanelArc(CircularArc(1.0, a0, a1), 20, (-1.0, -0.45, 0.35, 1.0))
    nd = arc.nodes()
    W = pn.log_table(arc)
    sp = np.concatenate([arc.speed(p, arc.s) for p in range(arc.P)])
    tau = CircularArc(1.0, a0, a1).parent_param(nd["t"])
    ref = np.array([float(mp.clsin(2, a0 - ti) - mp.clsin(2, a1 - ti)) for ti in tau])
    assert np.max(np.abs(W @ sp - ref)) < 1e-12


def test_log_table_ellipse_brute_force():
    """Entries of W against mpmath quadrature (30 digits) of the moments
    int log|y_i - y(s)| T_m(s) ds on a panel (the interpolant of T_m, m < n,
    is T_m itself): a target on the panel (log singularity), a target on
    the neighbouring panel next to the shared end (near singularity) and a
    distant one."""
    mp.mp.dps = 30
    ea, eb, s0, s1 = 1.3, 0.7, -0.4, 2.2
    br = (-1.0, -0.2, 0.5, 1.0)
    n = 12
    arc = pn.PanelArc(EllipseArc(ea, eb, s0, s1), n, br)
    nd = arc.nodes()
    W = pn.log_table(arc)

    def ypt(p, s):
        a = mp.mpf(br[p]), mp.mpf(br[p + 1])
        th = mp.cos(mp.pi * (1 - s) / 2)
        t = (a[0] + a[1]) / 2 + (a[1] - a[0]) / 2 * th
        tau = (mp.mpf(s0) + s1) / 2 + (mp.mpf(s1) - s0) / 2 * t
        return ea * mp.cos(tau), eb * mp.sin(tau)

    phi = [(2 * j + 1) * mp.pi / (2 * n) for j in range(n)]
    cases = [(1 * n + 4, 1), (1 * n + 0, 2), (2 * n + n - 1, 0), (0 * n + 3, 2)]
    for i, p in cases:
        pi_, j = divmod(i, n)
        yi = ypt(pi_, mp.cos(phi[j]))
        for m in (0, 3, n - 1):
            f = lambda s: mp.log(mp.sqrt((ypt(p, s)[0] - yi[0]) ** 2 + (ypt(p, s)[1] - yi[1]) ** 2)) * mp.chebyt(m, s)
            pts = [-1, mp.cos(phi[j]), 1] if pi_ == p else [-1, 1]
            ref = mp.quad(f, pts)
            got = W[i, p * n:(p + 1) * n] @ np.cos(m * arc.phi)
            assert abs(got - float(ref)) < 1e-12, (i, p, m, got, float(ref))


@pytest.mark.parametrize("curve", [Segment((-1.0, 0.2), (1.0, -0.1)), CircularArc(1.0, -0.5, 2.0)],
                         ids=["segment", "circular"])
def test_single_arc_matches_weighted_chebyshev(curve):
    """One open arc with smooth data: both discretisations converge
    spectrally to the same solution, so the panel scheme's field must agree
    with the single-panel weighted-Chebyshev field of ``oracle.nystrom``
    (96 nodes, exact to rounding), at far and near targets."""
    k = 7.0
    spec = IncidentSpec("plane", theta=0.5)
    z = np.array([[3 * math.cos(a), 3 * math.sin(a)] for a in np.linspace(0, 6, 7)] + [[0.1, 0.35]])
    nd = ny.arc_nodes(curve, 96)
    a = ny.solve(ny.assemble(nd, k), -inc.incident(spec, k, nd["y"]))
    ref = ny.field(k, z, curve, nd, a)
    arc = pn.PanelArc(curve, 24, (-1.0, -0.4, 0.3, 1.0))
    pnd = arc.nodes()
    mu = ny.solve(pn.assemble(pnd, k, pn.log_table(arc)), -inc.incident(spec, k, pnd["y"]))
    U = pn.field(k, z, pnd, mu)
    assert np.max(np.abs(U - ref)) < 1e-7 * np.max(np.abs(ref))
    # the densities agree too: mu = psi |dx/ds| at the panel nodes, with psi
    # = alpha / (sqrt(1 - t^2) |x'(t)|) from the weighted-Chebyshev
    # interpolant
    t = pnd["t"]
    co = ny.cheb_coeffs(a, nd["theta"])
    alpha_t = np.cos(np.outer(np.arccos(t), np.arange(co.size))) @ co
    d = curve.dx(t)
    psi_ref = alpha_t / (np.sqrt(1 - t * t) * np.hypot(d[:, 0], d[:, 1]))
    sp = np.concatenate([arc.speed(p, arc.s) for p in range(arc.P)])
    assert np.max(np.abs(mu - psi_ref * sp)) < 1e-5 * np.max(np.abs(mu))
    assert np.allclose(pn.density_per_length(arc, mu), mu / sp)


def test_ms_interior_exact_solution_converges_faster_with_panels():
    """Multiple scattering in the three-arc disc (Geometry 1 layout) at a
    complex wavenumber with a source outside: the MS sum tends to -U^i
    inside.  The single-panel scheme stalls near 1e-4 because of the induced
    square-root singularities at the ends of the truncated overlaps
    (Section 4.3); cutting the arcs there with the changes of variables of
    eq. cov restores fast convergence.  The window transition is widened
    (c0, c1 = 0.02, 0.98): with 1/3 and 2/3 the resolution of the steep
    C-infinity window eta limits both schemes at these sizes."""
    k = 5.0 + 2.0j
    errs = {}
    for scheme, n in (("panels", 12), ("panels", 16), ("cheb", 48), ("cheb", 72)):
        pb = disc_interior_case(n=n, omegas=(k,), M=6)
        pb.scheme = scheme
        pb.c0, pb.c1 = 0.02, 0.98
        lay = ms.Layout(pb)
        if scheme == "panels":
            assert np.allclose(lay.panel_breaks(0), (-1.0, -1.0 / 3.0, 1.0 / 3.0, 1.0))
        ui = inc.incident(pb.incident, k, pb.obs)
        U = ms.run_frequency(lay, k)["U"]
        errs[(scheme, n)] = float(np.max(np.abs(U + ui)) / np.max(np.abs(ui)))
    assert errs[("panels", 12)] < 1e-3
    assert errs[("panels", 16)] < 1e-4
    assert errs[("cheb", 48)] > 1e-4 and errs[("cheb", 72)] > 1e-4
    # 48 unknowns per arc with panels against 48 and 72 without
    assert errs[("panels", 16)] < 0.5 * min(errs[("cheb", 48)], errs[("cheb", 72)])
