"""Pins of the single-arc oracle (nodes, weights, matrix, solve, potentials)
against closed forms, textbook identities and independent brute force."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import incident as inc
from oracle import nystrom as ny
from workloads import CircularArc, Segment, EllipseArc


def test_symm_identity_weights():
    """W applied to cos(n theta) reproduces Symm's identity (Section 4.3
    weighted Chebyshev discretisation): -pi log 2 for n = 0 and
    -(pi/n) cos(n theta_i) for 1 <= n <= N-1."""
    for n in (3, 8, 33, 128):
        th, _ = ny.cheb_nodes(n)
        W = ny.log_weights(th)
        for m in range(n):
            v = np.cos(m * th)
            rhs = (-math.pi * math.log(2.0)) * v if m == 0 else -(math.pi / m) * v
            assert np.max(np.abs(W @ v - rhs)) < 2e-14 * max(1.0, n / 32)


def test_symm_identity_continuous():
    """The continuous identity the weights are built on, checked by mpmath
    quadrature at an off-node point (independent of the discrete sum)."""
    mp.mp.dps = 25
    x = mp.mpf("0.3141")
    for m in (0, 1, 4):
        f = lambda th: mp.log(abs(x - mp.cos(th))) * mp.cos(m * th)
        val = mp.quad(f, [0, mp.acos(x), mp.pi])
        ref = -mp.pi * mp.log(2) if m == 0 else -(mp.pi / m) * mp.cos(m * mp.acos(x))
        assert abs(val - ref) < 1e-18


def test_nodes_first_kind():
    th, t = ny.cheb_nodes(7)
    assert np.allclose(t, np.cos((2 * np.arange(1, 8) - 1) * np.pi / 14))
    assert np.all(np.abs(t) < 1.0)


def test_matrix_complex_symmetric():
    """A = A^T exactly (complex symmetric, not Hermitian)."""
    nd = ny.arc_nodes(CircularArc(1.0, -1.25, 1.25), 96)
    A = ny.assemble(nd, 17.3)
    assert np.max(np.abs(A - A.T)) < 1e-16
    assert np.max(np.abs(A - A.conj().T)) > 1e-3


@pytest.mark.parametrize("curve", [Segment((-0.3, 0.1), (2.3, 0.1)),
                                   CircularArc(1.2, 0.3, 2.1)])
def test_diagonal_limit(curve):
    """L2(t, t + h) tends to the closed-form diagonal value
    i/4 - (gamma + log(k s / 2)) / (2 pi) like h^2 (segment) or h (arc),
    with no stagnation from cancellation down to h = 1e-6."""
    k, t0 = 7.0, 0.17
    x0 = curve.x(np.array([t0]))
    s0 = np.hypot(*curve.dx(np.array([t0]))[0])
    _, d2 = ny.kernel_diag(k, s0)
    gaps = []
    for h in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6):
        x1 = curve.x(np.array([t0 + h]))
        _, L2 = ny.kernel_split(k, x0, x1, np.array([t0]), np.array([t0 + h]))
        gaps.append(abs(L2[0] - d2))
    gaps = np.array(gaps)
    assert gaps[-1] < 1e-5 * gaps[0] + 1e-13
    # monotone decay at a rate of at least one decade per decade of h
    assert np.all(gaps[1:] < 0.2 * gaps[:-1] + 1e-14)


def _mp_single_layer(k, curve_x, coeffs, t_target):
    """V[alpha_N / w](x(t_target)) at 25 digits (mpmath, tanh-sinh)."""
    mp.mp.dps = 25
    th0 = mp.acos(mp.mpf(t_target))
    zx, zy = curve_x(mp.mpf(t_target))

    def f(ph):
        px, py = curve_x(mp.cos(ph))
        r = mp.sqrt((px - zx) ** 2 + (py - zy) ** 2)
        h = mp.besselj(0, k * r) + 1j * mp.bessely(0, k * r)
        dens = sum(mp.mpc(c) * mp.cos(n * ph) for n, c in enumerate(coeffs))
        return 0.25j * h * dens

    return complex(mp.quad(f, [0, th0, mp.pi]))


@pytest.mark.parametrize("which", ["segment", "circle"])
def test_nystrom_matches_brute_force(which):
    """A alpha equals the boundary operator applied to the interpolated
    density, computed by 25-digit quadrature, for a tiny arc (k L ~ 1):
    pins W, L1, L2 and the diagonal limit at once."""
    k, n = 0.5, 16
    if which == "segment":
        curve = Segment((-1.0, 0.0), (1.0, 0.0))
        cx = lambda t: (t, mp.mpf(0))
    else:
        curve = CircularArc(1.0, 0.2, 1.4)
        cx = lambda t: (mp.cos(0.8 + 0.6 * t), mp.sin(0.8 + 0.6 * t))
    nd = ny.arc_nodes(curve, n)
    A = ny.assemble(nd, k)
    coeffs = [0.7 + 0.2j, -0.3 + 0.5j, 0.1 - 0.05j]
    a = np.zeros(n, dtype=complex)
    a[:3] = coeffs
    alpha = ny.density_at(a, nd["theta"])
    lhs = A @ alpha
    for i in (0, 5, 11, 15):
        ref = _mp_single_layer(k, cx, coeffs, nd["t"][i])
        assert abs(lhs[i] - ref) < 5e-15


def test_gauss_elimination_vs_lapack():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12))
    b = rng.standard_normal(12) + 1j * rng.standard_normal(12)
    x1 = ny.gauss_solve(A, b)
    x2 = ny.solve(A, b)
    assert np.linalg.norm(x1 - x2) < 1e-12 * np.linalg.norm(x2)
    assert np.linalg.norm(A @ x1 - b) < 1e-12 * np.linalg.norm(b)


def test_interpolant_reproduces_nodes():
    rng = np.random.default_rng(1)
    th, _ = ny.cheb_nodes(37)
    al = rng.standard_normal(37) + 1j * rng.standard_normal(37)
    a = ny.cheb_coeffs(al, th)
    assert np.max(np.abs(ny.density_at(a, th) - al)) < 1e-13


def test_self_convergence_flat_arc():
    """Spectral convergence on the flat arc at k = 32 (fields on the
    radius-3 circle): N = 64 is ~1e-5 off, N >= 96 agree to ~1e-14."""
    curve = Segment((-1.0, 0.0), (1.0, 0.0))
    k = 32.0
    p = 2 * np.pi * np.arange(64) / 64
    obs = 3.0 * np.stack([np.cos(p), np.sin(p)], -1)
    res = {}
    for n in (64, 96, 128, 192):
        nd = ny.arc_nodes(curve, n)
        al = ny.solve(ny.assemble(nd, k), -inc.plane(k, nd["y"], math.pi / 6))
        res[n] = ny.field_far(k, obs, nd["y"], al)
    ref = np.linalg.norm(res[192])
    e = {n: np.linalg.norm(res[n] - res[192]) / ref for n in res}
    assert 1e-7 < e[64] < 1e-4
    assert e[96] < 1e-13 and e[128] < 1e-13


@pytest.mark.parametrize("curve,k", [(Segment((-1.0, 0.0), (1.0, 0.0)), 7.0),
                                     (CircularArc(1.0, -1.25, 1.25), 12.0),
                                     (EllipseArc(1.3, 0.6, 0.4, 2.9), 9.5)])
def test_optical_theorem_and_reciprocity(curve, k):
    """Sound-soft arcs conserve energy: int |u_inf|^2 = -2 sqrt(2 pi / k)
    Re(e^{i pi/4} u_inf(d; d)); and u_inf(xh; d) = u_inf(-d; -xh).
    Pins the imaginary (J0) part of the kernel, the solve and the field."""
    n = 128
    nd = ny.arc_nodes(curve, n)
    A = ny.assemble(nd, k)
    th_d = 0.4
    al = ny.solve(A, -inc.plane(k, nd["y"], th_d))
    m = 2048
    ph = 2 * np.pi * np.arange(m) / m
    xh = np.stack([np.cos(ph), np.sin(ph)], -1)
    power = np.sum(np.abs(ny.far_field(k, xh, nd["y"], al)) ** 2) * 2 * np.pi / m
    d = np.array([[math.cos(th_d), math.sin(th_d)]])
    fwd = ny.far_field(k, d, nd["y"], al)[0]
    assert abs(power + 2 * math.sqrt(2 * math.pi / k)
               * np.real(np.exp(0.25j * math.pi) * fwd)) < 1e-12 * power
    th_x = 2.1
    al2 = ny.solve(A, -inc.plane(k, nd["y"], th_x + math.pi))
    u1 = ny.far_field(k, np.array([[math.cos(th_x), math.sin(th_x)]]), nd["y"], al)[0]
    u2 = ny.far_field(k, -d, nd["y"], al2)[0]
    assert abs(u1 - u2) < 1e-12 * abs(u1)


def test_near_field_against_mpmath():
    """The adaptive near-field rule matches 25-digit quadrature of the
    interpolated density at targets close to an arc, including one just
    past an endpoint on the curve's continuation."""
    mp.mp.dps = 20
    curve = CircularArc(1.0, 0.0, 1.5)
    n, k = 24, 6.0
    nd = ny.arc_nodes(curve, n)
    rng = np.random.default_rng(2)
    alpha = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    a = ny.cheb_coeffs(alpha, nd["theta"])
    targets = [(math.cos(0.7) * 1.01, math.sin(0.7) * 1.01),
               (math.cos(-0.003), math.sin(-0.003)),
               (0.5, 0.4)]
    for z in targets:
        got = ny.field_near(k, np.array(z), curve, a)
        zx, zy = mp.mpf(z[0]), mp.mpf(z[1])

        def f(ph):
            tau = 0.75 + 0.75 * mp.cos(ph)
            r = mp.sqrt((mp.cos(tau) - zx) ** 2 + (mp.sin(tau) - zy) ** 2)
            h = mp.besselj(0, k * r) + 1j * mp.bessely(0, k * r)
            dens = sum(mp.mpc(c) * mp.cos(j * ph) for j, c in enumerate(a))
            return 0.25j * h * dens

        phs = ny.nearest_param(curve, np.array(z))
        pts = [0, phs, mp.pi] if 0 < phs < math.pi else [0, mp.pi]
        ref = complex(mp.quad(f, pts, maxdegree=10))
        assert abs(got - ref) < 1e-12 * max(1.0, abs(ref))


def test_far_rule_matches_exact_at_far_targets():
    """Far targets (beyond the near radius) agree with exact quadrature of
    the interpolant, so the near/far switch is seamless."""
    curve = CircularArc(1.0, 0.0, 1.5)
    n, k = 32, 5.0
    nd = ny.arc_nodes(curve, n)
    rng = np.random.default_rng(3)
    alpha = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    a = ny.cheb_coeffs(alpha, nd["theta"])
    rad = ny.near_radius(nd["y"])
    z = np.array([[math.cos(0.6) * (1 + 1.05 * rad), math.sin(0.6) * (1 + 1.05 * rad)]])
    far = ny.field_far(k, z, nd["y"], alpha)[0]
    exact = ny.field_near(k, z[0], curve, a)
    assert abs(far - exact) < 1e-12 * max(1.0, abs(exact))


@pytest.mark.parametrize("scale", [1.0, 1e-12])
def test_near_rule_is_scale_free_against_dense_rule(scale):
    """The adaptive near-field integral of an oscillatory density meets its
    relative tolerance whatever the size of the field (the kite cavity's
    fields are ~1e-12 away from the source's centre frequency): checked
    against a dense composite Gauss-Legendre rule (2000 panels x 32 points)
    with the kernel from scipy and the density summed from its Chebyshev
    coefficients with numpy."""
    from numpy.polynomial import chebyshev as C
    from scipy.special import hankel1
    curve = CircularArc(1.0, -1.2, 1.2)
    rng = np.random.default_rng(4)
    coef = scale * (rng.standard_normal(48) + 1j * rng.standard_normal(48)) / (1 + np.arange(48))
    k = 30.0
    g, w = np.polynomial.legendre.leggauss(32)
    e = np.linspace(0.0, math.pi, 2001)
    phi = (0.5 * (e[1:] + e[:-1])[:, None] + 0.5 * np.diff(e)[:, None] * g[None, :]).ravel()
    wt = (0.5 * np.diff(e)[:, None] * w[None, :]).ravel()
    xy = curve.x(np.cos(phi))
    dens = C.chebval(np.cos(phi), coef)
    for z in (np.array([1.5, 0.2]), np.array([3.0, -1.0]), np.array([0.2, 0.1])):
        r = np.hypot(xy[:, 0] - z[0], xy[:, 1] - z[1])
        dense = np.sum(wt * 0.25j * hankel1(0, k * r) * dens)
        val = ny.field_near(k, z, curve, coef)
        assert abs(val - dense) <= 1e-12 * abs(dense), (z, abs(val - dense) / abs(dense))
