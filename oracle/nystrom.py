"""Oracle: single-layer Nystrom discretisation on one open arc.

Test infrastructure only (see the package header).

What is discretised (Section 3.2, eqs. FDBIEk-interior / FDsolk-interior):
the first-kind open-arc equation  V_Gamma[psi] = G  on the arc and the
single-layer potential  S_Gamma[psi]  off it, with the fundamental solution
Phi_k(x, y) = (i/4) H0^(1)(k |x - y|) (Section 2.1).

How (Section 4.3, eq. singularity; Chebyshev spectral discretisation):
  * the arc is x(t), t in [-1, 1]; nodes are first-kind Chebyshev points
    t_i = cos(theta_i), theta_i = (2i - 1) pi / (2N), i = 1..N;
  * the density carries the endpoint weight: psi(x(t)) |x'(t)| =
    alpha(t) / sqrt(1 - t^2), and the unknowns are alpha_i = alpha(t_i);
  * the kernel is split as Phi = L1 log|t - t'| + L2 with
    L1 = -J0(k r) / (2 pi) and L2 = Phi - L1 log|t - t'|; the log part is
    integrated exactly against the Chebyshev interpolant (Symm's identity
    int log|x - t| T_n(t) (1 - t^2)^(-1/2) dt = -pi log 2 (n = 0),
    -(pi / n) T_n(x) (n >= 1)), the smooth part by Gauss-Chebyshev;
  * A_ij = W_ij L1_ij + (pi / N) L2_ij with the diagonal limits
    L1_ii = -1/(2 pi),  L2_ii = i/4 - (gamma + log(k s_i / 2)) / (2 pi).

Every array is float64 / complex128.  Wavenumbers may be complex (used only
by the complex-frequency pins); the GPU path takes real k.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

EULER_GAMMA = 0.57721566490153286060651209008240243


# --------------------------------------------------------------------------
# nodes, geometry, weights
# --------------------------------------------------------------------------
def cheb_nodes(n):
    """First-kind Chebyshev nodes: theta_i = (2i-1) pi / (2n), t_i = cos."""
    i = np.arange(1, n + 1, dtype=float)
    theta = (2.0 * i - 1.0) * math.pi / (2.0 * n)
    return theta, np.cos(theta)


def arc_nodes(curve, n):
    """Node positions y_i = x(t_i) and speeds s_i = |x'(t_i)|."""
    theta, t = cheb_nodes(n)
    y = curve.x(t)
    d = curve.dx(t)
    return dict(theta=theta, t=t, y=y, s=np.hypot(d[:, 0], d[:, 1]), n=n)


def log_weights(theta):
    """Product-integration weights of log|t_i - t'| (1 - t'^2)^(-1/2) against
    the degree-(N-1) Chebyshev interpolant (Symm identity):
        W_ij = -(pi/N) [log 2 + 2 sum_{m=1}^{N-1} cos(m th_i) cos(m th_j) / m].
    """
    n = theta.size
    m = np.arange(1, n, dtype=float)
    C = np.cos(np.outer(theta, m))            # [N, N-1]
    S = (C / m) @ C.T
    return -(math.pi / n) * (math.log(2.0) + 2.0 * S)


def hankel0(z):
    return special.hankel1(0, z)


def bessel_j0(z):
    return special.jv(0, z)


def fundamental(k, r):
    """Phi_k(r) = (i/4) H0^(1)(k r)  (Section 2.1)."""
    return 0.25j * hankel0(k * r)


# --------------------------------------------------------------------------
# Nystrom matrix
# --------------------------------------------------------------------------
def kernel_split(k, x1, x2, t1, t2):
    """L1 and L2 of Phi_k = L1 log|t1 - t2| + L2 at distinct point pairs
    x1 = x(t1), x2 = x(t2) (arrays [..., 2] and [...])."""
    r = np.hypot(x1[..., 0] - x2[..., 0], x1[..., 1] - x2[..., 1])
    j0 = bessel_j0(k * r)
    L1 = -j0 / (2.0 * math.pi)
    L2 = (0.25j * hankel0(k * r)
          + j0 * np.log(np.abs(t1 - t2)) / (2.0 * math.pi))
    return L1, L2


def kernel_diag(k, s):
    """Limits of L1, L2 as t2 -> t1 at a point of speed s = |x'(t1)|."""
    L1 = np.full(np.shape(s), -1.0 / (2.0 * math.pi), dtype=complex)
    L2 = 0.25j - (EULER_GAMMA + np.log(k * np.asarray(s) / 2.0)) / (2.0 * math.pi)
    return L1, L2


def assemble(nodes, k):
    """Nystrom matrix A (complex128, N x N) of V_Gamma on one arc:
    A_ij = W_ij L1_ij + (pi/N) L2_ij."""
    theta, t, y, s = nodes["theta"], nodes["t"], nodes["y"], nodes["s"]
    n = t.size
    W = log_weights(theta)
    off = ~np.eye(n, dtype=bool)
    I, J = np.nonzero(off)
    L1 = np.empty((n, n), dtype=complex)
    L2 = np.empty((n, n), dtype=complex)
    L1[off], L2[off] = kernel_split(k, y[I], y[J], t[I], t[J])
    d = np.arange(n)
    L1[d, d], L2[d, d] = kernel_diag(k, s)
    return W * L1 + (math.pi / n) * L2


def solve(A, b):
    """Dense LU with partial pivoting (LAPACK zgesv through numpy)."""
    return np.linalg.solve(A, b)


def gauss_solve(A, b):
    """Textbook Gaussian elimination with partial pivoting (small N only)."""
    A = np.array(A, dtype=complex)
    x = np.array(b, dtype=complex)
    n = A.shape[0]
    for c in range(n):
        p = c + int(np.argmax(np.abs(A[c:, c])))
        if A[p, c] == 0:
            raise ZeroDivisionError("singular matrix")
        if p != c:
            A[[c, p]] = A[[p, c]]
            x[[c, p]] = x[[p, c]]
        for r in range(c + 1, n):
            f = A[r, c] / A[c, c]
            A[r, c:] -= f * A[c, c:]
            x[r] -= f * x[c]
    for c in range(n - 1, -1, -1):
        x[c] = (x[c] - A[c, c + 1:] @ x[c + 1:]) / A[c, c]
    return x


# --------------------------------------------------------------------------
# density interpolant
# --------------------------------------------------------------------------
def cheb_coeffs(alpha, theta):
    """a_n = ((2 - delta_n0) / N) sum_j alpha_j cos(n theta_j): the
    interpolant alpha_N(cos phi) = sum_n a_n cos(n phi)."""
    n = theta.size
    C = np.cos(np.outer(np.arange(n), theta))
    a = (C @ alpha) * (2.0 / n)
    a[0] *= 0.5
    return a


def density_at(a, phi):
    """alpha_N(cos phi) for an array of phi."""
    return np.cos(np.outer(phi, np.arange(a.size))) @ a


# --------------------------------------------------------------------------
# adaptive Gauss-Legendre (vectorised interval bisection)
# --------------------------------------------------------------------------
_GL = {}


def _gl(order):
    if order not in _GL:
        _GL[order] = np.polynomial.legendre.leggauss(order)
    return _GL[order]


def adaptive_gl(f, a, b, breaks=(), tol_abs=0.0, tol_rel=1e-14, order=16,
                max_rounds=120):
    """Integral of the vectorised complex function f over [a, b].

    Each interval is integrated by an ``order``-point Gauss-Legendre rule on
    the whole and on its two halves; an interval is accepted when the two
    estimates agree to its share of the tolerance (or to a small fixed
    fraction of the whole budget, which is what ends the bisection next to
    an integrable endpoint singularity), else it is bisected.  The tolerance
    is relative to the scale of the integrand, tol_rel * int |f| (first-round
    estimate), so that it means the same for a field of size 1e-12 as for
    one of size 1; tol_abs is an optional absolute floor.
    ``breaks`` are interior points (e.g. the nearest point of a curve to a
    target) at which the interval is split up front.
    """
    g, w = _gl(order)
    pts = sorted({a, b, *[p for p in breaks if a < p < b]})
    lo = np.array(pts[:-1], dtype=float)
    hi = np.array(pts[1:], dtype=float)
    span = b - a

    def rule(l, h, with_abs=False):
        c = 0.5 * (l + h)
        r = 0.5 * (h - l)
        x = c[:, None] + r[:, None] * g[None, :]
        fx = f(x.ravel()).reshape(x.shape)
        if with_abs:
            return (fx @ w) * r, (np.abs(fx) @ w) * r
        return (fx @ w) * r

    total = 0.0 + 0.0j
    tol = None
    for _ in range(max_rounds):
        if lo.size == 0:
            break
        mid = 0.5 * (lo + hi)
        whole = rule(lo, hi)
        if tol is None:
            h1, s1 = rule(lo, mid, True)
            h2, s2 = rule(mid, hi, True)
            halves = h1 + h2
            tol = max(tol_abs, tol_rel * float(np.sum(s1 + s2)))
            if tol == 0.0:
                return 0.0 + 0.0j
        else:
            halves = rule(lo, mid) + rule(mid, hi)
        err = np.abs(halves - whole)
        ok = (err <= tol * (hi - lo) / span) | (err <= 1e-3 * tol)
        ok |= (hi - lo) <= 1e-15 * span
        total += np.sum(halves[ok])
        lo, hi, mid = lo[~ok], hi[~ok], mid[~ok]
        lo, hi = np.concatenate([lo, mid]), np.concatenate([mid, hi])
    else:
        raise RuntimeError("adaptive_gl: no convergence")
    return total


# --------------------------------------------------------------------------
# potentials
# --------------------------------------------------------------------------
def max_spacing(y):
    """Largest distance between consecutive nodes of an arc."""
    return float(np.max(np.hypot(np.diff(y[:, 0]), np.diff(y[:, 1]))))


NEAR_FACTOR = 10.0


def near_radius(y):
    """Targets closer than this to some node use the near-field rule.

    The Gauss-Chebyshev rule applied to (kernel x degree-(N-1) interpolant)
    has error ~ exp(-pi d / h) for a target at distance d from an arc with
    node spacing h, so 10 h keeps the far rule at ~1e-14 relative."""
    return NEAR_FACTOR * max_spacing(y)


def field_far(k, z, y, alpha):
    """Gauss-Chebyshev rule (pi/N) sum_j Phi_k(z, y_j) alpha_j, z: [P, 2]."""
    n = y.shape[0]
    r = np.hypot(z[:, None, 0] - y[None, :, 0], z[:, None, 1] - y[None, :, 1])
    return (math.pi / n) * (fundamental(k, r) @ alpha)


def nearest_param(curve, z, samples=4001):
    """phi in [0, pi] of the point x(cos phi) nearest to z."""
    from scipy.optimize import minimize_scalar
    ph = np.linspace(0.0, math.pi, samples)
    p = curve.x(np.cos(ph))
    d = np.hypot(p[:, 0] - z[0], p[:, 1] - z[1])
    i = int(np.argmin(d))
    lo, hi = ph[max(i - 1, 0)], ph[min(i + 1, samples - 1)]
    if hi <= lo:
        return float(ph[i])

    def dist(q):
        x = curve.x(np.cos(np.array([q])))[0]
        return math.hypot(x[0] - z[0], x[1] - z[1])

    res = minimize_scalar(dist, bounds=(lo, hi), method="bounded",
                          options=dict(xatol=1e-13))
    return float(res.x)


def field_near(k, z, curve, a, tol_rel=1e-14):
    """Exact single-layer potential of the interpolated density at one target:
    int_0^pi Phi_k(z, x(cos phi)) alpha_N(cos phi) dphi (adaptive)."""
    phs = nearest_param(curve, z)

    def f(ph):
        x = curve.x(np.cos(ph))
        r = np.hypot(x[:, 0] - z[0], x[:, 1] - z[1])
        return fundamental(k, r) * density_at(a, ph)

    return adaptive_gl(f, 0.0, math.pi, breaks=(phs,), tol_rel=tol_rel)


def field(k, z, curve, nodes, alpha):
    """Single-layer potential at targets z [P, 2]: Gauss-Chebyshev for far
    targets, adaptive quadrature of the interpolant for near ones."""
    z = np.atleast_2d(np.asarray(z, dtype=float))
    y = nodes["y"]
    dmin = np.min(np.hypot(z[:, None, 0] - y[None, :, 0],
                           z[:, None, 1] - y[None, :, 1]), axis=1)
    near = dmin < near_radius(y)
    out = np.empty(z.shape[0], dtype=complex)
    if np.any(~near):
        out[~near] = field_far(k, z[~near], y, alpha)
    if np.any(near):
        a = cheb_coeffs(alpha, nodes["theta"])
        for p in np.nonzero(near)[0]:
            out[p] = field_near(k, z[p], curve, a)
    return out


def single_layer_on_arc(k, curve, a, t_target, tol_rel=1e-13):
    """V[alpha_N / w](x(t_target)): the boundary operator applied to the
    interpolated density, by adaptive quadrature with a break at the
    log singularity (brute-force reference for tiny arcs)."""
    z = curve.x(np.array([t_target]))[0]
    ph0 = math.acos(max(-1.0, min(1.0, t_target)))

    def f(ph):
        x = curve.x(np.cos(ph))
        r = np.hypot(x[:, 0] - z[0], x[:, 1] - z[1])
        r = np.where(r == 0.0, 1e-300, r)
        return fundamental(k, r) * density_at(a, ph)

    return adaptive_gl(f, 0.0, math.pi, breaks=(ph0,), tol_rel=tol_rel,
                       max_rounds=200)


def far_field(k, xhat, y, alpha):
    """Far-field pattern u_inf(xhat) = e^{i pi/4} / sqrt(8 pi k)
    * (pi/N) sum_j exp(-i k xhat . y_j) alpha_j."""
    n = y.shape[0]
    ph = np.exp(-1j * k * (xhat @ y.T))
    return (np.exp(0.25j * math.pi) / np.sqrt(8.0 * math.pi * k)
            * (math.pi / n) * (ph @ alpha))
