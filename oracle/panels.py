"""Oracle: composite-panel discretisation with cosine changes of variables.

Test infrastructure only (see the package header).

What is discretised: the same first-kind open-arc equation and potential as
``oracle.nystrom`` (Section 3.2, eqs. FDBIEk-interior / FDsolk-interior),
with the density resolved panel by panel (Section 4.3):

  * the arc x(t), t in [-1, 1], is cut at breakpoints into panels so that no
    endpoint of the arc or of its truncated overlap lies inside a panel;
  * each panel carries its own variable theta in [-1, 1] and, depending on
    where the panel has singular ends, the cosine change of variables
    theta = theta(s) of eq. cov (none, both ends, the -1 end, the +1 end);
  * the unknown is the density per unit s, mu(s) = psi(x) |dx/ds| (the
    Jacobian-carrying density of eq. psi-tilde, here including the arc
    speed), smooth when psi has the square-root end behaviour of
    eq. sqrt_sing;
  * in s, first-kind Chebyshev nodes s_i = cos(phi_i) and Fejer weights w_i
    (the interpolatory rule of int_{-1}^{1} f ds on those nodes).

Matrix.  With Phi_k = -(1/2pi) J0(kr) log r + S(r) and S smooth (S(0) =
i/4 - (gamma + log(k/2)) / (2pi)), the log part is integrated exactly
against the panel interpolant of J0 mu (product integration), the smooth
part by the Fejer rule:
    A_ij = -(1/2pi) J0(k r_ij) W_ij + w_j S(r_ij),
    W_ij = int_{panel(j)} log|y_i - y(s)| l_j(s) ds,
where l_j is the Lagrange basis of panel(j)'s nodes.  W depends only on the
geometry: one table serves every frequency (the kernel split of
Section 4.2).  The oracle computes each row of W by vector-valued adaptive
Gauss-Legendre quadrature of the Chebyshev moments, split at the target.

Field.  Far targets: sum_j w_j Phi_k(z, y_j) mu_j.  Near targets: the exact
integral of the panel interpolants, int_0^pi Phi_k(z, y(cos p)) mu_N(cos p)
sin p dp per panel, by adaptive quadrature.
"""
from __future__ import annotations

import math

import numpy as np
from . import nystrom as ny

COV_NONE, COV_BOTH, COV_LEFT, COV_RIGHT = 0, 1, 2, 3
_GL8 = np.polynomial.legendre.leggauss(8)


# --------------------------------------------------------------------------
# change of variables (eq. cov) and panel geometry
# --------------------------------------------------------------------------
def cov(kind, s):
    """theta(s) and theta'(s) of eq. cov on [-1, 1]."""
    s = np.asarray(s, dtype=float)
    if kind == COV_NONE:
        return s.copy(), np.ones_like(s)
    if kind == COV_BOTH:
        a = 0.5 * math.pi * (1.0 - s)
        return np.cos(a), 0.5 * math.pi * np.sin(a)
    if kind == COV_LEFT:
        a = 0.25 * math.pi * (1.0 + s)
        return 1.0 - 2.0 * np.cos(a), 0.5 * math.pi * np.sin(a)
    if kind == COV_RIGHT:
        a = 0.25 * math.pi * (1.0 - s)
        return 2.0 * np.cos(a) - 1.0, 0.5 * math.pi * np.sin(a)
    raise ValueError("unknown change of variables")


def fejer_weights(phi):
    """w_i = int_{-1}^{1} l_i(s) ds for the nodes s_i = cos(phi_i), phi_i =
    (2i-1) pi / (2n) (Fejer's first rule, from int T_m = 2/(1-m^2), m even):
    w_i = (2/n) [1 - 2 sum_{m=1}^{n/2} cos(2 m phi_i) / (4 m^2 - 1)]."""
    n = phi.size
    m = np.arange(1, n // 2 + 1, dtype=float)
    return (2.0 / n) * (1.0 - 2.0 * (np.cos(np.outer(phi, 2.0 * m))
                                     @ (1.0 / (4.0 * m * m - 1.0))))


class PanelArc:
    """An arc cut at ``breaks`` (t values, -1 = t_0 < ... < t_P = 1) into
    panels with change-of-variables kinds ``kinds`` and n nodes each."""

    def __init__(self, curve, n, breaks=(-1.0, 1.0), kinds=None):
        self.curve = curve
        self.n = int(n)
        self.breaks = np.asarray(breaks, dtype=float)
        self.P = self.breaks.size - 1
        self.kinds = list(kinds) if kinds is not None else [COV_BOTH] * self.P
        phi, s = ny.cheb_nodes(self.n)
        self.phi, self.s = phi, s
        self.w1 = fejer_weights(phi)

    def t_of(self, p, s):
        """Arc parameter t and dt/ds of panel p at s."""
        th, dth = cov(self.kinds[p], s)
        a, b = self.breaks[p], self.breaks[p + 1]
        return 0.5 * (a + b) + 0.5 * (b - a) * th, 0.5 * (b - a) * dth

    def y(self, p, s):
        t, _ = self.t_of(p, s)
        return self.curve.x(t)

    def dt(self, p, s, s0):
        """t(s) - t(s0) on panel p without cancellation: the cosine maps'
        differences are formed as products of sines
        (cos a - cos b = -2 sin((a+b)/2) sin((a-b)/2))."""
        s = np.asarray(s, dtype=float)
        kind = self.kinds[p]
        h = 0.5 * (self.breaks[p + 1] - self.breaks[p])
        if kind == COV_NONE:
            return h * (s - s0)
        if kind == COV_BOTH:
            a, a0, f = 0.5 * math.pi * (1.0 - s), 0.5 * math.pi * (1.0 - s0), 1.0
        elif kind == COV_LEFT:
            a, a0, f = 0.25 * math.pi * (1.0 + s), 0.25 * math.pi * (1.0 + s0), -2.0
        else:
            a, a0, f = 0.25 * math.pi * (1.0 - s), 0.25 * math.pi * (1.0 - s0), 2.0
        return h * f * (-2.0 * np.sin(0.5 * (a + a0)) * np.sin(0.5 * (a - a0)))

    def ydiff(self, p, s, s0):
        """x(t(s)) - x(t(s0)) on panel p: for |t - t0| < 0.05 as
        (t - t0) times the mean of x' over [t0, t] (8-point Gauss-Legendre),
        which keeps full relative precision for nearby points; else by
        subtraction."""
        s = np.asarray(s, dtype=float)
        t0, _ = self.t_of(p, np.array([s0]))
        d = self.dt(p, s, s0)
        out = self.y(p, s) - self.curve.x(t0)[0]
        small = np.abs(d) < 0.05
        if np.any(small):
            g, w = _GL8
            ds = d[small]
            tt = t0[0] + np.outer(ds, 0.5 * (g + 1.0))
            xd = self.curve.dx(tt.ravel()).reshape(tt.shape + (2,))
            out[small] = ds[:, None] * np.einsum("mqk,q->mk", xd, 0.5 * w)
        return out

    def speed(self, p, s):
        """|dx/ds| on panel p."""
        t, dt = self.t_of(p, s)
        d = self.curve.dx(t)
        return np.hypot(d[..., 0], d[..., 1]) * np.abs(dt)

    def nodes(self):
        """Node dictionary: arc parameters t, positions y, Fejer weights w,
        panel index, and (for overlap bookkeeping) n = total node count."""
        t = np.concatenate([self.t_of(p, self.s)[0] for p in range(self.P)])
        y = np.concatenate([self.y(p, self.s) for p in range(self.P)])
        w = np.tile(self.w1, self.P)
        pan = np.repeat(np.arange(self.P), self.n)
        return dict(t=t, y=y, w=w, panel=pan, n=self.P * self.n, arc=self)


# --------------------------------------------------------------------------
# frequency-independent log table
# --------------------------------------------------------------------------
def _coef_matrix(phi):
    """C[m, j] with l_j(cos p) = sum_m C[m, j] cos(m p)."""
    n = phi.size
    C = np.cos(np.outer(np.arange(n), phi)) * (2.0 / n)
    C[0] *= 0.5
    return C


def chebyshev_T(s, n):
    """[T_0(s), ..., T_{n-1}(s)] for points s in [-1, 1] (three-term
    recurrence), shape [len(s), n]."""
    s = np.asarray(s, dtype=float)
    T = np.empty((s.size, n))
    T[:, 0] = 1.0
    if n > 1:
        T[:, 1] = s
    for k in range(2, n):
        T[:, k] = 2.0 * s * T[:, k - 1] - T[:, k - 2]
    return T


def adaptive_gl_vec(f, a, b, breaks=(), tol=1e-14, order=16, max_rounds=200):
    """Integral over [a, b] of a vector-valued function f (f maps an array of
    points [q] to values [q, m]).  Each interval is integrated by an
    ``order``-point Gauss-Legendre rule on the whole and on its two halves
    and accepted when the two agree to its share of ``tol`` in the max norm
    (or to 1e-3 tol, which ends the bisection next to an integrable end
    singularity), else bisected; ``breaks`` split the interval up front.
    Bisection also stops at width 1e-12 (span): next to a log singularity
    the rule's error there is ~1e-15, while narrower intervals would place
    nodes within rounding of the singular point."""
    g, w = np.polynomial.legendre.leggauss(order)
    pts = sorted({a, b, *[p for p in breaks if a < p < b]})
    lo = np.array(pts[:-1], dtype=float)
    hi = np.array(pts[1:], dtype=float)
    span = b - a

    def rule(l, h):
        c, r = 0.5 * (l + h), 0.5 * (h - l)
        x = c[:, None] + r[:, None] * g[None, :]
        fx = f(x.ravel())
        fx = fx.reshape(x.shape + fx.shape[1:])
        return np.einsum("iq...,q->i...", fx, w) * r.reshape((-1,) + (1,) * (fx.ndim - 2))

    total = 0.0
    whole = rule(lo, hi)
    for _ in range(max_rounds):
        if lo.size == 0:
            return total
        mid = 0.5 * (lo + hi)
        left, right = rule(lo, mid), rule(mid, hi)
        halves = left + right
        err = np.abs(halves - whole).reshape(lo.size, -1).max(axis=1)
        ok = (err <= tol * (hi - lo) / span) | (err <= 1e-3 * tol)
        ok |= (hi - lo) <= 1e-12 * span
        total = total + halves[ok].sum(axis=0)
        # the halves of a bisected interval are its children's whole rules
        lo, hi, mid = lo[~ok], hi[~ok], mid[~ok]
        whole = np.concatenate([left[~ok], right[~ok]])
        lo, hi = np.concatenate([lo, mid]), np.concatenate([mid, hi])
    raise RuntimeError("adaptive_gl_vec: no convergence")


def log_table(arc, tol=1e-14, rows=None):
    """W_ij = int_{panel(j)} log|y_i - y(s)| l_j(s) ds for every node i of
    the arc and node j: adaptive Gauss-Legendre quadrature of the vector of
    Chebyshev moments int log|y_i - y(s)| T_m(s) ds, split at the target
    when it lies on the panel, then l_j = sum_m C[m, j] T_m (``rows``: only
    those rows; the others are NaN).  On the
    target's own panel the distances come from ``PanelArc.ydiff``: where the
    cosine maps cluster the nodes, plain subtraction of nearly equal points
    would lose ~1e-10 of the table."""
    nd = arc.nodes()
    N, n = nd["n"], arc.n
    C = _coef_matrix(arc.phi)
    W = np.full((N, N), np.nan)
    for i in (range(N) if rows is None else rows):
        yi = nd["y"][i]
        for p in range(arc.P):

            own = nd["panel"][i] == p
            si = float(arc.s[i % n])

            def f(s, p=p, yi=yi, own=own, si=si):
                if own:
                    d = arc.ydiff(p, s, si)
                else:
                    d = arc.y(p, s) - yi
                r = np.hypot(d[:, 0], d[:, 1])
                return np.log(np.maximum(r, 1e-300))[:, None] * chebyshev_T(s, n)

            brk = (si,) if own else ()
            W[i, p * n:(p + 1) * n] = adaptive_gl_vec(f, -1.0, 1.0, brk, tol) @ C
    return W


# --------------------------------------------------------------------------
# matrix, field
# --------------------------------------------------------------------------
def smooth_part(k, r):
    """S(r) = Phi_k(r) + J0(k r) log(r) / (2 pi) for r > 0."""
    return ny.fundamental(k, r) + ny.bessel_j0(k * r) * np.log(r) / (2.0 * math.pi)


def assemble(nodes, k, W):
    """A_ij = -(1/2pi) J0(k r_ij) W_ij + w_j S(r_ij), S(0) on the diagonal."""
    y, w = nodes["y"], nodes["w"]
    N = y.shape[0]
    r = np.hypot(y[:, None, 0] - y[None, :, 0], y[:, None, 1] - y[None, :, 1])
    off = ~np.eye(N, dtype=bool)
    J0 = np.ones((N, N), dtype=complex)
    S = np.full((N, N), 0.25j - (ny.EULER_GAMMA + np.log(k / 2.0)) / (2.0 * math.pi),
                dtype=complex)
    J0[off] = ny.bessel_j0(k * r[off])
    S[off] = smooth_part(k, r[off])
    return -J0 * W / (2.0 * math.pi) + S * w[None, :]


def panel_coeffs(arc, mu):
    """Chebyshev coefficients of each panel's interpolant of mu, [P, n]."""
    C = _coef_matrix(arc.phi)
    return np.stack([C @ mu[p * arc.n:(p + 1) * arc.n] for p in range(arc.P)])


def near_radius(nodes):
    """10 x the largest distance between nodes adjacent along the arc (in
    order of the arc parameter t; within a panel the node order runs
    against t, and consecutive panels follow each other)."""
    return ny.NEAR_FACTOR * ny.max_spacing(nodes["y"][np.argsort(nodes["t"])])


def field(k, z, nodes, mu, tol_rel=1e-14):
    """Single-layer potential of the panel densities at targets z [P, 2]."""
    arc = nodes["arc"]
    z = np.atleast_2d(np.asarray(z, dtype=float))
    y, w = nodes["y"], nodes["w"]
    r = np.hypot(z[:, None, 0] - y[None, :, 0], z[:, None, 1] - y[None, :, 1])
    near = np.min(r, axis=1) < near_radius(nodes)
    out = np.empty(z.shape[0], dtype=complex)
    if np.any(~near):
        out[~near] = ny.fundamental(k, r[~near]) @ (w * mu)
    if np.any(near):
        a = panel_coeffs(arc, mu)
        for q in np.nonzero(near)[0]:
            out[q] = sum(_panel_near(k, z[q], arc, p, a[p], tol_rel)
                         for p in range(arc.P))
    return out


def _panel_near(k, zq, arc, p, a, tol_rel):
    """int_0^pi Phi_k(z, y_p(cos t)) mu_N(cos t) sin t dt, split at the
    panel point nearest z."""
    ph = np.linspace(0.0, math.pi, 4001)
    pts = arc.y(p, np.cos(ph))
    i = int(np.argmin(np.hypot(pts[:, 0] - zq[0], pts[:, 1] - zq[1])))
    brk = (float(ph[i]),)

    def f(t):
        x = arc.y(p, np.cos(t))
        r = np.hypot(x[:, 0] - zq[0], x[:, 1] - zq[1])
        return ny.fundamental(k, r) * ny.density_at(a, t) * np.sin(t)

    return ny.adaptive_gl(f, 0.0, math.pi, breaks=brk, tol_rel=tol_rel)


def density_per_length(arc, mu):
    """psi at the nodes: mu / |dx/ds|."""
    sp = np.concatenate([arc.speed(p, arc.s) for p in range(arc.P)])
    return mu / sp
