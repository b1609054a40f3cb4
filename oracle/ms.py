"""Oracle: the multiple-scattering (MS) recursion in the frequency domain.

Test infrastructure only (see the package header).

Paper passages (Section 3.1):
  * window eta(t; t0, t1) .................................. eq. eta
  * POU chi_j on the patches, c0 = 1/3, c1 = 2/3 ............ eqs. POU1, POU2
  * g_{j,1} = -chi_j u^i;  g_{j,m+1} = -chi_j sum_{k != j} v~_{k,j,m}
    ........................................ eqs. criterion_int1/2 (Def. 3.x)
  * v~_{k,j,m} = 0 on the overlap of Gamma_j with an adjacent Gamma_k,
    v_{k,m} elsewhere ........................................ eq. vtilde
  * u_M = sum_{m<=M} sum_j v_{j,m} ......................... eq. mult-scatt-int

Readings taken where the text is silent or loose:
  * With a single time window the windows chi_j and the masking in vtilde are
    time-independent linear maps, so they commute with the Fourier transform;
    the recursion is run per frequency on boundary data G and densities.
  * d^ov(x) ("diameter of the arc joining x and the endpoint") is the chord
    |x - x_end| and A^ov is the chord between the two ends of the overlap.
  * Overlap membership of a node is decided by the parent-curve parameter
    interval of each arc, not by geometric distance.
  * The second line of eq. vtilde ("k = j-1 and k = j+1") means "or".
  * Several closed curves (the exterior problem of Section 3.3): every arc
    scatters onto every other one; the masking of eq. vtilde and the
    windows chi_j involve the neighbours on the same curve only, and an arc
    alone on its curve has chi = 1.
  * A closed curve may also be one patch of its own (Section 3.3): its
    density solves the combined-field equation and its field is
    (D - i eta S) Psi (``oracle.closed``); chi = 1 and nothing is masked.
    Targets of that field closer than five node spacings (another patch's
    nodes) take the adaptive integral over the curve of the density's
    trigonometric interpolant, the trapezoid rule's accuracy being lost
    there.
  * Discretisation: ``problem.scheme`` "cheb" is the single-panel
    weighted-Chebyshev scheme (``oracle.nystrom``); "panels" cuts each arc
    at the ends of its truncated overlap into three panels, each with the
    two-sided change of variables of eq. cov (``oracle.panels``), n nodes per
    panel.
"""
from __future__ import annotations

import math

import numpy as np

from . import closed as cl
from . import nystrom as ny
from . import panels as pn
from .incident import incident


def eta(t, t0, t1):
    """C-infinity cutoff: 1 for |t| <= t0, exp(2 e^{-1/s} / (s - 1)) with
    s = (|t| - t0)/(t1 - t0) between, 0 for |t| >= t1."""
    t = np.abs(np.asarray(t, dtype=float))
    out = np.zeros_like(t)
    out[t <= t0] = 1.0
    mid = (t > t0) & (t < t1)
    s = (t[mid] - t0) / (t1 - t0)
    out[mid] = np.exp(2.0 * np.exp(-1.0 / s) / (s - 1.0))
    return out


def in_interval(tau, a, b, period):
    """Parent parameter tau lies strictly inside (a, b) modulo period."""
    u = np.mod(np.asarray(tau, dtype=float) - a, period)
    return (u > 0.0) & (u < (b - a))


class Layout:
    """Node sets, overlap membership and POU values of cyclic partitions of
    one or several closed curves."""

    def __init__(self, problem):
        self.p = problem
        self.arcs = [a.curve for a in problem.arcs]
        self.J = len(self.arcs)
        self.group = [getattr(a, "group", 0) for a in problem.arcs]
        # cyclic neighbours on the same curve (None for an arc alone)
        self.nxt, self.prv = [None] * self.J, [None] * self.J
        for j in range(self.J):
            mem = [i for i in range(self.J) if self.group[i] == self.group[j]]
            if len(mem) > 1:
                q = mem.index(j)
                self.nxt[j] = mem[(q + 1) % len(mem)]
                self.prv[j] = mem[(q - 1) % len(mem)]
        self.scheme = getattr(problem, "scheme", "cheb")
        self.closed = [bool(getattr(a.curve, "closed", False)) for a in problem.arcs]
        for j in range(self.J):
            if self.closed[j] and self.nxt[j] is not None:
                raise ValueError("a closed patch is alone on its curve")
        self.nodes = []
        self.parcs = [None] * self.J
        for j, a in enumerate(problem.arcs):
            if self.closed[j]:
                nd = cl.nodes(a.curve, a.n)
                nd["t"] = nd["tau"]
            elif self.scheme == "panels":
                self.parcs[j] = pn.PanelArc(a.curve, a.n, self.panel_breaks(j))
                nd = self.parcs[j].nodes()
            else:
                nd = ny.arc_nodes(a.curve, a.n)
            self.nodes.append(nd)
        self._tables = {}
        self.tau = [c.parent_param(nd["t"]) for c, nd in zip(self.arcs,
                                                              self.nodes)]
        self.chi = [self._chi(j) for j in range(self.J)]
        # mask[k][j][i] = 0 where node i of arc j lies on adjacent arc k
        self.mask = [[None] * self.J for _ in range(self.J)]
        for j in range(self.J):
            for k in range(self.J):
                if k == j:
                    continue
                m = np.ones(self.nodes[j]["n"], dtype=bool)
                if k in (self.prv[j], self.nxt[j]):
                    a, b = self.arcs[k].interval
                    m &= ~in_interval(self.tau[j], a, b, problem.period)
                self.mask[k][j] = m

    def panel_breaks(self, j):
        """Breakpoints (arc parameter t) of arc j: its ends and the ends of
        its truncated overlap, where the overlaps with the neighbours on the
        same curve end."""
        br = [-1.0, 1.0]
        if self.nxt[j] is not None:
            a, b = self.arcs[j].interval
            for e in (self.arcs[self.prv[j]].interval[1], self.arcs[self.nxt[j]].interval[0]):
                u = (e - a) % self.p.period
                if 0.0 < u < b - a:
                    br.append(-1.0 + 2.0 * u / (b - a))
        return sorted(br)

    def assemble(self, j, k):
        """Matrix of arc j at wavenumber k in the problem's scheme."""
        if self.closed[j]:
            return cl.assemble(self.nodes[j], k)
        if self.scheme == "panels":
            if j not in self._tables:
                self._tables[j] = pn.log_table(self.parcs[j])
            return pn.assemble(self.nodes[j], k, self._tables[j])
        return ny.assemble(self.nodes[j], k)

    def field(self, j, k, z, alpha):
        """Potential of arc j's density at targets z."""
        if self.closed[j]:
            # the trapezoid rule where it is accurate (five node spacings and
            # more from every node), the adaptive integral over the curve nearer
            nd = self.nodes[j]
            z = np.atleast_2d(np.asarray(z, dtype=float))
            out = cl.field(k, z, nd, alpha)
            d = np.min(np.hypot(z[:, None, 0] - nd["y"][None, :, 0],
                                z[:, None, 1] - nd["y"][None, :, 1]), axis=1)
            near = d < cl.near_limit(nd)
            if np.any(near):
                out[near] = cl.field_near(k, z[near], self.arcs[j], nd, alpha)
            return out
        if self.scheme == "panels":
            return pn.field(k, z, self.nodes[j], alpha)
        return ny.field(k, z, self.arcs[j], self.nodes[j], alpha)

    def _chi(self, j):
        return self.chi_at(j, self.tau[j], self.nodes[j]["y"])

    def chi_at(self, j, tau, y):
        """chi_j (eq. POU1) at points y of the closed curve with parent
        parameters tau; zero off Gamma_j."""
        p = self.p
        nxt, prv = self.nxt[j], self.prv[j]
        c = self.arcs[j]
        if nxt is None:
            return np.ones(np.shape(tau))
        a0, b0 = c.interval
        chi = np.where(in_interval(tau, a0, b0, p.period), 1.0, 0.0)
        # overlap with the next arc: eta(A - d; c0 A, c1 A), d = chord to
        # the end point of Gamma_j inside that overlap
        xe = c.x(np.array([1.0]))[0]
        xs = self.arcs[nxt].x(np.array([-1.0]))[0]
        A = math.hypot(*(xs - xe))
        a, b = self.arcs[nxt].interval
        on = in_interval(tau, a, b, p.period) & (chi > 0)
        xs0 = c.x(np.array([-1.0]))[0]
        if nxt == prv:
            # two arcs on a curve overlap at both ends: the nearer end decides
            on &= (np.hypot(y[:, 0] - xe[0], y[:, 1] - xe[1])
                   <= np.hypot(y[:, 0] - xs0[0], y[:, 1] - xs0[1]))
        d = np.hypot(y[on, 0] - xe[0], y[on, 1] - xe[1])
        chi[on] = eta(A - d, p.c0 * A, p.c1 * A)
        # overlap with the previous arc: 1 - eta(A' - d'; c0 A', c1 A'),
        # d' = chord to the end point of Gamma_{j-1} inside that overlap
        xe2 = self.arcs[prv].x(np.array([1.0]))[0]
        xs2 = c.x(np.array([-1.0]))[0]
        A2 = math.hypot(*(xs2 - xe2))
        a2, b2 = self.arcs[prv].interval
        on2 = in_interval(tau, a2, b2, p.period) & (chi > 0) & ~on
        d2 = np.hypot(y[on2, 0] - xe2[0], y[on2, 1] - xe2[1])
        chi[on2] = 1.0 - eta(A2 - d2, p.c0 * A2, p.c1 * A2)
        return chi

    def delta_min(self, samples=4000):
        """delta_min = min_j dist(Gamma_j^tr, Gamma minus Gamma_j) (eq. dist),
        from dense samples of the arcs; Gamma_j^tr is where chi_j > 0."""
        best = np.inf
        pts, taus = [], []
        for c in self.arcs:
            t = np.linspace(-1.0, 1.0, samples)
            pts.append(c.x(t))
            taus.append(c.parent_param(t))
        for j, c in enumerate(self.arcs):
            chi = self.chi_at(j, taus[j], pts[j])
            tr = pts[j][chi > 0]
            a, b = c.interval
            for k in range(self.J):
                if k == j:
                    continue
                if self.group[k] == self.group[j]:
                    out = ~in_interval(taus[k], a, b, self.p.period)
                else:
                    out = np.ones(taus[k].shape, dtype=bool)
                q = pts[k][out]
                if q.shape[0] == 0 or tr.shape[0] == 0:
                    continue
                d = np.hypot(tr[:, None, 0] - q[None, ::4, 0],
                             tr[:, None, 1] - q[None, ::4, 1])
                best = min(best, float(d.min()))
        return best


def run_frequency(layout, k, keep_steps=False):
    """MS recursion at one wavenumber.  Returns the summed densities
    alpha_tot[j], the field U_M at the observation points and (optionally)
    every step's right-hand sides, densities and cross-arc fields."""
    p, J = layout.p, layout.J
    nodes = layout.nodes
    A = [layout.assemble(j, k) for j in range(J)]
    b = [-layout.chi[j] * incident(p.incident, k, nodes[j]["y"])
         for j in range(J)]
    alpha = [ny.solve(A[j], b[j]) for j in range(J)]
    tot = [a.copy() for a in alpha]
    steps = []
    for m in range(1, p.M):
        cross = [np.zeros(nodes[j]["n"], dtype=complex) for j in range(J)]
        for j in range(J):
            for kk in range(J):
                if kk == j:
                    continue
                msk = layout.mask[kk][j]
                tgt = nodes[j]["y"][msk]
                if tgt.shape[0]:
                    cross[j][msk] += layout.field(kk, k, tgt, alpha[kk])
        if keep_steps:
            steps.append(dict(b=b, alpha=alpha, cross=cross))
        b = [-layout.chi[j] * cross[j] for j in range(J)]
        alpha = [ny.solve(A[j], b[j]) for j in range(J)]
        for j in range(J):
            tot[j] += alpha[j]
    if keep_steps:
        steps.append(dict(b=b, alpha=alpha, cross=None))
    U = np.zeros(p.obs.shape[0], dtype=complex)
    for j in range(J):
        U += layout.field(j, k, p.obs, tot[j])
    return dict(alpha_tot=tot, U=U, steps=steps)


def run_traces(layout, omegas, weights, times, stop_tol=0.0):
    """Time traces of the MS sum at the observation points with the stop rule
    of the series in the time domain (reading of the 'update norm' stop: the
    increment of step m, F^{-1}[U of that step's densities] over all points
    and times, relative to the sum so far).  The recursion runs per frequency
    (eqs. criterion_int1/2, vtilde), each step's field is transformed with
    the trapezoid rule (eq. TDsol-interior), and the sum stops after the
    first step m with |u_m - u_{m-1}| <= stop_tol |u_m| or after M steps.
    Returns (traces [nt][nobs], steps taken)."""
    from .transform import freq_to_time
    p = layout.p
    nobs = p.obs.shape[0]
    per = np.zeros((p.M, len(omegas), nobs), dtype=complex)
    for l, k in enumerate(omegas):
        out = run_frequency(layout, k, keep_steps=True)
        for m, st in enumerate(out["steps"]):
            for j in range(layout.J):
                per[m, l] += layout.field(j, k, p.obs, st["alpha"][j])
    u = np.zeros((len(times), nobs), dtype=complex)
    for m in range(p.M):
        du = freq_to_time(omegas, weights, per[m], times)
        u = u + du
        if stop_tol > 0.0 and np.linalg.norm(du) <= stop_tol * np.linalg.norm(u):
            return u, m + 1
    return u, p.M
