"""Oracle: a closed curve as one patch with the combined-field equation.

Test infrastructure only (see the package header).

What is discretised (Section 3.3, eqs. FDsolk-closed / FDBIEk-closed): on a
closed curve Gamma the density Psi solves
    (1/2 I + K - i eta V) Psi = G        on Gamma,
and the patch's field is  (D - i eta S) Psi  outside it, with the
fundamental solution Phi_k = (i/4) H0^(1)(k r), V / S the single-layer
operator / potential, K / D the double-layer ones (normal derivative in y,
outward normal).  Reading: eta = Re k (the paper asks Re eta != 0).

How: the Nystrom method for periodic integrands with a logarithmic
singularity that the paper cites for closed curves (CK98): x(tau) is
2pi-periodic and counter-clockwise; 2n nodes tau_j = pi j / n; each kernel
is split as L(t, tau) = L1(t, tau) log(4 sin^2((t - tau)/2)) + L2(t, tau)
with smooth L1, L2; the log part is integrated exactly against the
trigonometric interpolant,
    int_0^{2pi} log(4 sin^2((t - tau)/2)) f(tau) dtau ~ sum_j R_j(t) f(tau_j),
    R_j(t) = -(2pi/n) sum_{m=1}^{n-1} cos(m(t - tau_j))/m - (pi/n^2) cos(n(t - tau_j)),
(from int log(4 sin^2(s/2)) cos(m s) ds = -2pi/m, m >= 1, and 0 for m = 0),
the smooth part by the trapezoid rule (pi/n) sum_j.  In tau, with
q(t, tau) = x2'(tau)(x1(t) - x1(tau)) - x1'(tau)(x2(t) - x2(tau)) and
r = |x(t) - x(tau)|:
    K(t, tau) = (ik/4) H1(kr) q / r,         K1 = -(k/4pi) J1(kr) q / r,
    V(t, tau) = (i/4) H0(kr) |x'(tau)|,      V1 = -(1/4pi) J0(kr) |x'(tau)|,
and on the diagonal K1 = 0, K2 = (x2' x1'' - x1' x2'') / (4 pi |x'|^2),
V2 = |x'| (i/4 - (log(k |x'| / 2) + gamma) / (2 pi)).  The far field of a
patch is the trapezoid rule applied to (D - i eta S) Psi.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

from .nystrom import EULER_GAMMA


def nodes(curve, n2):
    """2n equispaced parameters tau_j = 2 pi j / (2n) and the geometry there."""
    if n2 % 2:
        raise ValueError("closed patches take an even number of nodes")
    tau = 2.0 * math.pi * np.arange(n2) / n2
    return dict(tau=tau, y=curve.x(tau), dy=curve.dx(tau), ddy=curve.ddx(tau), n=n2,
                closed=True)


def kress_weights(t, n2):
    """R[i, j] = R_j(t_i) of the logarithmic quadrature on the 2n nodes
    tau_j = pi j / n, at evaluation points t."""
    n = n2 // 2
    tau = math.pi * np.arange(n2) / n
    d = np.asarray(t, dtype=float)[:, None] - tau[None, :]
    m = np.arange(1, n)
    R = -(2.0 * math.pi / n) * np.einsum("ijm,m->ij", np.cos(d[:, :, None] * m), 1.0 / m)
    return R - (math.pi / n ** 2) * np.cos(n * d)


def eta_of(k):
    return float(np.real(k))


def assemble(nd, k, eta=None):
    """Nystrom matrix of 1/2 I + K - i eta V on the closed patch."""
    if eta is None:
        eta = eta_of(k)
    y, dy, ddy, tau, n2 = nd["y"], nd["dy"], nd["ddy"], nd["tau"], nd["n"]
    n = n2 // 2
    N = n2
    sp = np.hypot(dy[:, 0], dy[:, 1])
    dx1 = y[:, None, 0] - y[None, :, 0]
    dx2 = y[:, None, 1] - y[None, :, 1]
    r = np.hypot(dx1, dx2)
    q = dy[None, :, 1] * dx1 - dy[None, :, 0] * dx2
    off = ~np.eye(N, dtype=bool)
    L = np.zeros((N, N))
    L[off] = np.log(4.0 * np.sin(0.5 * (tau[:, None] - tau[None, :])[off]) ** 2)
    K = np.zeros((N, N), dtype=complex)
    K1 = np.zeros((N, N), dtype=complex)
    V = np.zeros((N, N), dtype=complex)
    V1 = np.zeros((N, N), dtype=complex)
    z = k * r[off]
    K[off] = 0.25j * k * special.hankel1(1, z) * q[off] / r[off]
    K1[off] = -(k / (4.0 * math.pi)) * special.jv(1, z) * q[off] / r[off]
    spj = np.broadcast_to(sp[None, :], (N, N))[off]
    V[off] = 0.25j * special.hankel1(0, z) * spj
    V1[off] = -special.jv(0, z) * spj / (4.0 * math.pi)
    K2 = K - K1 * L
    V2 = V - V1 * L
    d = np.arange(N)
    K2[d, d] = (dy[:, 1] * ddy[:, 0] - dy[:, 0] * ddy[:, 1]) / (4.0 * math.pi * sp ** 2)
    V1[d, d] = -sp / (4.0 * math.pi)
    V2[d, d] = sp * (0.25j - (np.log(k * sp / 2.0) + EULER_GAMMA) / (2.0 * math.pi))
    R = kress_weights(tau, n2)
    return (0.5 * np.eye(N) + R * (K1 - 1j * eta * V1)
            + (math.pi / n) * (K2 - 1j * eta * V2))


def field(k, z, nd, psi, eta=None):
    """(D - i eta S)[Psi] at targets z [P, 2] off the curve (trapezoid rule;
    accurate for targets a few node spacings away)."""
    if eta is None:
        eta = eta_of(k)
    z = np.atleast_2d(np.asarray(z, dtype=float))
    y, dy, n2 = nd["y"], nd["dy"], nd["n"]
    n = n2 // 2
    sp = np.hypot(dy[:, 0], dy[:, 1])
    e1 = z[:, None, 0] - y[None, :, 0]
    e2 = z[:, None, 1] - y[None, :, 1]
    r = np.hypot(e1, e2)
    q = dy[None, :, 1] * e1 - dy[None, :, 0] * e2
    kern = (0.25j * k * special.hankel1(1, k * r) * q / r
            - 1j * eta * 0.25j * special.hankel1(0, k * r) * sp[None, :])
    return (math.pi / n) * (kern @ psi)


def trig_interp(psi, tau):
    """The trigonometric interpolant of the 2n node values psi at parameters
    tau: sum_{|m| < n} c_m e^{i m tau} + c_n cos(n tau), c_m from the DFT of
    the samples (the unique interpolant of that degree, Nyquist term split
    evenly between +n and -n)."""
    psi = np.asarray(psi, dtype=complex)
    n2 = psi.size
    n = n2 // 2
    c = np.fft.fft(psi) / n2            # c[m] for m = 0..n2-1 (negative m wrapped)
    tau = np.atleast_1d(np.asarray(tau, dtype=float))
    m = np.arange(-n + 1, n)
    cm = c[m % n2]
    out = np.exp(1j * np.outer(tau, m)) @ cm
    return out + c[n] * np.cos(n * tau)


def closest_param(curve, z, tau0, h):
    """Parameter of the point of the curve closest to z near tau0: the best
    of 129 samples on [tau0 - h, tau0 + h], then golden-section search."""
    dist = lambda t: float(np.hypot(*(curve.x(np.array([t]))[0] - z)))
    ts = tau0 + h * np.linspace(-1.0, 1.0, 129)
    xs = curve.x(ts)
    i = int(np.argmin(np.hypot(xs[:, 0] - z[0], xs[:, 1] - z[1])))
    a, b = ts[max(i - 1, 0)], ts[min(i + 1, ts.size - 1)]
    g = 0.5 * (math.sqrt(5.0) - 1.0)
    for _ in range(60):
        c, d = b - g * (b - a), a + g * (b - a)
        if dist(c) < dist(d):
            b = d
        else:
            a = c
    return 0.5 * (a + b)


def field_near(k, z, curve, nd, psi, eta=None, order=24):
    """(D - i eta S)[Psi] at targets z [P, 2] at any distance off the curve:
    the integral over one period of the curve x(tau) itself of the kernel
    against the trigonometric interpolant of the node densities, by
    composite Gauss-Legendre quadrature (``order`` points a panel) on panels
    graded geometrically toward the parameter t* of the curve's closest
    point: [t* - delta, t* + delta], then [t* + 2^m delta, t* + 2^(m+1) delta]
    and their mirrors, delta = d / (2 |x'(t*)|), d the distance -- every
    panel as long as its distance to t*, so the kernel's near-singularity at
    distance d stays outside each panel's region of analyticity -- and, once
    they reach the node spacing h = 2 pi / N, panels of length h up to half a
    period each side (delta itself at most h / 2)."""
    if eta is None:
        eta = eta_of(k)
    z = np.atleast_2d(np.asarray(z, dtype=float))
    psi = np.asarray(psi, dtype=complex)
    n2 = psi.size
    n = n2 // 2
    c = np.fft.fft(psi) / n2
    m = np.arange(-n + 1, n)
    cm = c[m % n2]
    gx, gw = np.polynomial.legendre.leggauss(order)
    h = 2.0 * math.pi / n2
    out = np.zeros(z.shape[0], dtype=complex)
    for p in range(z.shape[0]):
        zz = z[p]
        j = int(np.argmin(np.hypot(nd["y"][:, 0] - zz[0], nd["y"][:, 1] - zz[1])))
        ts = closest_param(curve, zz, nd["tau"][j], h)
        d = float(np.hypot(*(curve.x(np.array([ts]))[0] - zz)))
        delta = min(max(0.5 * d / float(np.hypot(*curve.dx(np.array([ts]))[0])), 1e-12), 0.5 * h)
        edges = [delta]
        while edges[-1] < math.pi:
            # doubling, but no panel longer than the node spacing (the
            # interpolant oscillates at up to n / 2 periods a period)
            edges.append(min(2.0 * edges[-1], edges[-1] + h, math.pi))
        brk = np.concatenate([-np.array(edges[::-1]), np.array(edges)])
        lo, hi = brk[:-1], brk[1:]
        t = ts + (0.5 * (hi - lo)[:, None] * gx[None, :] + 0.5 * (hi + lo)[:, None]).ravel()
        w = (0.5 * (hi - lo)[:, None] * gw[None, :]).ravel()
        x, dx = curve.x(t), curve.dx(t)
        e1, e2 = zz[0] - x[:, 0], zz[1] - x[:, 1]
        r = np.hypot(e1, e2)
        q = dx[:, 1] * e1 - dx[:, 0] * e2
        sp = np.hypot(dx[:, 0], dx[:, 1])
        kern = (0.25j * k * special.hankel1(1, k * r) * q / r
                + 0.25 * eta * sp * special.hankel1(0, k * r))
        dens = np.exp(1j * np.outer(t, m)) @ cm + c[n] * np.cos(n * t)
        out[p] = np.sum(w * kern * dens)
    return out


def near_limit(nd, factor=5.0):
    """Targets closer than this to a node are outside the trapezoid rule's
    accuracy (error ~ exp(-2 pi d / h))."""
    y = nd["y"]
    h = np.hypot(*(np.roll(y, -1, axis=0) - y).T)
    return factor * float(h.max())
