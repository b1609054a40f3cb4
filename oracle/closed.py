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


def near_limit(nd, factor=5.0):
    """Targets closer than this to a node are outside the trapezoid rule's
    accuracy (error ~ exp(-2 pi d / h))."""
    y = nd["y"]
    h = np.hypot(*(np.roll(y, -1, axis=0) - y).T)
    return factor * float(h.max())
