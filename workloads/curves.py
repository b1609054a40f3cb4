"""Parametrised arcs x(t), t in [-1, 1], and their derivatives dx/dt.

These are geometry *inputs*.  Each curve object is a plain description of a
smooth open arc; callers sample it wherever they need (the oracle samples it
at its own nodes and at quadrature points, the GPU path samples it at the
nodes the library reports).  Every method is vectorised over ``t``.

Shapes follow the paper's examples (Section 5) and the synthetic workloads
built on them: straight segments, circular arcs (the disc of Geometry 1 and
the circular cavity of Geometry 5), sub-arcs of a kite-shaped closed curve,
ellipse segments and sine-perturbed segments.
"""
from __future__ import annotations

import math
import numpy as np


class Curve:
    """Smooth open arc on the reference interval [-1, 1].

    Subclasses implement ``x(t)`` and ``dx(t)`` returning arrays of shape
    ``t.shape + (2,)``.  ``parent`` optionally names the closed curve the arc
    was cut from and ``interval`` its parameter interval on that curve (used
    to decide overlap membership in multi-arc problems).
    """

    parent: str | None = None
    interval: tuple[float, float] | None = None

    def x(self, t):  # pragma: no cover - abstract
        raise NotImplementedError

    def dx(self, t):  # pragma: no cover - abstract
        raise NotImplementedError

    def parent_param(self, t):
        """Parameter on the parent closed curve of the point x(t)."""
        a, b = self.interval
        t = np.asarray(t, dtype=float)
        return 0.5 * (a + b) + 0.5 * (b - a) * t

    def length(self, n: int = 200) -> float:
        """Arc length by Gauss-Legendre quadrature of |x'(t)| (input helper)."""
        g, w = np.polynomial.legendre.leggauss(n)
        d = self.dx(g)
        return float(np.sum(w * np.hypot(d[..., 0], d[..., 1])))


def _stack(a, b):
    return np.stack(np.broadcast_arrays(a, b), axis=-1)


class Segment(Curve):
    """Straight segment from A (t = -1) to B (t = +1)."""

    def __init__(self, A, B):
        self.A = np.asarray(A, dtype=float)
        self.B = np.asarray(B, dtype=float)

    def x(self, t):
        t = np.asarray(t, dtype=float)[..., None]
        return 0.5 * (1.0 - t) * self.A + 0.5 * (1.0 + t) * self.B

    def dx(self, t):
        t = np.asarray(t, dtype=float)
        return np.broadcast_to(0.5 * (self.B - self.A), t.shape + (2,)).copy()


class CircularArc(Curve):
    """Circle of radius R about ``center``, polar angle from ``a`` to ``b``."""

    def __init__(self, R, a, b, center=(0.0, 0.0)):
        self.R = float(R)
        self.a = float(a)
        self.b = float(b)
        self.c = np.asarray(center, dtype=float)
        self.parent = "circle"
        self.interval = (self.a, self.b)

    def x(self, t):
        tau = self.parent_param(t)
        return self.c + self.R * _stack(np.cos(tau), np.sin(tau))

    def dx(self, t):
        tau = self.parent_param(t)
        h = 0.5 * (self.b - self.a)
        return self.R * h * _stack(-np.sin(tau), np.cos(tau))


def kite_point(tau, scale=1.0, center=(0.0, 0.0), rot=0.0):
    """Kite curve (cos t + 0.65 cos 2t - 0.65, 1.5 sin t), scaled/rotated."""
    tau = np.asarray(tau, dtype=float)
    px = np.cos(tau) + 0.65 * np.cos(2.0 * tau) - 0.65
    py = 1.5 * np.sin(tau)
    c, s = math.cos(rot), math.sin(rot)
    return _stack(center[0] + scale * (c * px - s * py),
                  center[1] + scale * (s * px + c * py))


def kite_deriv(tau, scale=1.0, rot=0.0):
    tau = np.asarray(tau, dtype=float)
    dx = -np.sin(tau) - 1.3 * np.sin(2.0 * tau)
    dy = 1.5 * np.cos(tau)
    c, s = math.cos(rot), math.sin(rot)
    return _stack(scale * (c * dx - s * dy), scale * (s * dx + c * dy))


class KiteArc(Curve):
    """Sub-arc of the kite over parent parameter interval [a, b] (radians)."""

    def __init__(self, a, b, scale=1.0, center=(0.0, 0.0), rot=0.0):
        self.a = float(a)
        self.b = float(b)
        self.scale = float(scale)
        self.center = tuple(float(v) for v in center)
        self.rot = float(rot)
        self.parent = "kite"
        self.interval = (self.a, self.b)

    def x(self, t):
        return kite_point(self.parent_param(t), self.scale, self.center,
                          self.rot)

    def dx(self, t):
        h = 0.5 * (self.b - self.a)
        return h * kite_deriv(self.parent_param(t), self.scale, self.rot)


class EllipseArc(Curve):
    """Ellipse (a cos s, b sin s), rotated by ``rot`` about ``center``,
    parent parameter s from ``s0`` to ``s1``."""

    def __init__(self, a, b, s0, s1, center=(0.0, 0.0), rot=0.0):
        self.ea = float(a)
        self.eb = float(b)
        self.a = float(s0)
        self.b = float(s1)
        self.center = np.asarray(center, dtype=float)
        self.rot = float(rot)
        self.parent = "ellipse"
        self.interval = (self.a, self.b)

    def _rot(self, px, py):
        c, s = math.cos(self.rot), math.sin(self.rot)
        return _stack(c * px - s * py, s * px + c * py)

    def x(self, t):
        s = self.parent_param(t)
        return self.center + self._rot(self.ea * np.cos(s),
                                       self.eb * np.sin(s))

    def dx(self, t):
        s = self.parent_param(t)
        h = 0.5 * (self.b - self.a)
        return h * self._rot(-self.ea * np.sin(s), self.eb * np.cos(s))


class SineArc(Curve):
    """Segment of chord length ``ell`` from ``p0`` in direction ``angle`` with
    a normal offset amp * sin(pi * nu * (1 + t))."""

    def __init__(self, p0, ell, amp, nu, angle):
        self.p0 = np.asarray(p0, dtype=float)
        self.ell = float(ell)
        self.amp = float(amp)
        self.nu = int(nu)
        self.e = np.array([math.cos(angle), math.sin(angle)])
        self.n = np.array([-math.sin(angle), math.cos(angle)])

    def x(self, t):
        t = np.asarray(t, dtype=float)[..., None]
        off = self.amp * np.sin(np.pi * self.nu * (1.0 + t))
        return self.p0 + 0.5 * (1.0 + t) * self.ell * self.e + off * self.n

    def dx(self, t):
        t = np.asarray(t, dtype=float)[..., None]
        doff = self.amp * np.pi * self.nu * np.cos(np.pi * self.nu * (1.0 + t))
        return 0.5 * self.ell * self.e + doff * self.n


class ClosedCurve:
    """Smooth closed curve x(tau), tau in [0, 2 pi), counter-clockwise, with
    first and second derivatives (inputs for closed patches; vectorised)."""

    closed = True
    interval = (0.0, 2.0 * math.pi)

    def x(self, tau):  # pragma: no cover - abstract
        raise NotImplementedError

    def dx(self, tau):  # pragma: no cover - abstract
        raise NotImplementedError

    def ddx(self, tau):  # pragma: no cover - abstract
        raise NotImplementedError

    def parent_param(self, tau):
        return np.asarray(tau, dtype=float)


class ClosedEllipse(ClosedCurve):
    """(a cos tau, b sin tau) rotated by ``rot`` about ``center``."""

    def __init__(self, a, b, center=(0.0, 0.0), rot=0.0):
        self.ea, self.eb = float(a), float(b)
        self.center = np.asarray(center, dtype=float)
        self.rot = float(rot)

    def _rot(self, px, py):
        c, s = math.cos(self.rot), math.sin(self.rot)
        return _stack(c * px - s * py, s * px + c * py)

    def x(self, tau):
        tau = np.asarray(tau, dtype=float)
        return self.center + self._rot(self.ea * np.cos(tau), self.eb * np.sin(tau))

    def dx(self, tau):
        tau = np.asarray(tau, dtype=float)
        return self._rot(-self.ea * np.sin(tau), self.eb * np.cos(tau))

    def ddx(self, tau):
        tau = np.asarray(tau, dtype=float)
        return self._rot(-self.ea * np.cos(tau), -self.eb * np.sin(tau))


class ClosedKite(ClosedCurve):
    """The kite (cos t + 0.65 cos 2t - 0.65, 1.5 sin t), scaled, rotated and
    shifted."""

    def __init__(self, scale=1.0, center=(0.0, 0.0), rot=0.0):
        self.scale = float(scale)
        self.center = tuple(float(v) for v in center)
        self.rot = float(rot)

    def x(self, tau):
        return kite_point(tau, self.scale, self.center, self.rot)

    def dx(self, tau):
        return kite_deriv(tau, self.scale, self.rot)

    def ddx(self, tau):
        tau = np.asarray(tau, dtype=float)
        px = -np.cos(tau) - 2.6 * np.cos(2.0 * tau)
        py = -1.5 * np.sin(tau)
        c, s = math.cos(self.rot), math.sin(self.rot)
        return _stack(self.scale * (c * px - s * py), self.scale * (s * px + c * py))
