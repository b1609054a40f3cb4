"""Seeded synthetic workloads.

Every workload is a plain description: arcs (curve objects plus node counts),
wavenumber lists, incident-field parameters, observation points and time
samples.  Speed of propagation is 1 throughout, so wavenumber k equals angular
frequency omega.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .curves import (Curve, Segment, CircularArc, KiteArc, EllipseArc,
                     SineArc, kite_point, ClosedEllipse, ClosedKite)


@dataclass
class IncidentSpec:
    """Incident field parameters (Section 5, the incident fields list).

    kind = "plane"   : exp(i k x.d), d = (cos theta, sin theta)
    kind = "gplane"  : Gaussian-modulated plane wave (u2)
    kind = "point"   : Gaussian-modulated point source (u1), amplitude 5i/2
    """
    kind: str
    theta: float = 0.0
    z0: tuple = (0.0, 0.0)
    omega0: float = 0.0
    sigma: float = 1.0
    tau0: float = 0.0


@dataclass
class ArcSpec:
    curve: Curve
    n: int
    group: int = 0  # closed curve (obstacle) the arc belongs to


@dataclass
class MSProblem:
    """Closed curves split into overlapping arcs.  The arcs of one curve
    (equal ``group``) are cyclically ordered in list order: arc j overlaps
    its predecessor and successor on the same curve only.  A problem with
    several groups is an exterior problem with several obstacles."""
    arcs: list
    incident: IncidentSpec
    omegas: np.ndarray
    M: int
    obs: np.ndarray
    times: np.ndarray
    c0: float = 1.0 / 3.0
    c1: float = 2.0 / 3.0
    period: float = 2.0 * math.pi
    name: str = ""
    # "cheb": one weighted-Chebyshev panel per arc, n nodes; "panels": each
    # arc cut at the ends of its truncated overlap, n nodes per panel
    scheme: str = "cheb"


def _circle_points(n, radius, center=(0.0, 0.0)):
    p = 2.0 * np.pi * np.arange(n) / n
    return np.stack([center[0] + radius * np.cos(p),
                     center[1] + radius * np.sin(p)], axis=-1)


def plain_segment_case(n=128, nk=64):
    """One straight arc (-1,0)-(1,0), plane wave at 30 degrees, k uniform in
    [0.5, 32], fields on 256 points of the radius-3 circle."""
    k = 0.5 + 31.5 * np.arange(nk) / (nk - 1)
    return dict(curve=Segment((-1.0, 0.0), (1.0, 0.0)), n=n, k=k,
                incident=IncidentSpec("plane", theta=math.pi / 6.0),
                obs=_circle_points(256, 3.0), name="segment_n%d_k%d" % (n, nk))


def fixed512_case(nk=4096, n=512):
    """Circular arc R = 1 spanning 2.5 rad, N = 512, k uniform in [1, 120],
    plane wave at 30 degrees, fields on the 256 radius-3 circle points."""
    k = 1.0 + 119.0 * np.arange(nk) / max(nk - 1, 1)
    return dict(curve=CircularArc(1.0, -1.25, 1.25), n=n, k=k,
                incident=IncidentSpec("plane", theta=math.pi / 6.0),
                obs=_circle_points(256, 3.0), name="arc512_k%d" % nk)


def _kite_arcs(n, scale=1.0, center=(0.0, 0.0), rot=0.0, group=0):
    d = math.pi / 180.0
    arcs = []
    for j in range(4):
        a = (90.0 * j - 15.0) * d
        b = (90.0 * (j + 1) + 15.0) * d
        arcs.append(ArcSpec(KiteArc(a, b, scale, center, rot), n, group))
    return arcs


def _ellipse_arcs(n, ea, eb, center=(0.0, 0.0), rot=0.0, group=0):
    """Ellipse split like the kite: 4 arcs of 120 degrees of parameter with
    30 degree overlaps."""
    d = math.pi / 180.0
    return [ArcSpec(EllipseArc(ea, eb, (90.0 * j - 15.0) * d, (90.0 * (j + 1) + 15.0) * d,
                               center=center, rot=rot), n, group) for j in range(4)]


def two_arc_exterior_case(n=24, nobs=8):
    """Two facing circular arcs (open scatterers, one per group) 2.5 apart,
    a Gaussian-modulated plane wave (omega0 = 6, sigma = 1.5, tau0 = 4), 37
    frequencies on [1.5, 10.5] resolving the time window [0, 14], and
    observation points on the radius-4 circle: the multiple-scattering series
    settles within a few steps in the time domain."""
    arcs = [ArcSpec(CircularArc(0.8, 2.2, 4.1, center=(-1.3, 0.0)), n, 0),
            ArcSpec(CircularArc(0.7, -0.9, 0.9, center=(1.2, 0.2)), n, 1)]
    return MSProblem(arcs=arcs,
                     incident=IncidentSpec("gplane", theta=0.3, omega0=6.0, sigma=1.5,
                                           tau0=4.0),
                     omegas=np.arange(1.5, 10.51, 0.25), M=10,
                     obs=_circle_points(nobs, 4.0), times=np.linspace(0.0, 14.0, 57),
                     name="two_arcs_n%d" % n)


def two_obstacle_case(n=32, omegas=(5.0 + 2.0j,), M=8, nobs=8, times=None):
    """Exterior problem with two obstacles (an ellipse and a scaled kite,
    each split into 4 arcs), point source inside the ellipse -- the exact
    scattered field outside both is -u^i (the exact-solution idea of the
    paper's exterior geometry with a source inside an obstacle) -- and
    observation points on a circle around both."""
    arcs = _ellipse_arcs(n, 0.8, 0.5, center=(-1.0, 0.0), rot=0.3, group=0)
    arcs += _kite_arcs(n, scale=0.5, center=(1.2, 0.3), rot=-0.4, group=1)
    return MSProblem(arcs=arcs,
                     incident=IncidentSpec("point", z0=(-1.05, 0.1), sigma=0.0),
                     omegas=np.asarray(omegas), M=M, obs=_circle_points(nobs, 3.0),
                     times=np.zeros(0) if times is None else np.asarray(times),
                     name="two_obstacles_n%d" % n)


def closed_obstacles_case(n=64, omegas=(5.0 + 2.0j,), M=10, nobs=8, mixed=False, n_arc=32):
    """Exterior problem with two obstacles treated as closed patches (the
    combined-field option of Section 3.3): an ellipse and a scaled kite, a
    point source inside the ellipse (exact scattered field -u^i outside).
    With ``mixed`` the kite is split into 4 overlapping arcs of n_arc nodes
    instead, so closed and open patches interact."""
    from .curves import ClosedEllipse, ClosedKite
    arcs = [ArcSpec(ClosedEllipse(0.8, 0.5, (-1.0, 0.0), 0.3), n, group=0)]
    if mixed:
        arcs += _kite_arcs(n_arc, scale=0.5, center=(1.2, 0.3), rot=-0.4, group=1)
    else:
        arcs.append(ArcSpec(ClosedKite(0.5, (1.2, 0.3), -0.4), n, group=1))
    return MSProblem(arcs=arcs,
                     incident=IncidentSpec("point", z0=(-1.05, 0.1), sigma=0.0),
                     omegas=np.asarray(omegas), M=M, obs=_circle_points(nobs, 3.0),
                     times=np.zeros(0), name="closed_obstacles_n%d" % n)


def _inside_polygon(pts, poly):
    """Even-odd ray casting (input helper for sampling interior points)."""
    x, y = pts[:, 0][:, None], pts[:, 1][:, None]
    x0, y0 = poly[:, 0][None, :], poly[:, 1][None, :]
    x1, y1 = np.roll(poly[:, 0], -1)[None, :], np.roll(poly[:, 1], -1)[None, :]
    cond = (y0 > y) != (y1 > y)
    with np.errstate(divide="ignore", invalid="ignore"):
        xint = x0 + (y - y0) * (x1 - x0) / (y1 - y0)
    cross = cond & (x < xint)
    return (np.count_nonzero(cross, axis=1) % 2) == 1


def kite_interior_points(count, seed, min_dist=0.2):
    poly = kite_point(np.linspace(0.0, 2.0 * np.pi, 4000, endpoint=False))
    lo, hi = poly.min(axis=0), poly.max(axis=0)
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        p = lo + (hi - lo) * rng.random((256, 2))
        ok = _inside_polygon(p, poly)
        d = np.min(np.hypot(p[:, None, 0] - poly[None, :, 0],
                            p[:, None, 1] - poly[None, :, 1]), axis=1)
        for q in p[ok & (d >= min_dist)]:
            if len(out) < count:
                out.append(q)
    return np.array(out)


def kite_cavity_case(n=256, nfreq=512, M=6, nobs=64, nt=2001, dt=0.01):
    """Kite split into 4 arcs of 120 degrees of parameter (30 degree
    overlaps), point source at (0.1, 0.2) with omega0 = 20, sigma = 4,
    tau0 = 4; omega_l = 80 l / 512; time traces at 64 interior points."""
    omegas = 80.0 * np.arange(1, nfreq + 1) / nfreq
    return MSProblem(arcs=_kite_arcs(n),
                     incident=IncidentSpec("point", z0=(0.1, 0.2), omega0=20.0,
                                           sigma=4.0, tau0=4.0),
                     omegas=omegas, M=M,
                     obs=kite_interior_points(nobs, seed=2),
                     times=dt * np.arange(nt), name="kite4_n%d" % n)


def small_kite_case(n=40, omegas=(3.0, 7.5, 12.25), M=3, nobs=8, nt=64,
                    dt=0.05):
    """Reduced kite problem the oracle finishes in seconds."""
    return MSProblem(arcs=_kite_arcs(n),
                     incident=IncidentSpec("point", z0=(0.1, 0.2), omega0=8.0,
                                           sigma=3.0, tau0=4.0),
                     omegas=np.asarray(omegas), M=M,
                     obs=kite_interior_points(nobs, seed=2),
                     times=dt * np.arange(nt), name="kite4_small_n%d" % n)


def disc_interior_case(n=48, R=1.0, omegas=(6.0,), M=8, nobs=6,
                       incident=None):
    """Disc of radius R covered by three arcs of 180 degrees with 60 degree
    overlaps; the first arc is the polar interval (-pi/6, 5pi/6) (the layout
    of Geometry 1 and the density illustration of Section 4.3)."""
    arcs = []
    for j in range(3):
        a = -math.pi / 6.0 + j * 2.0 * math.pi / 3.0
        arcs.append(ArcSpec(CircularArc(R, a, a + math.pi), n))
    rng = np.random.default_rng(11)
    rr = 0.6 * R * np.sqrt(rng.random(nobs))
    pp = 2.0 * np.pi * rng.random(nobs)
    obs = np.stack([rr * np.cos(pp), rr * np.sin(pp)], axis=-1)
    if incident is None:
        incident = IncidentSpec("point", z0=(1.6 * R, 0.3 * R), omega0=0.0,
                                sigma=0.0, tau0=0.0)
    return MSProblem(arcs=arcs, incident=incident,
                     omegas=np.asarray(omegas, dtype=complex), M=M, obs=obs,
                     times=np.zeros(0), name="disc3_n%d" % n)


def _sine_length(ell, amp_ratio, nu):
    c = SineArc((0.0, 0.0), ell, amp_ratio * ell, nu, 0.0)
    return c.length(400)


def uneven_batch_case(seed=3, narcs=8, nk=2048, kmin=1.0, kmax=120.0,
                      nmax=1024, nmin=64, ppw=10.0, quantum=1):
    """Eight arcs of three kinds with lengths U[0.5, 4]; N per (arc, k) from
    ppw points per wavelength, clamped to [nmin, nmax], then rounded up to a
    multiple of `quantum` (1: the rule as stated; the GPU runs use 16 so that
    one frequency-independent table per (arc, N) serves a band of
    frequencies)."""
    rng = np.random.default_rng(seed)
    arcs = []
    for i in range(narcs):
        L = rng.uniform(0.5, 4.0)
        kind = i % 3
        if kind == 0:
            R = rng.uniform(0.5, 2.0)
            span = L / R
            if span > 1.5 * math.pi:
                R = L / (1.5 * math.pi)
                span = 1.5 * math.pi
            a = rng.uniform(0.0, 2.0 * math.pi)
            c = CircularArc(R, a, a + span,
                            center=tuple(rng.uniform(-3.0, 3.0, 2)))
        elif kind == 1:
            ea = rng.uniform(0.5, 2.0)
            eb = ea * rng.uniform(0.3, 1.0)
            sc = rng.uniform(0.0, 2.0 * math.pi)
            lo, hi = 1e-6, 0.75 * math.pi
            for _ in range(80):
                mid = 0.5 * (lo + hi)
                if EllipseArc(ea, eb, sc - mid, sc + mid).length() < L:
                    lo = mid
                else:
                    hi = mid
            h = 0.5 * (lo + hi)
            c = EllipseArc(ea, eb, sc - h, sc + h,
                           center=tuple(rng.uniform(-3.0, 3.0, 2)),
                           rot=rng.uniform(0.0, math.pi))
        else:
            ratio = rng.uniform(0.05, 0.2)
            nu = int(rng.integers(1, 4))
            ell = L / _sine_length(1.0, ratio, nu)
            c = SineArc(tuple(rng.uniform(-3.0, 3.0, 2)), ell, ratio * ell, nu,
                        rng.uniform(0.0, 2.0 * math.pi))
        theta = rng.uniform(0.0, 2.0 * math.pi)
        arcs.append(dict(curve=c, length=c.length(), theta=theta))
    k = kmin + (kmax - kmin) * np.arange(nk) / max(nk - 1, 1)
    for a in arcs:
        n = np.ceil(ppw * k * a["length"] / (2.0 * math.pi)).astype(int)
        n = np.minimum(nmax, np.maximum(nmin, n))
        a["n"] = np.minimum(nmax, quantum * ((n + quantum - 1) // quantum))
    return dict(arcs=arcs, k=k, name="uneven%d_k%d" % (narcs, nk))


def serving_requests(seed=5, count=32, max_obstacles=3, n_range=(32, 96),
                     nk_range=(48, 128), omega0_range=(3.0, 8.0), nobs=32,
                     dt=0.05, max_steps=100, stop_tol=1e-8):
    """Exterior scattering requests of different sizes for the serving loop
    (the shape of the serving workload at reduced size): 1..max_obstacles
    obstacles, each an ellipse (probability 1/2; semi-axes U[0.2, 1], random
    rotation) or a kite scaled by U[0.3, 1], centres rejection-sampled so
    that the obstacles keep a boundary distance of at least 0.5, each split
    into 4 arcs; n nodes per arc; J frequencies omega_l = 2 omega0 l / J;
    a Gaussian plane wave with sigma = 0.2 omega0, random direction and
    tau0 = R_cluster + 12 / sigma; observation points on the circle of radius
    R_cluster + 1; times 0 .. tau0 + 10 in steps of dt."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        nob = int(rng.integers(1, max_obstacles + 1))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        shapes, centres, radii = [], [], []
        while len(shapes) < nob:
            if rng.random() < 0.5:
                ea = rng.uniform(0.2, 1.0)
                eb = rng.uniform(0.2, 1.0)
                shp = ("ellipse", ea, eb, rng.uniform(0.0, math.pi))
                rad = max(ea, eb)
            else:
                sc = rng.uniform(0.3, 1.0)
                shp = ("kite", sc, rng.uniform(0.0, 2.0 * math.pi))
                rad = 1.65 * sc
            c = rng.uniform(-3.0, 3.0, 2)
            if all(math.hypot(*(c - c2)) - rad - r2 >= 0.5 for c2, r2 in zip(centres, radii)):
                shapes.append(shp)
                centres.append(c)
                radii.append(rad)
        arcs = []
        for g, (shp, c) in enumerate(zip(shapes, centres)):
            if shp[0] == "ellipse":
                arcs += _ellipse_arcs(n, shp[1], shp[2], center=tuple(c), rot=shp[3], group=g)
            else:
                arcs += _kite_arcs(n, scale=shp[1], center=tuple(c), rot=shp[2], group=g)
        cc = np.mean(centres, axis=0)
        rcl = max(math.hypot(*(c - cc)) + r for c, r in zip(centres, radii))
        omega0 = rng.uniform(*omega0_range)
        sigma = 0.2 * omega0
        nk = int(rng.integers(nk_range[0], nk_range[1] + 1))
        tau0 = rcl + 12.0 / sigma
        p = 2.0 * np.pi * np.arange(nobs) / nobs
        obs = np.stack([cc[0] + (rcl + 1.0) * np.cos(p), cc[1] + (rcl + 1.0) * np.sin(p)],
                       axis=-1)
        out.append(dict(arcs=arcs,
                        incident=IncidentSpec("gplane", theta=rng.uniform(0.0, 2.0 * math.pi),
                                              omega0=omega0, sigma=sigma, tau0=tau0),
                        omegas=2.0 * omega0 * np.arange(1, nk + 1) / nk, obs=obs,
                        times=dt * np.arange(int((tau0 + 10.0) / dt) + 1),
                        max_steps=max_steps, stop_tol=stop_tol, n=n, obstacles=nob,
                        name="request%d" % q))
    return out


def _perimeter(curve, m=2048):
    """Length of a closed curve by the trapezoid rule on m points (periodic:
    spectrally accurate)."""
    tau = 2.0 * np.pi * np.arange(m) / m
    d = curve.dx(tau)
    return float(np.sum(np.hypot(d[:, 0], d[:, 1])) * 2.0 * np.pi / m)


# largest distance of the unit kite (cos t + 0.65 cos 2t - 0.65, 1.5 sin t)
# from its centre (the origin), for bounding circles
_KITE_RADIUS = float(np.max(np.hypot(np.cos(np.linspace(0, 2 * np.pi, 20001))
                                     + 0.65 * np.cos(2 * np.linspace(0, 2 * np.pi, 20001)) - 0.65,
                                     1.5 * np.sin(np.linspace(0, 2 * np.pi, 20001)))))


def _max_speed(curve, m=4096):
    """max |x'(tau)| of a closed curve (dense sampling)."""
    tau = 2.0 * np.pi * np.arange(m) / m
    d = curve.dx(tau)
    return float(np.max(np.hypot(d[:, 0], d[:, 1])))


def serving_c5_requests(seed=5, count=200, max_obstacles=12, n_range=(64, 256),
                        nk_range=(128, 512), omega0_range=(5.0, 40.0), nobs=32, dt=0.05,
                        max_steps=100, stop_tol=1e-8, sep=0.5, precision=0):
    """Exterior scattering requests with the serving workload's
    distributions, each obstacle one closed patch (the paper's treatment of
    closed curves):

    * 1..max_obstacles obstacles, each an ellipse (probability 1/2; semi-axes
      U[0.2, 1], random rotation) or a kite scaled by U[0.3, 1] (random
      rotation); centres rejection-sampled in a square growing with the count
      so that the boundary-to-boundary distance (bounding circles) is at
      least ``sep``;
    * n nodes per obstacle ~ U{n_range}, raised where needed so that the
      largest node spacing (2 pi max |x'| / n) is at most sep / 5.25: the
      other obstacles then lie at least 5 node spacings away (the closed
      patches' far rule); rounded up to even;
    * J ~ U{nk_range} frequencies omega_l = 2 omega0 l / J, omega0 ~
      U[omega0_range], J raised where needed so that the grid's period
      2 pi / (2 omega0 / J) covers twice the time window (no wrap-around of
      late multiple-scattering arrivals into the traces);
    * a Gaussian plane wave, sigma = 0.2 omega0, random direction,
      tau0 = R_cluster + 12 / sigma; nobs points on the circle of radius
      R_cluster + 1 about the cluster centre; t = 0 .. tau0 + 10 in steps of
      dt; the time-domain stop rule at stop_tol within max_steps steps."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        nob = int(rng.integers(1, max_obstacles + 1))
        box = 1.5 + 1.2 * math.sqrt(nob)
        shapes, centres, radii = [], [], []
        while len(shapes) < nob:
            if rng.random() < 0.5:
                ea, eb = rng.uniform(0.2, 1.0), rng.uniform(0.2, 1.0)
                rot = rng.uniform(0.0, math.pi)
                rad = max(ea, eb)
                mk = ("ellipse", ea, eb, rot)
            else:
                sc = rng.uniform(0.3, 1.0)
                rot = rng.uniform(0.0, 2.0 * math.pi)
                rad = _KITE_RADIUS * sc
                mk = ("kite", sc, rot)
            c = rng.uniform(-box, box, 2)
            if all(math.hypot(*(c - c2)) - rad - r2 >= sep for c2, r2 in zip(centres, radii)):
                shapes.append(mk)
                centres.append(c)
                radii.append(rad)
        curves = []
        for shp, c in zip(shapes, centres):
            if shp[0] == "ellipse":
                curves.append(ClosedEllipse(shp[1], shp[2], center=tuple(c), rot=shp[3]))
            else:
                curves.append(ClosedKite(shp[1], center=tuple(c), rot=shp[2]))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        n = max(n, max(int(math.ceil(5.25 * 2.0 * math.pi * _max_speed(cv) / sep))
                       for cv in curves))
        n = min(1024, n + (n & 1))
        arcs = [ArcSpec(cv, n, g) for g, cv in enumerate(curves)]
        cc = np.mean(centres, axis=0)
        rcl = max(math.hypot(*(c - cc)) + r for c, r in zip(centres, radii))
        omega0 = rng.uniform(*omega0_range)
        sigma = 0.2 * omega0
        tau0 = rcl + 12.0 / sigma
        t_end = tau0 + 10.0
        nk = int(rng.integers(nk_range[0], nk_range[1] + 1))
        nk = max(nk, int(math.ceil(2.0 * omega0 * t_end / math.pi)))
        p = 2.0 * np.pi * np.arange(nobs) / nobs
        obs = np.stack([cc[0] + (rcl + 1.0) * np.cos(p), cc[1] + (rcl + 1.0) * np.sin(p)],
                       axis=-1)
        om = 2.0 * omega0 * np.arange(1, nk + 1) / nk
        # period of the frequency grid covers twice the time window
        assert 2.0 * np.pi / (om[1] - om[0]) >= 2.0 * t_end - 1e-9
        out.append(dict(arcs=arcs, closed=True, precision=precision,
                        incident=IncidentSpec("gplane", theta=rng.uniform(0.0, 2.0 * math.pi),
                                              omega0=omega0, sigma=sigma, tau0=tau0),
                        omegas=om, obs=obs, times=dt * np.arange(int(t_end / dt) + 1),
                        max_steps=max_steps, stop_tol=stop_tol, n=n, obstacles=nob,
                        name="c5request%d" % q))
    return out

