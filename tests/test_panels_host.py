"""The library's composite-panel set-up, built for the host, against the
oracle: the frequency-independent log table (Section 4.3) and the
per-panel near-target quadrature plan.

tests/native/panels_probe.cpp wraps the header the library uses (g++, CPU
only).  The test feeds it node samples of a panel arc (at the library's
panel nodes, computed here from eq. cov) and targets; it compares the table
with the oracle's independently computed table and with the segment's
closed form, and sums each planned near rule over the kernel and the panel
interpolants of a smooth density against the oracle's adaptive field."""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import nystrom as ny
from oracle import panels as pn
from workloads.curves import EllipseArc, Segment

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def probe():
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    d = tempfile.mkdtemp(prefix="pprobe")
    exe = os.path.join(d, "pprobe")
    subprocess.run([gxx, "-O2", "-std=c++17", "-pthread", "-o", exe,
                    os.path.join(HERE, "native", "panels_probe.cpp")],
                   check=True, capture_output=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def run(exe, arc, kmax, z):
    nd = arc.nodes()
    N = nd["n"]
    dx = np.concatenate([arc.curve.dx(arc.t_of(p, arc.s)[0]) for p in range(arc.P)])
    lines = ["%d %d %.17g %d" % (arc.P, arc.n, kmax, z.shape[0])]
    lines.append(" ".join("%.17g" % b for b in arc.breaks))
    lines.append(" ".join(str(k) for k in arc.kinds))
    lines += ["%.17g %.17g %.17g %.17g" % (*nd["y"][i], *dx[i]) for i in range(N)]
    lines += ["%.17g %.17g" % tuple(p) for p in z]
    out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True,
                         text=True, check=True).stdout.splitlines()
    assert out[0] == "W"
    W = np.array([[float(v) for v in out[1 + i].split()] for i in range(N)])
    cls, rules = {}, {}
    i = 1 + N
    while i < len(out):
        f = out[i].split()
        if f[0] == "C":
            cls[int(f[1])] = int(f[2])
            i += 1
        else:
            t, nq = int(f[1]), int(f[2])
            rules[t] = np.array([[float(v) for v in out[i + 1 + q].split()] for q in range(nq)])
            i += 1 + nq
    return W, cls, rules


def test_table_segment_closed_form(probe):
    """sum_j W_ij (dt/ds)_j = (1+t)log(1+t) + (1-t)log(1-t) - 2 on the
    segment x(t) = (t, 0), with three panels."""
    arc = pn.PanelArc(Segment((-1.0, 0.0), (1.0, 0.0)), 32, (-1.0, -0.3, 0.4, 1.0))
    W, _, _ = run(probe, arc, 1.0, np.zeros((0, 2)))
    t = arc.nodes()["t"]
    dts = np.concatenate([arc.t_of(p, arc.s)[1] for p in range(arc.P)])
    ref = (1 + t) * np.log(1 + t) + (1 - t) * np.log(1 - t) - 2.0
    assert np.max(np.abs(W @ dts - ref)) < 1e-12


def test_table_matches_oracle_ellipse(probe):
    """The library's table against the oracle's (adaptive quadrature on the
    exact curve) on an ellipse arc with three panels, at a panel size where
    the node samples resolve the geometry in s (the library interpolates it
    from them) to ~1e-14."""
    arc = pn.PanelArc(EllipseArc(1.3, 0.7, -0.4, 2.2), 24, (-1.0, -0.2, 0.5, 1.0))
    W, _, _ = run(probe, arc, 1.0, np.zeros((0, 2)))
    Wo = pn.log_table(arc)
    assert np.max(np.abs(W - Wo)) < 4e-12 * np.max(np.abs(Wo))


def test_near_plan_matches_oracle_field(probe):
    """Planned near rules (one per panel) summed over the fundamental
    solution and the panel interpolants of a smooth density, against the
    oracle's adaptive potential, for targets from 1e-6 to 0.3 off the arc,
    beyond its ends and next to the panel breaks."""
    curve = EllipseArc(1.3, 0.7, -0.4, 2.2)
    arc = pn.PanelArc(curve, 24, (-1.0, -0.2, 0.5, 1.0))
    nd = arc.nodes()
    k = 9.0
    rng = np.random.default_rng(4)
    c = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    mu = np.polynomial.chebyshev.chebval(nd["t"], c) * np.exp(1j * nd["t"])
    z = []
    for tt, off in ((0.1, 0.3), (-0.2, 1e-3), (0.5, 1e-6), (0.47, 2e-4), (-0.9, 5e-3)):
        x = curve.x(np.array([tt]))[0]
        d = curve.dx(np.array([tt]))[0]
        nrm = np.array([-d[1], d[0]]) / math.hypot(*d)
        z.append(x + off * nrm)
    # beyond the ends, along the tangent
    for e, sg in ((1.0, 1.0), (-1.0, -1.0)):
        x = curve.x(np.array([e]))[0]
        d = curve.dx(np.array([e]))[0]
        z.append(x + sg * 1e-4 * d / math.hypot(*d))
    z = np.array(z)
    _, cls, rules = run(probe, arc, k, z)
    a = pn.panel_coeffs(arc, mu)
    for p in range(z.shape[0]):
        assert cls[p] == 2
        r = rules[p]
        pan = r[:, 4].astype(int)
        dens = np.array([np.polynomial.chebyshev.chebval(r[q, 3], a[pan[q]]) for q in range(r.shape[0])])
        dist = np.hypot(r[:, 0] - z[p, 0], r[:, 1] - z[p, 1])
        got = np.sum(r[:, 2] * ny.fundamental(k, dist) * dens)
        ref = sum(pn._panel_near(k, z[p], arc, q, a[q], 1e-14) for q in range(arc.P))
        assert abs(got - ref) < 3e-11 * max(1.0, abs(ref)), (p, got, ref)
