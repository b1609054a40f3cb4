"""GPU parity of composite-panel arcs (Section 4.3, eqs. cov, psi-tilde):
the HIP path through the C-ABI against the CPU oracle ``oracle.panels``.

Bar: relative L2 error <= 1e-10 per solve, field and summed density, in FP64
and in the FP32-refined form.  Panel sizes resolve the geometry in s from
the node samples (the library interpolates it; the oracle uses the exact
curve), i.e. n_per >= 24 for these shapes."""
import sys

import numpy as np
import pytest

from oracle import incident as oinc
from oracle import ms as oms
from oracle import nystrom as ony
from oracle import panels as opn
from workloads import CircularArc, EllipseArc, IncidentSpec, Segment, disc_interior_case

pytestmark = pytest.mark.gpu
TOL = 1e-10


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def fth():
    import paper_2507_05725_amd as m  # raises if the HIP library is missing
    return m


@pytest.fixture(scope="module")
def ctx(fth):
    return fth.Context(0)


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def test_panel_table_and_weights(ctx, fth):
    """The table built by the library at arc creation against the oracle's."""
    curve = EllipseArc(1.3, 0.7, -0.4, 2.2)
    br = (-1.0, -0.2, 0.5, 1.0)
    say("panel table ellipse n_per=24")
    arc = ctx.panel_arc_from_curve(curve, 24, br)
    W, w = arc.panel_table()
    oarc = opn.PanelArc(curve, 24, br)
    Wo = opn.log_table(oarc)
    assert np.max(np.abs(W - Wo)) < 4e-12 * np.max(np.abs(Wo))
    assert np.max(np.abs(w - oarc.nodes()["w"])) < 1e-15


@pytest.mark.parametrize("n_per", [24, 40])
@pytest.mark.parametrize("prec", [0, 1])
def test_panel_single_arc_solve_and_field(ctx, fth, n_per, prec):
    """Solve and field of one panel arc (N = 72, and 120: two LU tiles with a
    ragged tail) at several wavenumbers, with far and near targets."""
    curve = EllipseArc(1.3, 0.7, -0.4, 2.2)
    br = (-1.0, -0.2, 0.5, 1.0)
    spec = IncidentSpec("plane", theta=0.7)
    ks = np.array([2.0, 7.5, 13.0])
    say("panel solve n_per", n_per, "prec", prec)
    arc = ctx.panel_arc_from_curve(curve, n_per, br)
    rhs = ctx.rhs(arc, ks, spec)
    mu, iters, relres = ctx.solve(arc, ks, rhs, prec)
    oarc = opn.PanelArc(curve, n_per, br)
    nd = oarc.nodes()
    W = opn.log_table(oarc)
    z = np.array([[0.0, 2.5], [-2.0, -1.5], [1.3 * np.cos(0.9) * 1.01, 0.7 * np.sin(0.9) * 1.01],
                  [1.3 * np.cos(2.2) + 1e-3, 0.7 * np.sin(2.2)]])
    U = ctx.eval_field(arc, ks, mu, z)
    for i, k in enumerate(ks):
        b = -oinc.incident(spec, k, nd["y"])
        assert rel(rhs[i], b) < 1e-14
        ref = ony.solve(opn.assemble(nd, k, W), b)
        assert rel(mu[i], ref) < TOL, (k, rel(mu[i], ref))
        Uref = opn.field(k, z, nd, ref)
        assert rel(U[i], Uref) < TOL, (k, rel(U[i], Uref))


def test_panel_ms_disc(ctx, fth):
    """Multiple scattering in the three-arc disc with panel arcs (each cut at
    the ends of its truncated overlap): fields and summed densities of the
    GPU recursion against the oracle's."""
    pb = disc_interior_case(n=24, omegas=(4.5,), M=3)
    pb.scheme = "panels"
    say("panel ms disc n_per=24")
    iv = np.array([a.curve.interval for a in pb.arcs])
    brs = fth.tov_breaks(iv, None, pb.period)
    arcs = [ctx.panel_arc_from_curve(a.curve, a.n, b) for a, b in zip(pb.arcs, brs)]
    prob = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M)
    om = np.real(np.asarray(pb.omegas)).astype(float)
    U, A = prob.run(om, want_alpha=True)
    lay = oms.Layout(pb)
    ref = oms.run_frequency(lay, om[0])
    assert rel(U[0], ref["U"]) < TOL, rel(U[0], ref["U"])
    assert rel(A[0], np.concatenate(ref["alpha_tot"])) < TOL


def test_panel_ms_kite(ctx, fth):
    """The four-arc kite (120 degree arcs, 30 degree overlaps) with panel
    arcs of 3 x 32 nodes: a point source inside, M = 2."""
    from workloads import small_kite_case
    pb = small_kite_case(n=32, omegas=(6.0,), M=2, nobs=6)
    pb.scheme = "panels"
    say("panel ms kite n_per=32")
    iv = np.array([a.curve.interval for a in pb.arcs])
    brs = fth.tov_breaks(iv, None, pb.period)
    arcs = [ctx.panel_arc_from_curve(a.curve, a.n, b) for a, b in zip(pb.arcs, brs)]
    prob = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M)
    om = np.real(np.asarray(pb.omegas)).astype(float)
    U, A = prob.run(om, want_alpha=True)
    ref = oms.run_frequency(oms.Layout(pb), om[0])
    assert rel(U[0], ref["U"]) < TOL, rel(U[0], ref["U"])
    assert rel(A[0], np.concatenate(ref["alpha_tot"])) < TOL


def test_panel_maximum_size(ctx, fth):
    """3 x 341 = 1023 nodes (the largest panel arc).  The table on the
    segment x(t) = (t, 0) against the closed form of the log integral
    (sum_j W_ij (dt/ds)_j = (1+t)log(1+t) + (1-t)log(1-t) - 2; the oracle's
    adaptive table is too slow at this size), and on an ellipse the field of
    a solve against the single-panel arc of 1024 nodes (both converged for
    this smooth problem)."""
    say("panel arc 3 x 341: segment table")
    br = (-1.0, -0.3, 0.4, 1.0)
    seg = ctx.panel_arc_from_curve(Segment((-1.0, 0.0), (1.0, 0.0)), 341, br)
    W, _ = seg.panel_table()
    oarc = opn.PanelArc(Segment((-1.0, 0.0), (1.0, 0.0)), 341, br)
    t = oarc.nodes()["t"]
    dts = np.concatenate([oarc.t_of(p, oarc.s)[1] for p in range(oarc.P)])
    ref = (1 + t) * np.log(1 + t) + (1 - t) * np.log(1 - t) - 2.0
    assert np.max(np.abs(W @ dts - ref)) < 1e-11
    say("panel arc 3 x 341: ellipse field")
    curve = EllipseArc(1.3, 0.7, -0.4, 2.2)
    arc = ctx.panel_arc_from_curve(curve, 341, (-1.0, -0.2, 0.5, 1.0))
    spec = IncidentSpec("plane", theta=0.7)
    ks = np.array([5.0, 40.0])
    mu, _, _ = ctx.solve(arc, ks, ctx.rhs(arc, ks, spec), 1)
    plain = ctx.arc_from_curve(curve, 1024)
    al, _, _ = ctx.solve(plain, ks, ctx.rhs(plain, ks, spec), 0)
    z = np.array([[0.0, 2.5], [-2.0, -1.5], [2.5, 0.3]])
    assert rel(ctx.eval_field(arc, ks, mu, z), ctx.eval_field(plain, ks, al, z)) < 1e-9


def test_panel_error_paths(ctx, fth):
    curve = CircularArc(1.0, 0.0, 1.5)
    with pytest.raises(fth.FthmsError):
        fth.panel_nodes([-1.0, 0.3, 0.1, 1.0], [1, 1, 1], 16)
    arc = ctx.panel_arc_from_curve(curve, 16, (-1.0, 1.0))
    # batches take single-panel arcs only
    with pytest.raises(fth.FthmsError):
        fth.Batch(ctx, [arc], np.array([3.0]), [IncidentSpec("plane", theta=0.1)])
    # the table of a single-panel arc is not available
    plain = ctx.arc_from_curve(curve, 16)
    with pytest.raises(fth.FthmsError):
        plain.panel_table()
