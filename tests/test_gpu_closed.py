"""GPU parity of closed patches (Section 3.3, eqs. FDsolk-closed,
FDBIEk-closed): the combined-field Nystrom solve and field through the C-ABI
against ``oracle.closed``, alone and inside multiple-scattering problems
(two closed obstacles; a closed obstacle beside one split into open arcs).

Bar: relative L2 error <= 1e-10 per solve, field and summed density, in FP64
and in the FP32-refined form."""
import math
import sys

import numpy as np
import pytest

from oracle import closed as ocl
from oracle import incident as oinc
from oracle import ms as oms
from workloads import (ClosedEllipse, ClosedKite, IncidentSpec, closed_obstacles_case)

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


@pytest.mark.parametrize("curve,n", [(ClosedEllipse(1.0, 0.6, (0.2, -0.1), 0.3), 64),
                                     (ClosedKite(1.0), 128), (ClosedKite(1.0), 250)],
                         ids=["ellipse64", "kite128", "kite250"])
@pytest.mark.parametrize("prec", [0, 1])
def test_closed_solve_and_field(ctx, fth, curve, n, prec):
    """Point source inside: solve and far field against the oracle, and the
    field against the exact -u^i outside (resolved sizes)."""
    spec = IncidentSpec("point", z0=(0.05, 0.1), sigma=0.0)
    ks = np.array([2.0, 7.5, 11.0])
    say("closed solve", n, "prec", prec)
    arc = ctx.closed_from_curve(curve, n)
    rhs = ctx.rhs(arc, ks, spec)
    psi, iters, relres = ctx.solve(arc, ks, rhs, prec)
    nd = ocl.nodes(curve, n)
    z = np.array([[3.0 * math.cos(a), 3.0 * math.sin(a)] for a in np.linspace(0, 6, 8)])
    U = ctx.eval_field(arc, ks, psi, z)
    for i, k in enumerate(ks):
        b = -oinc.incident(spec, k, nd["y"])
        assert rel(rhs[i], b) < 1e-14
        ref = np.linalg.solve(ocl.assemble(nd, k), b)
        assert rel(psi[i], ref) < TOL, (k, rel(psi[i], ref))
        Uref = ocl.field(k, z, nd, ref)
        assert rel(U[i], Uref) < TOL, (k, rel(U[i], Uref))
        if n >= 128:
            ui = oinc.incident(spec, k, z)
            assert rel(U[i], -ui) < 1e-11


@pytest.mark.parametrize("mixed", [False, True], ids=["two_closed", "closed_and_arcs"])
def test_closed_ms_problem(ctx, fth, mixed):
    """Exterior MS with closed patches: fields and summed densities of the
    GPU recursion against the oracle's (96 nodes per closed patch: the
    obstacles are 0.49 apart, beyond 5 node spacings)."""
    pb = closed_obstacles_case(n=96, omegas=(5.5,), M=4, mixed=mixed)
    say("closed ms mixed" if mixed else "closed ms two closed")
    arcs = []
    for a in pb.arcs:
        if getattr(a.curve, "closed", False):
            arcs.append(ctx.closed_from_curve(a.curve, a.n))
        else:
            arcs.append(ctx.arc_from_curve(a.curve, a.n))
    iv = np.array([a.curve.interval for a in pb.arcs])
    prob = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M,
                       groups=[a.group for a in pb.arcs])
    om = np.real(np.asarray(pb.omegas)).astype(float)
    U, A = prob.run(om, want_alpha=True)
    ref = oms.run_frequency(oms.Layout(pb), om[0])
    assert rel(U[0], ref["U"]) < TOL, rel(U[0], ref["U"])
    assert rel(A[0], np.concatenate(ref["alpha_tot"])) < TOL


@pytest.mark.parametrize("prec", [0, 1])
def test_closed_maximum_size(ctx, fth, prec):
    """1024 nodes (the largest closed patch) at a high wavenumber."""
    curve = ClosedKite(1.0)
    spec = IncidentSpec("point", z0=(0.05, 0.1), sigma=0.0)
    ks = np.array([60.0])
    say("closed 1024 prec", prec)
    arc = ctx.closed_from_curve(curve, 1024)
    rhs = ctx.rhs(arc, ks, spec)
    psi, _, _ = ctx.solve(arc, ks, rhs, prec)
    nd = ocl.nodes(curve, 1024)
    b = -oinc.incident(spec, ks[0], nd["y"])
    ref = np.linalg.solve(ocl.assemble(nd, ks[0]), b)
    assert rel(psi[0], ref) < TOL, rel(psi[0], ref)
    z = np.array([[3.0, 0.0], [0.0, -3.0]])
    assert rel(ctx.eval_field(arc, ks, psi, z)[0], -oinc.incident(spec, ks[0], z)) < 1e-9


def test_closed_error_paths(ctx, fth):
    curve = ClosedEllipse(1.0, 0.6)
    arc = ctx.closed_from_curve(curve, 32)
    psi = np.ones((1, 32), dtype=complex)
    # a target on the curve: refused (nearer than h / 25, h the node spacing)
    with pytest.raises(fth.FthmsError):
        ctx.eval_field(arc, np.array([3.0]), psi, np.array([[1.0, 0.0]]))
    # odd node count
    tau = 2 * np.pi * np.arange(31) / 31
    with pytest.raises(fth.FthmsError):
        fth.Arc(ctx, curve.x(tau), curve.dx(tau), ddxy=curve.ddx(tau))
    # not for batches
    with pytest.raises(fth.FthmsError):
        fth.Batch(ctx, [arc], np.array([3.0]), [IncidentSpec("plane", theta=0.1)])
    # a closed patch shares its group with nobody
    other = ctx.closed_from_curve(ClosedKite(0.3, (3.0, 0.0)), 32)
    with pytest.raises(fth.FthmsError):
        fth.Problem(ctx, [arc, other], IncidentSpec("plane"), np.array([[5.0, 5.0]]),
                    intervals=np.array([[0, 2 * np.pi]] * 2), M=2, groups=[0, 0])


@pytest.mark.parametrize("npts", [1, 33, 100, 200, 256, 300])
def test_closed_field_target_counts(ctx, fth, npts):
    """(D - i eta S) Psi at target counts that take every thread-per-target
    split (8, 4, 2 threads below 256 targets, one from 256 up, a ragged
    second block at 300) against the oracle's trapezoid sum."""
    curve = ClosedKite(1.0)
    n = 128
    arc = ctx.closed_from_curve(curve, n)
    rng = np.random.default_rng(200 + npts)
    ks = np.array([3.0, 17.0])
    psi = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    ang = rng.uniform(0.0, 2.0 * math.pi, npts)
    rad = rng.uniform(3.0, 4.0, npts)
    z = np.stack([rad * np.cos(ang), rad * np.sin(ang)], -1)
    say("closed field targets", npts)
    U = ctx.eval_field(arc, ks, psi, z)
    nd = ocl.nodes(curve, n)
    for i, k in enumerate(ks):
        Uref = ocl.field(k, z, nd, psi[i])
        assert rel(U[i], Uref) < 1e-12, (npts, k, rel(U[i], Uref))


def _exterior_points(curve, tt, dist):
    y, dy = curve.x(tt), curve.dx(tt)
    nrm = np.stack([dy[:, 1], -dy[:, 0]], -1) / np.hypot(dy[:, 0], dy[:, 1])[:, None]
    return y + dist * nrm


@pytest.mark.parametrize("curve,n", [(ClosedKite(1.0), 256),
                                     (ClosedEllipse(1.0, 0.6, (0.2, -0.1), 0.3), 128)],
                         ids=["kite256", "ellipse128"])
def test_closed_near_targets(ctx, fth, curve, n):
    """Targets from 6 node spacings down to 0.05 of one (every upsampling
    level, kappa = 2 .. 128, and the far rule) beside the oracle's
    near-target integral and the exact exterior field of an interior point
    source; a target at 0.03 of a node spacing is refused."""
    spec = IncidentSpec("point", z0=(0.05, 0.1), sigma=0.0)
    ks = np.array([2.0, 7.5])
    arc = ctx.closed_from_curve(curve, n)
    rhs = ctx.rhs(arc, ks, spec)
    psi, _, _ = ctx.solve(arc, ks, rhs, 0)
    nd = ocl.nodes(curve, n)
    h = ocl.near_limit(nd) / 5.0
    tt = np.array([0.31, 1.7, 2.95, 4.4, 5.9])
    fr = (0.05, 0.09, 0.2, 0.35, 0.7, 1.4, 2.0, 4.5, 6.0)
    z = np.concatenate([_exterior_points(curve, tt, f * h) for f in fr])
    say("closed near targets", n, z.shape[0])
    U = ctx.eval_field(arc, ks, psi, z)
    for i, k in enumerate(ks):
        ref = ocl.field_near(k, z, curve, nd, psi[i])
        assert np.max(np.abs(U[i] - ref)) < 1e-11 * np.max(np.abs(ref)), k
        ui = oinc.incident(spec, k, z)
        assert np.max(np.abs(U[i] + ui) / np.abs(ui)) < 1e-11, k
    with pytest.raises(fth.FthmsError):
        ctx.eval_field(arc, ks, psi, _exterior_points(curve, tt[:1], 0.03 * h))


@pytest.mark.parametrize("prec", [0, 1])
def test_closed_ms_near_obstacles(ctx, fth, prec):
    """Two obstacles 0.24 apart at 64 nodes each (nodes of each within five
    node spacings of the other: no stored operators, the near rule for the
    cross fields) and observation points in the gap: the GPU recursion
    against the oracle's."""
    E = ClosedEllipse(0.8, 0.5, (-1.0, 0.0))
    K = ClosedKite(0.5, (0.62, 0.2))
    gap = np.array([[-0.18017388, -0.19891766], [-0.13765677, -0.22256675],
                    [-0.09513967, -0.24621585]])
    far = np.stack([2.8 * np.cos(np.linspace(0, 6, 4)), 2.8 * np.sin(np.linspace(0, 6, 4))], -1)
    obs = np.concatenate([far, gap])
    from workloads.configs import ArcSpec, MSProblem
    pb = MSProblem(arcs=[ArcSpec(E, 64, group=0), ArcSpec(K, 64, group=1)],
                   incident=IncidentSpec("plane", theta=0.4), omegas=np.array([5.5]), M=4,
                   obs=obs, times=np.zeros(0))
    say("closed ms near obstacles prec", prec)
    arcs = [ctx.closed_from_curve(a.curve, a.n) for a in pb.arcs]
    iv = np.array([a.curve.interval for a in pb.arcs])
    prob = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M, groups=[0, 1],
                       precision=prec)
    U, A = prob.run(np.array([5.5]), want_alpha=True)
    ref = oms.run_frequency(oms.Layout(pb), 5.5)
    assert rel(U[0], ref["U"]) < TOL, rel(U[0], ref["U"])
    assert rel(A[0], np.concatenate(ref["alpha_tot"])) < TOL
