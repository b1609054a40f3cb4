"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Bar (per solve, field or trace): relative L2 error <= 1e-10 in FP64, and the
same for the FP32-refined form (it targets the FP64 solution).  Sizes span
several 32/64 tiles and ragged tails; full-size workloads are checked on
sampled wavenumbers the oracle computes one by one.
"""
import math
import sys

import numpy as np
import pytest

from oracle import incident as oinc
from oracle import ms as oms
from oracle import nystrom as ony
from oracle import transform as otr
from workloads import (CircularArc, EllipseArc, Segment, SineArc, IncidentSpec,
                       fixed512_case, kite_cavity_case, plain_segment_case, small_kite_case)

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


def oracle_solve(curve, n, k, inc):
    nd = ony.arc_nodes(curve, n)
    b = -oinc.incident(inc, k, nd["y"])
    return nd, ony.solve(ony.assemble(nd, k), b)


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", [0, 1])
def test_plain_segment_case_full(ctx, fth, prec):
    """Segment, N = 128, 64 wavenumbers in [0.5, 32], fields on 256 points
    of the radius-3 circle: every solve and field against the oracle."""
    case = plain_segment_case()
    say("segment n=128 nk=64 prec", prec)
    arc = ctx.arc_from_curve(case["curve"], case["n"])
    k = case["k"]
    rhs = ctx.rhs(arc, k, case["incident"])
    alpha, iters, relres = ctx.solve(arc, k, rhs, prec)
    U = ctx.eval_field(arc, k, alpha, case["obs"])
    for i, kk in enumerate(k):
        nd, a_ref = oracle_solve(case["curve"], case["n"], kk, case["incident"])
        assert rel(rhs[i], -oinc.incident(case["incident"], kk, nd["y"])) < 1e-14
        assert rel(alpha[i], a_ref) < TOL, (i, kk, rel(alpha[i], a_ref))
        assert rel(U[i], ony.field_far(kk, case["obs"], nd["y"], a_ref)) < TOL
    if prec == 1:
        assert np.all(iters >= 1), iters


def test_refined_fallback_to_fp64(ctx, fth):
    """A refinement tolerance no solve can reach sends every refined solve
    through its iteration cap to the FP64 redo (iters = -1): the redo
    factors the same FP64 matrix with the FP64 kernels, so it matches the
    FP64 form and the oracle."""
    case = plain_segment_case()
    k = case["k"][::8]
    say("refined fallback nk", k.size)
    arc = ctx.arc_from_curve(case["curve"], case["n"])
    rhs = ctx.rhs(arc, k, case["incident"])
    a64, it64, _ = ctx.solve(arc, k, rhs, fth.FP64)
    a32, it32, _ = ctx.solve(arc, k, rhs, fth.FP32_REFINED, 1e-300)
    assert np.all(it64 == 0), it64
    assert np.all(it32 == -1), it32
    assert rel(a32, a64) < 1e-13, rel(a32, a64)
    for i, kk in enumerate(k):
        _, a_ref = oracle_solve(case["curve"], case["n"], kk, case["incident"])
        assert rel(a32[i], a_ref) < TOL, (i, kk, rel(a32[i], a_ref))


@pytest.mark.parametrize("n", [2, 3, 7, 31, 33, 64, 65, 100, 257])
def test_ragged_sizes(ctx, fth, n):
    curves = [CircularArc(1.3, 0.2, 2.4), EllipseArc(1.2, 0.5, -0.4, 1.9),
              SineArc((0.1, -0.3), 2.2, 0.25, 2, 0.6)]
    curve = curves[n % 3]
    k = np.array([0.7, 3.1, 11.0, 23.5])
    inc = IncidentSpec("plane", theta=1.1)
    say("ragged n", n)
    arc = ctx.arc_from_curve(curve, n)
    rhs = ctx.rhs(arc, k, inc)
    for prec in (0, 1):
        alpha, _, _ = ctx.solve(arc, k, rhs, prec)
        for i, kk in enumerate(k):
            _, a_ref = oracle_solve(curve, n, kk, inc)
            assert rel(alpha[i], a_ref) < TOL, (n, prec, kk, rel(alpha[i], a_ref))


def test_fixed512_full_batch_sampled(ctx, fth):
    """The benchmark workload: N = 512 circular arc, all 4096 wavenumbers
    in [1, 120] in one call (same chunking as the benchmark), both forms;
    sampled wavenumbers against the oracle, all refined results against FP64."""
    case = fixed512_case()
    say("arc512 nk=4096")
    arc = ctx.arc_from_curve(case["curve"], case["n"])
    k = case["k"]
    rhs = ctx.rhs(arc, k, case["incident"])
    a64, _, _ = ctx.solve(arc, k, rhs, 0)
    a32, iters, _ = ctx.solve(arc, k, rhs, 1)
    errs = np.linalg.norm(a32 - a64, axis=1) / np.linalg.norm(a64, axis=1)
    assert errs.max() < TOL, errs.max()
    for i in (0, 1, 1500, 2731, 4094, 4095):
        _, a_ref = oracle_solve(case["curve"], case["n"], k[i], case["incident"])
        assert rel(a64[i], a_ref) < TOL, (i, rel(a64[i], a_ref))
        assert rel(a32[i], a_ref) < TOL, (i, rel(a32[i], a_ref))


def test_max_size_1024(ctx, fth):
    curve = EllipseArc(2.0, 1.1, 0.2, 4.6)
    k = np.array([2.0, 57.0, 119.0])
    inc = IncidentSpec("plane", theta=-0.3)
    say("n=1024")
    arc = ctx.arc_from_curve(curve, 1024)
    rhs = ctx.rhs(arc, k, inc)
    for prec in (0, 1):
        alpha, iters, _ = ctx.solve(arc, k, rhs, prec)
        if prec == 1:
            assert np.all(iters >= 1), iters  # refined in FP32, not redone in FP64
        for i in (0, 2):
            _, a_ref = oracle_solve(curve, 1024, k[i], inc)
            assert rel(alpha[i], a_ref) < TOL


def test_batch_invariance(ctx, fth):
    """Each solve is the same alone and inside a batch (bitwise)."""
    curve = CircularArc(1.0, -1.0, 1.3)
    k = np.linspace(2.0, 40.0, 37)
    inc = IncidentSpec("plane", theta=0.5)
    say("batch invariance")
    arc = ctx.arc_from_curve(curve, 96)
    rhs = ctx.rhs(arc, k, inc)
    for prec in (0, 1):
        batch, _, _ = ctx.solve(arc, k, rhs, prec)
        for i in (0, 17, 36):
            one, _, _ = ctx.solve(arc, k[i:i + 1], rhs[i:i + 1], prec)
            assert np.array_equal(one[0], batch[i])


def test_batch_invariance_large_refined(ctx, fth):
    """The refined form's solves are the same alone and inside a batch whose
    LU halves are large enough (over 1024 matrices each) to factor their
    diagonal blocks one wave per matrix, while a single solve takes the
    1024-thread panel: the two kernels must give the same bits.  N = 96 also
    has a partial last block."""
    curve = CircularArc(1.0, -1.0, 1.3)
    k = np.linspace(2.0, 40.0, 2100)
    inc = IncidentSpec("plane", theta=0.5)
    say("batch invariance, 2100 refined solves")
    arc = ctx.arc_from_curve(curve, 96)
    rhs = ctx.rhs(arc, k, inc)
    batch, iters, _ = ctx.solve(arc, k, rhs, 1)
    assert np.all(iters >= 1), iters.min()
    for i in (0, 1049, 1050, 2099):
        one, _, _ = ctx.solve(arc, k[i:i + 1], rhs[i:i + 1], 1)
        assert np.array_equal(one[0], batch[i]), (i, np.max(np.abs(one[0] - batch[i])))


@pytest.mark.parametrize("kind", ["gplane", "point"])
def test_incident_kinds(ctx, fth, kind):
    curve = SineArc((0.0, 0.0), 2.0, 0.2, 1, 0.3)
    spec = (IncidentSpec("gplane", theta=2.0, omega0=15.0, sigma=3.0, tau0=5.0) if kind == "gplane"
            else IncidentSpec("point", z0=(0.4, 1.7), omega0=20.0, sigma=4.0, tau0=4.0))
    k = np.linspace(5.0, 35.0, 13)
    arc = ctx.arc_from_curve(curve, 80)
    rhs = ctx.rhs(arc, k, spec)
    nd = ony.arc_nodes(curve, 80)
    for i, kk in enumerate(k):
        ref = -oinc.incident(spec, kk, nd["y"])
        assert np.max(np.abs(rhs[i] - ref)) < 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_near_field_targets(ctx, fth):
    """Targets within ten node spacings of the arc (including beyond an
    endpoint along the curve) use the near rule; compare with the oracle's
    adaptive quadrature."""
    curve = CircularArc(1.0, 0.0, 1.5)
    n = 48
    arc = ctx.arc_from_curve(curve, n)
    rng = np.random.default_rng(9)
    k = np.array([3.0, 14.0])
    alpha = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    ang = np.array([0.3, 0.75, 1.2, -0.02, 1.53, 0.9])
    rad = np.array([1.02, 0.97, 1.3, 1.0, 1.0, 0.6])
    pts = np.stack([rad * np.cos(ang), rad * np.sin(ang)], -1)
    say("near field")
    U = ctx.eval_field(arc, k, alpha, pts)
    nd = ony.arc_nodes(curve, n)
    for i, kk in enumerate(k):
        ref = ony.field(kk, pts, curve, nd, alpha[i])
        assert np.max(np.abs(U[i] - ref)) < 1e-11 * max(1.0, np.max(np.abs(ref))), (
            i, np.abs(U[i] - ref))


def test_freq_to_time(ctx, fth):
    rng = np.random.default_rng(12)
    om = 80.0 * np.arange(1, 131) / 130
    w = otr.trapezoid_weights(om)
    U = rng.standard_normal((130, 70)) + 1j * rng.standard_normal((130, 70))
    t = 0.01 * np.arange(150)
    say("freq_to_time")
    u = ctx.freq_to_time(om, w, U, t)
    ref = otr.freq_to_time(om, w, U, t)
    assert rel(u, ref) < 1e-13


def test_ms_small_kite(ctx, fth):
    """Kite split into 4 overlapping arcs, point source inside, M = 3: the
    GPU recursion (chi windows, overlap masks, cross-arc near/far fields)
    against the oracle's per-frequency recursion."""
    pb = small_kite_case(n=40, omegas=(3.0, 7.5, 12.25), M=3, nobs=8)
    say("ms small kite")
    arcs = [ctx.arc_from_curve(a.curve, a.n) for a in pb.arcs]
    iv = np.array([a.curve.interval for a in pb.arcs])
    prob = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M)
    U, A = prob.run(np.asarray(pb.omegas, dtype=float), want_alpha=True)
    lay = oms.Layout(pb)
    for i, kk in enumerate(pb.omegas):
        ref = oms.run_frequency(lay, kk)
        assert rel(U[i], ref["U"]) < TOL, (kk, rel(U[i], ref["U"]))
        assert rel(A[i], np.concatenate(ref["alpha_tot"])) < TOL


def test_ms_kite_cavity_full(ctx, fth):
    """The interior kite cavity at full size: 4 arcs of N = 256, 512
    frequencies up to 80, M = 6, 64 interior points, 2001 time samples.
    Sampled frequencies (the lowest and the source's centre frequency 20)
    against the oracle's recursion; the time traces against the trapezoid sum over the GPU's own
    frequency data; and the traces vanish before the source pulse starts."""
    import time
    pb = kite_cavity_case()
    say("ms kite cavity full", len(pb.omegas), "frequencies")
    arcs = [ctx.arc_from_curve(a.curve, a.n) for a in pb.arcs]
    iv = np.array([a.curve.interval for a in pb.arcs])
    prob = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M)
    om = np.asarray(pb.omegas, dtype=float)
    t0 = time.perf_counter()
    U, A = prob.run(om, want_alpha=True)
    say("kite cavity: %d frequencies x 4 arcs, M = 6: %.3f s" % (om.size, time.perf_counter() - t0))
    lay = oms.Layout(pb)
    for i in (0, int(np.argmin(np.abs(om - 20.0)))):
        say("kite cavity: oracle at omega = %g" % om[i])
        ref = oms.run_frequency(lay, om[i])
        assert rel(U[i], ref["U"]) < TOL, (om[i], rel(U[i], ref["U"]))
        assert rel(A[i], np.concatenate(ref["alpha_tot"])) < TOL, om[i]
    w = otr.trapezoid_weights(om)
    u = ctx.freq_to_time(om, w, U, pb.times)
    ref_u = (np.exp(-1j * np.outer(pb.times, om)) * w) @ U / (2.0 * np.pi)
    assert rel(u, ref_u) < 1e-12
    # the pulse is centred at tau0 = 4 with a time width of order 1/sigma
    early = np.abs(u[pb.times < 1.5]).max()
    assert early < 1e-6 * np.abs(u).max(), early


def test_ms_exterior_two_obstacles(ctx, fth):
    """Exterior problem with two closed obstacles (4 arcs each, cyclic within
    each obstacle, every arc scattering onto every other one): fields and
    summed densities against the oracle's recursion."""
    from workloads import two_obstacle_case
    pb = two_obstacle_case(n=20, omegas=np.array([7.25]), M=5)
    pb.incident = IncidentSpec("gplane", theta=0.4, omega0=7.5, sigma=1.5, tau0=3.0)
    say("ms two obstacles")
    arcs = [ctx.arc_from_curve(a.curve, a.n) for a in pb.arcs]
    iv = np.array([a.curve.interval for a in pb.arcs])
    prob = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M,
                       groups=[a.group for a in pb.arcs])
    U, A = prob.run(np.asarray(pb.omegas, dtype=float), want_alpha=True)
    ref = oms.run_frequency(oms.Layout(pb), pb.omegas[0])
    assert rel(U[0], ref["U"]) < TOL, rel(U[0], ref["U"])
    assert rel(A[0], np.concatenate(ref["alpha_tot"])) < TOL


def test_ms_exterior_traces_stop_rule(ctx, fth):
    """Two facing open arcs as separate scatterers: time traces with the
    time-domain stop rule (tolerance 0.1: the increments of steps 1-4 are
    1, 0.66, 0.24, 0.019 of the running sum), the step count, and the full
    M-step traces, against the oracle."""
    from workloads import two_arc_exterior_case
    pb = two_arc_exterior_case()
    om = np.asarray(pb.omegas, dtype=float)
    w = otr.trapezoid_weights(om)
    arcs = [ctx.arc_from_curve(a.curve, a.n) for a in pb.arcs]
    iv = np.array([a.curve.interval for a in pb.arcs])
    prob = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M, groups=[0, 1])
    lay = oms.Layout(pb)
    for tol, want in ((0.1, 4), (0.0, pb.M)):
        u, steps = prob.traces(om, w, pb.times, stop_tol=tol)
        ref, ref_steps = oms.run_traces(lay, om, w, pb.times, stop_tol=tol)
        say("two arcs: tol", tol, "steps", steps, "oracle", ref_steps)
        assert steps == ref_steps == want
        assert rel(u, ref) < TOL, rel(u, ref)


def test_error_paths(ctx, fth):
    curve = Segment((-1.0, 0.0), (1.0, 0.0))
    arc = ctx.arc_from_curve(curve, 16)
    k = np.array([1.0, 2.0])
    rhs = np.ones((2, 16), dtype=complex)
    rhs[1, 3] = np.nan
    with pytest.raises(fth.FthmsError) as e:
        ctx.solve(arc, k, rhs, 0)
    assert e.value.code == -2
    with pytest.raises(fth.FthmsError) as e:
        ctx.solve(arc, np.array([1.0, -2.0]), np.ones((2, 16), dtype=complex), 0)
    assert e.value.code == -2
    xy = np.zeros((8, 2))
    xy[:, 0] = np.linspace(0, 1, 8)
    xy[4] = xy[3]
    with pytest.raises(fth.FthmsError) as e:
        ctx.arc(xy, np.ones((8, 2)))
    assert e.value.code == -2
    small = fth.Context(0, hbm_budget=100_000)
    arc2 = small.arc_from_curve(curve, 64)
    with pytest.raises(fth.FthmsError) as e:
        small.solve(arc2, np.linspace(1, 5, 64), np.ones((64, 64), dtype=complex), 0)
    assert e.value.code == -3


@pytest.mark.parametrize("npts", [1, 33, 200, 256, 300, 600, 1100])
def test_far_field_target_counts(ctx, fth, npts):
    """Far-field sums at target counts that take every thread-per-target
    split (8 threads below 256 targets, 4 below 512, 2 below 1024, one
    from 1024 up; ragged last blocks at 300, 600 and 1100) against the
    oracle's Gauss-Chebyshev sum."""
    curve = CircularArc(1.0, -1.0, 1.0)
    n = 96
    arc = ctx.arc_from_curve(curve, n)
    rng = np.random.default_rng(100 + npts)
    k = np.array([4.0, 23.0])
    alpha = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    ang = rng.uniform(0.0, 2.0 * math.pi, npts)
    rad = rng.uniform(2.5, 3.5, npts)
    pts = np.stack([rad * np.cos(ang), rad * np.sin(ang)], -1)
    say("far field targets", npts)
    U = ctx.eval_field(arc, k, alpha, pts)
    y = ony.arc_nodes(curve, n)["y"]
    for i, kk in enumerate(k):
        ref = ony.field_far(kk, pts, y, alpha[i])
        err = np.linalg.norm(U[i] - ref) / np.linalg.norm(ref)
        assert err < 1e-12, (npts, kk, err)


def test_ms_refined_matches_oracle(ctx, fth):
    """The refined form inside the multiple-scattering recursion (FP32
    factors kept for all M steps, refined at every solve): the small kite
    and the two-obstacle exterior problem against the oracle's recursion."""
    from workloads import two_obstacle_case
    pb = small_kite_case(n=40, omegas=(3.0, 7.5, 12.25), M=3, nobs=8)
    say("ms small kite refined")
    arcs = [ctx.arc_from_curve(a.curve, a.n) for a in pb.arcs]
    iv = np.array([a.curve.interval for a in pb.arcs])
    prob = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M,
                       precision=fth.FP32_REFINED, tol=1e-12)
    U, A = prob.run(np.asarray(pb.omegas, dtype=float), want_alpha=True)
    lay = oms.Layout(pb)
    for i, kk in enumerate(pb.omegas):
        ref = oms.run_frequency(lay, kk)
        assert rel(U[i], ref["U"]) < TOL, (kk, rel(U[i], ref["U"]))
        assert rel(A[i], np.concatenate(ref["alpha_tot"])) < TOL
    pb = two_obstacle_case(n=20, omegas=np.array([7.25]), M=5)
    pb.incident = IncidentSpec("gplane", theta=0.4, omega0=7.5, sigma=1.5, tau0=3.0)
    say("ms two obstacles refined")
    arcs = [ctx.arc_from_curve(a.curve, a.n) for a in pb.arcs]
    iv = np.array([a.curve.interval for a in pb.arcs])
    prob = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M,
                       groups=[a.group for a in pb.arcs], precision=fth.FP32_REFINED,
                       tol=1e-12)
    U, A = prob.run(np.asarray(pb.omegas, dtype=float), want_alpha=True)
    ref = oms.run_frequency(oms.Layout(pb), pb.omegas[0])
    assert rel(U[0], ref["U"]) < TOL, rel(U[0], ref["U"])
    assert rel(A[0], np.concatenate(ref["alpha_tot"])) < TOL


def test_ms_kite_cavity_refined(ctx, fth):
    """The kite cavity at full size in the refined form: sampled frequencies
    against the oracle's recursion, every frequency against the GPU's FP64
    run, and the time traces against the FP64 run's traces."""
    pb = kite_cavity_case()
    say("ms kite cavity refined", len(pb.omegas), "frequencies")
    arcs = [ctx.arc_from_curve(a.curve, a.n) for a in pb.arcs]
    iv = np.array([a.curve.interval for a in pb.arcs])
    om = np.asarray(pb.omegas, dtype=float)
    p64 = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M)
    p32 = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M,
                      precision=fth.FP32_REFINED, tol=1e-12)
    U64, A64 = p64.run(om, want_alpha=True)
    U32, A32 = p32.run(om, want_alpha=True)
    err_a = max(rel(A32[i], A64[i]) for i in range(om.size))
    err_u = max(rel(U32[i], U64[i]) for i in range(om.size))
    say("kite cavity refined vs FP64: densities %.2e, fields %.2e" % (err_a, err_u))
    assert err_a < TOL and err_u < TOL
    lay = oms.Layout(pb)
    for i in (0, int(np.argmin(np.abs(om - 20.0)))):
        ref = oms.run_frequency(lay, om[i])
        assert rel(U32[i], ref["U"]) < TOL, (om[i], rel(U32[i], ref["U"]))
        assert rel(A32[i], np.concatenate(ref["alpha_tot"])) < TOL, om[i]
    w = otr.trapezoid_weights(om)
    u64 = ctx.freq_to_time(om, w, U64, pb.times)
    u32 = ctx.freq_to_time(om, w, U32, pb.times)
    assert rel(u32, u64) < TOL


def test_ms_refined_fp64_redo_paths(ctx, fth):
    """Refinement failures inside the recursion: with an unreachable
    tolerance every first solve is redone in FP64 and the matrices stay in
    FP64 (bit-identical to the FP64 problem); with the later solves' step
    cap at zero (a test hook) every later solve fails and is redone once in
    FP64, which must still agree with the oracle."""
    import os
    pb = small_kite_case(n=40, omegas=(3.0, 7.5, 12.25), M=4, nobs=8)
    arcs = [ctx.arc_from_curve(a.curve, a.n) for a in pb.arcs]
    iv = np.array([a.curve.interval for a in pb.arcs])
    om = np.asarray(pb.omegas, dtype=float)
    p64 = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M)
    U64, A64 = p64.run(om, want_alpha=True)
    say("ms refined, every solve redone")
    pall = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M,
                       precision=fth.FP32_REFINED, tol=1e-30)
    Ua, Aa = pall.run(om, want_alpha=True)
    assert np.array_equal(Ua, U64) and np.array_equal(Aa, A64)
    say("ms refined, later solves redone")
    plate = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M,
                        precision=fth.FP32_REFINED, tol=1e-12)
    os.environ["FTHMS_REFINE_LATE_MAXIT"] = "0"
    try:
        Ul, Al = plate.run(om, want_alpha=True)
    finally:
        del os.environ["FTHMS_REFINE_LATE_MAXIT"]
    lay = oms.Layout(pb)
    for i, kk in enumerate(om):
        ref = oms.run_frequency(lay, kk)
        assert rel(Ul[i], ref["U"]) < TOL, (kk, rel(Ul[i], ref["U"]))
        assert rel(Al[i], np.concatenate(ref["alpha_tot"])) < TOL
