"""Per-kernel GPU parity: device Bessel functions, Nystrom assembly, batched
LU (both precisions) and the triangular solves, each against the oracle or
an independent library result, through the C-ABI single-stage entry points."""
import sys

import numpy as np
import pytest
from scipy import special

from oracle import nystrom as ony
from workloads import CircularArc, EllipseArc, Segment, SineArc

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2507_05725_amd as fth
    ctx = fth.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    return fth, ctx, torch


def test_device_bessel(env):
    fth, ctx, torch = env
    rng = np.random.default_rng(1)
    z = np.concatenate([np.geomspace(1e-9, 1.0, 200), rng.uniform(0, 20, 4000) + 1e-4,
                        np.array([8.0, 16.5, 16.5 - 1e-13]), rng.uniform(20, 1500, 2000)])
    say("bessel", z.size)
    zt = torch.tensor(z, device="cuda", dtype=torch.float64)
    j0 = torch.empty_like(zt)
    y0 = torch.empty_like(zt)
    ctx.bessel_dev(zt, j0, y0)
    torch.cuda.synchronize()
    rj = special.j0(z)
    ry = special.y0(z)
    ej = np.abs(j0.cpu().numpy() - rj)
    ey = np.abs(y0.cpu().numpy() - ry) / np.maximum(1.0, np.abs(ry))
    assert ej.max() < 5e-15, (ej.max(), z[ej.argmax()])
    assert ey.max() < 5e-15, (ey.max(), z[ey.argmax()])


@pytest.mark.parametrize("curve,n", [(Segment((-1.0, 0.0), (1.0, 0.0)), 48),
                                     (CircularArc(1.0, -1.25, 1.25), 100),
                                     (EllipseArc(1.4, 0.6, 0.3, 2.8), 33),
                                     (SineArc((0.0, 0.2), 2.5, 0.3, 3, -0.4), 257)])
def test_assembly_matches_oracle(env, curve, n):
    fth, ctx, torch = env
    k = np.array([0.5, 7.3, 31.0, 118.0])
    say("assembly", n)
    arc = ctx.arc_from_curve(curve, n)
    kt = torch.tensor(k, device="cuda", dtype=torch.float64)
    A = torch.empty((k.size, n, n), device="cuda", dtype=torch.complex128)
    ctx.assemble_dev(arc, kt, A)
    torch.cuda.synchronize()
    # device layout: column-major per matrix -> transpose the row-major view
    Ag = A.cpu().numpy().transpose(0, 2, 1)
    nd = ony.arc_nodes(curve, n)
    for b, kk in enumerate(k):
        ref = ony.assemble(nd, kk)
        err = np.max(np.abs(Ag[b] - ref)) / np.max(np.abs(ref))
        assert err < 1e-13, (n, kk, err, np.unravel_index(np.argmax(np.abs(Ag[b] - ref)), ref.shape))


@pytest.mark.parametrize("kgrid", ["low", "high"])
def test_assembly_dense_wavenumber_grid(env, kgrid):
    """Dense, evenly spaced wavenumbers (the assembly takes eight
    wavenumbers per workgroup): ragged group counts (21 and 20), arguments
    k r crossing the series / modulus-phase boundaries at 4 and 8 (low) and
    large arguments (high), against the oracle entry by entry."""
    fth, ctx, torch = env
    curve = CircularArc(1.0, 0.3, 2.8)
    n = 97
    k = np.linspace(1.0, 5.0, 21) if kgrid == "low" else 40.0 + 0.05 * np.arange(20)
    say("assembly dense grid", kgrid)
    arc = ctx.arc_from_curve(curve, n)
    kt = torch.tensor(k, device="cuda", dtype=torch.float64)
    A = torch.empty((k.size, n, n), device="cuda", dtype=torch.complex128)
    ctx.assemble_dev(arc, kt, A)
    torch.cuda.synchronize()
    Ag = A.cpu().numpy().transpose(0, 2, 1)
    nd = ony.arc_nodes(curve, n)
    for b, kk in enumerate(k):
        ref = ony.assemble(nd, kk)
        err = np.max(np.abs(Ag[b] - ref)) / np.max(np.abs(ref))
        assert err < 1e-13, (kgrid, b, kk, err)


def _lu_reconstruct(LU, piv):
    n = LU.shape[0]
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    P = np.arange(n)
    for i in range(n):
        p = piv[i]
        P[i], P[p] = P[p], P[i]
    return L @ U, P


@pytest.mark.parametrize("n", [1, 5, 8, 9, 16, 64, 65, 130, 300, 512, 777, 1024])
@pytest.mark.parametrize("prec", [0, 1])
def test_batched_lu(env, n, prec):
    # n > 512 (FP32) and n > 256 (FP64) take the LDS panel kernel for their
    # first blocks, the register panel for the rest
    fth, ctx, torch = env
    rng = np.random.default_rng(n)
    nb = 3
    M = rng.standard_normal((nb, n, n)) + 1j * rng.standard_normal((nb, n, n))
    say("lu n", n, "prec", prec)
    dt = torch.complex128 if prec == 0 else torch.complex64
    # column-major storage: pass the transpose's contiguous copy
    A = torch.tensor(np.ascontiguousarray(M.transpose(0, 2, 1)), dtype=dt, device="cuda")
    piv = torch.empty((nb, n), dtype=torch.int32, device="cuda")
    info = torch.empty(nb, dtype=torch.int32, device="cuda")
    ctx.lu_dev(A, piv, info, precision=prec)
    torch.cuda.synchronize()
    LUs = A.cpu().numpy().astype(np.complex128).transpose(0, 2, 1)
    pv = piv.cpu().numpy()
    assert np.all(info.cpu().numpy() == 0)
    for b in range(nb):
        assert np.all((pv[b] >= np.arange(n)) & (pv[b] < n))
        LU, P = _lu_reconstruct(LUs[b], pv[b])
        err = np.linalg.norm(LU - M[b][P]) / np.linalg.norm(M[b])
        if prec == 0:
            tol = 1e-13
        else:
            # backward error of LU with partial pivoting, |PA - LU| <= g |L||U|,
            # with g ~ sqrt(n) u for rounding errors of random sign (u = 2^-24;
            # the constant covers complex products and blocked accumulation)
            L = np.tril(LUs[b], -1) + np.eye(n)
            ref = np.linalg.norm(np.abs(L) @ np.abs(np.triu(LUs[b]))) / np.linalg.norm(M[b])
            tol = 8.0 * np.sqrt(n) * 2.0 ** -24 * ref
        assert err < tol, (n, prec, b, err, tol)
        # pivots maximise |re| + |im| over the column, so |L| <= sqrt(2)
        assert np.max(np.abs(np.tril(LUs[b], -1))) <= np.sqrt(2.0) + 1e-6


@pytest.mark.parametrize("n", [1, 7, 64, 65, 200, 512])
def test_lu_solve(env, n):
    fth, ctx, torch = env
    rng = np.random.default_rng(100 + n)
    nb = 2
    M = rng.standard_normal((nb, n, n)) + 1j * rng.standard_normal((nb, n, n)) + 3 * np.eye(n)
    bvec = rng.standard_normal((nb, n)) + 1j * rng.standard_normal((nb, n))
    say("lu_solve n", n)
    A = torch.tensor(np.ascontiguousarray(M.transpose(0, 2, 1)), device="cuda")
    piv = torch.empty((nb, n), dtype=torch.int32, device="cuda")
    ctx.lu_dev(A, piv)
    bt = torch.tensor(bvec, device="cuda")
    x = torch.empty_like(bt)
    ctx.lu_solve_dev(A, piv, bt, x)
    torch.cuda.synchronize()
    xs = x.cpu().numpy()
    for b in range(nb):
        ref = np.linalg.solve(M[b], bvec[b])
        assert np.linalg.norm(xs[b] - ref) / np.linalg.norm(ref) < 1e-12


def test_dev_calls_follow_torch_default_stream(env):
    """A context on torch's current stream (HIP's null stream; the binding
    passes handle 0 as NULL) orders its _dev calls after torch's earlier work
    on it: an LU enqueued right behind a slow product and the copy that fills
    its input factors the whole input, with no synchronisation between.  A
    private stream (OWN_STREAM) gives the same factors once the caller has
    synchronised."""
    fth, ctx, torch = env
    n, nb = 512, 64
    g = torch.Generator(device="cuda").manual_seed(3)
    A0 = torch.randn((nb, n, n), dtype=torch.complex64, device="cuda", generator=g)
    X = torch.randn((4096, 4096), dtype=torch.float32, device="cuda", generator=g)
    piv = torch.empty((nb, n), dtype=torch.int32, device="cuda")
    ref = A0.clone()
    torch.cuda.synchronize()
    ctx.lu_dev(ref, piv, precision=1)
    torch.cuda.synchronize()
    ref_piv = piv.clone()
    say("lu behind torch work", n, nb)
    for _ in range(3):
        A = torch.empty_like(A0)
        Y = X @ X  # keeps the stream busy for a while
        A.copy_(A0)
        ctx.lu_dev(A, piv, precision=1)
        torch.cuda.synchronize()
        assert torch.equal(A, ref) and torch.equal(piv, ref_piv)
        del Y
    own = fth.Context(0, stream=fth.OWN_STREAM)
    try:
        A = A0.clone()
        piv2 = torch.empty_like(piv)
        torch.cuda.synchronize()
        own.lu_dev(A, piv2, precision=1)
        own.sync()
        assert torch.equal(A, ref) and torch.equal(piv2, ref_piv)
    finally:
        own.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_lu_split_batch_bitwise(env, prec):
    """Large batches are factored as two halves on two streams; every matrix
    must come out bit-identical to factoring it alone."""
    fth, ctx, torch = env
    n, nb = 70, 301
    rng = np.random.default_rng(7)
    M = rng.standard_normal((nb, n, n)) + 1j * rng.standard_normal((nb, n, n))
    say("lu split batch", nb, "prec", prec)
    dt = torch.complex128 if prec == 0 else torch.complex64
    A = torch.tensor(np.ascontiguousarray(M.transpose(0, 2, 1)), dtype=dt, device="cuda")
    A1 = A.clone()
    piv = torch.empty((nb, n), dtype=torch.int32, device="cuda")
    ctx.lu_dev(A, piv, precision=prec)
    # the same batch with the two-stream split switched off
    import os
    A2 = A1.clone()
    piv2 = torch.empty_like(piv)
    os.environ["FTHMS_LU_SPLIT"] = "0"
    try:
        ctx.lu_dev(A2, piv2, precision=prec)
    finally:
        del os.environ["FTHMS_LU_SPLIT"]
    torch.cuda.synchronize()
    assert torch.equal(A2, A) and torch.equal(piv2, piv)
    piv1 = torch.empty((1, n), dtype=torch.int32, device="cuda")
    for b in (0, 1, 150, 151, 152, 153, 299, 300):
        one = A1[b:b + 1].clone()
        ctx.lu_dev(one, piv1, precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(one[0], A[b]), b
        assert torch.equal(piv1[0], piv[b]), b


@pytest.mark.parametrize("n", [7, 65, 300, 512, 1024])
def test_refined_solve_with_row_interchanges(env, n):
    """The refined solve (FP32 factors with pivoting, FP64 residuals) on
    random complex matrices, whose partial pivoting moves rows in every
    block: the gather of the permutation inside the refinement kernel and the
    FP32 substitutions after real swaps.  Every solve must converge by
    refinement alone (no FP64 redo) to the oracle's direct solve."""
    fth, ctx, torch = env
    rng = np.random.default_rng(500 + n)
    nb = 3
    M = rng.standard_normal((nb, n, n)) + 1j * rng.standard_normal((nb, n, n))
    bvec = rng.standard_normal((nb, n)) + 1j * rng.standard_normal((nb, n))
    say("lu_refine n", n)
    Acm = np.ascontiguousarray(M.transpose(0, 2, 1))
    A64 = torch.tensor(Acm, dtype=torch.complex128, device="cuda")
    LU32 = torch.tensor(Acm, dtype=torch.complex64, device="cuda")
    piv = torch.empty((nb, n), dtype=torch.int32, device="cuda")
    info = torch.empty(nb, dtype=torch.int32, device="cuda")
    ctx.lu_dev(LU32, piv, info, precision=1)
    bt = torch.tensor(bvec, device="cuda")
    x = torch.empty_like(bt)
    iters = torch.empty(nb, dtype=torch.int32, device="cuda")
    relres = torch.empty(nb, dtype=torch.float64, device="cuda")
    ctx.lu_refine_dev(A64, LU32, piv, bt, x, tol=1e-12, max_iter=10, iters=iters,
                      relres=relres)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    pv = piv.cpu().numpy()
    it = iters.cpu().numpy()
    xs = x.cpu().numpy()
    # the input is untouched (it is the FP64 residual's matrix)
    assert torch.equal(A64.cpu(), torch.tensor(Acm))
    for b in range(nb):
        if n > 1:
            assert np.any(pv[b] != np.arange(n)), "test matrix did not pivot"
        assert it[b] >= 1, (n, b, it[b])
        ref = ony.solve(M[b], bvec[b])
        err = np.linalg.norm(xs[b] - ref) / np.linalg.norm(ref)
        assert err < 1e-10, (n, b, err, it[b])


def _symmetric_dominant(rng, nb, n):
    """Complex symmetric matrices whose columns are dominated by their
    diagonal (|re| + |im| of the diagonal above the column sum of the rest),
    so that partial pivoting makes no interchange at any step."""
    R = rng.standard_normal((nb, n, n)) + 1j * rng.standard_normal((nb, n, n))
    S = 0.5 * (R + R.transpose(0, 2, 1))
    return S + (2.0 * n) * (1 + 1j) * np.eye(n)


def _pp_swaps(M):
    """Row interchanges of partial pivoting (largest |re| + |im|, first row on
    ties) in FP64, plain right-looking elimination."""
    A = M.astype(np.complex128).copy()
    n = A.shape[0]
    swaps = 0
    for c in range(n):
        mag = np.abs(A[c:, c].real) + np.abs(A[c:, c].imag)
        p = c + int(np.argmax(mag))
        if mag[p - c] > mag[0]:
            swaps += 1
            A[[c, p]] = A[[p, c]]
        A[c + 1:, c] /= A[c, c]
        A[c + 1:, c + 1:] -= np.outer(A[c + 1:, c], A[c, c + 1:])
    return swaps


@pytest.mark.parametrize("n", [1, 5, 64, 65, 130, 300, 512])
def test_symmetric_lu(env, n):
    """The symmetric form (complex symmetric A, no row interchanges, updates
    on and below the diagonal only) on matrices that partial pivoting would
    not permute: identity pivots, info 0, factors with the FP32 backward
    error of an LU, and the refined solve with those factors converging by
    refinement alone to the oracle's direct solve."""
    fth, ctx, torch = env
    rng = np.random.default_rng(700 + n)
    nb = 3
    M = _symmetric_dominant(rng, nb, n)
    assert all(_pp_swaps(M[b]) == 0 for b in range(nb))
    bvec = rng.standard_normal((nb, n)) + 1j * rng.standard_normal((nb, n))
    say("symmetric lu n", n)
    Acm = np.ascontiguousarray(M.transpose(0, 2, 1))
    LU32 = torch.tensor(Acm, dtype=torch.complex64, device="cuda")
    A64 = torch.tensor(Acm, dtype=torch.complex128, device="cuda")
    piv = torch.empty((nb, n), dtype=torch.int32, device="cuda")
    info = torch.empty(nb, dtype=torch.int32, device="cuda")
    ctx.lu_dev(LU32, piv, info, precision=fth.FP32_SYM)
    bt = torch.tensor(bvec, device="cuda")
    x = torch.empty_like(bt)
    iters = torch.empty(nb, dtype=torch.int32, device="cuda")
    ctx.lu_refine_dev(A64, LU32, piv, bt, x, tol=1e-12, max_iter=10, iters=iters)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    assert np.array_equal(piv.cpu().numpy(), np.tile(np.arange(n), (nb, 1)))
    LUs = LU32.cpu().numpy().astype(np.complex128).transpose(0, 2, 1)
    it = iters.cpu().numpy()
    xs = x.cpu().numpy()
    for b in range(nb):
        L = np.tril(LUs[b], -1) + np.eye(n)
        U = np.triu(LUs[b])
        err = np.linalg.norm(L @ U - M[b]) / np.linalg.norm(M[b])
        ref = np.linalg.norm(np.abs(L) @ np.abs(U)) / np.linalg.norm(M[b])
        assert err < 8.0 * np.sqrt(n) * 2.0 ** -24 * ref, (n, b, err)
        assert it[b] >= 1, (n, b, it[b])
        sol = ony.solve(M[b], bvec[b])
        assert np.linalg.norm(xs[b] - sol) / np.linalg.norm(sol) < 1e-10


@pytest.mark.parametrize("n", [65, 300, 512])
def test_symmetric_lu_flags_pivoting(env, n):
    """The symmetric form refuses what partial pivoting would permute: a
    random complex symmetric matrix (interchanges from the first column on)
    and a dominant one with one small diagonal entry late in the matrix (an
    interchange at that column only) get info -2; the dominant ones beside
    them in the batch get 0.  Sizes beyond 512 are refused."""
    fth, ctx, torch = env
    rng = np.random.default_rng(900 + n)
    M = _symmetric_dominant(rng, 4, n)
    R = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    M[1] = 0.5 * (R + R.T)
    k = n - 40
    M[3][k, k] = 1e-3
    expect = [0, -2, 0, -2]
    for b in range(4):
        assert (_pp_swaps(M[b]) > 0) == (expect[b] == -2)
    say("symmetric lu flags n", n)
    LU32 = torch.tensor(np.ascontiguousarray(M.transpose(0, 2, 1)), dtype=torch.complex64,
                        device="cuda")
    piv = torch.empty((4, n), dtype=torch.int32, device="cuda")
    info = torch.empty(4, dtype=torch.int32, device="cuda")
    ctx.lu_dev(LU32, piv, info, precision=fth.FP32_SYM)
    torch.cuda.synchronize()
    assert list(info.cpu().numpy()) == expect
    big = torch.zeros((1, 513, 513), dtype=torch.complex64, device="cuda")
    p2 = torch.empty((1, 513), dtype=torch.int32, device="cuda")
    with pytest.raises(fth.FthmsError):
        ctx.lu_dev(big, p2, precision=fth.FP32_SYM)


def test_symmetric_lu_large_batch_flags(env):
    """A batch large enough (2100 matrices, halves of 1050) that the
    diagonal blocks are factored one wave per matrix: matrices with a small
    diagonal entry in the first 64 x 64 block, in the partial last block
    (N = 96) or an exactly zero pivot get info -2, all others 0 with
    identity pivots, and every factor equals the factor of the same matrix
    alone (the 1024-thread register panel) bit for bit."""
    fth, ctx, torch = env
    rng = np.random.default_rng(4242)
    n, nb = 96, 2100
    M = _symmetric_dominant(rng, nb, n)
    planted = {5: 20, 1500: 70, 2000: 40}
    M[5][20, 20] = 1e-3
    M[1500][70, 70] = 1e-3
    M[2000][40, 40] = 0.0
    for b in planted:
        assert _pp_swaps(M[b]) > 0
    for b in (0, 1049, 1050, 2099):
        assert _pp_swaps(M[b]) == 0
    say("symmetric lu, batch of", nb)
    Acm = np.ascontiguousarray(M.transpose(0, 2, 1))
    LU32 = torch.tensor(Acm, dtype=torch.complex64, device="cuda")
    piv = torch.empty((nb, n), dtype=torch.int32, device="cuda")
    info = torch.empty(nb, dtype=torch.int32, device="cuda")
    ctx.lu_dev(LU32, piv, info, precision=fth.FP32_SYM)
    torch.cuda.synchronize()
    inf = info.cpu().numpy()
    expect = np.zeros(nb, dtype=inf.dtype)
    for b in planted:
        expect[b] = -2
    assert np.array_equal(inf, expect), np.nonzero(inf != expect)
    ok = inf == 0
    assert np.array_equal(piv.cpu().numpy()[ok], np.tile(np.arange(n), (int(ok.sum()), 1)))
    LUb = LU32.cpu().numpy()
    for b in (0, 17, 1049, 1050, 2099):
        one = torch.tensor(Acm[b:b + 1], dtype=torch.complex64, device="cuda")
        p1 = torch.empty((1, n), dtype=torch.int32, device="cuda")
        i1 = torch.empty(1, dtype=torch.int32, device="cuda")
        ctx.lu_dev(one, p1, i1, precision=fth.FP32_SYM)
        torch.cuda.synchronize()
        assert int(i1.cpu().numpy()[0]) == 0
        assert np.array_equal(one.cpu().numpy()[0], LUb[b]), b


def test_refined_solve_reports_cap(env):
    """With a cap of one step and an unreachable tolerance the refinement
    reports -1 (not converged) and still returns its last iterate."""
    fth, ctx, torch = env
    n, nb = 200, 2
    rng = np.random.default_rng(77)
    M = rng.standard_normal((nb, n, n)) + 1j * rng.standard_normal((nb, n, n))
    bvec = rng.standard_normal((nb, n)) + 1j * rng.standard_normal((nb, n))
    Acm = np.ascontiguousarray(M.transpose(0, 2, 1))
    A64 = torch.tensor(Acm, dtype=torch.complex128, device="cuda")
    LU32 = torch.tensor(Acm, dtype=torch.complex64, device="cuda")
    piv = torch.empty((nb, n), dtype=torch.int32, device="cuda")
    ctx.lu_dev(LU32, piv, precision=1)
    bt = torch.tensor(bvec, device="cuda")
    x = torch.empty_like(bt)
    iters = torch.empty(nb, dtype=torch.int32, device="cuda")
    say("lu_refine cap", n)
    ctx.lu_refine_dev(A64, LU32, piv, bt, x, tol=1e-30, max_iter=1, iters=iters)
    torch.cuda.synchronize()
    assert np.all(iters.cpu().numpy() == -1)
    xs = x.cpu().numpy()
    for b in range(nb):
        ref = ony.solve(M[b], bvec[b])
        assert np.linalg.norm(xs[b] - ref) / np.linalg.norm(ref) < 1e-6
    with pytest.raises(fth.FthmsError):
        ctx.lu_refine_dev(A64, LU32, piv, bt, x, tol=1e-12, max_iter=0)
