"""The allocation-free solve entry point against the ordinary one, through
the C-ABI: two calls in a row (the second with a smaller batch and a smaller
n, so the shared fixed scratch keeps the first call's contents), each
bit-identical to fthms_lu_solve_dev on the same factors; and the refusal of
a batch beyond the fixed scratch."""
import sys

import numpy as np
import pytest

from oracle import nystrom as ony

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2507_05725_amd as fth
    ctx = fth.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    return fth, ctx, torch


def _factored(torch, ctx, rng, n, nb):
    M = rng.standard_normal((nb, n, n)) + 1j * rng.standard_normal((nb, n, n))
    A = torch.tensor(np.ascontiguousarray(M.transpose(0, 2, 1)), device="cuda")
    piv = torch.empty((nb, n), dtype=torch.int32, device="cuda")
    ctx.lu_dev(A, piv)
    b = torch.tensor(rng.standard_normal((nb, n)) + 1j * rng.standard_normal((nb, n)),
                     device="cuda")
    return M, A, piv, b


def test_noalloc_solve_matches_solve_twice(env):
    fth, ctx, torch = env
    rng = np.random.default_rng(2024)
    for n, nb in ((300, 37), (65, 5)):
        say("noalloc lu_solve n", n, "nb", nb)
        M, A, piv, b = _factored(torch, ctx, rng, n, nb)
        x_ref = torch.empty_like(b)
        x_na = torch.empty_like(b)
        ctx.lu_solve_dev(A, piv, b, x_ref)
        ctx.lu_solve_noalloc_dev(A, piv, b, x_na)
        torch.cuda.synchronize()
        assert torch.equal(x_na, x_ref)
        xs = x_na.cpu().numpy()
        bs = b.cpu().numpy()
        for i in range(nb):
            ref = ony.solve(M[i], bs[i])
            assert np.linalg.norm(xs[i] - ref) / np.linalg.norm(ref) < 1e-10


def test_noalloc_solve_refuses_oversize_batch(env):
    fth, ctx, torch = env
    n, nb = 2, 4097
    A = torch.zeros((nb, n, n), dtype=torch.complex128, device="cuda")
    piv = torch.zeros((nb, n), dtype=torch.int32, device="cuda")
    b = torch.zeros((nb, n), dtype=torch.complex128, device="cuda")
    x = torch.empty_like(b)
    with pytest.raises(fth.FthmsError) as ei:
        ctx.lu_solve_noalloc_dev(A, piv, b, x)
    assert ei.value.code == -1
