"""GPU: the high-frequency transform of real signals (Section 4.1, eqs.
ft_appr, backwardFT1, int1, int2) through the C-ABI against the oracle's
weights, and against the time signal whose exact spectrum is transformed
(the single pulse u3 of Section 5, eq. planewave)."""
import sys

import numpy as np
import pytest

from oracle import hftransform as hf

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def env():
    import paper_2507_05725_amd as fth
    return fth, fth.Context(0)


@pytest.mark.parametrize("grid,nt", [((1.0, 20.0, 8, 10.0, 11, 800), 301),
                                     ((0.7, 14.0, 6, 8.0, 9, 150), 67)])
def test_hf_transform_matches_oracle(env, grid, nt):
    fth, ctx = env
    X = np.array([[0.5, 0.0], [-0.3, 0.7], [0.1, -0.9], [1.2, 0.4]])
    fs = hf.FreqSet(*grid)
    om = fth.hf_frequencies(fth.hf_grid(*grid))
    assert np.max(np.abs(om - fs.omega)) < 1e-14 * grid[1]
    # smooth samples: the spectrum of a single pulse at several points and
    # its product with a slowly varying factor
    U = hf.u3_spectrum(X, om, 0.4)
    U = np.concatenate([U, U * np.exp(-0.05 * om)[:, None] * (1 + 0.3j)], axis=1)
    t0, dt = -3.0, 0.2
    say("hf transform", om.size, "frequencies,", nt, "times")
    u = ctx.hf_to_time(fth.hf_grid(*grid), U, t0, dt, nt)
    t = t0 + dt * np.arange(nt)
    ref = hf.real_signal(fs, U, t)
    err = np.max(np.abs(u - ref)) / np.max(np.abs(ref))
    say("hf transform vs oracle: %.2e" % err)
    assert err < 1e-10
    exact = hf.u3(X, t, 0.4)
    assert np.max(np.abs(u[:, :4] - exact)) < (1e-8 if grid[5] >= 800 else 1e-5)
