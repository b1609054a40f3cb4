"""Pins of the special functions the oracle calls: SciPy's H0^(1) and J0
against mpmath (an independent arbitrary-precision implementation) over the
argument range of the workloads, plus the Wronskian identity."""
import mpmath as mp
import numpy as np
from scipy import special

from oracle import nystrom as ny


def test_hankel_against_mpmath():
    mp.mp.dps = 30
    z = np.concatenate([np.geomspace(1e-8, 1.0, 25), np.linspace(1.0, 30.0, 60),
                        np.geomspace(30.0, 1500.0, 40)])
    h = ny.hankel0(z)
    for zi, hi in zip(z, h):
        ref = complex(mp.besselj(0, zi) + 1j * mp.bessely(0, zi))
        assert abs(hi - ref) < 4e-15 * max(1.0, abs(ref))


def test_complex_argument_against_mpmath():
    mp.mp.dps = 30
    for z in (0.3 + 0.1j, 5.0 + 2.0j, 12.5 + 3.0j, 40.0 + 16.0j):
        ref = complex(mp.hankel1(0, z))
        assert abs(ny.hankel0(z) - ref) < 1e-14 * abs(ref)
        assert abs(ny.bessel_j0(z) - complex(mp.besselj(0, z))) < 1e-14 * max(
            1.0, abs(complex(mp.besselj(0, z))))


def test_wronskian():
    z = np.linspace(0.05, 400.0, 5000)
    w = special.j1(z) * special.y0(z) - special.j0(z) * special.y1(z)
    assert np.max(np.abs(w - 2.0 / (np.pi * z)) * z) < 1e-13
