"""The device Bessel routines, compiled for the host, against mpmath.

The same header the HIP kernels include is built into a small CPU probe
(tests/native/bessel_probe.cpp) with hipcc; nothing runs on a GPU.  The
absolute error bound 1.5e-15 holds uniformly over [0, 1500], covering every
regime boundary of the order-zero routines (series below 4, fitted modulus
functions on [4, 8), [8, 24) and beyond) and of the order-one routine (1e-6, 8,
16.5); the order-zero values also satisfy the Wronskian with the order-one
values of the independent order-one routine."""
import os
import shutil
import subprocess
import tempfile

import mpmath as mp
import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def probe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp(prefix="bprobe")
    exe = os.path.join(d, "bprobe")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O2", "-o", exe,
                    os.path.join(HERE, "native", "bessel_probe.cpp")],
                   check=True, capture_output=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def _run(exe, z):
    out = subprocess.run([exe], input="\n".join("%.17g" % v for v in z),
                         capture_output=True, text=True, check=True).stdout
    return np.array([[float(x) for x in l.split()] for l in out.strip().splitlines()])


def test_phase_sincos_against_mpmath(probe):
    """The phase sine and cosine of the modulus-phase form (Cody-Waite
    reduction, Taylor polynomials) within 2e-16 of mpmath on [0, 1e5],
    next to multiples of pi/2 included, and the library's beyond 1e6."""
    mp.mp.dps = 40
    rng = np.random.default_rng(11)
    k = rng.integers(1, 60000, 200)
    z = np.concatenate([rng.uniform(0.0, 100.0, 300), rng.uniform(100.0, 1e5, 300),
                        k * (np.pi / 2) + rng.uniform(-1e-9, 1e-9, 200),
                        np.array([0.0, 1e-300, np.pi / 4, 3 * np.pi / 4, 2e6])])
    res = _run(probe, z)
    worst = 0.0
    for row in res:
        zz = mp.mpf(row[0])
        worst = max(worst, float(abs(row[9] - mp.sin(zz))), float(abs(row[10] - mp.cos(zz))))
    assert worst < 2e-16, worst


def test_device_bessel_against_mpmath(probe):
    mp.mp.dps = 30
    rng = np.random.default_rng(7)
    z = np.concatenate([
        np.geomspace(1e-9, 1e-5, 20),
        np.array([1e-6, 4.0 - 1e-12, 4.0, 8.0 - 1e-12, 8.0, 16.5, 24.0 - 1e-12, 24.0]),
        rng.uniform(0.0, 20.0, 600) + 1e-3, rng.uniform(20.0, 30.0, 200),
        rng.uniform(20.0, 1500.0, 300)])
    res = _run(probe, z)
    g = mp.euler
    worst = 0.0
    for row in res:
        zz = mp.mpf(row[0])
        j0 = mp.besselj(0, zz)
        y0 = mp.bessely(0, zz)
        yh = y0 - 2 / mp.pi * (mp.log(zz / 2) + g) * j0
        e = max(abs(row[1] - j0), abs(row[2] - y0) / max(1, abs(y0)),
                abs(row[3] - j0), abs(row[4] - yh))
        worst = max(worst, float(e))
    assert worst < 1.5e-15


def test_device_bessel_order_one_against_mpmath(probe):
    """J1, Y1 (and J0, Y0 from the same routine) of the double-layer kernel:
    absolute error, relative where |Y| > 1 (Y1 ~ -2/(pi z) at small z)."""
    mp.mp.dps = 30
    rng = np.random.default_rng(8)
    z = np.concatenate([
        np.geomspace(1e-9, 1e-5, 20),
        np.array([1e-6 * (1 - 1e-12), 1e-6, 8.0 - 1e-12, 8.0, 16.5 - 1e-12, 16.5]),
        rng.uniform(0.0, 20.0, 600) + 1e-3,
        rng.uniform(20.0, 1500.0, 300)])
    res = _run(probe, z)
    worst = 0.0
    for row in res:
        zz = mp.mpf(row[0])
        j0, y0 = mp.besselj(0, zz), mp.bessely(0, zz)
        j1, y1 = mp.besselj(1, zz), mp.bessely(1, zz)
        e = max(abs(row[5] - j0), abs(row[6] - y0) / max(1, abs(y0)),
                abs(row[7] - j1), abs(row[8] - y1) / max(1, abs(y1)))
        worst = max(worst, float(e))
    assert worst < 2e-15


def test_device_bessel_wronskian(probe):
    """J1 Y0 - J0 Y1 = 2 / (pi z) (DLMF 10.5.2) with J0, Y0 from the order-zero
    routines and J1, Y1 from the order-one routine (a different method in
    every regime), relative to the size of the two products."""
    rng = np.random.default_rng(9)
    z = np.concatenate([np.geomspace(1e-4, 4.0, 200), rng.uniform(3.9, 8.1, 300),
                        rng.uniform(8.0, 20.0, 300), rng.uniform(20.0, 28.0, 200),
                        rng.uniform(20.0, 1500.0, 300)])
    res = _run(probe, z)
    zz, j0, y0, j1, y1 = res[:, 0], res[:, 1], res[:, 2], res[:, 7], res[:, 8]
    w = j1 * y0 - j0 * y1
    scale = np.abs(j1 * y0) + np.abs(j0 * y1)
    assert np.max(np.abs(w - 2.0 / (np.pi * zz)) / scale) < 4e-15
