"""Pins of the windowed recursion oracle (Section 2.1, eqs. windowing,
Fourierk, TDsol; the window function of Section 5): the window functions
form a smooth partition of unity, the pulse train is the time-domain form of
the Gaussian plane-wave spectrum, splitting the data into windows is exact
(different window layouts give the same traces to rounding), and with the
data resolved the windowed recursion reproduces the single-window
frequency-domain recursion."""
import math

import numpy as np
import pytest

from oracle import ms as oms
from oracle import transform as otr
from oracle import windowed as ow
from workloads import IncidentSpec, disc_interior_case


@pytest.mark.parametrize("Q,H", [(1, 10.0), (3, 4.0), (6, 10.0)])
def test_windows_partition_of_unity(Q, H):
    s = 1.5 * H * np.arange(Q)
    t = np.linspace(0.0, s[-1] + 0.5 * H, 4001)
    tot = sum(ow.pou(t - sq, H) for sq in s)
    assert np.max(np.abs(tot - 1.0)) < 1e-14
    # support [-H, H], values in [0, 1], continuous derivative
    u = np.linspace(-1.5 * H, 1.5 * H, 30001)
    P = ow.pou(u, H)
    assert np.all(P[np.abs(u) >= H] == 0.0) and np.all((P >= 0) & (P <= 1))
    d = np.diff(P) / np.diff(u)
    assert np.max(np.abs(np.diff(d))) < 1e-2


def test_pulse_is_the_gaussian_plane_wave_spectrum():
    """int f(tau) exp(i w tau) dtau = exp(-(w - w0)^2/sigma^2) exp(i w tau0)."""
    w0, sig, tau0 = 9.0, 1.3, 6.0
    tau = np.linspace(-40.0, 60.0, 200001)
    f = ow.pulse_train(np.zeros((1, 2)), tau, 0.0, w0, sig, tau0, 1, 0.0)[:, 0]
    for w in (5.0, 8.5, 9.0, 11.0):
        num = np.trapezoid(f * np.exp(1j * w * tau), tau)
        ref = math.exp(-(w - w0) ** 2 / sig ** 2) * np.exp(1j * w * tau0)
        assert abs(num - ref) < 1e-12


def _disc(nf, om0=9.0, sig=1.0, tau0=7.0, theta=0.3):
    om = np.linspace(om0 - 6 * sig, om0 + 6 * sig, nf)
    pb = disc_interior_case(n=12, omegas=om, M=2)
    pb.incident = IncidentSpec("gplane", theta=theta, omega0=om0, sigma=sig, tau0=tau0)
    inc = dict(theta=theta, omega0=om0, sigma=sig, tau0=tau0, npulse=1, period=0.0)
    return pb, om, otr.trapezoid_weights(om), inc


def test_window_layouts_agree():
    """Linearity: the traces do not depend on how the data are cut into
    windows (two layouts covering the same interval)."""
    pb, om, w, inc = _disc(31)
    lay = oms.Layout(pb)
    u1 = ow.run_windowed(lay, om, w, 0.1, 131, 2, 10.0, inc)
    u2 = ow.run_windowed(lay, om, w, 0.1, 131, 3, 6.5, inc)
    assert np.linalg.norm(u1 - u2) <= 1e-12 * np.linalg.norm(u1)


def test_windowed_matches_frequency_domain_recursion():
    """With the frequency grid and the time samples resolving the data, the
    windowed recursion gives the traces of the single-window recursion run
    per frequency (agreement limited by the finite time interval)."""
    pb, om, w, inc = _disc(61)
    lay = oms.Layout(pb)
    t = 0.1 * np.arange(151)
    uf, _ = oms.run_traces(lay, om, w, t)
    uw = ow.run_windowed(lay, om, w, 0.1, 151, 2, 10.0, inc)
    assert np.linalg.norm(uw - uf) <= 1e-3 * np.linalg.norm(uf)
