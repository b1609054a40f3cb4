"""Pins of the frequency-to-time oracle and of the incident-field
conventions: the modulated point source against the closed-form
time-domain convolution with the 2D wave Green's function, and the
modulated plane wave against its closed form."""
import math

import numpy as np

from oracle import incident as inc
from oracle import transform as tr


def test_trapezoid_weights():
    om = 0.5 + 0.25 * np.arange(9)
    w = tr.trapezoid_weights(om)
    assert np.isclose(w.sum(), om[-1] - om[0])
    assert w[0] == w[-1] == 0.125


def test_free_space_point_source_pulse():
    """u1 through the trapezoid transform (omega_l = 80 l / 512) equals
    10 (G2 * f)(t), G2 = H(t - r) / (2 pi sqrt(t^2 - r^2)): pins the
    transform sign, the 1/2pi, the weights and the outgoing H0^(1)."""
    om = 80.0 * np.arange(1, 513) / 512
    w = tr.trapezoid_weights(om)
    x = np.array([[1.0, 0.0]])
    U = np.array([inc.u1(k, x, (0.0, 0.0), 20.0, 4.0, 4.0) for k in om])
    ts = np.array([3.5, 4.8, 5.0, 5.3, 6.0, 7.5])
    u = tr.freq_to_time(om, w, U, ts)[:, 0]
    ref = np.array([tr.free_space_pulse(1.0, t, 20.0, 4.0, 4.0) for t in ts])
    assert np.max(np.abs(u - ref)) < 2e-11
    assert np.max(np.abs(ref)) > 0.4


def test_gaussian_plane_wave_closed_form():
    """u2 through the transform equals f(t - x.d) with the closed-form
    Gaussian pulse f (eq. planewave2 and the convention eq. backwardFT)."""
    om = 40.0 * np.arange(1, 401) / 400
    w = tr.trapezoid_weights(om)
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, (5, 2))
    U = np.stack([inc.u2(k, x, 0.7, 15.0, 2.5, 5.0) for k in om])
    ts = np.linspace(0.0, 12.0, 41)
    u = tr.freq_to_time(om, w, U, ts)
    ref = np.stack([inc.u2_time(x, t, 0.7, 15.0, 2.5, 5.0) for t in ts])
    assert np.max(np.abs(u - ref)) < 1e-12
