"""Oracle: frequency-domain incident fields (Section 5, the list of incident
fields: eqs. pointsource and planewave2) and their closed-form time signals.

Test infrastructure only (see the package header).  Convention: forward
transform G(w) = int g(t) e^{+i w t} dt, inverse (1/2pi) int G e^{-i w t} dw
(Section 2.1, eqs. forwardFT / backwardFT); c = 1 so k = w.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special


def gaussian_factor(k, omega0, sigma, tau0):
    """exp(-(k - w0)^2 / sigma^2) exp(i k tau0)."""
    return np.exp(-((k - omega0) ** 2) / sigma ** 2) * np.exp(1j * k * tau0)


def plane(k, y, theta):
    """exp(i k y . d), d = (cos theta, sin theta)."""
    d = np.array([math.cos(theta), math.sin(theta)])
    return np.exp(1j * k * (y @ d))


def u1(k, y, z0, omega0, sigma, tau0):
    """Gaussian-modulated point source (5i/2) H0^(1)(k |y - z0|) * gauss.
    sigma = 0 means no modulation (a plain point source, amplitude 5i/2)."""
    r = np.hypot(y[..., 0] - z0[0], y[..., 1] - z0[1])
    f = 2.5j * special.hankel1(0, k * r)
    if sigma > 0:
        f = f * gaussian_factor(k, omega0, sigma, tau0)
    return f


def u2(k, y, theta, omega0, sigma, tau0):
    """Gaussian-modulated plane wave exp(i k y.d) * gauss."""
    return plane(k, y, theta) * gaussian_factor(k, omega0, sigma, tau0)


def incident(spec, k, y):
    if spec.kind == "plane":
        return plane(k, y, spec.theta)
    if spec.kind == "gplane":
        return u2(k, y, spec.theta, spec.omega0, spec.sigma, spec.tau0)
    if spec.kind == "point":
        return u1(k, y, spec.z0, spec.omega0, spec.sigma, spec.tau0)
    raise ValueError(spec.kind)


def pulse_signal(t, omega0, sigma, tau0):
    """Inverse transform of the Gaussian factor:
    f(t) = sigma / (2 sqrt(pi)) e^{-i w0 (t - tau0)} e^{-sigma^2 (t-tau0)^2/4}."""
    s = t - tau0
    return (sigma / (2.0 * math.sqrt(math.pi)) * np.exp(-1j * omega0 * s)
            * np.exp(-(sigma * s) ** 2 / 4.0))


def u2_time(x, t, theta, omega0, sigma, tau0):
    """Time-domain Gaussian plane wave: f(t - x.d) with f = pulse_signal."""
    d = np.array([math.cos(theta), math.sin(theta)])
    return pulse_signal(t - x @ d, omega0, sigma, tau0)
