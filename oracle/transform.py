"""Oracle: frequency-to-time transform.

Test infrastructure only (see the package header).

u(x, t) = (1/2pi) int U(x, w) e^{-i w t} dw (Section 2.1, eq. backwardFT;
eq. TDsol-interior with a single window, s_1 = 0), truncated to the band
where the incident spectrum is non-negligible (Section 4.1, eq. ft_appr) and
evaluated by the trapezoid rule on a uniform positive-frequency grid:

    u(x_p, t_n) = (1/2pi) sum_l w_l U(x_p, w_l) e^{-i w_l t_n}.
"""
from __future__ import annotations

import math

import numpy as np


def trapezoid_weights(omegas):
    """Trapezoid weights on a uniform grid (half weight at both ends)."""
    om = np.asarray(omegas, dtype=float)
    h = np.diff(om)
    if om.size < 2 or not np.allclose(h, h[0], rtol=1e-12, atol=0.0):
        raise ValueError("uniform grid with at least two points required")
    w = np.full(om.size, h[0])
    w[0] *= 0.5
    w[-1] *= 0.5
    return w


def freq_to_time(omegas, weights, U, times):
    """U: [J, P] complex -> u: [T, P] complex (plain double sum)."""
    E = np.exp(-1j * np.outer(times, omegas)) * weights[None, :]
    return (E @ U) / (2.0 * math.pi)


def free_space_pulse(r, t, omega0, sigma, tau0, amp=10.0):
    """Closed form of the modulated point source in the time domain:
    amp * (G2 * f)(t) with the 2D wave Green's function
    G2(r, t) = H(t - r) / (2 pi sqrt(t^2 - r^2)) and
    f(t) = sigma/(2 sqrt pi) e^{-i w0 (t - tau0)} e^{-sigma^2 (t-tau0)^2/4};
    written as (amp / 2pi) int_0^inf f(t - r cosh v) dv."""
    from .incident import pulse_signal
    from .nystrom import adaptive_gl
    width = 12.0 / sigma
    hi_arg = (t - tau0 + width) / r
    if hi_arg <= 1.0:
        return 0.0 + 0.0j
    vmax = math.acosh(hi_arg)
    lo_arg = (t - tau0 - width) / r
    vmin = math.acosh(lo_arg) if lo_arg > 1.0 else 0.0
    br = []
    if (t - tau0) / r > 1.0:
        br.append(math.acosh((t - tau0) / r))

    def f(v):
        return pulse_signal(t - r * np.cosh(v), omega0, sigma, tau0)

    val = adaptive_gl(f, vmin, vmax, breaks=tuple(br), tol_abs=1e-16,
                      tol_rel=1e-14)
    return amp * val / (2.0 * math.pi)
