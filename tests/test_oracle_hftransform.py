"""Pins of the oracle's high-frequency transforms and pulses (Section 4.1,
eqs. ft_appr, backwardFT1, int1, int2; Section 5, eqs. planewave, multi)
against closed forms, brute-force quadrature and the time signals
themselves."""
import math

import numpy as np
import pytest

from oracle import hftransform as hf


X = np.array([[0.5, 0.0], [-0.3, 0.7], [0.1, -0.9]])


def test_pulse_definitions():
    """u3 by hand at one point and time (eq. planewave, t_lag = 2); u4 is five
    copies 10 apart (eq. multi)."""
    th = 0.4
    x = X[:1]
    t = np.array([6.3])
    ell = 6.3 - 2.0 - 0.5 * math.cos(th)
    want = -math.sin(4 * ell) * math.exp(-1.6 * (ell - 3.0) ** 2)
    assert abs(hf.u3(x, t, th)[0, 0] - want) < 1e-15
    tt = np.linspace(0, 60, 601)
    u4 = hf.u4(X, tt, th)
    ref = sum(hf.u3(X, tt - 10.0 * j, th) for j in range(5))
    assert np.array_equal(u4, ref)


def test_pulse_spectra_against_quadrature():
    """The closed-form transforms equal the trapezoid sum of the time signal
    over a window holding the whole (Gaussian-decaying) signal: spectral
    accuracy for a smooth signal decaying like e^{-1.6 s^2}."""
    th = 1.1
    t = np.linspace(-30.0, 90.0, 96001)
    dt = t[1] - t[0]
    w = np.array([0.05, 0.7, 3.2, 4.0, 5.5, 9.0, 13.0, 19.5])
    for sig, spec in ((hf.u3(X, t, th), hf.u3_spectrum(X, w, th)),
                      (hf.u4(X, t, th), hf.u4_spectrum(X, w, th))):
        num = (np.exp(1j * np.outer(w, t)) * dt) @ sig
        assert np.max(np.abs(num - spec)) < 1e-11 * np.max(np.abs(spec))


def test_chebyshev_moments_closed_forms():
    """mu_0 = 2 sin(k)/k and mu_1 = -2i (sin k - k cos k)/k^2 (int of T_0, T_1
    against e^{-ikx} over [-1, 1]), and mu_k(0) = int T_k = (1 + (-1)^k)/(1 - k^2)."""
    for kap in (1e-3, 0.7, 5.0, 37.5, 150.0):
        m = hf.cheb_moments(6, kap)
        assert abs(m[0] - 2 * math.sin(kap) / kap) < 1e-13
        assert abs(m[1] - (-2j) * (math.sin(kap) - kap * math.cos(kap)) / kap ** 2) < 1e-13
    m0 = hf.cheb_moments(9, 0.0)
    for k in range(9):
        want = 0.0 if k == 1 else (1 + (-1) ** k) / (1 - k * k)
        assert abs(m0[k] - want) < 1e-13


def test_filon_exact_for_polynomials():
    """Filon-Clenshaw-Curtis integrates p(w) e^{-iwt} exactly for p of degree
    < n, at small and large t (reference: high-order Gauss-Legendre of the
    same integrand, resolved)."""
    rng = np.random.default_rng(4)
    c = rng.standard_normal(9)
    a, b, n = 0.3, 1.7, 9
    xw = 0.5 * (a + b) + 0.5 * (b - a) * hf.cc_points(n)[::-1]
    p = np.polynomial.polynomial.polyval(xw, c)
    tt = np.array([0.0, 3.0, 40.0, 400.0])
    v = hf.filon_cc_weights(a, b, n, tt)
    xg, wg = np.polynomial.legendre.leggauss(2000)
    wq = 0.5 * (a + b) + 0.5 * (b - a) * xg
    for i, t in enumerate(tt):
        ref = 0.5 * (b - a) * np.sum(wg * np.polynomial.polynomial.polyval(wq, c)
                                     * np.exp(-1j * wq * t))
        # rounding of the interpolation (values up to max|p|) and moments
        assert abs(v[i] @ p - ref) < 1e-12 * max(1.0, abs(ref), np.max(np.abs(p)))


def test_fourier_continuation_integrals():
    """The continuation's term-wise integrals of e^{i a w} and of a
    Gaussian-modulated e^{i a w} over [w0, w0 + D] against their closed
    forms, for times from 0 to far beyond the band (eq. int1)."""
    w0, D, L = 1.0, 19.0, 400
    s = w0 + D * np.arange(L + 1) / L
    tt = np.array([0.0, 0.37, 6.0, 25.0, 80.0, 300.0])
    U = hf.fc_weights(D, L, tt, w0=w0)
    for a in (0.0, 3.3, -7.1):
        f = np.exp(1j * a * s)
        for i, t in enumerate(tt):
            kap = a - t
            ref = (np.exp(1j * kap * (w0 + D)) - np.exp(1j * kap * w0)) / (1j * kap) \
                if abs(kap) > 1e-12 else D + 0j
            assert abs(U[i] @ f - ref) < 1e-11 * max(1.0, abs(ref)), (a, t)
    # a smooth non-periodic function with a known transform: the Gaussian
    # e^{-(w-6)^2/4} e^{2.5 i w}; the reference is resolved quadrature
    g = np.exp(-(s - 6.0) ** 2 / 4.0) * np.exp(2.5j * s)
    xg, wg = np.polynomial.legendre.leggauss(3000)
    wq = w0 + 0.5 * D * (xg + 1.0)
    for i, t in enumerate(tt):
        ref = 0.5 * D * np.sum(wg * np.exp(-(wq - 6.0) ** 2 / 4.0) * np.exp(2.5j * wq)
                               * np.exp(-1j * wq * t))
        assert abs(U[i] @ g - ref) < 1e-11


def test_log_singular_half_interval():
    """The graded Filon-Clenshaw-Curtis part integrates a spectrum with a
    logarithmic singularity at w = 0 (eq. int2), G(w) = log(w) e^{-w},
    against mpmath quadrature of int_0^{w_c} log(w) e^{-w} e^{-iwt} dw.  With
    enough points per interval the error is the left-out piece (0, mu_1), of
    order mu_1 |log mu_1|; finer grading brings it below 1e-9."""
    import mpmath
    tt = np.array([0.0, 2.0, 15.0, 60.0])
    refs = []
    for t in tt:
        f = lambda w, t=t: mpmath.log(w) * mpmath.exp(-w) * mpmath.exp(-1j * w * t)
        refs.append(complex(mpmath.quad(f, mpmath.linspace(0, 1, 9))))
    for (P, p, ncc, bound) in ((8, 10.0, 15, None), (10, 12.0, 15, 1e-9)):
        fs = hf.FreqSet(1.0, 20.0, P, p, ncc, 80)
        cc = np.array([w for w in fs.omega if w <= fs.wc + 1e-15])
        G = np.log(cc) * np.exp(-cc)
        Wt = np.zeros((tt.size, cc.size), dtype=complex)
        for (a, b) in fs.intervals:
            x = 0.5 * (a + b) + 0.5 * (b - a) * hf.cc_points(fs.ncc)[::-1]
            v = hf.filon_cc_weights(a, b, fs.ncc, tt)
            for i, w in enumerate(x):
                Wt[:, int(np.argmin(np.abs(cc - w)))] += v[:, i]
        err = np.abs(Wt @ G - np.array(refs))
        mu1 = fs.mu[0]
        lim = bound if bound is not None else 1.5 * mu1 * abs(math.log(mu1))
        assert np.all(err < lim), (P, p, ncc, err, lim)


@pytest.mark.slow
def test_real_signal_round_trip():
    """The whole transform of a real signal: the exact spectrum of u3 on the
    frequency set (graded Clenshaw-Curtis near 0, uniform on [w_c, W])
    gives back u3(t) for t up to 200 (no periodic images: the transform is
    a quadrature, not a discrete Fourier series)."""
    fs = hf.FreqSet(1.0, 20.0, 8, 10.0, 11, 800)
    tt = np.linspace(0.0, 200.0, 201)
    g = hf.real_signal(fs, hf.u3_spectrum(X, fs.omega, 0.4), tt)
    assert np.max(np.abs(g - hf.u3(X, tt, 0.4))) < 1e-8
    # the set: no repeated frequency, all positive, graded points below w_c
    assert np.all(np.diff(fs.omega) > 0) and fs.omega[0] > 0
    assert fs.omega.size == (fs.P - 1) * (fs.ncc - 1) + fs.L + 1
