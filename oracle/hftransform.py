"""Oracle: high-frequency Fourier transforms of real time signals and the
pulse incident fields u3, u4.

Test infrastructure only (see the package header).

Paper passages:
  * truncated inverse transform g(t) ~ (1/2pi) int_{-W}^{W} G(w) e^{-iwt} dw
    ............................................... Section 4.1, eq. ft_appr
  * split at +-w_c ...................................... eq. backwardFT1
  * regular integrals I_a^b[G] on [w_c, W]: Fourier continuation of the
    uniform samples, then term-wise exact integration ........... eq. int1
  * half-interval integrals I_0^{w_c}[G] with the log singularity at w = 0:
    graded points mu_j = w_c (j/P)^p, Clenshaw-Curtis on every
    (mu_j, mu_{j+1}), integrated against e^{-iwt} exactly (Filon) .. eq. int2
  * the frequency set: uniform on [w_c, W], Clenshaw-Curtis points on the
    graded intervals ........................................... Section 5
  * u3 = -sin(4 l) exp(-1.6 (l - 3)^2), l = t - t_lag - x.d, t_lag = 2;
    u4 = sum_{j=0}^{4} u3(x, t - 10 j) ............. eqs. planewave, multi

Readings (the cited constructions are not in the text):
  * Real signals: G(-w) = conj G(w), so
        g(t) ~ (1/pi) Re [ I_0^{w_c}[G](t) + I_{w_c}^{W}[G](t) ].
  * The graded intervals are (mu_j, mu_{j+1}), j = 1..P-1, mu_P = w_c; the
    piece (0, mu_1) of length w_c P^{-p} is left out (it holds the
    singularity; its contribution is of order mu_1 log mu_1).  Adjacent
    intervals share their end points (one frequency each).
  * Fourier continuation: least squares in the space of trigonometric
    polynomials sum_{|k| <= K} a_k exp(2 pi i k s / b) on s = w - w_c in
    [0, D], D = W - w_c, period b = 2 D, K = L/4 (about two samples per
    unknown), solved by a QR factorisation with column pivoting truncated at
    |R_ii| <= 1e-13 |R_00| -- a least-squares Fourier continuation, the form
    of the method in which the continuation is a plain linear least-squares
    fit.
  * Filon: on each interval the degree-(n-1) polynomial through the n
    Clenshaw-Curtis values (cos(pi i / (n-1)) mapped to the interval) is
    integrated against e^{-iwt} exactly; the oracle forms its Chebyshev
    coefficients by solving the interpolation system and the moments
    int_{-1}^{1} T_k(x) e^{-i kappa x} dx by Gauss-Legendre quadrature of
    enough points for the oscillation.

Every transform here is a linear map of the samples G(w_l) on the
frequency set, returned as a weight matrix Wt [nt][J] so that
g(t_n) ~ (1/pi) Re sum_l Wt[n, l] G(w_l).
"""
from __future__ import annotations

import math

import numpy as np


# ---------------------------------------------------------------------------
# pulses (Section 5, eqs. planewave and multi)
# ---------------------------------------------------------------------------
T_LAG = 2.0


def u3(x, t, theta):
    """u3(x, t) at points x [P, 2] and times t [T] -> [T, P] (real)."""
    d = np.array([math.cos(theta), math.sin(theta)])
    xd = np.asarray(x, dtype=float) @ d
    ell = np.asarray(t, dtype=float)[:, None] - T_LAG - xd[None, :]
    return -np.sin(4.0 * ell) * np.exp(-1.6 * (ell - 3.0) ** 2)


def u4(x, t, theta, npulse=5, period=10.0):
    """u4 = sum_{j < npulse} u3(x, t - period j) (the paper: 5 pulses, 10 apart)."""
    t = np.asarray(t, dtype=float)
    return sum(u3(x, t - period * j, theta) for j in range(npulse))


def u3_spectrum(x, w, theta):
    """Fourier transform int u3(x, t) e^{iwt} dt in closed form (Gaussian
    integrals: -sin(4s) = -(e^{4is} - e^{-4is}) / (2i) and
    int e^{ias} e^{-1.6 (s-3)^2} ds = sqrt(pi/1.6) e^{3ia} e^{-a^2/6.4}),
    shifted by the delay t_lag + x.d: [J, P]."""
    d = np.array([math.cos(theta), math.sin(theta)])
    xd = np.asarray(x, dtype=float) @ d
    w = np.asarray(w, dtype=float)[:, None]
    c = math.sqrt(math.pi / 1.6)

    def gauss(a):
        return c * np.exp(3j * a) * np.exp(-a * a / 6.4)

    core = -(gauss(w + 4.0) - gauss(w - 4.0)) / 2j
    return core * np.exp(1j * w * (T_LAG + xd[None, :]))


def u4_spectrum(x, w, theta, npulse=5, period=10.0):
    w = np.asarray(w, dtype=float)
    ph = sum(np.exp(1j * w * period * j) for j in range(npulse))
    return u3_spectrum(x, w, theta) * ph[:, None]


# ---------------------------------------------------------------------------
# the frequency set (Section 5)
# ---------------------------------------------------------------------------
def cc_points(n):
    """Clenshaw-Curtis points cos(pi i / (n-1)), i = 0..n-1 (decreasing)."""
    return np.cos(math.pi * np.arange(n) / (n - 1))


class FreqSet:
    """Frequencies of the transform: the Clenshaw-Curtis points of the graded
    intervals (mu_j, mu_{j+1}), j = 1..P-1 (mu_j = w_c (j/P)^p), then the
    uniform grid w_c + l (W - w_c)/L, l = 0..L.  ``omega`` is sorted and
    has no repeated point (shared interval ends and w_c appear once)."""

    def __init__(self, wc, W, P, p, ncc, L):
        self.wc, self.W, self.P, self.p, self.ncc, self.L = wc, W, P, p, ncc, L
        mu = wc * (np.arange(1, P + 1) / P) ** p
        self.mu = mu
        pts = []
        self.intervals = []
        for a, b in zip(mu[:-1], mu[1:]):
            x = 0.5 * (a + b) + 0.5 * (b - a) * cc_points(ncc)[::-1]  # increasing
            self.intervals.append((a, b))
            pts.append(x)
        self.uniform = wc + (W - wc) * np.arange(L + 1) / L
        allp = np.concatenate(pts + [self.uniform])
        # one frequency per distinct point (interval ends and w_c repeat)
        allp = np.sort(allp)
        keep = np.concatenate([[True], np.diff(allp) > 1e-14 * max(1.0, W)])
        self.omega = allp[keep]

    def index(self, w):
        """Position of frequency w in ``omega``."""
        i = int(np.argmin(np.abs(self.omega - w)))
        assert abs(self.omega[i] - w) <= 1e-13 * max(1.0, self.W)
        return i


# ---------------------------------------------------------------------------
# Filon-Clenshaw-Curtis on one interval (eq. int2)
# ---------------------------------------------------------------------------
def gauss_legendre(n):
    return np.polynomial.legendre.leggauss(n)


def cheb_moments(nk, kappa):
    """mu_k(kappa) = int_{-1}^{1} T_k(x) e^{-i kappa x} dx, k < nk, by
    Gauss-Legendre quadrature with enough points for degree nk and the
    oscillation (error far below double precision)."""
    npts = int(nk + 2.0 * abs(kappa) + 40)
    x, wq = gauss_legendre(npts)
    T = np.cos(np.outer(np.arange(nk), np.arccos(np.clip(x, -1.0, 1.0))))
    return T @ (wq * np.exp(-1j * kappa * x))


def filon_cc_weights(a, b, n, t):
    """Weights v_i(t) such that int_a^b p(w) e^{-iwt} dw = sum_i v_i f_i for
    the polynomial p of degree n-1 through the values f_i at the
    Clenshaw-Curtis points of [a, b] in increasing order: [len(t), n]."""
    x = cc_points(n)[::-1]
    V = np.cos(np.outer(np.arccos(np.clip(x, -1.0, 1.0)), np.arange(n)))  # V[i,k] = T_k(x_i)
    Vinv = np.linalg.inv(V)  # Chebyshev coefficients c = Vinv f
    m, r = 0.5 * (a + b), 0.5 * (b - a)
    out = np.empty((np.size(t), n), dtype=complex)
    for it, tt in enumerate(np.atleast_1d(t)):
        mom = cheb_moments(n, r * tt)
        out[it] = r * np.exp(-1j * m * tt) * (mom @ Vinv)
    return out


# ---------------------------------------------------------------------------
# Fourier continuation on [w_c, W] (eq. int1)
# ---------------------------------------------------------------------------
def fc_modes(L):
    """Number of modes on each side: K = floor(L / 4) (about two samples per
    unknown)."""
    return L // 4


def fc_weights(D, L, t, w0=0.0, rtol=1e-13):
    """Weights u_l(t) with int_{w0}^{w0+D} G(w) e^{-iwt} dw ~ sum_l u_l G(w0 + l D/L)
    for the least-squares Fourier continuation of the L+1 uniform samples
    (period b = 2D, modes |k| <= K): [len(t), L+1].

    The least-squares problem A a = G, A[l, k] = exp(2 pi i k s_l / b), is
    severely ill-conditioned (the continuation is far from unique); it is
    solved by a QR factorisation with column pivoting, A P = Q R, keeping the
    leading r columns with |R_ii| > rtol |R_00|, so that a = P R_r^{-1}
    Q_r^H G.  The weights follow without forming that inverse:
    u(t) = conj(Q_r) y with R_r^T y = (P^T E(t)), E_k(t) = int_0^D
    exp(i (2 pi k / b - t) s) ds exp(-i w0 t)."""
    from scipy.linalg import qr, solve_triangular
    s = D * np.arange(L + 1) / L
    K = fc_modes(L)
    ks = np.arange(-K, K + 1)
    b = 2.0 * D
    A = np.exp(2j * math.pi * np.outer(s, ks) / b)
    Q, R, P = qr(A, pivoting=True, mode="economic")
    d = np.abs(np.diag(R))
    r = int(np.sum(d > rtol * d[0]))
    out = np.empty((np.size(t), L + 1), dtype=complex)
    for it, tt in enumerate(np.atleast_1d(t)):
        kap = 2.0 * math.pi * ks / b - tt
        # int_0^D e^{i kap s} ds, with its limit D at kap = 0
        small = np.abs(kap * D) < 1e-8
        e = np.where(small, D + 0.5j * kap * D * D,
                     (np.exp(1j * kap * D) - 1.0) / (1j * np.where(small, 1.0, kap)))
        e = np.exp(-1j * w0 * tt) * e
        y = solve_triangular(R[:r, :r], e[P[:r]], trans="T")
        out[it] = Q[:, :r].conj() @ y
    return out


# ---------------------------------------------------------------------------
# the whole transform of a real signal
# ---------------------------------------------------------------------------
def transform_weights(fs, t, rtol=1e-13):
    """Wt [nt][J] on the frequency set fs: g(t_n) ~ (1/pi) Re sum_l Wt[n,l] G(w_l)."""
    t = np.atleast_1d(np.asarray(t, dtype=float))
    Wt = np.zeros((t.size, fs.omega.size), dtype=complex)
    for (a, b) in fs.intervals:
        x = 0.5 * (a + b) + 0.5 * (b - a) * cc_points(fs.ncc)[::-1]
        v = filon_cc_weights(a, b, fs.ncc, t)
        for i, w in enumerate(x):
            Wt[:, fs.index(w)] += v[:, i]
    u = fc_weights(fs.W - fs.wc, fs.L, t, w0=fs.wc, rtol=rtol)
    for l, w in enumerate(fs.uniform):
        Wt[:, fs.index(w)] += u[:, l]
    return Wt


def real_signal(fs, G, t, rtol=1e-13):
    """g(t) for the samples G [J, ...] on fs: (1/pi) Re(Wt G)."""
    Wt = transform_weights(fs, t, rtol)
    return np.real(Wt @ G) / math.pi
