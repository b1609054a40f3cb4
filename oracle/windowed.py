"""Oracle: windowing and time recentering of the multiple-scattering
recursion (Section 2.1, eqs. windowing, Fourierk, TDsol; Algorithm 1 with
Q windows; the window function of Section 5).

Test infrastructure only (see the package header).

Each step m works on boundary data g_{j,m}(x, t) in the time domain at the
nodes of every arc: for every window q the data are multiplied by
P_q(t) = P(t - s_q) and transformed about the window centre s_q (the slow
transform of eq. Fourierk, trapezoid rule on the time samples), the
frequency-domain integral equations are solved for every frequency (the
factors of step one are reused: only the right-hand sides change), the
field of the density is evaluated at the other arcs' nodes and at the
observation points, and transformed back with the shift of eq. TDsol:
    v_{j,m}(x, t) += (1/2pi) sum_l w_l V_{j,m,q}(x, w_l) exp(-i w_l (t - s_q)).
The next step's data follow from eqs. criterion_int2 and vtilde in time,
g_{k,m+1} = -chi_k sum_{j != k} v~_{j,k,m}, and u_M accumulates the fields
at the observation points.  Window function (Section 5): s_q = 3/2 (q-1) H,
P(s) = eta(s/H; 1/2, 1) on [-H/2, H], 1 - eta(s/H + 3/2; 1/2, 1) on
(-H, -H/2), 0 elsewhere; sum_q P_q = 1 on [0, s_Q + H/2].

Signals are complex and frequencies positive, as in the single-window
pipeline (the transform of eq. backwardFT over the band where the incident
spectrum lives).  The long-duration incident field is a train of Gaussian
plane-wave pulses (u2 of Section 5 in the time domain):
    u(x, t) = sum_p f(t - p T_p - x.d),
    f(tau) = (sigma / (2 sqrt(pi))) exp(-i w0 (tau - tau0)) exp(-sigma^2 (tau - tau0)^2 / 4),
the inverse transform of exp(-(w - w0)^2/sigma^2) exp(i w tau0).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import lu_factor, lu_solve

from .ms import eta


def pou(s, H):
    """P(s) of the windowing partition of unity."""
    s = np.asarray(s, dtype=float)
    out = np.zeros_like(s)
    a = (s >= -0.5 * H) & (s <= H)
    out[a] = eta(s[a] / H, 0.5, 1.0)
    b = (s > -H) & (s < -0.5 * H)
    out[b] = 1.0 - eta(s[b] / H + 1.5, 0.5, 1.0)
    return out


def pulse_train(x, t, theta, omega0, sigma, tau0, npulse, period):
    """u(x, t) of the pulse train at points x [P, 2] and times t [T] -> [T, P]."""
    d = np.array([math.cos(theta), math.sin(theta)])
    xd = np.asarray(x, dtype=float) @ d
    out = np.zeros((np.size(t), xd.size), dtype=complex)
    for p in range(npulse):
        tau = np.asarray(t, dtype=float)[:, None] - p * period - xd[None, :] - tau0
        out += (sigma / (2.0 * math.sqrt(math.pi))) * np.exp(-1j * omega0 * tau
                                                             - 0.25 * sigma ** 2 * tau ** 2)
    return out


def data_len(nt, dt, Q, H):
    """Samples of the time mesh of the real-signal recursion: the nt
    requested, and at least enough to cover [0, s_Q + H], the whole support
    of the last window (Section 5 takes the time mesh on [0, s_Q + H]; a
    window cut short would give its data a jump, and its spectrum a slowly
    decaying tail that no band-limited transform reproduces)."""
    return max(nt, int(math.ceil((1.5 * (Q - 1) * H + H) / dt - 1e-9)) + 1)


def run_windowed(layout, omegas, weights, dt, nt, Q, H, inc):
    """Traces u_M(x_p, t_n), t_n = n dt (n < nt), of the windowed recursion;
    inc = dict(theta, omega0, sigma, tau0, npulse, period).  The time mesh
    is the nt samples asked for: the trapezoid transform on a uniform
    frequency grid is periodic in time (period 2 pi / spacing), so the mesh
    must stay inside one period and the caller sizes both."""
    p, J = layout.p, layout.J
    om = np.asarray(omegas, dtype=float)
    w = np.asarray(weights, dtype=float)
    t = dt * np.arange(nt)
    sq = 1.5 * H * np.arange(Q)
    nodes = layout.nodes
    # factors of every (arc, frequency) matrix, reused by all steps and windows
    F = [[lu_factor(layout.assemble(j, k)) for k in om] for j in range(J)]
    g = [-layout.chi[j][None, :] * pulse_train(nodes[j]["y"], t, **inc) for j in range(J)]
    u = np.zeros((nt, p.obs.shape[0]), dtype=complex)
    for m in range(p.M):
        cross = [np.zeros((nt, nodes[k]["n"]), dtype=complex) for k in range(J)]
        for j in range(J):
            for q in range(Q):
                win = dt * pou(t - sq[q], H)
                E = np.exp(1j * np.outer(om, t - sq[q]))
                G = E @ (win[:, None] * g[j])                     # [nk][n_j]
                psi = [lu_solve(F[j][l], G[l]) for l in range(om.size)]
                back = np.exp(-1j * np.outer(t - sq[q], om)) * w / (2.0 * math.pi)
                for k in range(J):
                    if k == j:
                        continue
                    msk = layout.mask[j][k]
                    tgt = nodes[k]["y"][msk]
                    if tgt.shape[0] == 0:
                        continue
                    V = np.array([layout.field(j, om[l], tgt, psi[l]) for l in range(om.size)])
                    cross[k][:, msk] += back @ V
                Vo = np.array([layout.field(j, om[l], p.obs, psi[l]) for l in range(om.size)])
                u += back @ Vo
        g = [-layout.chi[k][None, :] * cross[k] for k in range(J)]
    return u


def run_windowed_real(layout, fs, dt, nt, Q, H, inc):
    """Traces u_M(x_p, t_n) (real), t_n = n dt (n < nt), of the windowed
    recursion for the real pulse field u4 of Section 5 (eq. multi; inc =
    dict(theta, npulse, period)) on the frequency set fs of
    ``oracle.hftransform``: the slow transforms of eq. Fourierk are taken at
    the frequencies of fs (positive; real data have G(-w) = conj G(w)), and
    the way back is the real-signal transform of Section 4.1 (Filon-Clenshaw-
    Curtis near 0, Fourier continuation on [w_c, W]) at the shifted times
    t - s_q of eq. TDsol.  The recursion runs on the time mesh of data_len
    samples (these transforms are quadratures, with no period in time); the
    first nt rows are returned."""
    from . import hftransform as hf
    p, J = layout.p, layout.J
    om = np.asarray(fs.omega, dtype=float)
    nt_out, nt = nt, data_len(nt, dt, Q, H)
    t = dt * np.arange(nt)
    sq = 1.5 * H * np.arange(Q)
    nodes = layout.nodes
    F = [[lu_factor(layout.assemble(j, k)) for k in om] for j in range(J)]
    npulse, period = inc.get("npulse", 5), inc.get("period", 10.0)
    g = [-layout.chi[j][None, :] * hf.u4(nodes[j]["y"], t, inc["theta"], npulse, period)
         for j in range(J)]
    back = [hf.transform_weights(fs, t - sq[q]) / math.pi for q in range(Q)]
    u = np.zeros((nt, p.obs.shape[0]))
    for m in range(p.M):
        cross = [np.zeros((nt, nodes[k]["n"])) for k in range(J)]
        for j in range(J):
            for q in range(Q):
                win = dt * pou(t - sq[q], H)
                E = np.exp(1j * np.outer(om, t - sq[q]))
                G = E @ (win[:, None] * g[j])                     # [nk][n_j]
                psi = [lu_solve(F[j][l], G[l]) for l in range(om.size)]
                for k in range(J):
                    if k == j:
                        continue
                    msk = layout.mask[j][k]
                    tgt = nodes[k]["y"][msk]
                    if tgt.shape[0] == 0:
                        continue
                    V = np.array([layout.field(j, om[l], tgt, psi[l]) for l in range(om.size)])
                    cross[k][:, msk] += np.real(back[q] @ V)
                Vo = np.array([layout.field(j, om[l], p.obs, psi[l]) for l in range(om.size)])
                u += np.real(back[q] @ Vo)
        g = [-layout.chi[k][None, :] * cross[k] for k in range(J)]
    return u[:nt_out]

