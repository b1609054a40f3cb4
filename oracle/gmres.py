"""Oracle: GMRES for the dense per-(arc, frequency) systems.

Test infrastructure only (see the package header).

The paper solves its frequency-domain integral equations with GMRES or
direct solvers and uses GMRES iteration counts to show what the
decomposition into non-trapping patches buys (Section 5, Geometries 5).
This is the textbook method: x0 = 0, Arnoldi with modified Gram-Schmidt on
the Krylov space of A and b, the least-squares problem kept triangular by
Givens rotations, stop after the first iteration j with
|residual estimate| <= tol |b| (the estimate is exact in exact arithmetic)
or after maxit iterations; no restarts.  Complex Givens rotation of (a, b):
c = |a| / sqrt(|a|^2 + |b|^2), s = (a / |a|) conj(b) / sqrt(|a|^2 + |b|^2),
applied as (a, b) -> (c a + s b, -conj(s) a + c b).
"""
from __future__ import annotations

import numpy as np


def givens(a, b):
    """(c, s) with [[c, s], [-conj(s), c]] [a, b] = [r, 0], c real."""
    if b == 0:
        return 1.0, 0.0
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    h = np.hypot(abs(a), abs(b))
    return abs(a) / h, (a / abs(a)) * np.conj(b) / h


def gmres(A, b, tol=1e-12, maxit=None):
    """Returns (x, iterations, residual estimates per iteration)."""
    A = np.asarray(A, dtype=complex)
    b = np.asarray(b, dtype=complex)
    n = b.size
    maxit = n if maxit is None else min(maxit, n)
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return np.zeros(n, dtype=complex), 0, []
    V = np.zeros((maxit + 1, n), dtype=complex)
    R = np.zeros((maxit + 1, maxit), dtype=complex)
    g = np.zeros(maxit + 1, dtype=complex)
    cs = np.zeros(maxit)
    sn = np.zeros(maxit, dtype=complex)
    V[0] = b / beta
    g[0] = beta
    hist = []
    j = 0
    for j in range(maxit):
        w = A @ V[j]
        for i in range(j + 1):
            h = np.vdot(V[i], w)
            R[i, j] = h
            w = w - h * V[i]
        hn = np.linalg.norm(w)
        R[j + 1, j] = hn
        if hn > 0.0:
            V[j + 1] = w / hn
        for i in range(j):
            a, bb = R[i, j], R[i + 1, j]
            R[i, j] = cs[i] * a + sn[i] * bb
            R[i + 1, j] = -np.conj(sn[i]) * a + cs[i] * bb
        cs[j], sn[j] = givens(R[j, j], R[j + 1, j])
        R[j, j] = cs[j] * R[j, j] + sn[j] * R[j + 1, j]
        R[j + 1, j] = 0.0
        g[j + 1] = -np.conj(sn[j]) * g[j]
        g[j] = cs[j] * g[j]
        hist.append(abs(g[j + 1]) / beta)
        if hist[-1] <= tol or hn == 0.0:
            break
    k = j + 1
    y = np.linalg.solve(np.triu(R[:k, :k]), g[:k])
    return V[:k].T @ y, k, hist
