"""Pins of the GMRES oracle: exact termination (at most n iterations in
exact arithmetic, here to rounding), agreement with the direct solve,
residual estimates that are true residuals and never increase, and the
textbook behaviour on matrices with known spectra (identity plus a rank-r
perturbation converges in r + 1 iterations)."""
import numpy as np
import pytest

from oracle import gmres as og
from oracle import nystrom as ony
from oracle import incident as oinc
from workloads import CircularArc, IncidentSpec


def test_givens_annihilates():
    rng = np.random.default_rng(1)
    for _ in range(20):
        a, b = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        c, s = og.givens(a, b)
        assert abs(c * a + s * b) == pytest.approx(np.hypot(abs(a), abs(b)), rel=1e-14)
        assert abs(-np.conj(s) * a + c * b) < 1e-15 * abs(b) + 1e-300
        assert abs(c * c + abs(s) ** 2 - 1.0) < 1e-15


def test_random_system_exact_and_monotone():
    rng = np.random.default_rng(2)
    n = 40
    A = np.eye(n) * 3 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it, hist = og.gmres(A, b, tol=1e-13)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-12 * np.linalg.norm(x)
    assert it <= n
    assert all(h2 <= h1 * (1 + 1e-12) for h1, h2 in zip(hist, hist[1:]))
    # the final estimate is the true relative residual
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) == pytest.approx(hist[-1], rel=1e-3, abs=1e-14)


@pytest.mark.parametrize("r", [1, 3, 7])
def test_low_rank_perturbation_of_identity(r):
    """A = I + U W^H of rank r: the Krylov space of dimension r + 1
    contains the solution."""
    rng = np.random.default_rng(3 + r)
    n = 60
    U = rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))
    W = rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))
    A = np.eye(n) + 0.1 * U @ W.conj().T
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it, _ = og.gmres(A, b, tol=1e-12)
    assert it <= r + 1
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-10 * np.linalg.norm(x)


def test_open_arc_system():
    """On a first-kind open-arc matrix (the systems of the hot path) GMRES
    reaches the direct solution to its tolerance."""
    nd = ony.arc_nodes(CircularArc(1.0, -1.0, 1.4), 48)
    k = 9.0
    A = ony.assemble(nd, k)
    b = -oinc.incident(IncidentSpec("plane", theta=0.4), k, nd["y"])
    x, it, hist = og.gmres(A, b, tol=1e-12)
    ref = np.linalg.solve(A, b)
    assert np.linalg.norm(x - ref) < 1e-10 * np.linalg.norm(ref)
    assert hist[-1] <= 1e-12 and it < 48
