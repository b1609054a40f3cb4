"""Pins of the closed-patch oracle (Section 3.3, eqs. FDsolk-closed,
FDBIEk-closed; the Nystrom method the paper cites for closed curves): the
logarithmic quadrature against its defining integrals, the combined-field
solution against the exact exterior field of an interior point source
(exponential convergence), and the multiple-scattering sum over closed
patches against the exact field of two obstacles."""
import math

import numpy as np
import pytest
from scipy.special import hankel1

from oracle import closed as cl
from oracle import incident as oinc
from oracle import ms
from workloads import ClosedEllipse, ClosedKite, IncidentSpec
from workloads.configs import ArcSpec, MSProblem


def test_log_quadrature_exact_on_trigonometric_polynomials():
    """int_0^{2pi} log(4 sin^2((t - tau)/2)) cos(m tau) dtau = -(2pi/m) cos(m t)
    (m >= 1), 0 (m = 0): the weights reproduce it for m < n at every node
    and at an off-node t, and for sin(m tau) likewise."""
    n2 = 24
    n = n2 // 2
    tau = 2.0 * math.pi * np.arange(n2) / n2
    t = np.concatenate([tau, [0.37, 2.9]])
    Rt = cl.kress_weights(t, n2)
    assert np.max(np.abs(Rt @ np.ones(n2))) < 1e-13
    for m in range(1, n):
        assert np.max(np.abs(Rt @ np.cos(m * tau) + (2 * math.pi / m) * np.cos(m * t))) < 1e-13
        assert np.max(np.abs(Rt @ np.sin(m * tau) + (2 * math.pi / m) * np.sin(m * t))) < 1e-13
    # one further check by quadrature of the log integral itself (m = n - 1,
    # t off the nodes), independent of the closed form
    from scipy.integrate import quad
    f = lambda s: math.log(4.0 * math.sin(0.5 * (0.37 - s)) ** 2) * math.cos((n - 1) * s)
    ref = quad(f, 0.0, 0.37, limit=200)[0] + quad(f, 0.37, 2 * math.pi, limit=200)[0]
    assert abs(Rt[n2] @ np.cos((n - 1) * tau) - ref) < 1e-10


@pytest.mark.parametrize("curve,z0", [(ClosedEllipse(1.0, 0.6, (0.2, -0.1), 0.3), (0.3, 0.0)),
                                      (ClosedKite(1.0), (-0.2, 0.3))], ids=["ellipse", "kite"])
@pytest.mark.parametrize("k", [2.0, 7.5, 5.0 + 2.0j])
def test_exterior_point_source_exact(curve, z0, k):
    """Data -Phi(., z0) with z0 inside: the radiating solution outside is
    -Phi(x, z0) exactly; the combined-field Nystrom solution reaches it
    exponentially (1e-13 at 128 nodes on the kite, 64 on the ellipse)."""
    zt = np.array([[3.0 * math.cos(a), 3.0 * math.sin(a)] for a in np.linspace(0, 6, 8)])

    def ui(p):
        return 0.25j * hankel1(0, k * np.hypot(p[:, 0] - z0[0], p[:, 1] - z0[1]))

    errs = []
    for n2 in (32, 64, 128):
        nd = cl.nodes(curve, n2)
        psi = np.linalg.solve(cl.assemble(nd, k), -ui(nd["y"]))
        U = cl.field(k, zt, nd, psi)
        errs.append(float(np.max(np.abs(U + ui(zt))) / np.max(np.abs(ui(zt)))))
    assert errs[2] < 1e-12
    assert errs[1] < 1e-4
    assert errs[2] < 1e-3 * errs[0]


def test_ms_two_closed_patches_exact():
    """Two obstacles, each one closed patch, point source inside the first:
    at a complex wavenumber the MS sum converges geometrically and its limit
    is -U^i outside both (exact to 1e-12 at 64 nodes per obstacle)."""
    k = 5.0 + 2.0j
    obs = np.stack([2.8 * np.cos(np.linspace(0, 6, 8)), 2.8 * np.sin(np.linspace(0, 6, 8))], -1)
    errs = []
    for n2 in (32, 64):
        arcs = [ArcSpec(ClosedEllipse(0.8, 0.5, (-1.0, 0.0)), n2, group=0),
                ArcSpec(ClosedKite(0.5, (1.2, 0.3)), n2, group=1)]
        pb = MSProblem(arcs=arcs, incident=IncidentSpec("point", z0=(-1.1, 0.1), sigma=0.0),
                       omegas=np.array([k]), M=12, obs=obs, times=np.zeros(0))
        lay = ms.Layout(pb)
        assert lay.closed == [True, True] and np.all(lay.chi[0] == 1.0)
        out = ms.run_frequency(lay, k)
        ui = oinc.incident(pb.incident, k, obs)
        errs.append(float(np.max(np.abs(out["U"] + ui)) / np.max(np.abs(ui))))
    assert errs[0] < 1e-6 and errs[1] < 1e-12


def test_closed_patch_must_be_alone_on_its_curve():
    arcs = [ArcSpec(ClosedEllipse(0.8, 0.5), 16, group=0), ArcSpec(ClosedKite(0.5, (2, 0)), 16, group=0)]
    pb = MSProblem(arcs=arcs, incident=IncidentSpec("plane"), omegas=np.array([3.0]), M=2,
                   obs=np.zeros((1, 2)), times=np.zeros(0))
    with pytest.raises(ValueError):
        ms.Layout(pb)
