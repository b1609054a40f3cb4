"""Host logic of the composite-panel entry points (no GPU needed): the
panel breakpoints at the ends of the truncated overlaps and the panel node
parameters, against the oracle's layout and panel arcs."""
import math

import numpy as np
import pytest

from oracle import ms as oms
from oracle import panels as opn
from workloads import disc_interior_case, small_kite_case, two_obstacle_case


@pytest.fixture(scope="module")
def fth():
    import paper_2507_05725_amd as m
    return m


@pytest.mark.parametrize("make", [lambda: disc_interior_case(n=8), lambda: small_kite_case(n=8),
                                  lambda: two_obstacle_case(n=8)],
                         ids=["disc", "kite", "two_obstacles"])
def test_tov_breaks_match_oracle_layout(fth, make):
    pb = make()
    lay = oms.Layout(pb)
    iv = np.array([a.curve.interval for a in pb.arcs])
    br = fth.tov_breaks(iv, [a.group for a in pb.arcs], pb.period)
    for j in range(len(pb.arcs)):
        assert np.allclose(br[j], lay.panel_breaks(j), atol=1e-15, rtol=0)


def test_tov_breaks_lone_arc_is_one_panel(fth):
    br = fth.tov_breaks([[0.0, 1.0], [2.0, 3.0]], [0, 1])
    assert [b.tolist() for b in br] == [[-1.0, 1.0], [-1.0, 1.0]]


@pytest.mark.parametrize("kinds", [[1, 1, 1], [0, 2, 3]])
def test_panel_nodes_match_oracle(fth, kinds):
    from workloads import CircularArc
    breaks = [-1.0, -0.35, 0.2, 1.0]
    arc = opn.PanelArc(CircularArc(1.0, 0.0, 2.0), 11, breaks, kinds)
    t = fth.panel_nodes(breaks, kinds, 11)
    assert np.max(np.abs(t - arc.nodes()["t"])) < 1e-15


def test_panel_nodes_reject_bad_layouts(fth):
    with pytest.raises(fth.FthmsError):
        fth.panel_nodes([-1.0, 0.5, 0.2, 1.0], [1, 1, 1], 8)   # not increasing
    with pytest.raises(fth.FthmsError):
        fth.panel_nodes([-0.9, 1.0], [1], 8)                   # must start at -1
    with pytest.raises(fth.FthmsError):
        fth.panel_nodes([-1.0, 1.0], [7], 8)                   # unknown map
    with pytest.raises(fth.FthmsError):
        fth.panel_nodes([-1.0, 0.0, 1.0], [1, 1], 600)         # over 1024 nodes
