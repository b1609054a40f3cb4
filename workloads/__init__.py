"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds *inputs only*: parametrised curves (position and derivative
on the reference interval [-1, 1]), frequency lists, observation points,
incident-field descriptors (plain parameters) and the seeds that produce them.
It contains none of the discretisation, quadrature, special-function, solve,
multiple-scattering or transform arithmetic of the method; both the oracle and
the GPU path build those themselves from what is returned here.

The workloads are shaped like the paper's numerical examples (Section 5: arcs,
closed curves split into overlapping arcs, Gaussian-modulated incident fields,
hundreds to thousands of frequencies).  The paper prints no dataset; every
workload here is synthetic and seeded.
"""
from .curves import (Curve, Segment, CircularArc, KiteArc, EllipseArc,
                     SineArc, kite_point, kite_deriv, ClosedCurve, ClosedEllipse,
                     ClosedKite)
from .configs import (plain_segment_case, kite_cavity_case, uneven_batch_case,
                      fixed512_case, small_kite_case, disc_interior_case,
                      two_obstacle_case, two_arc_exterior_case, serving_requests, serving_c5_requests, IncidentSpec, ArcSpec, MSProblem,
                      closed_obstacles_case)

__all__ = [
    "Curve", "Segment", "CircularArc", "KiteArc", "EllipseArc", "SineArc",
    "kite_point", "kite_deriv", "ClosedCurve", "ClosedEllipse", "ClosedKite",
    "closed_obstacles_case",
    "plain_segment_case", "kite_cavity_case", "uneven_batch_case",
    "fixed512_case", "small_kite_case", "disc_interior_case",
    "two_obstacle_case", "two_arc_exterior_case", "serving_requests", "serving_c5_requests", "IncidentSpec", "ArcSpec", "MSProblem",
]
