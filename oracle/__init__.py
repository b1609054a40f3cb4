"""CPU oracle for the open-arc Helmholtz solve path -- TEST INFRASTRUCTURE.

A plain, slow, FP64 / complex128 NumPy+SciPy implementation of every step of
the frequency-domain FTH-MS hot path, written from the paper:

  nodes, weights, Nystrom matrix ........ ``oracle.nystrom``
  composite panels with changes of
  variables (eq. cov) .................... ``oracle.panels``
  closed patches, combined-field
  equation (Section 3.3) ................. ``oracle.closed``
  GMRES for the dense systems ............ ``oracle.gmres``
  windowing and time recentering ......... ``oracle.windowed``
  incident fields ....................... ``oracle.incident``
  multiple-scattering recursion ......... ``oracle.ms``
  frequency-to-time transform ........... ``oracle.transform``

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding) never
imports, links or calls it, and shares no code with it; the only common
module is ``workloads`` (seeded inputs, no method arithmetic).

Parity status: every function here is pinned by ``-m "not gpu"`` tests
against closed forms, textbook identities, brute-force quadrature or
library routines (see the pin tests under tests/).  None is "parity
unpinned".
"""
from . import closed, gmres, nystrom, incident, ms, panels, transform, windowed  # noqa: F401
