"""MI355X-native open-arc Helmholtz solves for the FTH-MS method.

The compute path is libfthms.so (HIP for gfx950, C-ABI in include/fthms.h);
this package is its Python binding.  Build the library with
``python -m paper_2507_05725_amd.build``.  The binding is loaded on first
use of any name below; it raises ImportError when the library is missing
(there is no CPU fallback).
"""
_NAMES = ("FP64", "FP32_REFINED", "GMRES", "FP32_SYM", "FP16_GMRES_IR", "INC_PLANE", "INC_GPLANE", "INC_POINT",
          "Arc", "Batch", "Context", "FthmsError", "Problem", "Server", "cheb_nodes",
          "JOB_QUEUED", "JOB_RUNNING", "JOB_DONE", "JOB_FAILED", "JOB_CANCELLED",
          "incident_struct", "lib", "EXPORTED", "request_from_workload", "panel_nodes", "tov_breaks",
          "COV_NONE", "COV_BOTH", "COV_LEFT", "COV_RIGHT", "OWN_STREAM", "hf_grid",
          "hf_frequencies")

__all__ = list(_NAMES)


def __getattr__(name):
    if name in _NAMES:
        from . import _binding
        return getattr(_binding, name)
    raise AttributeError(name)
