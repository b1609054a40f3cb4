"""ctypes binding to libfthms (include/fthms.h).

Argument marshalling only: every step of the solve path runs in the HIP
library.  Host functions take NumPy arrays; the *_dev functions take torch
tensors on the GPU (device pointers) and run on the context's stream.  If the
shared library is missing this module raises at import time -- there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfthms.so")

FP64 = 0
FP32_REFINED = 1
GMRES = 2
FP32_SYM = 3  # fthms_lu_dev only: complex symmetric matrices, no row interchanges
FP16_GMRES_IR = 4  # FP64 GMRES preconditioned by an FP16-MFMA LU
# Context(stream=OWN_STREAM): the context creates a private stream
OWN_STREAM = "own"
_OWN_STREAM_HANDLE = (1 << 64) - 1  # FTHMS_OWN_STREAM, (void *)(intptr_t)-1
INC_PLANE, INC_GPLANE, INC_POINT = 0, 1, 2

_ERR = {0: "OK", -1: "EINVAL", -2: "EINVAL_DATA", -3: "ENOMEM",
        -4: "ESINGULAR", -5: "ENOCONV", -6: "EDEVICE", -7: "EAGAIN", -8: "ECANCELLED"}
JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED, JOB_CANCELLED = 0, 1, 2, 3, 4


class FthmsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_ERR.get(code, "?"), code, msg))
        self.code = code


class Incident(C.Structure):
    _fields_ = [("kind", C.c_int), ("theta", C.c_double),
                ("z0", C.c_double * 2), ("omega0", C.c_double),
                ("sigma", C.c_double), ("tau0", C.c_double)]


class ProblemDesc(C.Structure):
    _fields_ = [("narcs", C.c_int), ("arcs", C.POINTER(C.c_void_p)),
                ("interval", C.POINTER(C.c_double)), ("period", C.c_double),
                ("c0", C.c_double), ("c1", C.c_double), ("M", C.c_int),
                ("precision", C.c_int), ("tol", C.c_double),
                ("incident", Incident), ("nobs", C.c_int),
                ("obs_xy", C.POINTER(C.c_double)), ("group", C.POINTER(C.c_int))]


class PulseTrain(C.Structure):
    _fields_ = [("theta", C.c_double), ("omega0", C.c_double), ("sigma", C.c_double),
                ("tau0", C.c_double), ("period", C.c_double), ("npulse", C.c_int)]


class HfGrid(C.Structure):
    _fields_ = [("wc", C.c_double), ("W", C.c_double), ("p", C.c_double), ("P", C.c_int),
                ("ncc", C.c_int), ("L", C.c_int)]


class Pulse3(C.Structure):
    _fields_ = [("theta", C.c_double), ("period", C.c_double), ("npulse", C.c_int)]


class Request(C.Structure):
    _fields_ = [("narcs", C.c_int), ("n", C.c_int), ("xy", C.POINTER(C.c_double)),
                ("dxy", C.POINTER(C.c_double)), ("interval", C.POINTER(C.c_double)),
                ("group", C.POINTER(C.c_int)), ("period", C.c_double), ("nk", C.c_int),
                ("k", C.POINTER(C.c_double)), ("w", C.POINTER(C.c_double)),
                ("incident", Incident), ("nobs", C.c_int), ("obs_xy", C.POINTER(C.c_double)),
                ("nt", C.c_int), ("t", C.POINTER(C.c_double)), ("max_steps", C.c_int),
                ("stop_tol", C.c_double), ("closed", C.c_int),
                ("ddxy", C.POINTER(C.c_double)), ("precision", C.c_int)]


if not os.path.exists(LIB_PATH):
    raise ImportError("libfthms.so is not built (run `python -m "
                      "paper_2507_05725_amd.build`); there is no CPU fallback")
_lib = C.CDLL(LIB_PATH)

_vp, _i, _d, _sz = C.c_void_p, C.c_int, C.c_double, C.c_size_t
_SIGS = {
    "fthms_abi_version": ([], _i),
    "fthms_create": ([C.POINTER(_vp), _i, _sz, _vp], _i),
    "fthms_destroy": ([_vp], _i),
    "fthms_last_error": ([_vp], C.c_char_p),
    "fthms_sync": ([_vp], _i),
    "fthms_timing_enable": ([_vp, _i], _i),
    "fthms_timing_reset": ([_vp], _i),
    "fthms_timing_read": ([_vp, C.c_char_p, C.POINTER(_d), C.POINTER(_i)], _i),
    "fthms_cheb_nodes": ([_i, _vp], _i),
    "fthms_arc_create": ([_vp, _i, _vp, _vp, C.POINTER(_vp)], _i),
    "fthms_arc_destroy": ([_vp], _i),
    "fthms_arc_size": ([_vp], _i),
    "fthms_panel_nodes": ([_i, _vp, _vp, _i, _vp], _i),
    "fthms_arc_create_panels": ([_vp, _i, _vp, _vp, _i, _vp, _vp, C.POINTER(_vp)], _i),
    "fthms_arc_panel_table": ([_vp, _vp, _vp], _i),
    "fthms_tov_breaks": ([_i, _vp, _vp, _d, _vp, _vp], _i),
    "fthms_closed_create": ([_vp, _i, _vp, _vp, _vp, C.POINTER(_vp)], _i),
    "fthms_gmres_dev": ([_vp, _i, _i, _vp, _vp, _vp, _d, _i, _vp, _vp], _i),
    "fthms_problem_traces_windowed": ([_vp, _i, _vp, _vp, _i, _d, _i, _d,
                                       C.POINTER(PulseTrain), _vp], _i),
    "fthms_solve": ([_vp, _vp, _i, _vp, _vp, _vp, _i, _d, _vp, _vp], _i),
    "fthms_solve_dev": ([_vp, _vp, _i, _vp, _vp, _vp, _i, _d, _vp, _vp], _i),
    "fthms_rhs": ([_vp, _vp, _i, _vp, C.POINTER(Incident), _vp], _i),
    "fthms_rhs_dev": ([_vp, _vp, _i, _vp, C.POINTER(Incident), _vp], _i),
    "fthms_eval_field": ([_vp, _vp, _i, _vp, _vp, _i, _vp, _vp], _i),
    "fthms_eval_field_dev": ([_vp, _vp, _i, _vp, _vp, _i, _vp, _vp], _i),
    "fthms_freq_to_time": ([_vp, _i, _vp, _vp, _i, _vp, _i, _vp, _vp], _i),
    "fthms_freq_to_time_dev": ([_vp, _i, _vp, _vp, _i, _vp, _i, _vp, _vp], _i),
    "fthms_assemble_dev": ([_vp, _vp, _i, _vp, _vp], _i),
    "fthms_lu_dev": ([_vp, _i, _i, _i, _vp, _vp, _vp], _i),
    "fthms_lu_solve_dev": ([_vp, _i, _i, _vp, _vp, _vp, _vp], _i),
    "fthms_lu_solve_noalloc_dev": ([_vp, _i, _i, _vp, _vp, _vp, _vp], _i),
    "fthms_lu_refine_dev": ([_vp, _i, _i, _vp, _vp, _vp, _vp, _vp, _d, _i, _vp, _vp], _i),
    "fthms_bessel_dev": ([_vp, _i, _vp, _vp, _vp], _i),
    "fthms_problem_traces_windowed_real": ([_vp, C.POINTER(HfGrid), _i, _d, _i, _d,
                                            C.POINTER(Pulse3), _vp], _i),
    "fthms_hf_frequencies": ([C.POINTER(HfGrid), _vp, C.POINTER(_i)], _i),
    "fthms_hf_to_time_dev": ([_vp, C.POINTER(HfGrid), _i, _vp, _d, _d, _i, _vp], _i),
    "fthms_hf_to_time": ([_vp, C.POINTER(HfGrid), _i, _vp, _d, _d, _i, _vp], _i),
    "fthms_problem_create": ([_vp, C.POINTER(ProblemDesc), C.POINTER(_vp)], _i),
    "fthms_problem_destroy": ([_vp], _i),
    "fthms_problem_run": ([_vp, _i, _vp, _vp, _vp], _i),
    "fthms_problem_run_dev": ([_vp, _i, _vp, _vp, _vp], _i),
    "fthms_problem_traces": ([_vp, _i, _vp, _vp, _i, _vp, _d, _vp, C.POINTER(_i)], _i),
    "fthms_problem_traces_dev": ([_vp, _i, _vp, _vp, _i, _vp, _d, _vp, C.POINTER(_i)], _i),
    "fthms_batch_create": ([_vp, _i, _vp, _vp, C.POINTER(Incident), _i, _d, C.POINTER(_vp)],
                           _i),
    "fthms_batch_destroy": ([_vp], _i),
    "fthms_batch_layout": ([_vp, C.POINTER(C.c_longlong), _vp], _i),
    "fthms_batch_run_dev": ([_vp, _vp, _vp], _i),
    "fthms_batch_run": ([_vp, _vp, _vp], _i),
    "fthms_batch_tune": ([_vp, _i], _i),
    "fthms_batch_buckets": ([_vp, C.POINTER(_i), _vp, _vp, _vp, _vp], _i),
    "fthms_server_create": ([_i, _sz, _i, C.POINTER(_vp)], _i),
    "fthms_server_destroy": ([_vp], _i),
    "fthms_server_error": ([_vp], C.c_char_p),
    "fthms_submit": ([_vp, C.POINTER(Request), C.POINTER(C.c_uint64)], _i),
    "fthms_poll": ([_vp, C.c_uint64, C.POINTER(_i)], _i),
    "fthms_fetch": ([_vp, C.c_uint64, _vp, C.POINTER(_i), C.POINTER(_d)], _i),
    "fthms_cancel": ([_vp, C.c_uint64], _i),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIGS)


def lib():
    return _lib


def _ptr(a):
    """Host pointer of a C-contiguous NumPy array (or None)."""
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def _dptr(t):
    """Device pointer of a contiguous torch tensor (or None)."""
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


def hf_grid(wc, W, P, p, ncc, L):
    g = HfGrid()
    g.wc, g.W, g.p, g.P, g.ncc, g.L = float(wc), float(W), float(p), int(P), int(ncc), int(L)
    return g


def hf_frequencies(grid):
    """The frequency set of fthms_hf_grid `grid` (see hf_grid)."""
    nk = C.c_int()
    rc = _lib.fthms_hf_frequencies(C.byref(grid), None, C.byref(nk))
    if rc:
        raise FthmsError(rc, "bad high-frequency grid")
    om = np.empty(nk.value)
    _lib.fthms_hf_frequencies(C.byref(grid), _ptr(om), C.byref(nk))
    return om


def cheb_nodes(n):
    t = np.empty(n)
    rc = _lib.fthms_cheb_nodes(n, _ptr(t))
    if rc:
        raise FthmsError(rc, "fthms_cheb_nodes")
    return t


COV_NONE, COV_BOTH, COV_LEFT, COV_RIGHT = 0, 1, 2, 3


def tov_breaks(intervals, groups=None, period=2 * np.pi):
    """Per arc: the panel breakpoints at the ends of its truncated overlap
    (list of arrays, 2 or 4 entries)."""
    iv = np.ascontiguousarray(intervals, dtype=np.float64).reshape(-1, 2)
    na = iv.shape[0]
    gr = None if groups is None else np.ascontiguousarray(groups, dtype=np.int32)
    br = np.empty((na, 4))
    npan = np.empty(na, dtype=np.int32)
    rc = _lib.fthms_tov_breaks(na, _ptr(iv), _ptr(gr), float(period), _ptr(br), _ptr(npan))
    if rc:
        raise FthmsError(rc, "fthms_tov_breaks")
    return [br[j, :npan[j] + 1].copy() for j in range(na)]


def panel_nodes(breaks, kinds, n_per):
    """Arc parameters t of a composite-panel arc's nodes (panel by panel)."""
    br = np.ascontiguousarray(breaks, dtype=np.float64)
    kd = np.ascontiguousarray(kinds, dtype=np.int32)
    t = np.empty((br.size - 1) * n_per)
    rc = _lib.fthms_panel_nodes(br.size - 1, _ptr(br), _ptr(kd), n_per, _ptr(t))
    if rc:
        raise FthmsError(rc, "fthms_panel_nodes")
    return t


def incident_struct(spec):
    """workloads.IncidentSpec -> fthms_incident."""
    kind = {"plane": INC_PLANE, "gplane": INC_GPLANE, "point": INC_POINT}[spec.kind]
    inc = Incident()
    inc.kind = kind
    inc.theta = float(spec.theta)
    inc.z0[0], inc.z0[1] = float(spec.z0[0]), float(spec.z0[1])
    inc.omega0 = float(spec.omega0)
    inc.sigma = float(spec.sigma)
    inc.tau0 = float(spec.tau0)
    return inc


class Context:
    def __init__(self, device=0, hbm_budget=0, stream=None):
        """stream: a hipStream_t handle (an int), None for HIP's null stream
        (torch's default stream), or OWN_STREAM for a private one."""
        h = C.c_void_p()
        if stream is None or (not isinstance(stream, str) and int(stream) == 0):
            st = None
        elif stream == OWN_STREAM:
            st = C.c_void_p(_OWN_STREAM_HANDLE)
        else:
            st = C.c_void_p(int(stream))
        rc = _lib.fthms_create(C.byref(h), int(device), int(hbm_budget), st)
        if rc:
            raise FthmsError(rc, _lib.fthms_last_error(None).decode())
        self.h = h
        self.device = device

    def check(self, rc, what=""):
        if rc:
            raise FthmsError(rc, "%s: %s" % (what, _lib.fthms_last_error(self.h).decode()))

    def sync(self):
        self.check(_lib.fthms_sync(self.h), "sync")

    def timing(self, enable=True):
        self.check(_lib.fthms_timing_enable(self.h, int(bool(enable))), "timing")

    def timing_reset(self):
        self.check(_lib.fthms_timing_reset(self.h), "timing_reset")

    def timing_read(self, name):
        ms, cnt = C.c_double(), C.c_int()
        self.check(_lib.fthms_timing_read(self.h, name.encode(), C.byref(ms),
                                          C.byref(cnt)), "timing_read")
        return ms.value, cnt.value

    def close(self):
        if self.h:
            _lib.fthms_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- single arc -------------------------------------------------------
    def arc(self, xy, dxy):
        return Arc(self, xy, dxy)

    def arc_from_curve(self, curve, n):
        t = cheb_nodes(n)
        return Arc(self, curve.x(t), curve.dx(t))

    def closed_from_curve(self, curve, n):
        """Closed patch sampled at tau_j = 2 pi j / n (curve: x, dx, ddx)."""
        tau = 2.0 * np.pi * np.arange(n) / n
        return Arc(self, curve.x(tau), curve.dx(tau), ddxy=curve.ddx(tau))

    def panel_arc_from_curve(self, curve, n_per, breaks, kinds=None):
        """Composite-panel arc sampled at panel_nodes (default: the two-sided
        change of variables on every panel)."""
        breaks = np.asarray(breaks, dtype=np.float64)
        if kinds is None:
            kinds = [COV_BOTH] * (breaks.size - 1)
        t = panel_nodes(breaks, kinds, n_per)
        return Arc(self, curve.x(t), curve.dx(t), breaks=breaks, kinds=kinds, n_per=n_per)

    def solve(self, arc, k, rhs, precision=FP64, tol=0.0):
        k = np.ascontiguousarray(k, dtype=np.float64)
        rhs = np.ascontiguousarray(rhs, dtype=np.complex128)
        nk = k.size
        alpha = np.empty((nk, arc.n), dtype=np.complex128)
        iters = np.empty(nk, dtype=np.int32)
        relres = np.empty(nk, dtype=np.float64)
        self.check(_lib.fthms_solve(self.h, arc.h, nk, _ptr(k), _ptr(rhs), _ptr(alpha),
                                    precision, tol, _ptr(iters), _ptr(relres)), "solve")
        return alpha, iters, relres

    def solve_dev(self, arc, k, rhs, alpha, precision=FP64, tol=0.0, iters=None,
                  relres=None):
        self.check(_lib.fthms_solve_dev(self.h, arc.h, k.numel(), _dptr(k), _dptr(rhs),
                                        _dptr(alpha), precision, tol, _dptr(iters),
                                        _dptr(relres)), "solve_dev")

    def rhs(self, arc, k, spec):
        k = np.ascontiguousarray(k, dtype=np.float64)
        out = np.empty((k.size, arc.n), dtype=np.complex128)
        inc = incident_struct(spec)
        self.check(_lib.fthms_rhs(self.h, arc.h, k.size, _ptr(k), C.byref(inc), _ptr(out)),
                   "rhs")
        return out

    def rhs_dev(self, arc, k, spec, out):
        inc = incident_struct(spec)
        self.check(_lib.fthms_rhs_dev(self.h, arc.h, k.numel(), _dptr(k), C.byref(inc),
                                      _dptr(out)), "rhs_dev")

    def eval_field(self, arc, k, alpha, pts):
        k = np.ascontiguousarray(k, dtype=np.float64)
        alpha = np.ascontiguousarray(alpha, dtype=np.complex128)
        pts = np.ascontiguousarray(pts, dtype=np.float64)
        U = np.empty((k.size, pts.shape[0]), dtype=np.complex128)
        self.check(_lib.fthms_eval_field(self.h, arc.h, k.size, _ptr(k), _ptr(alpha),
                                         pts.shape[0], _ptr(pts), _ptr(U)), "eval_field")
        return U

    def eval_field_dev(self, arc, k, alpha, pts, U):
        self.check(_lib.fthms_eval_field_dev(self.h, arc.h, k.numel(), _dptr(k), _dptr(alpha),
                                             pts.shape[0], _dptr(pts), _dptr(U)),
                   "eval_field_dev")

    def freq_to_time(self, omega, w, U, t):
        omega = np.ascontiguousarray(omega, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        U = np.ascontiguousarray(U, dtype=np.complex128)
        t = np.ascontiguousarray(t, dtype=np.float64)
        out = np.empty((t.size, U.shape[1]), dtype=np.complex128)
        self.check(_lib.fthms_freq_to_time(self.h, omega.size, _ptr(omega), _ptr(w), U.shape[1],
                                           _ptr(U), t.size, _ptr(t), _ptr(out)), "freq_to_time")
        return out

    def freq_to_time_dev(self, omega, w, U, t, out):
        self.check(_lib.fthms_freq_to_time_dev(self.h, omega.numel(), _dptr(omega), _dptr(w),
                                               U.shape[1], _dptr(U), t.numel(), _dptr(t),
                                               _dptr(out)), "freq_to_time_dev")


    def hf_to_time(self, grid, U, t0, dt, nt):
        """Real signal u[nt][np] from complex samples U[nk][np] on the set."""
        U = np.ascontiguousarray(U, dtype=np.complex128)
        u = np.empty((nt, U.shape[1]))
        self.check(_lib.fthms_hf_to_time(self.h, C.byref(grid), U.shape[1], _ptr(U), float(t0),
                                         float(dt), int(nt), _ptr(u)), "hf_to_time")
        return u

    # ---- single stages (torch tensors on the device) ----------------------
    def assemble_dev(self, arc, k, A):
        self.check(_lib.fthms_assemble_dev(self.h, arc.h, k.numel(), _dptr(k), _dptr(A)),
                   "assemble_dev")

    def lu_dev(self, A, piv, info=None, precision=FP64):
        nb, n = A.shape[0], A.shape[-1]
        self.check(_lib.fthms_lu_dev(self.h, n, nb, precision, _dptr(A), _dptr(piv),
                                     _dptr(info)), "lu_dev")

    def gmres_dev(self, A, b, x, iters, relres, tol=1e-12, maxit=None):
        nb, n = A.shape[0], A.shape[-1]
        maxit = min(n, 256) if maxit is None else maxit
        self.check(_lib.fthms_gmres_dev(self.h, n, nb, _dptr(A), _dptr(b), _dptr(x), tol,
                                        int(maxit), _dptr(iters), _dptr(relres)), "gmres_dev")

    def lu_solve_dev(self, LU, piv, b, x):
        nb, n = LU.shape[0], LU.shape[-1]
        self.check(_lib.fthms_lu_solve_dev(self.h, n, nb, _dptr(LU), _dptr(piv), _dptr(b),
                                           _dptr(x)), "lu_solve_dev")

    def lu_solve_noalloc_dev(self, LU, piv, b, x):
        nb, n = LU.shape[0], LU.shape[-1]
        self.check(_lib.fthms_lu_solve_noalloc_dev(self.h, n, nb, _dptr(LU), _dptr(piv),
                                                   _dptr(b), _dptr(x)), "lu_solve_noalloc_dev")

    def lu_refine_dev(self, A, LU32, piv, b, x, tol=1e-12, max_iter=10, iters=None,
                      relres=None):
        nb, n = A.shape[0], A.shape[-1]
        self.check(_lib.fthms_lu_refine_dev(self.h, n, nb, _dptr(A), _dptr(LU32), _dptr(piv),
                                            _dptr(b), _dptr(x), tol, int(max_iter),
                                            _dptr(iters), _dptr(relres)), "lu_refine_dev")

    def bessel_dev(self, z, j0, y0):
        self.check(_lib.fthms_bessel_dev(self.h, z.numel(), _dptr(z), _dptr(j0), _dptr(y0)),
                   "bessel_dev")


class Arc:
    """An arc from samples at fthms_cheb_nodes (one weighted panel); with
    ``breaks``/``kinds``/``n_per`` a composite-panel arc sampled at
    panel_nodes(breaks, kinds, n_per); with ``ddxy`` a closed patch sampled at
    tau_j = 2 pi j / n."""

    def __init__(self, ctx, xy, dxy, breaks=None, kinds=None, n_per=None, ddxy=None):
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        dxy = np.ascontiguousarray(dxy, dtype=np.float64)
        n = xy.shape[0]
        h = C.c_void_p()
        if ddxy is not None:
            ddxy = np.ascontiguousarray(ddxy, dtype=np.float64)
            ctx.check(_lib.fthms_closed_create(ctx.h, n, _ptr(xy), _ptr(dxy), _ptr(ddxy),
                                               C.byref(h)), "closed_create")
        elif breaks is None:
            ctx.check(_lib.fthms_arc_create(ctx.h, n, _ptr(xy), _ptr(dxy), C.byref(h)),
                      "arc_create")
        else:
            br = np.ascontiguousarray(breaks, dtype=np.float64)
            kd = np.ascontiguousarray(kinds, dtype=np.int32)
            ctx.check(_lib.fthms_arc_create_panels(ctx.h, br.size - 1, _ptr(br), _ptr(kd),
                                                   int(n_per), _ptr(xy), _ptr(dxy), C.byref(h)),
                      "arc_create_panels")
        self.ctx, self.h, self.n = ctx, h, n

    def panel_table(self):
        """(W [n][n], w [n]) of a composite-panel arc."""
        W = np.empty((self.n, self.n))
        w = np.empty(self.n)
        self.ctx.check(_lib.fthms_arc_panel_table(self.h, _ptr(W), _ptr(w)), "arc_panel_table")
        return W, w

    def close(self):
        if self.h:
            _lib.fthms_arc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """Cyclic multi-arc (or single-arc) problem; see fthms_problem_desc."""

    def __init__(self, ctx, arcs, incident, obs, intervals=None, period=2 * np.pi,
                 c0=1.0 / 3.0, c1=2.0 / 3.0, M=1, precision=FP64, tol=0.0, groups=None):
        self.ctx = ctx
        self.arcs = list(arcs)
        self.nsum = sum(a.n for a in self.arcs)
        self.obs = np.ascontiguousarray(obs, dtype=np.float64)
        self._arr = (C.c_void_p * len(self.arcs))(*[a.h.value for a in self.arcs])
        self._iv = None
        d = ProblemDesc()
        d.narcs = len(self.arcs)
        d.arcs = C.cast(self._arr, C.POINTER(C.c_void_p))
        if intervals is not None:
            self._iv = np.ascontiguousarray(intervals, dtype=np.float64).reshape(-1)
            d.interval = self._iv.ctypes.data_as(C.POINTER(C.c_double))
        d.period, d.c0, d.c1, d.M = period, c0, c1, M
        d.precision, d.tol = precision, tol
        d.incident = incident_struct(incident)
        d.nobs = self.obs.shape[0]
        d.obs_xy = self.obs.ctypes.data_as(C.POINTER(C.c_double))
        self._grp = None
        if groups is not None:
            self._grp = np.ascontiguousarray(groups, dtype=np.int32)
            d.group = self._grp.ctypes.data_as(C.POINTER(C.c_int))
        h = C.c_void_p()
        ctx.check(_lib.fthms_problem_create(ctx.h, C.byref(d), C.byref(h)), "problem_create")
        self.h = h

    def run(self, k, want_alpha=False):
        k = np.ascontiguousarray(k, dtype=np.float64)
        U = np.empty((k.size, self.obs.shape[0]), dtype=np.complex128)
        A = np.empty((k.size, self.nsum), dtype=np.complex128) if want_alpha else None
        self.ctx.check(_lib.fthms_problem_run(self.h, k.size, _ptr(k), _ptr(U), _ptr(A)),
                       "problem_run")
        return (U, A) if want_alpha else U

    def traces(self, k, w, t, stop_tol=0.0):
        """Time traces u_m at the observation points; returns (traces, steps)."""
        k = np.ascontiguousarray(k, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        t = np.ascontiguousarray(t, dtype=np.float64)
        out = np.empty((t.size, self.obs.shape[0]), dtype=np.complex128)
        steps = C.c_int()
        self.ctx.check(_lib.fthms_problem_traces(self.h, k.size, _ptr(k), _ptr(w), t.size, _ptr(t),
                                                 stop_tol, _ptr(out), C.byref(steps)),
                       "problem_traces")
        return out, steps.value

    def traces_windowed(self, k, w, dt, nt, Q, H, theta, omega0, sigma, tau0, npulse=1,
                        period=0.0):
        """Time traces of the recursion run through the time domain with Q
        windows, for a pulse-train incident field; returns [nt][nobs]."""
        k = np.ascontiguousarray(k, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        out = np.empty((nt, self.obs.shape[0]), dtype=np.complex128)
        inc = PulseTrain(theta, omega0, sigma, tau0, period, npulse)
        self.ctx.check(_lib.fthms_problem_traces_windowed(self.h, k.size, _ptr(k), _ptr(w), nt,
                                                          dt, Q, H, C.byref(inc), _ptr(out)),
                       "problem_traces_windowed")
        return out

    def traces_windowed_real(self, grid, dt, nt, Q, H, theta, npulse=5, period=10.0):
        """Real traces [nt][nobs] of the windowed recursion for the pulses u3
        (u4 for 5 pulses 10 apart) on the frequency set of `grid`."""
        inc = Pulse3()
        inc.theta, inc.period, inc.npulse = float(theta), float(period), int(npulse)
        u = np.empty((nt, self.obs.shape[0]))
        self.ctx.check(_lib.fthms_problem_traces_windowed_real(
            self.h, C.byref(grid), int(nt), float(dt), int(Q), float(H), C.byref(inc), _ptr(u)),
            "problem_traces_windowed_real")
        return u

    def run_dev(self, k, U, alpha=None):
        self.ctx.check(_lib.fthms_problem_run_dev(self.h, k.numel(), _dptr(k), _dptr(U),
                                                  _dptr(alpha)), "problem_run_dev")

    def close(self):
        if self.h:
            _lib.fthms_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Uneven batch of single-arc solves (see fthms_batch_create): solve i
    on arcs[i] at k[i] with incidents[i] (one spec for all, or a list)."""

    def __init__(self, ctx, arcs, k, incidents, precision=FP64, tol=0.0):
        self.ctx = ctx
        self.arcs = list(arcs)
        k = np.ascontiguousarray(k, dtype=np.float64)
        nb = k.size
        if len(self.arcs) != nb:
            raise ValueError("one arc per wavenumber required")
        if not isinstance(incidents, (list, tuple)):
            incidents = [incidents] * nb
        self._inc = (Incident * nb)(*[incident_struct(s) for s in incidents])
        self._arr = (C.c_void_p * nb)(*[a.h.value for a in self.arcs])
        h = C.c_void_p()
        ctx.check(_lib.fthms_batch_create(ctx.h, nb, self._arr, _ptr(k), self._inc, precision,
                                          tol, C.byref(h)), "batch_create")
        self.h = h
        self.nb = nb
        total = C.c_longlong()
        self.offsets = np.empty(nb, dtype=np.int64)
        ctx.check(_lib.fthms_batch_layout(h, C.byref(total), _ptr(self.offsets)), "batch_layout")
        self.total = total.value

    def run(self):
        alpha = np.empty(self.total, dtype=np.complex128)
        iters = np.empty(self.nb, dtype=np.int32)
        self.ctx.check(_lib.fthms_batch_run(self.h, _ptr(alpha), _ptr(iters)), "batch_run")
        return alpha, iters

    def run_dev(self, alpha, iters=None):
        self.ctx.check(_lib.fthms_batch_run_dev(self.h, _dptr(alpha), _dptr(iters)),
                       "batch_run_dev")

    def tune(self, reps=2):
        self.ctx.check(_lib.fthms_batch_tune(self.h, int(reps)), "batch_tune")

    def buckets(self):
        ng = C.c_int()
        self.ctx.check(_lib.fthms_batch_buckets(self.h, C.byref(ng), None, None, None, None),
                       "batch_buckets")
        arr = [np.empty(ng.value, dtype=np.int32) for _ in range(4)]
        self.ctx.check(_lib.fthms_batch_buckets(self.h, C.byref(ng), *[_ptr(a) for a in arr]),
                       "batch_buckets")
        return dict(n=arr[0], count=arr[1], split=arr[2], reg_panel=arr[3])

    def density(self, alpha, i):
        o = int(self.offsets[i])
        return alpha[o:o + self.arcs[i].n]

    def close(self):
        if self.h:
            _lib.fthms_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Server:
    """Request loop on one GPU (see fthms_server_create).  Requests are dicts
    of NumPy arrays: xy, dxy [narcs, n, 2], interval [narcs, 2], group
    [narcs], k, w [nk], incident (IncidentSpec), obs [nobs, 2], t [nt],
    max_steps, stop_tol, period."""

    def __init__(self, device=0, hbm_budget=0, workers=4):
        h = C.c_void_p()
        rc = _lib.fthms_server_create(int(device), int(hbm_budget), int(workers), C.byref(h))
        if rc:
            raise FthmsError(rc, _lib.fthms_last_error(None).decode())
        self.h = h
        self._shape = {}

    def _err(self, rc, what):
        raise FthmsError(rc, "%s: %s" % (what, _lib.fthms_server_error(self.h).decode()))

    def submit(self, req):
        closed = bool(req.get("closed", False))
        nob = len(req["xy"])
        keep = dict(xy=np.ascontiguousarray(req["xy"], dtype=np.float64),
                    dxy=np.ascontiguousarray(req["dxy"], dtype=np.float64),
                    ddxy=(np.ascontiguousarray(req["ddxy"], dtype=np.float64) if closed
                          else None),
                    iv=np.ascontiguousarray(req["interval"] if not closed
                                            else np.zeros((nob, 2)), dtype=np.float64),
                    grp=np.ascontiguousarray(req["group"] if not closed
                                             else np.arange(nob), dtype=np.int32),
                    k=np.ascontiguousarray(req["k"], dtype=np.float64),
                    w=np.ascontiguousarray(req["w"], dtype=np.float64),
                    obs=np.ascontiguousarray(req["obs"], dtype=np.float64),
                    t=np.ascontiguousarray(req["t"], dtype=np.float64))
        r = Request()
        r.narcs, r.n = keep["xy"].shape[0], keep["xy"].shape[1]
        r.xy, r.dxy, r.interval = _dp(keep["xy"]), _dp(keep["dxy"]), _dp(keep["iv"])
        r.group = keep["grp"].ctypes.data_as(C.POINTER(C.c_int))
        r.period = float(req.get("period", 2 * np.pi))
        r.nk, r.k, r.w = keep["k"].size, _dp(keep["k"]), _dp(keep["w"])
        r.incident = incident_struct(req["incident"])
        r.nobs, r.obs_xy = keep["obs"].shape[0], _dp(keep["obs"])
        r.nt, r.t = keep["t"].size, _dp(keep["t"])
        r.max_steps = int(req.get("max_steps", 100))
        r.stop_tol = float(req.get("stop_tol", 1e-8))
        r.closed = 1 if closed else 0
        if closed:
            r.ddxy = _dp(keep["ddxy"])
        r.precision = int(req.get("precision", FP64))
        ticket = C.c_uint64()
        rc = _lib.fthms_submit(self.h, C.byref(r), C.byref(ticket))
        if rc:
            self._err(rc, "submit")
        self._shape[ticket.value] = (r.nt, r.nobs)
        return ticket.value

    def poll(self, ticket):
        st = C.c_int()
        rc = _lib.fthms_poll(self.h, ticket, C.byref(st))
        if rc:
            self._err(rc, "poll")
        return st.value

    def fetch(self, ticket):
        """(traces [nt, nobs], steps, latency seconds); raises FthmsError
        with code EAGAIN while the request is not finished."""
        nt, nobs = self._shape[ticket]
        out = np.empty((nt, nobs), dtype=np.complex128)
        steps, lat = C.c_int(), C.c_double()
        rc = _lib.fthms_fetch(self.h, ticket, _ptr(out), C.byref(steps), C.byref(lat))
        if rc:
            if rc != -7:
                self._shape.pop(ticket, None)
            self._err(rc, "fetch")
        self._shape.pop(ticket, None)
        return out, steps.value, lat.value

    def wait(self, ticket, poll_s=0.001):
        import time
        while self.poll(ticket) in (JOB_QUEUED, JOB_RUNNING):
            time.sleep(poll_s)
        return self.fetch(ticket)

    def cancel(self, ticket):
        rc = _lib.fthms_cancel(self.h, ticket)
        if rc:
            self._err(rc, "cancel")

    def close(self):
        if self.h:
            _lib.fthms_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def request_from_workload(req):
    """Server request dict from a workloads.serving_requests entry: node
    samples of every arc at the Chebyshev nodes, parent intervals, groups,
    and trapezoid weights on the uniform frequency grid (half weight at the
    ends)."""
    arcs = req["arcs"]
    n = arcs[0].n
    om = np.asarray(req["omegas"], dtype=np.float64)
    w = np.full(om.size, om[1] - om[0] if om.size > 1 else 1.0)
    w[0] *= 0.5
    w[-1] *= 0.5
    if req.get("closed", False):
        # every obstacle one closed patch: samples at tau_j = 2 pi j / n
        tau = 2.0 * np.pi * np.arange(n) / n
        return dict(closed=True, xy=np.stack([a.curve.x(tau) for a in arcs]),
                    dxy=np.stack([a.curve.dx(tau) for a in arcs]),
                    ddxy=np.stack([a.curve.ddx(tau) for a in arcs]), k=om, w=w,
                    incident=req["incident"], obs=req["obs"], t=req["times"],
                    max_steps=req["max_steps"], stop_tol=req["stop_tol"],
                    precision=req.get("precision", FP64))
    t = cheb_nodes(n)
    return dict(xy=np.stack([a.curve.x(t) for a in arcs]),
                dxy=np.stack([a.curve.dx(t) for a in arcs]),
                interval=np.array([a.curve.interval for a in arcs]),
                group=np.array([a.group for a in arcs]), k=om, w=w,
                incident=req["incident"], obs=req["obs"], t=req["times"],
                max_steps=req["max_steps"], stop_tol=req["stop_tol"])
