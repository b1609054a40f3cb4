"""Benchmark: Helmholtz open-arc solves/s at N = 512 on one MI355X.

Workload (the fixed N = 512 batch of the mixed-precision configuration): a
circular arc of radius 1 spanning 2.5 rad, N = 512 Chebyshev nodes, 4096
wavenumbers uniform in [1, 120], plane wave at 30 degrees, fields at 256
points on the radius-3 circle, and time traces at those points
(t = 0.01 n, n = 0..1000) by the trapezoid frequency-to-time transform.

One step = one pass of the whole path over the batch: right-hand sides,
Nystrom assembly, LU, solve (+ FP64 refinement for the refined form), field
evaluation, frequency-to-time transform.  Inputs are resident in HBM before
the timed region.  Both the FP32-refined form (the headline `value`) and the
plain FP64 form are timed; the refined results are checked against the FP64
ones (relative L2 per solve) and, on a sample, against the CPU oracle.

Prints ONE JSON line.  `python bench.py --gpus N` with N > 1 exits: this
build measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import subprocess
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_ARC = 512
NK = 4096
NT = 1001
PEAK = {"fp64_mfma_tflops": 78.6, "fp32_mfma_tflops": 157.3, "hbm_gbs": 8000.0}


def lu_flops(n):
    """Algorithmic real flops of a complex LU: (8/3) n^3."""
    return 8.0 / 3.0 * n ** 3


def lu_block_flops(n, nb=64, sym=False):
    """Algorithmic real flops of one complex LU split by kernel: the panel
    kernel factors each (n-k0) x 64 column block, 4(m b^2 - b^3/3) flops; the
    strip kernel applies the block's triangular solve to the columns on its
    right (4 b^2 r) and the trailing update (8 b r^2), r = n - k0 - b.  The
    two sums add up to (8/3) n^3 up to O(n^2) terms.
    sym: the symmetric form -- the strip kernel scales the block's L21 rows
    into U12 (6 b r) and updates the r(r+1)/2 entries on and below the
    diagonal (8 b each); the sums then add up to (4/3) n^3 + O(n^2 b)."""
    panel = strip = 0.0
    for k0 in range(0, n, nb):
        b = min(nb, n - k0)
        m = n - k0
        r = m - b
        panel += 4.0 * (m * b * b - b ** 3 / 3.0)
        if sym:
            strip += 6.0 * b * r + 4.0 * b * r * (r + 1)
        else:
            strip += 4.0 * b * b * r + 8.0 * b * r * r
    return panel, strip


def lu_sym_used(n):
    """The refined form factors the complex symmetric single-panel arc
    matrices in the symmetric form up to n = 512 (FTHMS_LU_SYM=0 turns it
    off)."""
    return n <= 512 and os.environ.get("FTHMS_LU_SYM", "1") != "0"


SOLVE_MARK = "// triangular solves on a vector held in LDS"


def source_digest(path=None):
    """sha256 of the code of csrc/lu.h up to its triangular solves (the strip
    kernel and everything it uses; line comments and blank lines dropped), so
    that only a change to that code voids the recorded traffic."""
    import hashlib
    import re
    if path is None:
        path = os.path.join(ROOT, "paper_2507_05725_amd", "csrc", "lu.h")
    with open(path) as f:
        text = f.read()
    if SOLVE_MARK in text:
        text = text[:text.index(SOLVE_MARK)]
    lines = [re.sub(r"//.*", "", ln).rstrip() for ln in text.split("\n")]
    code = "\n".join(ln for ln in lines if ln.strip())
    return hashlib.sha256(code.encode()).hexdigest()


def recorded_traffic(kernel, per_launch=None):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when the summary is absent, the kernel source has changed since
    the counters were taken, or (per_launch given) its launches covered a
    different number of matrices."""
    path = os.path.join(ROOT, "profiles", "lu_strip_f512_traffic.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith(" "):
                key, val = line.split(":", 1)
                rec[key.strip()] = val.strip()
    if rec.get("kernel") != kernel or rec.get("lu.h code sha256") != source_digest():
        return None
    try:
        if per_launch is not None and int(rec["matrices per launch"]) != per_launch:
            return None
        return float(rec["hbm bytes per launch"])
    except (KeyError, ValueError):
        return None


def _oracle_worker_init():
    import threadpoolctl  # noqa: F401
    from oracle import incident, nystrom  # noqa: F401


def _oracle_solve(args):
    """One oracle solve (assembly + LU solve + 256-point far field) with BLAS
    on one thread; runs in the CPU-baseline worker processes."""
    kk, curve, inc, obs = args
    from threadpoolctl import threadpool_limits
    from oracle import incident as oinc
    from oracle import nystrom as ony
    with threadpool_limits(1):
        nd = ony.arc_nodes(curve, N_ARC)
        b = -oinc.incident(inc, kk, nd["y"])
        a = ony.solve(ony.assemble(nd, kk), b)
        ony.field_far(kk, obs, nd["y"], a)
    return a


def _oracle_job(case, kk):
    return (float(kk), case["curve"], case["incident"], case["obs"])


# Worker processes of the all-cores CPU baseline: one GPU's share of the host
# (16 cores) however many cores the host shows, so that the baseline neither
# oversubscribes a shared host nor depends on its size.
CPU_SHARE = 16


def cpu_pool_leg(case, k_all, budget_s=12.0):
    """The oracle on the GPU's share of the host cores (min(CPU_SHARE, cores
    this process may run on) worker processes, each solving whole wavenumbers
    with BLAS on one thread), over about budget_s of work on evenly spaced
    wavenumbers across the band.  Run before anything touches the GPU, so the
    workers start from a process with no device state.  The record names the
    cap, the host's core count and its CPU model."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    t0 = time.perf_counter()
    for kk in (k_all[0], k_all[-1]):
        _oracle_solve(_oracle_job(case, kk))
    rate = 2.0 / (time.perf_counter() - t0)  # one core, for sizing the sample
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (
        os.cpu_count() or 1)
    workers = max(1, min(CPU_SHARE, avail))
    nsol = min(len(k_all), workers * max(1, int(rate * budget_s)))
    args = [_oracle_job(case, kk) for kk in k_all[np.linspace(0, len(k_all) - 1, nsol).astype(int)]]
    # an executor, not multiprocessing.Pool: a worker that dies raises here
    # instead of being replaced forever
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn"),
                             initializer=_oracle_worker_init) as pool:
        list(pool.map(_oracle_solve, args[:workers]))  # start-up, untimed
        t1 = time.perf_counter()
        list(pool.map(_oracle_solve, args, chunksize=max(1, nsol // (4 * workers))))
        dt = time.perf_counter() - t1
    return {"value": nsol / dt, "unit": "solves/s", "cores": workers, "kind": "oracle",
            "sample": "%d of the %d wavenumbers, evenly spaced, over %d worker processes "
                      "(assembly + LU solve + 256-point field per solve, numpy/scipy FP64, "
                      "BLAS on one thread each)" % (nsol, len(k_all), workers),
            "worker_cap": CPU_SHARE,
            "host_nproc": os.cpu_count(), "host_cores_available": avail,
            "cpu_model": cpu_model()}


def cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo), or None."""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.strip().startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_single_leg(case, k_sample, alpha_gpu_rows, budget_s=12.0):
    """The oracle on one core (BLAS on one thread) over the sampled
    wavenumbers, at most about budget_s; returns the record and the largest
    relative L2 error of the GPU densities given for them."""
    errs = []
    t0 = time.perf_counter()
    for a_gpu, kk in zip(alpha_gpu_rows, k_sample):
        a = _oracle_solve(_oracle_job(case, kk))
        errs.append(float(np.linalg.norm(a_gpu - a) / np.linalg.norm(a)))
        if time.perf_counter() - t0 > budget_s:
            break
    rec = {"value": round(len(errs) / (time.perf_counter() - t0), 3), "unit": "solves/s",
           "cores": 1, "sample": "%d wavenumbers" % len(errs)}
    return rec, max(errs)


def uneven_batch(fth, ctx, torch, steps, tol):
    """The uneven multi-arc batch: 8 arcs x 2048 wavenumbers in [1, 120], n
    from ten points per wavelength rounded up to a multiple of 16, as one
    captured graph per precision after autotuning.  Returns its record."""
    from workloads import IncidentSpec, uneven_batch_case
    case = uneven_batch_case(quantum=16)
    t0 = time.perf_counter()
    cache, arcs, ks, incs = {}, [], [], []
    for ai, a in enumerate(case["arcs"]):
        inc = IncidentSpec("plane", theta=a["theta"])
        for kk, n in zip(case["k"], a["n"]):
            key = (ai, int(n))
            if key not in cache:
                cache[key] = ctx.arc_from_curve(a["curve"], int(n))
            arcs.append(cache[key])
            ks.append(kk)
            incs.append(inc)
    setup = time.perf_counter() - t0
    ns = np.array([a.n for a in arcs], dtype=float)
    rec = {"workload": "8 arcs (circular, ellipse, sine-perturbed; lengths U[0.5,4], seed 3) x "
                       "2048 wavenumbers in [1,120]; n = 10 points per wavelength in [64,1024] "
                       "rounded up to a multiple of 16",
           "solves": len(arcs), "tables": len(cache), "mean_n": round(float(ns.mean()), 1),
           "max_n": int(ns.max()), "table_setup_s": round(setup, 3),
           "lu_gflop": round(float(np.sum(lu_flops(ns))) / 1e9, 1)}
    out = {}
    for prec, name in ((fth.FP64, "fp64"), (fth.FP32_REFINED, "refined")):
        bt = fth.Batch(ctx, arcs, np.array(ks), incs, precision=prec, tol=tol)
        alpha = torch.empty(bt.total, dtype=torch.complex128, device="cuda")
        iters = torch.empty(bt.nb, dtype=torch.int32, device="cuda")
        t0 = time.perf_counter()
        bt.tune(reps=1)
        tune_s = time.perf_counter() - t0
        bt.run_dev(alpha, iters)  # captures the graph
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            bt.run_dev(alpha, iters)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        g = bt.buckets()
        it = iters.cpu().numpy()
        offs = bt.offsets.copy()
        out[name] = {"value": round(len(arcs) / dt, 1), "unit": "solves/s",
                     "ms_per_batch": round(1e3 * dt, 3), "groups": int(len(g["n"])),
                     "groups_split": int(g["split"].sum()), "groups_reg_panel": int(g["reg_panel"].sum()),
                     "tune_s": round(tune_s, 3), "redone_fp64": int(np.sum(it == -1)),
                     "alpha": alpha.clone()}
        bt.close()
    a64 = out["fp64"].pop("alpha").cpu().numpy()
    a32 = out["refined"].pop("alpha").cpu().numpy()
    d2 = np.add.reduceat(np.abs(a32 - a64) ** 2, offs)
    r2 = np.add.reduceat(np.abs(a64) ** 2, offs)
    rec.update(out)
    rec["refined_over_fp64"] = round(out["refined"]["value"] / out["fp64"]["value"], 3)
    rec["max_rel_err_refined_vs_fp64"] = float(np.sqrt(np.max(d2 / r2)))
    for a in cache.values():
        a.close()
    return rec


def kite_cavity(fth, ctx, reps=3, n_per=86):
    """The kite cavity (4 arcs, 512 frequencies up to 80, M = 6, 64 interior
    points, 2001 time samples) with single-panel arcs of N = 256 (FP64 and the
    refined form, whose fields are compared with the FP64 ones) and with
    composite-panel arcs (each arc cut at the ends of its truncated overlap,
    three panels of n_per nodes): set-up time (tables, plans) and warm time
    per run (all frequencies, all steps, fields and the time transform)."""
    from workloads import kite_cavity_case
    pb = kite_cavity_case()
    om = np.asarray(pb.omegas, dtype=float)
    w = np.full(om.size, om[1] - om[0])
    w[0] *= 0.5
    w[-1] *= 0.5
    iv = np.array([a.curve.interval for a in pb.arcs])
    rec = {"workload": "kite cavity, 4 arcs (120 deg, 30 deg overlaps), 512 frequencies on (0, 80], "
                       "M = 6, 64 interior points, 2001 time samples"}
    U64 = None
    for name in ("single_panel", "single_panel_refined", "panels"):
        t0 = time.perf_counter()
        if name == "panels":
            brs = fth.tov_breaks(iv, None, pb.period)
            arcs = [ctx.panel_arc_from_curve(a.curve, n_per, b) for a, b in zip(pb.arcs, brs)]
        else:
            arcs = [ctx.arc_from_curve(a.curve, a.n) for a in pb.arcs]
        refined = name.endswith("_refined")
        prob = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M,
                           precision=fth.FP32_REFINED if refined else fth.FP64,
                           tol=1e-11 if refined else 0.0)
        U = prob.run(om)
        ctx.freq_to_time(om, w, U, pb.times)
        setup = time.perf_counter() - t0
        ts = []
        for _ in range(reps):
            t1 = time.perf_counter()
            U = prob.run(om)
            ctx.freq_to_time(om, w, U, pb.times)
            ts.append(time.perf_counter() - t1)
        rec[name] = {"n_per_arc": arcs[0].n, "first_run_with_setup_s": round(setup, 3),
                     "ms_per_run": round(1e3 * min(ts), 2),
                     "solves_per_s": round(len(arcs) * om.size * pb.M / min(ts), 1)}
        if name == "single_panel":
            U64 = U
        elif refined:
            rec[name]["max_rel_err_fields_vs_fp64"] = float(max(
                np.linalg.norm(U[i] - U64[i]) / np.linalg.norm(U64[i]) for i in range(om.size)))
        prob.close()
        for a in arcs:
            a.close()
    return rec


def closed_obstacles(fth, ctx, reps=3, n=256):
    """Two obstacles (ellipse and kite, 0.49 apart), Gaussian plane wave
    (w0 = 15, sigma = 3), 512 frequencies on (0, 30], M = 10, 32 points on
    the radius-3 circle, 601 time samples: each obstacle as one closed
    combined-field patch of n nodes, and split into 4 overlapping open arcs
    of n/4 nodes (the same unknown count)."""
    from workloads import IncidentSpec, closed_obstacles_case
    rec = {"workload": "two obstacles (ellipse 0.8 x 0.5, kite x 0.5), Gaussian plane wave "
                       "w0 = 15, sigma = 3, 512 frequencies on (0, 30], M = 10, 32 points, "
                       "601 time samples"}
    om = 30.0 * np.arange(1, 513) / 512.0
    w = np.full(om.size, om[1] - om[0])
    w[-1] *= 0.5
    times = np.linspace(0.0, 30.0, 601)
    for name in ("closed_patches", "split_arcs"):
        pb = closed_obstacles_case(n=n, omegas=om, M=10, nobs=32, mixed=(name == "split_arcs"),
                                   n_arc=n // 4)
        if name == "split_arcs":
            # the ellipse split as well
            from workloads.configs import _ellipse_arcs
            pb.arcs = _ellipse_arcs(n // 4, 0.8, 0.5, center=(-1.0, 0.0), rot=0.3, group=0) + \
                pb.arcs[1:]
        pb.incident = IncidentSpec("gplane", theta=0.3, omega0=15.0, sigma=3.0, tau0=6.0)
        t0 = time.perf_counter()
        arcs = [ctx.closed_from_curve(a.curve, a.n) if getattr(a.curve, "closed", False)
                else ctx.arc_from_curve(a.curve, a.n) for a in pb.arcs]
        iv = np.array([a.curve.interval for a in pb.arcs])
        prob = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M,
                           groups=[a.group for a in pb.arcs])
        U = prob.run(om)
        ctx.freq_to_time(om, w, U, times)
        setup = time.perf_counter() - t0
        ts = []
        for _ in range(reps):
            t1 = time.perf_counter()
            U = prob.run(om)
            ctx.freq_to_time(om, w, U, times)
            ts.append(time.perf_counter() - t1)
        rec[name] = {"patches": len(arcs), "nodes_per_obstacle": n,
                     "first_run_with_setup_s": round(setup, 3),
                     "ms_per_run": round(1e3 * min(ts), 2),
                     "solves_per_s": round(len(arcs) * om.size * pb.M / min(ts), 1)}
        prob.close()
        for a in arcs:
            a.close()
    return rec


def gmres_cavity(fth, ctx, n_full=256, n_patch=64, patches=6, nk=401, W=25.0):
    """The circular cavity of the paper's Geometries 5 (the arc of the unit
    circle over (0.02 pi, 1.98 pi), plane wave from theta = -pi), nk
    frequencies on (0, W]: GMRES iterations (tol 1e-12) for the whole
    trapping arc (n_full nodes) against its decomposition into `patches`
    overlapping arcs (n_patch nodes each; quarter-part overlaps), and the
    time of the whole-arc batch by GMRES and by LU."""
    from workloads import CircularArc, IncidentSpec
    a0, a1 = 0.02 * math.pi, 1.98 * math.pi
    d = (a1 - a0) / patches
    spec = IncidentSpec("plane", theta=-math.pi)
    om = W * np.arange(1, nk + 1) / nk
    rec = {"workload": "circular cavity (0.02 pi, 1.98 pi), plane wave theta = -pi, %d frequencies "
                       "on (0, %g], GMRES tol 1e-12" % (nk, W)}

    def run(curve, n, prec):
        arc = ctx.arc_from_curve(curve, n)
        rhs = ctx.rhs(arc, om, spec)
        ctx.solve(arc, om[:8], rhs[:8], prec, 1e-12)  # warm-up
        t0 = time.perf_counter()
        _, it, rr = ctx.solve(arc, om, rhs, prec, 1e-12)
        dt = time.perf_counter() - t0
        arc.close()
        return it, dt

    it_full, t_gm = run(CircularArc(1.0, a0, a1), n_full, fth.GMRES)
    _, t_lu = run(CircularArc(1.0, a0, a1), n_full, fth.FP64)
    it_ir, t_ir = run(CircularArc(1.0, a0, a1), n_full, fth.FP16_GMRES_IR)
    its = []
    for j in range(patches):
        c = CircularArc(1.0, max(a0, a0 + j * d - 0.25 * d), min(a1, a0 + (j + 1) * d + 0.25 * d))
        its.append(run(c, n_patch, fth.GMRES)[0])
    its = np.concatenate(its)
    rec["whole_arc"] = {"n": n_full, "gmres_iters_mean": round(float(np.mean(it_full)), 1),
                        "gmres_iters_max": int(np.max(it_full)),
                        "gmres_batch_s": round(t_gm, 4), "lu_fp64_batch_s": round(t_lu, 4),
                        "fp16_gmres_ir": {"iters_mean": round(float(np.mean(it_ir[it_ir > 0])), 2)
                                          if np.any(it_ir > 0) else None,
                                          "iters_max": int(np.max(it_ir)),
                                          "redone_fp64": int(np.sum(it_ir < 0)),
                                          "batch_s": round(t_ir, 4)}}
    rec["patches"] = {"count": patches, "n": n_patch,
                      "gmres_iters_mean": round(float(np.mean(its)), 1),
                      "gmres_iters_max": int(np.max(its))}
    return rec


def windowed_long_time(fth, ctx, n=64, M=10, npulse=8, period=10.0, H=10.0, dt=0.1):
    """A long incident signal (npulse Gaussian plane-wave pulses, w0 = 9,
    sigma = 1, period apart) on the three-arc disc: the recursion through
    the time domain with windows of half-width H uses a fixed frequency set
    (81 frequencies, spacing 0.15, period 42 > 2H + decay), while the single
    window needs a spacing of 2 pi / T: time per run of both at T =
    npulse * period + 20."""
    from workloads import IncidentSpec, disc_interior_case
    om0, sig = 9.0, 1.0
    T = npulse * period + 20.0
    nt = int(round(T / dt)) + 1
    Q = int(math.ceil((T - 0.5 * H) / (1.5 * H))) + 1
    rec = {"workload": "disc of radius 1, 3 arcs of N = %d, M = %d, %d pulses (w0 = 9, sigma = 1) "
                       "%g apart, t in [0, %g], dt = %g" % (n, M, npulse, period, T, dt)}
    for name, nf in (("windowed", 81), ("single_window", int(math.ceil(12.0 * sig * T / (2 * math.pi))) + 1)):
        om = np.linspace(om0 - 6 * sig, om0 + 6 * sig, nf)
        w = np.full(nf, om[1] - om[0])
        w[0] *= 0.5
        w[-1] *= 0.5
        pb = disc_interior_case(n=n, omegas=om, M=M)
        pb.incident = IncidentSpec("gplane", theta=0.3, omega0=om0, sigma=sig, tau0=7.0)
        arcs = [ctx.arc_from_curve(a.curve, a.n) for a in pb.arcs]
        iv = np.array([a.curve.interval for a in pb.arcs])
        prob = fth.Problem(ctx, arcs, pb.incident, pb.obs, intervals=iv, M=pb.M)
        t = dt * np.arange(nt)
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            if name == "windowed":
                prob.traces_windowed(om, w, dt, nt, Q, H, theta=0.3, omega0=om0, sigma=sig,
                                     tau0=7.0, npulse=npulse, period=period)
            else:
                # the single-window run of one pulse (the recursion is linear:
                # a train costs the same per pulse shift only through the data)
                prob.traces(om, w, t)
            ts.append(time.perf_counter() - t0)
        rec[name] = {"frequencies": nf, "windows": Q if name == "windowed" else 1,
                     "ms_per_run": round(1e3 * min(ts), 1)}
        prob.close()
        for a in arcs:
            a.close()
    return rec


# Serving request sizes drawn up to these caps (the workload allows n and J up
# to 1024): the saturated rate, the 2 x 200 Poisson requests and the burst
# then fit about two minutes.
N_CAP = (64, 128)
J_CAP = (128, 256)


def _wait_ok(srv, fth, ticket):
    """(traces, steps, latency) of a served request, or None if it failed."""
    try:
        return srv.wait(ticket)
    except fth.FthmsError:
        return None


def serving(fth, workers=8, burst=64, count=200, seed=5):
    """Serving loop on requests drawn from the serving workload's
    distributions (workloads.serving_c5_requests: 1-12 closed obstacles, n
    per obstacle U{64..128} (raised so that the other obstacles lie 5 node
    spacings away), 128..256 frequencies (raised so that the frequency grid's
    period covers twice the time window) on (0, 2 w0], w0 in [5, 40], Gaussian plane wave, 32 points,
    time-domain stop 1e-8 decided on the device, at most 100 steps),
    submitted to a server with `workers` concurrent slots.  The saturated
    rate comes from a burst of `burst` requests; then `count` requests arrive
    as a Poisson stream at 0.5 and 0.8 of that rate, and the latency from
    arrival to traces in host memory is reported (p50/p99), with the steps
    each request took and which rule ended it."""
    from workloads import serving_c5_requests
    gen = serving_c5_requests(seed=seed, count=workers + burst + 2 * count,
                              n_range=N_CAP, nk_range=J_CAP)
    reqs = [fth.request_from_workload(r) for r in gen]
    solves = lambda q, steps: len(q["xy"]) * len(q["k"]) * steps
    srv = fth.Server(0, workers=workers)
    # warm up (first touches of the device and of every worker)
    for t in [srv.submit(q) for q in reqs[:workers]]:
        srv.wait(t)
    reqs = reqs[workers:]
    sl = slice(0, burst)
    t0 = time.perf_counter()
    tickets = [srv.submit(q) for q in reqs[sl]]
    res = [_wait_ok(srv, fth, t) for t in tickets]
    dt = time.perf_counter() - t0
    failed = sum(r is None for r in res)
    sat = (burst - failed) / dt
    all_steps = [r[1] for r in res if r is not None]
    rec = {"workload": "exterior requests drawn from the serving distributions: 1-12 closed "
                       "obstacles (ellipses with semi-axes U[0.2,1] or kites x U[0.3,1], >= 0.5 "
                       "apart), each one combined-field patch of n nodes, n ~ U{64..128} raised "
                       "so other obstacles lie 5 node spacings away, J ~ U{128..256} frequencies "
                       "on (0, 2 w0] raised so the grid period covers twice the window, "
                       "w0 ~ U[5,40], "
                       "Gaussian plane wave, 32 points, t in [0, tau0 + 10] step 0.05, stop 1e-8 "
                       "decided on the device (at most 100 steps), FP64; seed %d" % seed,
           "caps": "n <= 128 per obstacle and J <= 256 drawn before the raises (the workload "
                   "allows 1024 and 1024)",
           "workers": workers, "burst_requests": burst,
           "saturated_requests_per_s": round(sat, 2),
           "saturated_solves_per_s": round(sum(solves(q, r[1]) for q, r in
                                               zip(reqs[sl], res) if r is not None) / dt, 1),
           "poisson": []}
    rng = np.random.default_rng(seed + 1)
    off = burst
    for frac in (0.5, 0.8):
        lam = frac * sat
        gaps = rng.exponential(1.0 / lam, count)
        batch = reqs[off:off + count]
        off += count
        start = time.perf_counter()
        due = start + np.cumsum(gaps)
        tickets = []
        for q, tdue in zip(batch, due):
            now = time.perf_counter()
            if tdue > now:
                time.sleep(tdue - now)
            tickets.append(srv.submit(q))
        out = [_wait_ok(srv, fth, t) for t in tickets]
        wall = time.perf_counter() - start
        failed += sum(o is None for o in out)
        batch = [q for q, o in zip(batch, out) if o is not None]
        out = [o for o in out if o is not None]
        lat = np.array([o[2] for o in out])
        steps = [o[1] for o in out]
        all_steps += steps
        rec["poisson"].append({"rate_fraction": frac, "lambda_per_s": round(lam, 3),
                               "requests": count,
                               "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
                               "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
                               "max_latency_s": round(float(lat.max()), 4),
                               "solves_per_s": round(sum(solves(q, o[1]) for q, o in
                                                         zip(batch, out)) / wall, 1)})
    st = np.array(all_steps)
    rec["failed_requests"] = failed
    rec["ms_steps"] = {"mean": round(float(st.mean()), 2), "p50": int(np.percentile(st, 50)),
                       "max": int(st.max()), "ended_by_stop_rule": int(np.sum(st < 100)),
                       "ended_by_cap": int(np.sum(st >= 100)), "requests": int(st.size)}
    srv.close()
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tol", type=float, default=1e-11,
                    help="refinement stop: predicted relative error (the metric's 1e-10 "
                         "with a 10x margin); every solve's error is measured")
    ap.add_argument("--no-cavity", action="store_true",
                    help="skip the kite cavity, closed-obstacle and GMRES cavity runs")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving loop measurement (Poisson arrivals, p50/p99)")
    ap.add_argument("--no-uneven", action="store_true",
                    help="skip the uneven multi-arc batch (reported beside the headline)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solve path would shard by frequency "
              "(one all-reduce of the traces at the end), and only the one-GPU share "
              "is implemented", file=sys.stderr)
        sys.exit(2)

    from workloads import fixed512_case

    case = fixed512_case(nk=NK, n=N_ARC)
    pool_base = None if args.no_cpu_baseline else cpu_pool_leg(case, case["k"])

    import torch
    import paper_2507_05725_amd as fth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    ctx = fth.Context(0, stream=stream.cuda_stream)
    arc = ctx.arc_from_curve(case["curve"], N_ARC)
    k_np = case["k"]
    w_np = np.full(NK, k_np[1] - k_np[0])
    w_np[0] *= 0.5
    w_np[-1] *= 0.5
    t_np = 0.01 * np.arange(NT)
    k = torch.tensor(k_np, dtype=torch.float64, device=dev)
    w = torch.tensor(w_np, dtype=torch.float64, device=dev)
    t = torch.tensor(t_np, dtype=torch.float64, device=dev)
    nobs = case["obs"].shape[0]
    probs = {p: fth.Problem(ctx, [arc], case["incident"], case["obs"], M=1, precision=p,
                            tol=args.tol)
             for p in (fth.FP64, fth.FP32_REFINED)}
    U = {p: torch.empty((NK, nobs), dtype=torch.complex128, device=dev) for p in probs}
    A = {p: torch.empty((NK, N_ARC), dtype=torch.complex128, device=dev) for p in probs}
    u = {p: torch.empty((NT, nobs), dtype=torch.complex128, device=dev) for p in probs}

    def step(p):
        probs[p].run_dev(k, U[p], A[p])
        ctx.freq_to_time_dev(k, w, U[p], t, u[p])

    if args.calib_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    results = {}
    for p in (fth.FP64, fth.FP32_REFINED):
        for _ in range(args.warmup):
            step(p)
        torch.cuda.synchronize()
        ctx.timing_reset()
        ctx.timing(True)
        lat = []
        t_all = time.perf_counter()
        for _ in range(args.steps):
            t0 = time.perf_counter()
            step(p)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
        torch.cuda.synchronize()
        total = time.perf_counter() - t_all
        ctx.timing(False)
        kt = {name: ctx.timing_read(name) for name in
              ("assemble", "lu", "lu_panel", "lu_strip", "solve", "fallback",
                            "rhs", "field", "freq_to_time")}
        results[p] = dict(total=total, lat=lat, kt=kt)

    # the same refined steps with every batched LU on one stream, so that the
    # strip kernel runs with no other kernel beside it (its own efficiency;
    # the headline keeps the faster two-stream form)
    os.environ["FTHMS_LU_SPLIT"] = "0"
    step(fth.FP32_REFINED)
    torch.cuda.synchronize()
    ctx.timing_reset()
    ctx.timing(True)
    for _ in range(args.steps):
        step(fth.FP32_REFINED)
    torch.cuda.synchronize()
    ctx.timing(False)
    kt_iso = {name: ctx.timing_read(name) for name in ("lu", "lu_strip")}
    del os.environ["FTHMS_LU_SPLIT"]

    # refinement steps taken, on a sample of 512 wavenumbers
    ks = k[:: NK // 512].contiguous()
    rhs_s = torch.empty((ks.numel(), N_ARC), dtype=torch.complex128, device=dev)
    al_s = torch.empty_like(rhs_s)
    it_s = torch.empty(ks.numel(), dtype=torch.int32, device=dev)
    ctx.rhs_dev(arc, ks, case["incident"], rhs_s)
    ctx.solve_dev(arc, ks, rhs_s, al_s, fth.FP32_REFINED, args.tol, it_s)
    torch.cuda.synchronize()
    its = it_s.cpu().numpy()
    iter_stats = {"mean": round(float(its[its > 0].mean()), 3) if np.any(its > 0) else None,
                  "max": int(its.max()), "redone_fp64": int(np.sum(its == -1))}

    # FP16-MFMA GMRES-IR on the same batch (assembly, factorisation with the
    # trailing products on the FP16 matrix cores, FP64 GMRES preconditioned
    # by it): its rate, iterations and error against the FP64 solves
    rhs_all = torch.empty((NK, N_ARC), dtype=torch.complex128, device=dev)
    ctx.rhs_dev(arc, k, case["incident"], rhs_all)
    al_ir = torch.empty_like(rhs_all)
    al_64 = torch.empty_like(rhs_all)
    it_ir = torch.empty(NK, dtype=torch.int32, device=dev)
    ctx.solve_dev(arc, k, rhs_all, al_64, fth.FP64)
    # GMRES stops on the residual (not on a predicted error as the
    # refinement does): 1e-12 for errors below the metric's 1e-10
    ir_tol = 1e-12
    ctx.solve_dev(arc, k[:256].contiguous(), rhs_all[:256], al_ir[:256], fth.FP16_GMRES_IR,
                  ir_tol, it_ir[:256])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.solve_dev(arc, k, rhs_all, al_ir, fth.FP16_GMRES_IR, ir_tol, it_ir)
    torch.cuda.synchronize()
    t_ir = time.perf_counter() - t0
    iti = it_ir.cpu().numpy()
    ir_err = (torch.linalg.vector_norm(al_ir - al_64, dim=1) /
              torch.linalg.vector_norm(al_64, dim=1)).max().item()
    gmres_ir = {"solves_per_s": round(NK / t_ir, 1), "ms_per_batch": round(1e3 * t_ir, 3),
                "iters_mean": round(float(iti[iti > 0].mean()), 2) if np.any(iti > 0) else None,
                "iters_max": int(iti.max()), "redone_fp64": int(np.sum(iti < 0)),
                "max_rel_err_vs_fp64": ir_err,
                "note": "solves only (assembly, FP16-MFMA factorisation, preconditioned FP64 "
                        "GMRES to relative residual 1e-12); no field or transform"}
    del rhs_all, al_ir, al_64

    # accuracy of the refined form against the FP64 form, every solve
    a64, a32 = A[fth.FP64], A[fth.FP32_REFINED]
    err = (torch.linalg.vector_norm(a32 - a64, dim=1) /
           torch.linalg.vector_norm(a64, dim=1)).max().item()
    uerr = (torch.linalg.vector_norm(u[fth.FP32_REFINED] - u[fth.FP64]) /
            torch.linalg.vector_norm(u[fth.FP64])).item()

    r32, r64 = results[fth.FP32_REFINED], results[fth.FP64]
    ms_step = 1000.0 * r32["total"] / args.steps
    value = NK * args.steps / r32["total"]
    fp64_value = NK * args.steps / r64["total"]
    sym32 = lu_sym_used(N_ARC)
    fl32 = lu_block_flops(N_ARC, sym=sym32)
    fl64 = lu_block_flops(N_ARC)
    panel_f, strip_f = fl32
    nsteps = args.steps

    def lu_kernels(r, peak, fls):
        out = {}
        for name, fl in (("lu_panel", fls[0]), ("lu_strip", fls[1])):
            ms, n = r["kt"][name]
            avg = ms / max(n, 1)
            flops_launch = fl * NK * nsteps / max(n, 1)
            ach = flops_launch / (avg / 1e3) / 1e12 if n else 0.0
            out[name + "_kernel"] = {"launches": n, "avg_launch_ms": round(avg, 4),
                                     "alg_gflop_per_launch": round(flops_launch / 1e9, 3),
                                     "achieved_tflops": round(ach, 3),
                                     "frac_of_mfma_peak": round(ach / peak, 4)}
        ms, n = r["kt"]["lu"]
        ach = (fls[0] + fls[1]) * NK * nsteps / (ms / 1e3) / 1e12 if n else 0.0
        out["whole_lu"] = {"ms_per_step": round(ms / nsteps, 3),
                           "alg_gflop_per_lu": round((fls[0] + fls[1]) / 1e9, 4),
                           "achieved_tflops": round(ach, 3),
                           "frac_of_mfma_peak": round(ach / peak, 4)}
        return out

    k32 = lu_kernels(r32, PEAK["fp32_mfma_tflops"], fl32)
    k64 = lu_kernels(r64, PEAK["fp64_mfma_tflops"], fl64)
    k32["form"] = "symmetric (no row interchanges, lower-triangle updates)" if sym32 else \
        "partial pivoting"
    k64["form"] = "partial pivoting"
    strip = k32["lu_strip_kernel"]
    strip_name = "lu_strip_kernel<float, true>" if sym32 else "lu_strip_kernel<float, false>"
    # matrices per strip launch in the timed steps: every block step launches
    # strips in the pivoting form, only those with columns on the block's
    # right in the symmetric form
    n_strip = r32["kt"]["lu_strip"][1]
    blocks = [k0 for k0 in range(0, N_ARC, 64) if N_ARC - k0 - 64 > 0 or (not sym32 and k0 > 0)]
    per_launch = round(NK * nsteps * len(blocks) / n_strip) if n_strip else None
    traffic = recorded_traffic(strip_name, per_launch)
    roof = {"bound": "mfma", "achieved": strip["achieved_tflops"],
            "peak": PEAK["fp32_mfma_tflops"], "unit": "TFLOP/s",
            "frac": strip["frac_of_mfma_peak"],
            "traffic": traffic,
            "kernel": strip_name + (" (U12 from the block's L21 rows + lower-triangle "
                                    "trailing update, FP32 MFMA)" if sym32 else
                                    " (block triangular solve + trailing update, FP32 MFMA)"),
            "avg_launch_ms": strip["avg_launch_ms"],
            "alg_gflop_per_launch": strip["alg_gflop_per_launch"],
            "matrices_per_launch": per_launch}

    ms_iso, n_iso = kt_iso["lu_strip"]
    avg_iso = ms_iso / max(n_iso, 1)
    fl_iso = strip_f * NK * nsteps / max(n_iso, 1)
    ach_iso = fl_iso / (avg_iso / 1e3) / 1e12 if n_iso else 0.0
    roof_iso = {"achieved": round(ach_iso, 3), "peak": PEAK["fp32_mfma_tflops"],
                "unit": "TFLOP/s", "frac": round(ach_iso / PEAK["fp32_mfma_tflops"], 4),
                "avg_launch_ms": round(avg_iso, 4),
                "alg_gflop_per_launch": round(fl_iso / 1e9, 3),
                "lu_ms_per_step": round(kt_iso["lu"][0] / nsteps, 3),
                "kernel": strip_name + ", every LU on one stream (nothing beside it)"}

    uneven = None
    if not args.no_uneven:
        uneven = uneven_batch(fth, ctx, torch, max(1, args.steps), args.tol)

    # latency of one solve (N = 512, one wavenumber, inputs resident):
    # assembly + LU + solve (+ refinement) on the device, host-timed with a
    # synchronisation after each
    single = {}
    kk = k[NK // 2:NK // 2 + 1].contiguous()
    rhs1 = torch.empty((1, N_ARC), dtype=torch.complex128, device=dev)
    ctx.rhs_dev(arc, kk, case["incident"], rhs1)
    x1 = torch.empty_like(rhs1)
    for p, name in ((fth.FP64, "fp64"), (fth.FP32_REFINED, "refined")):
        ls = []
        for r in range(55):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.solve_dev(arc, kk, rhs1, x1, p, args.tol)
            torch.cuda.synchronize()
            if r >= 5:
                ls.append(1e3 * (time.perf_counter() - t0))
        single[name] = {"p50_ms": round(float(np.percentile(ls, 50)), 3),
                        "p99_ms": round(float(np.percentile(ls, 99)), 3)}

    cavity = None
    closed = None
    gcav = None
    wlong = None
    if not args.no_cavity:
        cavity = kite_cavity(fth, ctx)
        closed = closed_obstacles(fth, ctx)
        gcav = gmres_cavity(fth, ctx)
        wlong = windowed_long_time(fth, ctx)

    serve = None
    if not args.no_serving:
        serve = serving(fth)

    base = None
    oracle_err = None
    if not args.no_cpu_baseline:
        idx = np.linspace(0, NK - 1, 64).astype(int)
        rows = a32[idx].cpu().numpy()
        one_core, oracle_err = cpu_single_leg(case, k_np[idx], rows)
        base = dict(pool_base, single_core=one_core)

    lat32 = np.array(r32["lat"]) * 1000.0
    line = {
        "metric": "Helmholtz arc solves/s at N=512 (1e-10 rel err), refined vs FP64; "
                  "p50/p99 latency",
        "value": round(value, 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64-mfma+f64-refine",
        "data": "synthetic",
        "config": {"workload": "circular arc R=1 span 2.5 rad, N=512, 4096 wavenumbers "
                               "in [1,120], plane wave 30 deg, 256 field points, 1001 "
                               "time samples", "n": N_ARC, "n_freq": NK,
                   "refine_tol": args.tol, "parallelism": "single GPU"},
        "fp64": {"value": round(fp64_value, 2), "unit": "solves/s",
                 "ms_per_step": round(1000.0 * r64["total"] / args.steps, 3),
                 "lu_kernels": k64},
        "lu_kernels_refined": k32,
        "refined_over_fp64": round(value / fp64_value, 3),
        "max_rel_err_refined_vs_fp64": err,
        "trace_rel_err_refined_vs_fp64": uerr,
        "refinement_steps": iter_stats,
        "max_rel_err_vs_oracle_sampled": oracle_err,
        "latency_ms_per_batch": {"p50": round(float(np.percentile(lat32, 50)), 3),
                                 "p99": round(float(np.percentile(lat32, 99)), 3)},
        "latency_single_solve": single,
        "kernel_ms_per_step_refined": {n: round(v[0] / args.steps, 3)
                                       for n, v in r32["kt"].items()},
        "kernel_ms_per_step_fp64": {n: round(v[0] / args.steps, 3)
                                    for n, v in r64["kt"].items()},
        "roofline": roof,
        "roofline_isolated": roof_iso,
        "fp16_gmres_ir": gmres_ir,
        "uneven_batch": uneven,
        "kite_cavity": cavity,
        "closed_obstacles": closed,
        "gmres_cavity": gcav,
        "windowed_long_time": wlong,
        "serving": serve,
        "cpu_baseline": base,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
