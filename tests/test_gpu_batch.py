"""GPU: uneven batches (solves of different n in one captured graph).

The batch is the uneven multi-arc workload (eight arcs of three kinds, n
from ten points per wavelength, rounded up to a multiple of 16) at reduced
size.  Checks: sampled solves against the oracle (1e-10, both precisions);
every solve bit-identical to the single-arc path on the same arc and
wavenumber; graph replays bit-identical to the first run with eager work in
between; the autotuner's choice still within the parity bar."""
import math
import sys

import numpy as np
import pytest

from oracle import incident as oinc
from oracle import nystrom as ony
from workloads import IncidentSpec, uneven_batch_case

pytestmark = pytest.mark.gpu
TOL = 1e-10


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def setup():
    # torch first (device memory for the _dev tests); the context runs on
    # torch's current stream, the legacy default stream
    import torch
    import paper_2507_05725_amd as fth
    ctx = fth.Context(0, stream=torch.cuda.current_stream().cuda_stream)
    case = uneven_batch_case(nk=40, kmax=30.0, quantum=16)
    arcs_cache = {}
    arcs, ks, incs, meta = [], [], [], []
    for ai, a in enumerate(case["arcs"]):
        inc = IncidentSpec("plane", theta=a["theta"])
        for kk, n in zip(case["k"], a["n"]):
            key = (ai, int(n))
            if key not in arcs_cache:
                arcs_cache[key] = ctx.arc_from_curve(a["curve"], int(n))
            arcs.append(arcs_cache[key])
            ks.append(kk)
            incs.append(inc)
            meta.append((ai, int(n), kk))
    yield fth, ctx, case, arcs, np.array(ks), incs, meta
    ctx.sync()


def _oracle(case, ai, n, kk):
    a = case["arcs"][ai]
    nd = ony.arc_nodes(a["curve"], n)
    b = -oinc.incident(IncidentSpec("plane", theta=a["theta"]), kk, nd["y"])
    return ony.solve(ony.assemble(nd, kk), b)


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_against_oracle_and_single_path(setup, prec):
    fth, ctx, case, arcs, ks, incs, meta = setup
    say("batch", len(arcs), "solves, precision", prec)
    bt = fth.Batch(ctx, arcs, ks, incs, precision=prec)
    g = bt.buckets()
    say("groups", len(g["n"]), "n from", g["n"].min(), "to", g["n"].max())
    alpha, iters = bt.run()
    assert np.all(iters >= 0)
    ns = np.array([m[1] for m in meta])
    for i in sorted({int(np.argmax(ns)), 0, len(meta) // 3, len(meta) - 1, int(np.argmin(ns))}):
        ai, n, kk = meta[i]
        ref = _oracle(case, ai, n, kk)
        got = bt.density(alpha, i)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err < TOL, (i, n, kk, err)
        # the single-arc path on the same arc and wavenumber: same kernels
        rhs = ctx.rhs(arcs[i], np.array([kk]), incs[i])
        one = ctx.solve(arcs[i], np.array([kk]), rhs, prec)[0][0]
        assert np.array_equal(one, got), (i, np.max(np.abs(one - got)))
    bt.close()


def test_batch_graph_replays(setup):
    fth, ctx, case, arcs, ks, incs, meta = setup
    import torch
    bt = fth.Batch(ctx, arcs, ks, incs, precision=1)
    first = torch.empty(bt.total, dtype=torch.complex128, device="cuda")
    it0 = torch.empty(bt.nb, dtype=torch.int32, device="cuda")
    bt.run_dev(first, it0)
    ctx.sync()
    for r in range(3):
        # eager work of the program between the replays
        rhs = ctx.rhs(arcs[5], ks[5:6], incs[5])
        ctx.solve(arcs[5], ks[5:6], rhs, 1)
        again = torch.zeros_like(first)
        it = torch.zeros_like(it0)
        bt.run_dev(again, it)
        ctx.sync()
        say("replay", r)
        assert torch.equal(again, first)
        assert torch.equal(it, it0)
    bt.close()


def test_batch_tune(setup):
    fth, ctx, case, arcs, ks, incs, meta = setup
    bt = fth.Batch(ctx, arcs, ks, incs, precision=1)
    before, _ = bt.run()
    bt.tune(reps=1)
    g = bt.buckets()
    say("tuned: split", g["split"].tolist(), "reg", g["reg_panel"].tolist())
    after, iters = bt.run()
    assert np.all(iters >= 0)
    for i in range(0, len(meta), 7):
        a, b = bt.density(before, i), bt.density(after, i)
        assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-11, i
    bt.close()
