// Uneven batches: many (arc, wavenumber) solves whose arcs have different
// node counts, run as one captured graph.
//
// Solves are grouped by node count n into buckets; a bucket is assembled
// (each matrix from its own arc's table), factored and solved with the
// batched kernels, and its densities are scattered to the caller's packed
// layout.  The whole sequence of bucket launches (right-hand sides,
// assembly, both LU kernels on one or two streams, the row permutation,
// the solve or refinement and the FP64 redo pass) is captured into one HIP
// graph on the first run and replayed afterwards, so a run costs one graph
// launch on the host.  fthms_batch_tune times every launch variant of the
// LU per bucket on the batch's own data (two streams or one; register or
// LDS panel) and keeps the fastest; the graph is captured again after.
#pragma once

struct fthms_batch {
  fthms_ctx *ctx = nullptr;
  int nb = 0;
  int precision = FTHMS_FP64;
  double tol = 1e-12;
  long long total = 0;              // sum of n over the solves
  std::vector<long long> off;       // packed offset of each solve
  struct Bucket {
    int n = 0, count = 0;
    std::vector<int> items;
    const double2 **d_y = nullptr;  // per matrix: arc nodes, table
    const double **d_G = nullptr;
    double *d_k = nullptr;
    IncidentDev *d_inc = nullptr;
    long long *d_off = nullptr;     // packed offset of each matrix's density
    int *d_item = nullptr;          // solve index of each matrix
    LuOpts opts;
  };
  std::vector<Bucket> buckets;
  // workspace shared by the buckets (they run one after the other)
  void *ws = nullptr;
  size_t ws_bytes = 0;
  double2 *d_alpha = nullptr;       // packed densities written by the graph
  int *d_iters = nullptr;           // per solve: refinement steps / status
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // the graph is captured and replayed on a private stream (default
  // priority), ordered after / before the context's stream by events, so
  // that any caller stream works, the legacy default stream included
  hipStream_t cs = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  bool tuned = false;
  // concurrent lanes: the buckets are dealt to up to kBatchLanes streams
  // (balanced by LU work, count n^3), each with its own workspace, so that
  // small buckets no longer wait for each other; the captured graph forks
  // from cs to the lanes and joins back
  int lanes = 1;
  std::vector<int> lane_of;           // per bucket
  std::vector<size_t> lane_off;       // workspace offset of each lane
  hipStream_t ls[4] = {};
  hipEvent_t lev[4] = {}, ev_fork = nullptr;
};

constexpr int kBatchLanes = 4;

namespace {

struct BucketWs {
  double2 *A64, *rhs, *x;
  float2 *A32;
  int *piv, *status;
  void *scr;
};

size_t bucket_bytes(int n, int count, bool fp32) {
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t nn = (size_t)n * n * count;
  return al(nn * sizeof(double2)) + (fp32 ? al(nn * sizeof(float2)) : 0) +
         al(sizeof(int) * (size_t)n * count) + al(kLuScratchBytes * count) +
         al(sizeof(int) * count) + 2 * al(sizeof(double2) * (size_t)n * count);
}

BucketWs bucket_ws(void *base, int n, int count, bool fp32) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = (char *)base + off;
    off += (bytes + 255) & ~(size_t)255;
    return (void *)p;
  };
  const size_t nn = (size_t)n * n * count;
  BucketWs w;
  w.A64 = (double2 *)take(nn * sizeof(double2));
  w.A32 = fp32 ? (float2 *)take(nn * sizeof(float2)) : nullptr;
  w.piv = (int *)take(sizeof(int) * (size_t)n * count);
  w.scr = take(kLuScratchBytes * count);
  w.status = (int *)take(sizeof(int) * count);
  w.rhs = (double2 *)take(sizeof(double2) * (size_t)n * count);
  w.x = (double2 *)take(sizeof(double2) * (size_t)n * count);
  return w;
}

// alpha[off[b] + i] = x[b][i]; iters[item[b]] = status[b]
__global__ __launch_bounds__(256) void batch_scatter_kernel(const double2 *__restrict__ x, int n,
                                                            const long long *__restrict__ off,
                                                            const int *__restrict__ status,
                                                            const int *__restrict__ item,
                                                            double2 *__restrict__ alpha,
                                                            int *__restrict__ iters) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) alpha[off[b] + i] = x[(long long)b * n + i];
  if (i == 0) iters[item[b]] = status[b];
}

}  // namespace

// Everything up to and including the factorisation of one bucket.
static int batch_factor(fthms_batch *bt, const fthms_batch::Bucket &bk, const BucketWs &w) {
  fthms_ctx *ctx = bt->ctx;
  const bool fp32 = bt->precision == FTHMS_FP32_REFINED;
  const int n = bk.n, c = bk.count;
  const long long ms = (long long)n * n;
  const int T = (n + 31) / 32;
  dim3 g(T * (T + 1) / 2, c), blk(256);
  // single-panel arc matrices are complex symmetric: the symmetric form
  // (lower block triangle, symmetric LU and residual) wherever it applies
  const bool sym = fp32 && lu_sym_fits(true, n);
  tbeg(ctx, "assemble");
  if (fp32)
    assemble_kernel<true, false><<<g, blk, 0, ctx->stream>>>(
        nullptr, nullptr, n, bk.d_k, w.A64, w.A32, ms, bk.d_y, bk.d_G, nullptr, sym ? 1 : 0);
  else
    assemble_kernel<false, false><<<g, blk, 0, ctx->stream>>>(
        nullptr, nullptr, n, bk.d_k, w.A64, nullptr, ms, bk.d_y, bk.d_G, nullptr);
  tend(ctx);
  int rc = check_launch(ctx, "assemble_kernel (batch)");
  if (rc) return rc;
  tbeg(ctx, "lu");
  LuOpts o = bk.opts;
  o.sym = sym;
  // the two-half split shares the context's second stream: not across lanes
  if (bt->lanes > 1) o.split = false;
  rc = launch_lu(ctx, fp32, fp32 ? (void *)w.A32 : (void *)w.A64, n, ms, w.piv, w.scr, w.status, c,
                 0, o);
  tend(ctx);
  return rc;
}

static int batch_enqueue(fthms_batch *bt) {
  fthms_ctx *ctx = bt->ctx;
  const bool fp32 = bt->precision == FTHMS_FP32_REFINED;
  const hipStream_t origin = ctx->stream;
  if (bt->lanes > 1) {
    HIPCK(ctx, hipEventRecord(bt->ev_fork, origin));
    for (int l = 0; l < bt->lanes; ++l) HIPCK(ctx, hipStreamWaitEvent(bt->ls[l], bt->ev_fork, 0));
  }
  for (size_t bi = 0; bi < bt->buckets.size(); ++bi) {
    const auto &bk = bt->buckets[bi];
    const int lane = bt->lanes > 1 ? bt->lane_of[bi] : 0;
    if (bt->lanes > 1) ctx->stream = bt->ls[lane];
    const int n = bk.n, c = bk.count;
    const long long ms = (long long)n * n;
    BucketWs w = bucket_ws((char *)bt->ws + bt->lane_off[lane], n, c, fp32);
    dim3 gv((n + 255) / 256, c);
    tbeg(ctx, "rhs");
    batch_rhs_kernel<<<gv, 256, 0, ctx->stream>>>(bk.d_inc, bk.d_y, bk.d_k, n, w.rhs, n);
    tend(ctx);
    int rc = check_launch(ctx, "batch_rhs_kernel");
    if (!rc) rc = batch_factor(bt, bk, w);
    if (rc) {
      ctx->stream = origin;
      return rc;
    }
    const bool sym = fp32 && lu_sym_fits(true, n);
    tbeg(ctx, "solve");
    if (fp32)
      launch_refine(ctx->stream, sym, c, w.A32, lu_perm(w.scr, c), w.A64, n, ms, w.rhs, w.x, n,
                    bt->tol, 10, w.status, nullptr, 0);
    else
      lu_solve64_kernel<<<c, kLuThreads, 0, ctx->stream>>>(w.A64, lu_perm(w.scr, c), n, ms, w.rhs,
                                                           w.x, n);
    tend(ctx);
    rc = check_launch(ctx, "batch solve");
    if (!rc && fp32) {
      tbeg(ctx, "fallback");
      rc = launch_fallback(ctx, w.A64, n, ms, w.piv, w.scr, w.rhs, w.x, w.status, c, kRedoFailed,
                           sym);
      tend(ctx);
    }
    if (rc) {
      ctx->stream = origin;
      return rc;
    }
    batch_scatter_kernel<<<gv, 256, 0, ctx->stream>>>(w.x, n, bk.d_off, w.status, bk.d_item,
                                                      bt->d_alpha, bt->d_iters);
    if ((rc = check_launch(ctx, "batch_scatter_kernel"))) {
      ctx->stream = origin;
      return rc;
    }
  }
  ctx->stream = origin;
  if (bt->lanes > 1)
    for (int l = 0; l < bt->lanes; ++l) {
      HIPCK(ctx, hipEventRecord(bt->lev[l], bt->ls[l]));
      HIPCK(ctx, hipStreamWaitEvent(origin, bt->lev[l], 0));
    }
  return FTHMS_OK;
}

static void batch_drop_graph(fthms_batch *bt) {
  if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  bt->exec = nullptr;
  bt->graph = nullptr;
}

extern "C" {

int fthms_batch_destroy(fthms_batch *bt) {
  if (!bt) return FTHMS_EINVAL;
  fthms_ctx *ctx = bt->ctx;
  (void)hipStreamSynchronize(ctx->stream);
  batch_drop_graph(bt);
  for (auto &bk : bt->buckets) {
    dev_free(ctx, (void *)bk.d_y, sizeof(void *) * bk.count);
    dev_free(ctx, (void *)bk.d_G, sizeof(void *) * bk.count);
    dev_free(ctx, bk.d_k, sizeof(double) * bk.count);
    dev_free(ctx, bk.d_inc, sizeof(IncidentDev) * bk.count);
    dev_free(ctx, bk.d_off, sizeof(long long) * bk.count);
    dev_free(ctx, bk.d_item, sizeof(int) * bk.count);
  }
  if (bt->cs) {
    (void)hipStreamSynchronize(bt->cs);
    (void)hipStreamDestroy(bt->cs);
  }
  if (bt->ev_in) (void)hipEventDestroy(bt->ev_in);
  if (bt->ev_out) (void)hipEventDestroy(bt->ev_out);
  for (int l = 0; l < kBatchLanes; ++l) {
    if (bt->ls[l]) {
      (void)hipStreamSynchronize(bt->ls[l]);
      (void)hipStreamDestroy(bt->ls[l]);
    }
    if (bt->lev[l]) (void)hipEventDestroy(bt->lev[l]);
  }
  if (bt->ev_fork) (void)hipEventDestroy(bt->ev_fork);
  dev_free(ctx, bt->ws, bt->ws_bytes);
  dev_free(ctx, bt->d_alpha, sizeof(double2) * std::max<long long>(1, bt->total));
  dev_free(ctx, bt->d_iters, sizeof(int) * std::max(1, bt->nb));
  delete bt;
  return FTHMS_OK;
}

int fthms_batch_create(fthms_ctx *ctx, int nb, const fthms_arc *const *arcs, const double *k,
                       const fthms_incident *inc, int precision, double tol,
                       fthms_batch **out) {
  if (!ctx || !out || nb < 1 || !arcs || !k || !inc)
    return fail(ctx, FTHMS_EINVAL, "bad argument to fthms_batch_create");
  if (precision != FTHMS_FP64 && precision != FTHMS_FP32_REFINED)
    return fail(ctx, FTHMS_EINVAL, "unknown precision");
  *out = nullptr;
  HIPCK(ctx, hipSetDevice(ctx->device));
  std::vector<IncidentDev> incd(nb);
  for (int i = 0; i < nb; ++i) {
    if (!arcs[i] || arcs[i]->ctx != ctx)
      return fail(ctx, FTHMS_EINVAL, "solve " + std::to_string(i) + ": arc missing or of another context");
    if (arcs[i]->d_w || arcs[i]->closed)
      return fail(ctx, FTHMS_EINVAL, "solve " + std::to_string(i) +
                                         ": composite-panel arcs and closed patches are not batched");
    if (!(k[i] > 0.0) || !std::isfinite(k[i]))
      return fail(ctx, FTHMS_EINVAL_DATA, "solve " + std::to_string(i) + ": wavenumber must be > 0");
    int rc = to_incident(ctx, &inc[i], incd[i]);
    if (rc) return rc;
  }
  fthms_batch *bt = new (std::nothrow) fthms_batch;
  if (!bt) return fail(ctx, FTHMS_ENOMEM, "host allocation failed");
  bt->ctx = ctx;
  bt->nb = nb;
  bt->precision = precision;
  bt->tol = tol > 0.0 ? tol : 1e-12;
  bt->off.resize(nb);
  for (int i = 0; i < nb; ++i) {
    bt->off[i] = bt->total;
    bt->total += arcs[i]->n;
  }
  const bool fp32 = precision == FTHMS_FP32_REFINED;
  // buckets by n (largest first), each cut so that its workspace stays
  // within kChunkBytes (or half the context's remaining budget)
  std::map<int, std::vector<int>, std::greater<int>> byn;
  for (int i = 0; i < nb; ++i) byn[arcs[i]->n].push_back(i);
  size_t cap = kChunkBytes;
  if (ctx->budget) cap = std::min(cap, ctx->budget > ctx->held ? (ctx->budget - ctx->held) / 2 : 0);
  size_t need = 0;
  for (auto &kv : byn) {
    const int n = kv.first;
    const size_t per = bucket_bytes(n, 1, fp32);
    if (per > cap) {
      fthms_batch_destroy(bt);
      return fail(ctx, FTHMS_ENOMEM, "no room for one matrix of n = " + std::to_string(n));
    }
    const int maxc = (int)std::min<size_t>(65535, cap / per);
    const int nparts = ((int)kv.second.size() + maxc - 1) / maxc;
    const int chunk = ((int)kv.second.size() + nparts - 1) / nparts;  // even split
    for (size_t s = 0; s < kv.second.size(); s += chunk) {
      fthms_batch::Bucket bk;
      bk.n = n;
      bk.items.assign(kv.second.begin() + s,
                      kv.second.begin() + std::min(kv.second.size(), s + chunk));
      bk.count = (int)bk.items.size();
      need = std::max(need, bucket_bytes(n, bk.count, fp32));
      bt->buckets.push_back(bk);
    }
  }
  int rc = FTHMS_OK;
  for (auto &bk : bt->buckets) {
    const int c = bk.count;
    std::vector<const double2 *> ys(c);
    std::vector<const double *> gs(c);
    std::vector<double> ks(c);
    std::vector<IncidentDev> is(c);
    std::vector<long long> os(c);
    for (int m = 0; m < c; ++m) {
      const int i = bk.items[m];
      ys[m] = arcs[i]->d_y;
      gs[m] = arcs[i]->d_G;
      ks[m] = k[i];
      is[m] = incd[i];
      os[m] = bt->off[i];
    }
    if ((rc = dev_alloc(ctx, (void **)&bk.d_y, sizeof(void *) * c)) ||
        (rc = dev_alloc(ctx, (void **)&bk.d_G, sizeof(void *) * c)) ||
        (rc = dev_alloc(ctx, (void **)&bk.d_k, sizeof(double) * c)) ||
        (rc = dev_alloc(ctx, (void **)&bk.d_inc, sizeof(IncidentDev) * c)) ||
        (rc = dev_alloc(ctx, (void **)&bk.d_off, sizeof(long long) * c)) ||
        (rc = dev_alloc(ctx, (void **)&bk.d_item, sizeof(int) * c)))
      break;
    if (hipMemcpy(bk.d_y, ys.data(), sizeof(void *) * c, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(bk.d_G, gs.data(), sizeof(void *) * c, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(bk.d_k, ks.data(), sizeof(double) * c, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(bk.d_inc, is.data(), sizeof(IncidentDev) * c, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(bk.d_off, os.data(), sizeof(long long) * c, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(bk.d_item, bk.items.data(), sizeof(int) * c, hipMemcpyHostToDevice) !=
            hipSuccess) {
      rc = fail(ctx, FTHMS_EDEVICE, "hipMemcpy of the batch tables failed");
      break;
    }
  }
  // deal the buckets to lanes, largest LU work first to the least loaded
  // lane; each lane's workspace holds its largest bucket.  One lane when the
  // lanes' workspaces would not fit twice the single-lane cap.
  if (rc == FTHMS_OK) {
    const int nbk = (int)bt->buckets.size();
    int L = std::min(kBatchLanes, nbk);
    for (; L >= 1; --L) {
      std::vector<double> work(L, 0.0);
      std::vector<size_t> lneed(L, 0);
      std::vector<int> order(nbk);
      for (int i = 0; i < nbk; ++i) order[i] = i;
      auto w_of = [&](int i) {
        const double nn = bt->buckets[i].n;
        return bt->buckets[i].count * nn * nn * nn;
      };
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return w_of(a) > w_of(b); });
      bt->lane_of.assign(nbk, 0);
      for (int i : order) {
        const int l = (int)(std::min_element(work.begin(), work.end()) - work.begin());
        bt->lane_of[i] = l;
        work[l] += w_of(i);
        lneed[l] = std::max(lneed[l], bucket_bytes(bt->buckets[i].n, bt->buckets[i].count, fp32));
      }
      size_t tot = 0;
      bt->lane_off.assign(L, 0);
      for (int l = 0; l < L; ++l) {
        bt->lane_off[l] = tot;
        tot += (lneed[l] + 255) & ~(size_t)255;
      }
      if (L == 1 || tot <= 2 * cap) {
        bt->lanes = L;
        need = tot;
        break;
      }
    }
    for (int l = 0; l < bt->lanes && bt->lanes > 1 && rc == FTHMS_OK; ++l)
      if (hipStreamCreateWithFlags(&bt->ls[l], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&bt->lev[l], hipEventDisableTiming) != hipSuccess)
        rc = fail(ctx, FTHMS_EDEVICE, "stream/event creation failed");
    if (rc == FTHMS_OK && bt->lanes > 1 &&
        hipEventCreateWithFlags(&bt->ev_fork, hipEventDisableTiming) != hipSuccess)
      rc = fail(ctx, FTHMS_EDEVICE, "event creation failed");
  }
  if (rc == FTHMS_OK) rc = dev_alloc(ctx, &bt->ws, need);
  if (rc == FTHMS_OK) bt->ws_bytes = need;
  if (rc == FTHMS_OK)
    rc = dev_alloc(ctx, (void **)&bt->d_alpha, sizeof(double2) * std::max<long long>(1, bt->total));
  if (rc == FTHMS_OK) rc = dev_alloc(ctx, (void **)&bt->d_iters, sizeof(int) * nb);
  if (rc == FTHMS_OK &&
      (hipStreamCreateWithFlags(&bt->cs, hipStreamNonBlocking) != hipSuccess ||
       hipEventCreateWithFlags(&bt->ev_in, hipEventDisableTiming) != hipSuccess ||
       hipEventCreateWithFlags(&bt->ev_out, hipEventDisableTiming) != hipSuccess))
    rc = fail(ctx, FTHMS_EDEVICE, "stream/event creation failed");
  if (rc) {
    fthms_batch_destroy(bt);
    return rc;
  }
  *out = bt;
  return FTHMS_OK;
}

int fthms_batch_layout(const fthms_batch *bt, long long *total, long long *offsets) {
  if (!bt) return FTHMS_EINVAL;
  if (total) *total = bt->total;
  if (offsets) std::copy(bt->off.begin(), bt->off.end(), offsets);
  return FTHMS_OK;
}

int fthms_batch_run_dev(fthms_batch *bt, fthms_c64 *alpha_dev, int *iters_dev) {
  if (!bt || !alpha_dev) return fail(bt ? bt->ctx : nullptr, FTHMS_EINVAL, "bad argument to fthms_batch_run_dev");
  fthms_ctx *ctx = bt->ctx;
  HIPCK(ctx, hipSetDevice(ctx->device));
  if (!bt->exec) {
    // capture the whole batch once on the private stream; the graph writes
    // the batch's own buffers, copied to the caller's below
    hipStream_t user = ctx->stream;
    HIPCK(ctx, hipStreamBeginCapture(bt->cs, hipStreamCaptureModeThreadLocal));
    ctx->stream = bt->cs;
    ctx->capturing = true;
    int rc = batch_enqueue(bt);
    ctx->capturing = false;
    ctx->stream = user;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(bt->cs, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess)
      return fail(ctx, FTHMS_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    bt->graph = g;
    if (hipGraphInstantiate(&bt->exec, g, nullptr, nullptr, 0) != hipSuccess) {
      batch_drop_graph(bt);
      return fail(ctx, FTHMS_EDEVICE, "hipGraphInstantiate failed");
    }
  }
  tbeg(ctx, "batch");
  HIPCK(ctx, hipEventRecord(bt->ev_in, ctx->stream));
  HIPCK(ctx, hipStreamWaitEvent(bt->cs, bt->ev_in, 0));
  HIPCK(ctx, hipGraphLaunch(bt->exec, bt->cs));
  HIPCK(ctx, hipEventRecord(bt->ev_out, bt->cs));
  HIPCK(ctx, hipStreamWaitEvent(ctx->stream, bt->ev_out, 0));
  tend(ctx);
  HIPCK(ctx, hipMemcpyAsync(alpha_dev, bt->d_alpha, sizeof(double2) * bt->total,
                            hipMemcpyDeviceToDevice, ctx->stream));
  if (iters_dev)
    HIPCK(ctx, hipMemcpyAsync(iters_dev, bt->d_iters, sizeof(int) * bt->nb,
                              hipMemcpyDeviceToDevice, ctx->stream));
  return FTHMS_OK;
}

int fthms_batch_run(fthms_batch *bt, fthms_c64 *alpha, int *iters) {
  if (!bt || !alpha) return fail(bt ? bt->ctx : nullptr, FTHMS_EINVAL, "bad argument to fthms_batch_run");
  fthms_ctx *ctx = bt->ctx;
  int rc = fthms_batch_run_dev(bt, (fthms_c64 *)bt->d_alpha, nullptr);
  if (rc) return rc;
  HIPCK(ctx, hipMemcpyAsync(alpha, bt->d_alpha, sizeof(double2) * bt->total,
                            hipMemcpyDeviceToHost, ctx->stream));
  std::vector<int> it(bt->nb);
  HIPCK(ctx, hipMemcpyAsync(it.data(), bt->d_iters, sizeof(int) * bt->nb, hipMemcpyDeviceToHost,
                            ctx->stream));
  HIPCK(ctx, hipStreamSynchronize(ctx->stream));
  if (iters) std::copy(it.begin(), it.end(), iters);
  for (int i = 0; i < bt->nb; ++i)
    if (it[i] == -2)
      return fail(ctx, FTHMS_ESINGULAR, "zero pivot in solve " + std::to_string(i));
  return FTHMS_OK;
}

int fthms_batch_tune(fthms_batch *bt, int reps) {
  if (!bt) return FTHMS_EINVAL;
  fthms_ctx *ctx = bt->ctx;
  HIPCK(ctx, hipSetDevice(ctx->device));
  if (reps < 1) reps = 2;
  const bool fp32 = bt->precision == FTHMS_FP32_REFINED;
  hipEvent_t e0, e1;
  HIPCK(ctx, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(ctx, FTHMS_EDEVICE, "hipEventCreate failed");
  }
  const bool timing = ctx->timing;
  ctx->timing = false;
  int rc = FTHMS_OK;
  for (size_t bi = 0; bi < bt->buckets.size(); ++bi) {
    auto &bk = bt->buckets[bi];
    BucketWs w = bucket_ws((char *)bt->ws + bt->lane_off[bt->lanes > 1 ? bt->lane_of[bi] : 0],
                           bk.n, bk.count, fp32);
    std::vector<LuOpts> cand;
    for (int s = 0; s < 2; ++s)
      for (int r = 0; r < 2; ++r) {
        LuOpts o;
        o.split = s == 0;
        o.reg_panel = r == 0;
        o.sym = fp32 && lu_sym_fits(true, bk.n);
        if (!o.split && bk.count < kLuSplitMin) continue;  // same launches as split
        if (o.split && bt->lanes > 1) continue;  // lanes run their LUs on one stream each
        if (!o.reg_panel && bk.n > (fp32 ? 512 : 256)) continue;
        // the symmetric form always takes the register panel
        if (!o.reg_panel && lu_sym_fits(fp32, bk.n)) continue;
        cand.push_back(o);
      }
    float best = 1e30f;
    LuOpts pick = bk.opts;
    for (const LuOpts &o : cand) {
      bk.opts = o;
      float tot = 0.f;
      const int n = bk.n, c = bk.count;
      const long long ms = (long long)n * n;
      const int T = (n + 31) / 32;
      dim3 g(T * (T + 1) / 2, c), blk(256);
      for (int r = 0; r < reps && rc == FTHMS_OK; ++r) {
        // fresh matrices, then the factorisation alone between events
        if (fp32)
          assemble_kernel<true, false><<<g, blk, 0, ctx->stream>>>(
              nullptr, nullptr, n, bk.d_k, w.A64, w.A32, ms, bk.d_y, bk.d_G, nullptr);
        else
          assemble_kernel<false, false><<<g, blk, 0, ctx->stream>>>(
              nullptr, nullptr, n, bk.d_k, w.A64, nullptr, ms, bk.d_y, bk.d_G, nullptr);
        if ((rc = check_launch(ctx, "assemble_kernel (tune)"))) break;
        (void)hipEventRecord(e0, ctx->stream);
        rc = launch_lu(ctx, fp32, fp32 ? (void *)w.A32 : (void *)w.A64, n, ms, w.piv, w.scr,
                       w.status, c, 0, o);
        (void)hipEventRecord(e1, ctx->stream);
        if (rc) break;
        if (hipEventSynchronize(e1) != hipSuccess) {
          rc = fail(ctx, FTHMS_EDEVICE, "hipEventSynchronize failed");
          break;
        }
        float ms_t = 0.f;
        (void)hipEventElapsedTime(&ms_t, e0, e1);
        tot += ms_t;
      }
      if (rc) break;
      if (tot < best) {
        best = tot;
        pick = o;
      }
    }
    bk.opts = pick;
    if (rc) break;
  }
  ctx->timing = timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  batch_drop_graph(bt);  // captured again with the chosen launches
  bt->tuned = rc == FTHMS_OK;
  return rc;
}

int fthms_batch_buckets(const fthms_batch *bt, int *nbuckets, int *n, int *count, int *split,
                        int *reg_panel) {
  if (!bt) return FTHMS_EINVAL;
  if (nbuckets) *nbuckets = (int)bt->buckets.size();
  for (size_t b = 0; b < bt->buckets.size(); ++b) {
    if (n) n[b] = bt->buckets[b].n;
    if (count) count[b] = bt->buckets[b].count;
    if (split) split[b] = bt->buckets[b].opts.split ? 1 : 0;
    if (reg_panel) reg_panel[b] = bt->buckets[b].opts.reg_panel ? 1 : 0;
  }
  return FTHMS_OK;
}

}  // extern "C"
