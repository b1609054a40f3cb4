// Multiple-scattering driver (included at the end of fthms.hip).
//
// Frequency-domain form of the FTH-MS recursion of Section 3.1 (Definition
// inductive_int with a single time window, so the spatial windows chi_j and
// the overlap masking of eq. vtilde commute with the Fourier transform):
//
//   b_{j,1}   = -chi_j U^inc                              eq. criterion_int1
//   b_{j,m+1} = -chi_j sum_{k != j} v~_{k,j,m}            eq. criterion_int2
//   v~_{k,j,m} = 0 on the overlap of Gamma_j with an adjacent Gamma_k,
//                S_k[alpha_{k,m}] elsewhere               eq. vtilde
//   V_j alpha_{j,m} = b_{j,m}                             eq. FDBIEk-interior
//   U_M = sum_j S_j[sum_m alpha_{j,m}]                    eq. mult-scatt-int
//
// Per chunk of wavenumbers every arc matrix is assembled and factored once;
// the factors are reused for all M steps.  Everything stays on the device;
// the host only plans (chi values, overlap masks, near-target quadrature).
//
// Readings: d^ov(x) in eq. POU1 is the chord |x - x_end| and A^ov the chord
// between the two ends of the overlap; overlap membership of a node is
// decided by the parent-curve parameter interval of each arc.

namespace fthms {

__global__ void zero_kernel(double2 *p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = make_double2(0.0, 0.0);
}

// dst[b][i] = -chi[i] * src[b][i]
__global__ void chi_scale_kernel(const double2 *src, const double *chi, int n, long long nn,
                                 double2 *dst) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const double c = -chi[e % n];
    dst[e] = make_double2(c * src[e].x, c * src[e].y);
  }
}

__global__ void axpy_kernel(double2 *y, const double2 *x, long long nn) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x)
    y[e] = make_double2(y[e].x + x[e].x, y[e].y + x[e].y);
}

// dst[b][i] = src[b][off + i], b < nb, i < n (the inverse of place_kernel)
__global__ void take_kernel(const double2 *src, long long sstride, long long off, int n, int nb,
                            double2 *dst) {
  const long long nn = (long long)n * nb;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x)
    dst[e] = src[(e / n) * sstride + off + e % n];
}

// y += x unless the run has stopped (gate[0] != 0: the step at which the
// time-domain stop rule held)
__global__ void axpy_gated_kernel(double2 *y, const double2 *x, long long nn, const int *gate) {
  if (gate[0] != 0) return;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x)
    y[e] = make_double2(y[e].x + x[e].x, y[e].y + x[e].y);
}

// The stop rule on the device: after step `step`, gate[0] = step if the
// step's change |du| (nrm[0] = |du|^2) is at most tol |u| (nrm[1] = |u|^2)
// and no earlier step stopped the run.
__global__ void stop_check_kernel(const double *nrm, double tol, int step, int *gate) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && gate[0] == 0 &&
      sqrt(nrm[0]) <= tol * sqrt(nrm[1]))
    gate[0] = step;
}

// dst[b][off + i] = src[b][i], b < nb, i < n
__global__ void place_kernel(const double2 *src, int n, int nb, double2 *dst, long long dstride,
                             long long off) {
  const long long nn = (long long)n * nb;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x)
    dst[(e / n) * dstride + off + e % n] = src[e];
}

}  // namespace fthms

// out[0] += sum |x|^2 (block partial sums, one atomic add per block)
__global__ __launch_bounds__(256) void norm2_kernel(const double2 *__restrict__ x, long long n,
                                                    double *out) {
  __shared__ double red[4];
  double s = 0.0;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x)
    s += x[i].x * x[i].x + x[i].y * x[i].y;
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, red[0] + red[1] + red[2] + red[3]);
}

static dim3 grid1d(long long n) {
  long long b = (n + 255) / 256;
  return dim3((unsigned)std::max<long long>(1, std::min<long long>(b, 65535)));
}

// ---------------------------------------------------------------------------
// near-target plans on the device
// ---------------------------------------------------------------------------
void near_plan_free(fthms_ctx *ctx, NearPlan &p) {
  dev_free(ctx, p.d_cls, (size_t)p.np);
  dev_free(ctx, p.d_tgt, sizeof(int) * p.ntgt);
  dev_free(ctx, p.d_qoff, sizeof(int) * (p.ntgt + 1));
  dev_free(ctx, p.d_xq, sizeof(double2) * p.nq);
  dev_free(ctx, p.d_wq, sizeof(double) * p.nq);
  dev_free(ctx, p.d_cq, sizeof(double) * p.nq);
  dev_free(ctx, p.d_pq, sizeof(int) * p.nq);
  for (int l = 0; l < kClosedLevels; ++l) {
    const size_t M = (size_t)p.lev_kappa[l] * p.np_nodes;
    dev_free(ctx, p.d_yf[l], sizeof(double2) * M);
    dev_free(ctx, p.d_dyf[l], sizeof(double2) * M);
    dev_free(ctx, p.d_Tf[l], sizeof(double) * M);
  }
  p = NearPlan();
}

// The periodic interpolation kernel of N (even) equispaced samples:
// T(t) = (1/N) sin(N t / 2) cot(t / 2), T(0) = 1.
static double closed_interp_kernel(double t, int N) {
  const double s = std::sin(0.5 * t);
  if (std::fabs(s) < 1e-15) return 1.0;
  return std::sin(0.5 * N * t) * std::cos(0.5 * t) / (s * N);
}

// Near targets of a closed patch: the distance of each target to the
// curve's trigonometric interpolant (sampled around the nearest node, then
// a golden-section refinement), its upsampling level (the smallest
// kappa = 2, 4, ..., 128 with h / kappa <= d / 5.2, h the largest node
// spacing), and per level in use the fine geometry and interpolation kernel.
static int closed_near_plan(fthms_ctx *ctx, const fthms_arc *arc, int np, const double *xy,
                            const unsigned char *skip, NearPlanHost &h, NearPlan &plan) {
  const int N = arc->n;
  const double hs = arc->hmax, dtau = 2.0 * kPi / N;
  auto point = [&](double t, double &x, double &y) {
    x = y = 0.0;
    for (int j = 0; j < N; ++j) {
      const double w = closed_interp_kernel(t - dtau * j, N);
      x += w * arc->xy[2 * j];
      y += w * arc->xy[2 * j + 1];
    }
  };
  h.cls.assign(np, 0);
  h.qoff.assign(1, 0);
  std::vector<std::vector<int>> lev(kClosedLevels);
  for (int p = 0; p < np; ++p) {
    if (skip && skip[p]) continue;
    const double zx = xy[2 * p], zy = xy[2 * p + 1];
    double dmin = 1e300;
    int jn = 0;
    for (int j = 0; j < N; ++j) {
      const double d = std::hypot(zx - arc->xy[2 * j], zy - arc->xy[2 * j + 1]);
      if (d < dmin) {
        dmin = d;
        jn = j;
      }
    }
    if (dmin >= 5.0 * hs) {
      h.cls[p] = 1;
      continue;
    }
    auto dist = [&](double t) {
      double x, y;
      point(t, x, y);
      return std::hypot(zx - x, zy - y);
    };
    // the curve's nearest point lies within a node spacing of the nearest
    // node: sample, then golden-section search around the best sample
    double best = dmin, tb = dtau * jn;
    for (int i = -32; i <= 32; ++i) {
      const double t = dtau * (jn + i / 16.0), d = dist(t);
      if (d < best) {
        best = d;
        tb = t;
      }
    }
    double a = tb - dtau / 16.0, b = tb + dtau / 16.0;
    const double g = 0.5 * (std::sqrt(5.0) - 1.0);
    for (int it = 0; it < 40; ++it) {
      const double c = b - g * (b - a), d = a + g * (b - a);
      if (dist(c) < dist(d)) b = d;
      else a = c;
    }
    const double dc = std::min(best, dist(0.5 * (a + b)));
    int l = 0;
    while (l < kClosedLevels && hs / (double)(2 << l) > dc / 5.2) ++l;
    if (l == kClosedLevels)
      return fail(ctx, FTHMS_EINVAL_DATA,
                  "target closer than h/25 to a closed patch (h its largest node spacing)");
    h.cls[p] = 2;
    lev[l].push_back(p);
  }
  for (int l = 0; l < kClosedLevels; ++l) {
    plan.lev_first[l] = (int)h.tgt.size();
    for (int p : lev[l]) h.tgt.push_back(p);
  }
  plan.lev_first[kClosedLevels] = (int)h.tgt.size();
  plan.np_nodes = N;
  for (int l = 0; l < kClosedLevels; ++l) {
    if (lev[l].empty()) continue;
    const int kappa = 2 << l, M = kappa * N;
    std::vector<double2> yf(M), dyf(M);
    std::vector<double> T(M);
    for (int q = 0; q < M; ++q) T[q] = closed_interp_kernel(2.0 * kPi * q / M, N);
    for (int q = 0; q < M; ++q) {
      double x = 0.0, y = 0.0, dx = 0.0, dy = 0.0;
      for (int j = 0; j < N; ++j) {
        int d = q - kappa * j;
        d %= M;
        if (d < 0) d += M;
        const double w = T[d];
        x += w * arc->xy[2 * j];
        y += w * arc->xy[2 * j + 1];
        dx += w * arc->dxy[2 * j];
        dy += w * arc->dxy[2 * j + 1];
      }
      yf[q] = make_double2(x, y);
      dyf[q] = make_double2(dx, dy);
    }
    int rc;
    plan.lev_kappa[l] = kappa;  // before the allocations: near_plan_free sizes by it
    if ((rc = dev_alloc(ctx, (void **)&plan.d_yf[l], sizeof(double2) * M)) ||
        (rc = dev_alloc(ctx, (void **)&plan.d_dyf[l], sizeof(double2) * M)) ||
        (rc = dev_alloc(ctx, (void **)&plan.d_Tf[l], sizeof(double) * M)))
      return rc;
    HIPCK(ctx, hipMemcpy(plan.d_yf[l], yf.data(), sizeof(double2) * M, hipMemcpyHostToDevice));
    HIPCK(ctx, hipMemcpy(plan.d_dyf[l], dyf.data(), sizeof(double2) * M, hipMemcpyHostToDevice));
    HIPCK(ctx, hipMemcpy(plan.d_Tf[l], T.data(), sizeof(double) * M, hipMemcpyHostToDevice));
  }
  return FTHMS_OK;
}

int near_plan_build(fthms_ctx *ctx, const fthms_arc *arc, int np, const double *xy,
                    NearPlan &plan, const unsigned char *skip, double kmax) {
  NearPlanHost h;
  if (arc->closed) {
    // far targets (five node spacings away and more): the trapezoid rule;
    // nearer ones: the same rule on an upsampled grid
    int rc = closed_near_plan(ctx, arc, np, xy, skip, h, plan);
    if (rc) {
      near_plan_free(ctx, plan);
      return rc;
    }
  } else if (arc->d_w) {
    std::vector<double> smax(arc->npan, 0.0);
    for (int i = 0; i < arc->n; ++i)
      smax[i / arc->nper] = std::max(smax[i / arc->nper], arc->s[i]);
    plan_near_panels(arc->npan, arc->nper, arc->xy.data(), arc->cgx.data(), arc->cgy.data(),
                     arc->hmax, smax.data(), kmax, np, xy, skip, h);
  } else {
    double smax = 0.0;
    for (double v : arc->s) smax = std::max(smax, v);
    plan_near(arc->n, arc->xy.data(), arc->cgx, arc->cgy, arc->hmax, smax, kmax, np, xy, skip,
              h);
  }
  plan.np = np;
  plan.ntgt = (int)h.tgt.size();
  plan.nq = (int)h.wq.size();
  int rc;
  if ((rc = dev_alloc(ctx, (void **)&plan.d_cls, (size_t)std::max(np, 1)))) return rc;
  HIPCK(ctx, hipMemcpy(plan.d_cls, h.cls.data(), (size_t)np, hipMemcpyHostToDevice));
  if (plan.ntgt > 0 && arc->closed) {
    if ((rc = dev_alloc(ctx, (void **)&plan.d_tgt, sizeof(int) * plan.ntgt))) return rc;
    HIPCK(ctx, hipMemcpy(plan.d_tgt, h.tgt.data(), sizeof(int) * plan.ntgt, hipMemcpyHostToDevice));
  } else if (plan.ntgt > 0) {
    if ((rc = dev_alloc(ctx, (void **)&plan.d_tgt, sizeof(int) * plan.ntgt)) ||
        (rc = dev_alloc(ctx, (void **)&plan.d_qoff, sizeof(int) * (plan.ntgt + 1))) ||
        (rc = dev_alloc(ctx, (void **)&plan.d_xq, sizeof(double2) * plan.nq)) ||
        (rc = dev_alloc(ctx, (void **)&plan.d_wq, sizeof(double) * plan.nq)) ||
        (rc = dev_alloc(ctx, (void **)&plan.d_cq, sizeof(double) * plan.nq)))
      return rc;
    HIPCK(ctx, hipMemcpy(plan.d_tgt, h.tgt.data(), sizeof(int) * plan.ntgt, hipMemcpyHostToDevice));
    HIPCK(ctx, hipMemcpy(plan.d_qoff, h.qoff.data(), sizeof(int) * (plan.ntgt + 1),
                         hipMemcpyHostToDevice));
    HIPCK(ctx, hipMemcpy(plan.d_xq, h.xq.data(), sizeof(double2) * plan.nq, hipMemcpyHostToDevice));
    HIPCK(ctx, hipMemcpy(plan.d_wq, h.wq.data(), sizeof(double) * plan.nq, hipMemcpyHostToDevice));
    HIPCK(ctx, hipMemcpy(plan.d_cq, h.cq.data(), sizeof(double) * plan.nq, hipMemcpyHostToDevice));
    if (!h.pq.empty()) {
      if ((rc = dev_alloc(ctx, (void **)&plan.d_pq, sizeof(int) * plan.nq))) return rc;
      HIPCK(ctx, hipMemcpy(plan.d_pq, h.pq.data(), sizeof(int) * plan.nq, hipMemcpyHostToDevice));
    }
  }
  return FTHMS_OK;
}

// ---------------------------------------------------------------------------
// problems
// ---------------------------------------------------------------------------
struct fthms_problem {
  fthms_ctx *ctx = nullptr;
  int narcs = 0, M = 1, precision = FTHMS_FP64;
  double tol = 1e-13, period = 0.0, c0 = 1.0 / 3.0, c1 = 2.0 / 3.0;
  IncidentDev inc;
  std::vector<const fthms_arc *> arcs;
  std::vector<int> group;           // obstacle (closed curve) of each arc
  std::vector<int> nxt, prv;        // cyclic neighbours within the group (-1: none)
  std::vector<double> interval;
  std::vector<double *> d_chi;
  std::vector<std::vector<unsigned char>> skip;  // [k * narcs + j][i]
  int nobs = 0;
  std::vector<double> obs;
  double2 *d_obs = nullptr;
  double planned_kmax = -1.0;
  std::vector<NearPlan> pair_plan;  // [k * narcs + j]
  std::vector<NearPlan> obs_plan;   // [j]
};

static bool in_interval(double tau, double a, double b, double period) {
  double u = std::fmod(tau - a, period);
  if (u < 0) u += period;
  return u > 0.0 && u < (b - a);
}

// eq. eta: 1 for |t| <= t0, exp(2 e^{-1/s} / (s - 1)) between, 0 for |t| >= t1
static double eta_window(double t, double t0, double t1) {
  t = std::fabs(t);
  if (t <= t0) return 1.0;
  if (t >= t1) return 0.0;
  const double s = (t - t0) / (t1 - t0);
  return std::exp(2.0 * std::exp(-1.0 / s) / (s - 1.0));
}

// End point x(-1) (side < 0) or x(+1) of an arc from its geometry
// coefficients: the start of the first panel (s = -1) or the end of the
// last (s = +1).
static void arc_end(const fthms_arc *a, int side, double &x, double &y) {
  x = 0.0;
  y = 0.0;
  const int n = a->nper;
  const size_t off = side < 0 ? 0 : (size_t)(a->npan - 1) * n;
  for (int m = 0; m < n; ++m) {
    const double sg = (side < 0 && (m & 1)) ? -1.0 : 1.0;
    x += sg * a->cgx[off + m];
    y += sg * a->cgy[off + m];
  }
}

static void problem_free_plans(fthms_problem *pb) {
  (void)hipStreamSynchronize(pb->ctx->stream);
  for (auto &p : pb->pair_plan) near_plan_free(pb->ctx, p);
  for (auto &p : pb->obs_plan) near_plan_free(pb->ctx, p);
  pb->pair_plan.clear();
  pb->obs_plan.clear();
  pb->planned_kmax = -1.0;
}

static int problem_plan(fthms_problem *pb, double kmax) {
  if (kmax <= pb->planned_kmax) return FTHMS_OK;
  problem_free_plans(pb);
  fthms_ctx *ctx = pb->ctx;
  const int J = pb->narcs;
  pb->pair_plan.resize((size_t)J * J);
  pb->obs_plan.resize(J);
  int rc;
  for (int j = 0; j < J; ++j) {
    if ((rc = near_plan_build(ctx, pb->arcs[j], pb->nobs, pb->obs.data(), pb->obs_plan[j],
                              nullptr, kmax)))
      return rc;
    for (int k = 0; k < J && J > 1; ++k) {
      if (k == j) continue;
      if ((rc = near_plan_build(ctx, pb->arcs[k], pb->arcs[j]->n, pb->arcs[j]->xy.data(),
                                pb->pair_plan[(size_t)k * J + j], pb->skip[(size_t)k * J + j].data(),
                                kmax)))
        return rc;
    }
  }
  pb->planned_kmax = kmax;
  return FTHMS_OK;
}

extern "C" {

int fthms_problem_create(fthms_ctx *ctx, const fthms_problem_desc *d, fthms_problem **out) {
  if (!ctx || !d || !out) return fail(ctx, FTHMS_EINVAL, "NULL argument");
  *out = nullptr;
  if (d->narcs < 1 || !d->arcs) return fail(ctx, FTHMS_EINVAL, "narcs must be >= 1");
  if (d->M < 1) return fail(ctx, FTHMS_EINVAL, "M must be >= 1");
  if (d->precision != FTHMS_FP64 && d->precision != FTHMS_FP32_REFINED)
    return fail(ctx, FTHMS_EINVAL, "unknown precision");
  if (d->narcs > 1 && (!d->interval || !(d->period > 0.0) || !(d->c0 > 0.0) ||
                       !(d->c0 < 0.5) || !(d->c1 > 0.5) || !(d->c1 < 1.0)))
    return fail(ctx, FTHMS_EINVAL, "multi-arc problems need intervals, period > 0, "
                                   "0 < c0 < 1/2 < c1 < 1");
  if (d->nobs < 0 || (d->nobs > 0 && !d->obs_xy)) return fail(ctx, FTHMS_EINVAL, "bad obs");
  for (int j = 0; j < d->narcs; ++j)
    if (!d->arcs[j] || d->arcs[j]->ctx != ctx) return fail(ctx, FTHMS_EINVAL, "bad arc");
  fthms_problem *pb = new (std::nothrow) fthms_problem;
  if (!pb) return fail(ctx, FTHMS_ENOMEM, "host allocation failed");
  pb->ctx = ctx;
  pb->narcs = d->narcs;
  pb->M = d->narcs > 1 ? d->M : 1;
  pb->precision = d->precision;
  pb->tol = d->tol > 0.0 ? d->tol : 1e-12;
  pb->period = d->period;
  pb->c0 = d->c0;
  pb->c1 = d->c1;
  int rc = to_incident(ctx, &d->incident, pb->inc);
  if (rc) {
    delete pb;
    return rc;
  }
  pb->arcs.assign(d->arcs, d->arcs + d->narcs);
  const int J = pb->narcs;
  if (J > 1) pb->interval.assign(d->interval, d->interval + 2 * J);
  pb->nobs = d->nobs;
  pb->obs.assign(d->obs_xy, d->obs_xy + 2 * (size_t)d->nobs);
  if (!finite_all(pb->obs.data(), pb->obs.size())) {
    delete pb;
    return fail(ctx, FTHMS_EINVAL_DATA, "non-finite observation point");
  }
  if ((rc = dev_alloc(ctx, (void **)&pb->d_obs, sizeof(double2) * std::max(1, pb->nobs)))) {
    delete pb;
    return rc;
  }
  if (pb->nobs)
    HIPCK(ctx, hipMemcpy(pb->d_obs, pb->obs.data(), sizeof(double2) * pb->nobs,
                         hipMemcpyHostToDevice));
  // groups: arcs of one closed curve in cyclic order (d->group NULL: one curve)
  pb->group.assign(J, 0);
  if (d->group)
    for (int j = 0; j < J; ++j) pb->group[j] = d->group[j];
  pb->nxt.assign(J, -1);
  pb->prv.assign(J, -1);
  for (int j = 0; j < J; ++j) {
    std::vector<int> mem;
    for (int i = 0; i < J; ++i)
      if (pb->group[i] == pb->group[j]) mem.push_back(i);
    const int sz = (int)mem.size();
    if (sz < 2) continue;
    const int pos = (int)(std::find(mem.begin(), mem.end(), j) - mem.begin());
    pb->nxt[j] = mem[(pos + 1) % sz];
    pb->prv[j] = mem[(pos + sz - 1) % sz];
  }
  for (int j = 0; j < J; ++j)
    if (pb->arcs[j]->closed && pb->nxt[j] >= 0) {
      fthms_problem_destroy(pb);
      return fail(ctx, FTHMS_EINVAL, "a closed patch must be alone in its group");
    }
  if (J > 1) {
    // chi_j at the nodes (eq. POU1, chord reading) and overlap masks
    pb->d_chi.assign(J, nullptr);
    pb->skip.assign((size_t)J * J, std::vector<unsigned char>());
    for (int j = 0; j < J; ++j) {
      const fthms_arc *a = pb->arcs[j];
      const int nxt = pb->nxt[j], prv = pb->prv[j];
      std::vector<double> chi(a->n, 1.0), tau(a->n);
      if (nxt < 0) {  // an arc alone in its group: chi = 1, nothing masked
        if ((rc = dev_alloc(ctx, (void **)&pb->d_chi[j], sizeof(double) * a->n))) {
          fthms_problem_destroy(pb);
          return rc;
        }
        HIPCK(ctx, hipMemcpy(pb->d_chi[j], chi.data(), sizeof(double) * a->n,
                             hipMemcpyHostToDevice));
        for (int k = 0; k < J; ++k)
          if (k != j) pb->skip[(size_t)k * J + j].assign(a->n, 0);
        continue;
      }
      const double aj = pb->interval[2 * j], bj = pb->interval[2 * j + 1];
      for (int i = 0; i < a->n; ++i) tau[i] = 0.5 * (aj + bj) + 0.5 * (bj - aj) * a->t[i];
      double xe, ye, xs, ys;
      arc_end(a, +1, xe, ye);                // end of Gamma_j (in overlap with next)
      arc_end(pb->arcs[nxt], -1, xs, ys);   // start of Gamma_{j+1}
      const double A = std::hypot(xs - xe, ys - ye);
      double xe2, ye2, xs2, ys2;
      arc_end(pb->arcs[prv], +1, xe2, ye2);  // end of Gamma_{j-1} (in overlap with j)
      arc_end(a, -1, xs2, ys2);              // start of Gamma_j
      const double A2 = std::hypot(xs2 - xe2, ys2 - ye2);
      for (int i = 0; i < a->n; ++i) {
        const double px = a->xy[2 * i], py = a->xy[2 * i + 1];
        const bool on_nxt =
            in_interval(tau[i], pb->interval[2 * nxt], pb->interval[2 * nxt + 1], pb->period);
        const bool on_prv =
            in_interval(tau[i], pb->interval[2 * prv], pb->interval[2 * prv + 1], pb->period);
        // two arcs in a group overlap at both ends: the nearer end decides
        const bool use_nxt = on_nxt && (nxt != prv || std::hypot(px - xe, py - ye) <=
                                                          std::hypot(px - xs2, py - ys2));
        if (use_nxt) {
          const double dd = std::hypot(px - xe, py - ye);
          chi[i] = eta_window(A - dd, pb->c0 * A, pb->c1 * A);
        } else if (on_prv) {
          const double dd = std::hypot(px - xe2, py - ye2);
          chi[i] = 1.0 - eta_window(A2 - dd, pb->c0 * A2, pb->c1 * A2);
        }
      }
      if ((rc = dev_alloc(ctx, (void **)&pb->d_chi[j], sizeof(double) * a->n))) {
        fthms_problem_destroy(pb);
        return rc;
      }
      HIPCK(ctx, hipMemcpy(pb->d_chi[j], chi.data(), sizeof(double) * a->n, hipMemcpyHostToDevice));
      for (int k = 0; k < J; ++k) {
        if (k == j) continue;
        std::vector<unsigned char> sk(a->n, 0);
        if (k == nxt || k == prv)
          for (int i = 0; i < a->n; ++i)
            sk[i] = in_interval(tau[i], pb->interval[2 * k], pb->interval[2 * k + 1], pb->period)
                        ? 1
                        : 0;
        pb->skip[(size_t)k * J + j] = sk;
      }
    }
  }
  *out = pb;
  return FTHMS_OK;
}

int fthms_problem_destroy(fthms_problem *pb) {
  if (!pb) return FTHMS_EINVAL;
  fthms_ctx *ctx = pb->ctx;
  (void)hipStreamSynchronize(ctx->stream);
  problem_free_plans(pb);
  for (size_t j = 0; j < pb->d_chi.size(); ++j)
    dev_free(ctx, pb->d_chi[j], sizeof(double) * pb->arcs[j]->n);
  dev_free(ctx, pb->d_obs, sizeof(double2) * std::max(1, pb->nobs));
  delete pb;
  return FTHMS_OK;
}

}  // extern "C"

// Time-domain output of a run: traces[nt][nobs] of u_m = F^{-1}[U_m] at the
// observation points (trapezoid weights w), updated after every step m, and
// the stop rule |u_m - u_{m-1}| <= stop_tol |u_m| (stop_tol <= 0: run all M
// steps); steps receives the number of steps taken.
struct TraceReq {
  const double *w;
  int nt;
  const double *t;
  double stop_tol;
  double2 *traces;
  int *steps;
};

static int problem_run_impl(fthms_problem *pb, int nk, const double *k_dev, double kmax,
                            double2 *U, double2 *alpha_tot, const TraceReq *tr = nullptr) {
  fthms_ctx *ctx = pb->ctx;
  const int J = pb->narcs;
  const bool fp32 = pb->precision == FTHMS_FP32_REFINED;
  int rc = problem_plan(pb, kmax);
  if (rc) return rc;
  // per-wavenumber bytes of all arcs' matrices, factors and vectors
  size_t per = 0;
  int nsum = 0;
  for (int j = 0; j < J; ++j) {
    const size_t n = pb->arcs[j]->n;
    per += n * n * sizeof(double2) + (fp32 ? n * n * sizeof(float2) : 0) + n * sizeof(int) +
           kLuScratchBytes + 4 * n * sizeof(double2) + sizeof(int) + sizeof(double) + 2048;
    nsum += (int)n;
  }
  size_t cap = kChunkBytes;
  if (ctx->budget) {
    const size_t avail = ctx->budget > ctx->held ? ctx->budget - ctx->held + ctx->ws_bytes : 0;
    cap = std::min(cap, avail);
  }
  // Problems made only of closed patches (obstacles of an exterior problem,
  // each one patch) store every pair's cross operator once per wavenumber
  // (S x S, S = all nodes) when all wavenumbers fit with it, and apply it at
  // every step instead of evaluating the fields again.
  bool use_ops = J > 1 && nsum <= kCrossMaxS;
  for (int j = 0; j < J; ++j) use_ops = use_ops && pb->arcs[j]->closed;
  // the stored operators take the plain trapezoid rule: every node must lie
  // five node spacings or more from the other patches; nearer patches take
  // the field kernels, whose near plans upsample
  for (int j = 0; use_ops && j < J; ++j)
    for (int k = 0; use_ops && k < J; ++k) {
      if (k == j) continue;
      const fthms_arc *ak = pb->arcs[k], *aj = pb->arcs[j];
      for (int i = 0; use_ops && i < aj->n; ++i)
        for (int l = 0; use_ops && l < ak->n; ++l)
          if (!(std::hypot(aj->xy[2 * i] - ak->xy[2 * l], aj->xy[2 * i + 1] - ak->xy[2 * l + 1]) >=
                5.0 * ak->hmax))
            use_ops = false;
    }
  const size_t op_per = (size_t)nsum * nsum * sizeof(double2) + 2 * (size_t)nsum * sizeof(double2);
  if (use_ops && (size_t)nk * (per + op_per) + (size_t)(4 * nsum + 64) * 16 > cap) use_ops = false;
  if (use_ops) per += op_per;
  int C = (int)std::min<size_t>((size_t)nk, cap / per);
  C = std::min(C, 4096);
  if (C < 1) return fail(ctx, FTHMS_ENOMEM, "no room for one wavenumber");
  const int nchunks = (nk + C - 1) / C;  // even split of the batch
  C = (nk + nchunks - 1) / nchunks;
  if (tr && nchunks > 1)
    return fail(ctx, FTHMS_ENOMEM, "the time-domain stop rule needs every frequency resident "
                                   "(" + std::to_string(nk) + " do not fit)");
  struct ArcWs {
    double2 *A64;
    float2 *A32;
    int *piv, *status;
    void *swp;
    double *relres;
    double2 *b, *al, *cr, *tot;
  };
  std::vector<ArcWs> w(J);
  std::vector<size_t> ops_off;
  double2 *Tops = nullptr, *xcat = nullptr, *ycat = nullptr;
  double2 *Ustep = nullptr, *du = nullptr;
  double *nrm = nullptr;
  int *gate = nullptr;
  {
    size_t off = 0;
    std::vector<size_t> o((size_t)J * 10);
    auto take = [&](size_t bytes) {
      size_t r = off;
      off += (bytes + 255) & ~(size_t)255;
      return r;
    };
    for (int j = 0; j < J; ++j) {
      const size_t n = pb->arcs[j]->n;
      o[10 * j + 0] = take(n * n * sizeof(double2) * C);
      o[10 * j + 1] = fp32 ? take(n * n * sizeof(float2) * C) : 0;
      o[10 * j + 2] = take(n * sizeof(int) * C);
      o[10 * j + 3] = take(sizeof(int) * C);
      o[10 * j + 4] = take(sizeof(double) * C);
      for (int v = 0; v < 4; ++v) o[10 * j + 5 + v] = take(n * sizeof(double2) * C);
      o[10 * j + 9] = take(kLuScratchBytes * C);
    }
    // stored cross operators: T [C][S][S], gathered densities and fields
    // [C][S], node tables [S]
    const size_t oT = use_ops ? take(sizeof(double2) * (size_t)C * nsum * nsum) : 0;
    const size_t oX = use_ops ? take(sizeof(double2) * (size_t)C * nsum) : 0;
    const size_t oY = use_ops ? take(sizeof(double2) * (size_t)C * nsum) : 0;
    const size_t oNy = use_ops ? take(sizeof(double2) * (size_t)nsum) : 0;
    const size_t oNd = use_ops ? take(sizeof(double2) * (size_t)nsum) : 0;
    const size_t oNp = use_ops ? take(sizeof(int) * (size_t)nsum) : 0;
    const size_t oNh = use_ops ? take(sizeof(double) * (size_t)nsum) : 0;
    ops_off = {oT, oX, oY, oNy, oNd, oNp, oNh};
    if (tr) {
      o.push_back(take(sizeof(double2) * (size_t)C * std::max(1, pb->nobs)));   // U of a step
      o.push_back(take(sizeof(double2) * (size_t)tr->nt * std::max(1, pb->nobs)));  // its trace
      o.push_back(take(sizeof(double2) + 2 * sizeof(int)));  // two norms, then the gate
    }
    if ((rc = ensure_ws(ctx, off))) return rc;
    char *base = (char *)ctx->ws;
    for (int j = 0; j < J; ++j) {
      w[j].A64 = (double2 *)(base + o[10 * j + 0]);
      w[j].A32 = fp32 ? (float2 *)(base + o[10 * j + 1]) : nullptr;
      w[j].piv = (int *)(base + o[10 * j + 2]);
      w[j].status = (int *)(base + o[10 * j + 3]);
      w[j].relres = (double *)(base + o[10 * j + 4]);
      w[j].b = (double2 *)(base + o[10 * j + 5]);
      w[j].al = (double2 *)(base + o[10 * j + 6]);
      w[j].cr = (double2 *)(base + o[10 * j + 7]);
      w[j].tot = (double2 *)(base + o[10 * j + 8]);
      w[j].swp = (void *)(base + o[10 * j + 9]);
    }
    if (use_ops) {
      Tops = (double2 *)(base + ops_off[0]);
      xcat = (double2 *)(base + ops_off[1]);
      ycat = (double2 *)(base + ops_off[2]);
      // node tables of all patches, concatenated in arc order
      std::vector<double2> hy(nsum), hd(nsum);
      std::vector<int> hp(nsum);
      std::vector<double> hh(nsum);
      int q = 0;
      for (int j = 0; j < J; ++j) {
        const fthms_arc *a = pb->arcs[j];
        for (int i = 0; i < a->n; ++i, ++q) {
          hy[q] = make_double2(a->xy[2 * i], a->xy[2 * i + 1]);
          hd[q] = make_double2(a->dxy[2 * i], a->dxy[2 * i + 1]);
          hp[q] = j;
          hh[q] = 2.0 * kPi / a->n;
        }
      }
      HIPCK(ctx, hipMemcpy(base + ops_off[3], hy.data(), sizeof(double2) * nsum,
                           hipMemcpyHostToDevice));
      HIPCK(ctx, hipMemcpy(base + ops_off[4], hd.data(), sizeof(double2) * nsum,
                           hipMemcpyHostToDevice));
      HIPCK(ctx, hipMemcpy(base + ops_off[5], hp.data(), sizeof(int) * nsum,
                           hipMemcpyHostToDevice));
      HIPCK(ctx, hipMemcpy(base + ops_off[6], hh.data(), sizeof(double) * nsum,
                           hipMemcpyHostToDevice));
    }
    if (tr) {
      Ustep = (double2 *)(base + o[(size_t)10 * J]);
      du = (double2 *)(base + o[(size_t)10 * J + 1]);
      nrm = (double *)(base + o[(size_t)10 * J + 2]);
      gate = (int *)(nrm + 2);
    }
  }
  // later: a solve after the first with the same factors (the FP32 factors
  // of every arc are kept for all M steps; a matrix whose refinement fails
  // is refactored in FP64 once and solved with those factors afterwards)
  // FTHMS_REFINE_LATE_MAXIT=<n> in the environment caps the refinement
  // steps of later solves (a test hook: 0 makes every later refinement fail,
  // which exercises the late FP64 redo)
  int late_maxit = 10;
  if (const char *e = getenv("FTHMS_REFINE_LATE_MAXIT")) late_maxit = std::max(0, atoi(e));
  auto solve_arc = [&](int j, int c, bool later = false) -> int {
    const int n = pb->arcs[j]->n;
    const long long ms = (long long)n * n;
    if (!fp32) {
      tbeg(ctx, "solve");
      lu_solve64_kernel<<<c, kLuThreads, 0, ctx->stream>>>(w[j].A64, lu_perm(w[j].swp, c), n, ms,
                                                           w[j].b, w[j].al, n);
      tend(ctx);
      return check_launch(ctx, "lu_solve64_kernel");
    }
    const bool sym = use_sym_form(fp32, pb->arcs[j]);
    tbeg(ctx, "solve");
    launch_refine(ctx->stream, sym, c, w[j].A32, lu_perm(w[j].swp, c), w[j].A64, n, ms, w[j].b,
                  w[j].al, n, pb->tol, later ? late_maxit : 10, w[j].status, w[j].relres,
                  later ? 1 : 0);
    tend(ctx);
    int r = check_launch(ctx, "refine_kernel");
    if (r) return r;
    tbeg(ctx, "fallback");
    r = launch_fallback(ctx, w[j].A64, n, ms, w[j].piv, w[j].swp, w[j].b, w[j].al, w[j].status,
                        c, later ? kRedoLate : kRedoFailed, sym);
    tend(ctx);
    return r;
  };
  // fold the densities of step `step` into the traces.  With a stop
  // tolerance the rule is decided on the device: every accumulation of a
  // step after the one that met it is skipped (gate), so the host may run
  // ahead of the decision and reads it one step late.
  const bool gated = tr && tr->stop_tol > 0.0;
  auto trace_step = [&](int c, const double *kc, int step) -> int {
    const int P = pb->nobs;
    if (P == 0 || tr->nt == 0) return FTHMS_OK;
    zero_kernel<<<grid1d((long long)c * P), 256, 0, ctx->stream>>>(Ustep, (long long)c * P);
    int r;
    for (int j = 0; j < J; ++j) {
      const fthms_arc *a = pb->arcs[j];
      if ((r = field_dev_impl(ctx, a, c, kc, w[j].al, a->n, P, pb->d_obs, pb->obs_plan[j], Ustep,
                              P, 1)))
        return r;
    }
    if ((r = launch_freq_to_time(ctx, c, kc, tr->w, P, Ustep, tr->nt, tr->t, du))) return r;
    const long long nn = (long long)tr->nt * P;
    if (step == 1)
      HIPCK(ctx, hipMemcpyAsync(tr->traces, du, sizeof(double2) * nn, hipMemcpyDeviceToDevice,
                                ctx->stream));
    else if (gated)
      axpy_gated_kernel<<<grid1d(nn), 256, 0, ctx->stream>>>(tr->traces, du, nn, gate);
    else
      axpy_kernel<<<grid1d(nn), 256, 0, ctx->stream>>>(tr->traces, du, nn);
    if (!gated) return check_launch(ctx, "axpy_kernel");
    zero_kernel<<<1, 256, 0, ctx->stream>>>((double2 *)nrm, 1);
    const int nb = (int)std::min<long long>(1024, (nn + 255) / 256);
    norm2_kernel<<<nb, 256, 0, ctx->stream>>>(du, nn, nrm);
    norm2_kernel<<<nb, 256, 0, ctx->stream>>>(tr->traces, nn, nrm + 1);
    stop_check_kernel<<<1, 64, 0, ctx->stream>>>(nrm, tr->stop_tol, step, gate);
    return check_launch(ctx, "stop_check_kernel");
  };
  // the host's view of the gate: copied to pinned memory after each step,
  // read one step later (so the device never waits for the host)
  int *hgate = nullptr;
  if (gated) {
    if ((rc = ctx_pinned(ctx, &hgate))) return rc;
    hgate[0] = hgate[1] = 0;
    HIPCK(ctx, hipMemsetAsync(gate, 0, 2 * sizeof(int), ctx->stream));
  }
  auto publish_gate = [&](int slot) -> int {
    HIPCK(ctx, hipMemcpyAsync(hgate + slot, gate, sizeof(int), hipMemcpyDeviceToHost,
                              ctx->stream));
    HIPCK(ctx, hipEventRecord(ctx->ev_step[slot], ctx->stream));
    return FTHMS_OK;
  };
  auto read_gate = [&](int slot) -> int {
    HIPCK(ctx, hipEventSynchronize(ctx->ev_step[slot]));
    return hgate[slot];
  };
  long long aoff = 0;
  for (int f0 = 0; f0 < nk; f0 += C) {
    const int c = std::min(C, nk - f0);
    const double *kc = k_dev + f0;
    for (int j = 0; j < J; ++j) {
      const fthms_arc *a = pb->arcs[j];
      const int n = a->n;
      const bool sym = use_sym_form(fp32, a);
      tbeg(ctx, "assemble");
      rc = assemble_launch(ctx, a, kc, c, w[j].A64, fp32 ? w[j].A32 : nullptr, sym);
      tend(ctx);
      if (rc) return rc;
      tbeg(ctx, "lu");
      LuOpts lo;
      lo.sym = sym;
      rc = launch_lu(ctx, fp32, fp32 ? (void *)w[j].A32 : (void *)w[j].A64, n, (long long)n * n,
                     w[j].piv, w[j].swp, w[j].status, c, 0, lo);
      tend(ctx);
      if (rc) return rc;
      tbeg(ctx, "rhs");
      dim3 g((n + 255) / 256, c);
      incident_kernel<<<g, 256, 0, ctx->stream>>>(pb->inc, a->d_y, J > 1 ? pb->d_chi[j] : nullptr,
                                                   n, kc, -1.0, w[j].b, n);
      tend(ctx);
      if ((rc = check_launch(ctx, "incident_kernel"))) return rc;
      if ((rc = solve_arc(j, c))) return rc;
      HIPCK(ctx, hipMemcpyAsync(w[j].tot, w[j].al, sizeof(double2) * n * c,
                                hipMemcpyDeviceToDevice, ctx->stream));
    }
    if (use_ops && pb->M > 1) {
      tbeg(ctx, "field_cross");
      const long long ss = (long long)nsum * nsum;
      dim3 gb((unsigned)((ss + 255) / 256), c);
      closed_cross_build_kernel<<<gb, 256, 0, ctx->stream>>>(
          (const double2 *)((char *)ctx->ws + ops_off[3]),
          (const double2 *)((char *)ctx->ws + ops_off[4]), (const int *)((char *)ctx->ws + ops_off[5]),
          (const double *)((char *)ctx->ws + ops_off[6]), nsum, kc, Tops);
      tend(ctx);
      if ((rc = check_launch(ctx, "closed_cross_build_kernel"))) return rc;
    }
    int steps = 1, stop = 0;
    if (tr && (rc = trace_step(c, kc, 1))) return rc;
    if (gated && (rc = publish_gate(0))) return rc;
    for (int m = 1; m < pb->M && !stop; ++m) {
      tbeg(ctx, "field_cross");
      if (use_ops) {
        // the stored operators: gather every patch's densities, one product
        // per wavenumber, scatter the fields to the patches
        long long off = 0;
        for (int j = 0; j < J; ++j) {
          const int n = pb->arcs[j]->n;
          place_kernel<<<grid1d((long long)n * c), 256, 0, ctx->stream>>>(w[j].al, n, c, xcat,
                                                                          nsum, off);
          off += n;
        }
        dim3 ga((nsum + 15) / 16, c);
        cross_apply_kernel<<<ga, 256, 0, ctx->stream>>>(Tops, nsum, xcat, ycat);
        off = 0;
        for (int j = 0; j < J; ++j) {
          const int n = pb->arcs[j]->n;
          take_kernel<<<grid1d((long long)n * c), 256, 0, ctx->stream>>>(ycat, nsum, off, n, c,
                                                                         w[j].cr);
          off += n;
        }
        if ((rc = check_launch(ctx, "cross_apply_kernel"))) return rc;
      } else {
        for (int j = 0; j < J; ++j) {
          const long long nn = (long long)pb->arcs[j]->n * c;
          zero_kernel<<<grid1d(nn), 256, 0, ctx->stream>>>(w[j].cr, nn);
        }
        for (int j = 0; j < J; ++j)
          for (int k = 0; k < J; ++k) {
            if (k == j) continue;
            const fthms_arc *ak = pb->arcs[k], *aj = pb->arcs[j];
            if ((rc = field_dev_impl(ctx, ak, c, kc, w[k].al, ak->n, aj->n, aj->d_y,
                                     pb->pair_plan[(size_t)k * J + j], w[j].cr, aj->n, 1)))
              return rc;
          }
      }
      tend(ctx);
      for (int j = 0; j < J; ++j) {
        const int n = pb->arcs[j]->n;
        const long long nn = (long long)n * c;
        chi_scale_kernel<<<grid1d(nn), 256, 0, ctx->stream>>>(w[j].cr, pb->d_chi[j], n, nn, w[j].b);
        if ((rc = check_launch(ctx, "chi_scale_kernel"))) return rc;
        if ((rc = solve_arc(j, c, true))) return rc;
        if (gated)
          axpy_gated_kernel<<<grid1d(nn), 256, 0, ctx->stream>>>(w[j].tot, w[j].al, nn, gate);
        else
          axpy_kernel<<<grid1d(nn), 256, 0, ctx->stream>>>(w[j].tot, w[j].al, nn);
        if ((rc = check_launch(ctx, "axpy_kernel"))) return rc;
      }
      steps = m + 1;
      if (tr && (rc = trace_step(c, kc, m + 1))) return rc;
      if (gated) {
        // step m + 1 is enqueued; the decision after step m is read now
        if ((rc = publish_gate(m & 1))) return rc;
        stop = read_gate((m - 1) & 1) != 0;
      }
    }
    if (gated) {
      HIPCK(ctx, hipStreamSynchronize(ctx->stream));
      int g = 0;
      HIPCK(ctx, hipMemcpy(&g, gate, sizeof(int), hipMemcpyDeviceToHost));
      if (g) steps = g;
    }
    if (tr && tr->steps) *tr->steps = steps;
    if (pb->nobs > 0 && U) {
      double2 *Uc = U + (long long)f0 * pb->nobs;
      zero_kernel<<<grid1d((long long)c * pb->nobs), 256, 0, ctx->stream>>>(
          Uc, (long long)c * pb->nobs);
      tbeg(ctx, "field");
      for (int j = 0; j < J; ++j) {
        const fthms_arc *a = pb->arcs[j];
        if ((rc = field_dev_impl(ctx, a, c, kc, w[j].tot, a->n, pb->nobs, pb->d_obs,
                                 pb->obs_plan[j], Uc, pb->nobs, 1)))
          return rc;
      }
      tend(ctx);
    }
    if (alpha_tot) {
      long long off = 0;
      for (int j = 0; j < J; ++j) {
        const int n = pb->arcs[j]->n;
        place_kernel<<<grid1d((long long)n * c), 256, 0, ctx->stream>>>(
            w[j].tot, n, c, alpha_tot + (long long)f0 * nsum, nsum, off);
        if ((rc = check_launch(ctx, "place_kernel"))) return rc;
        off += n;
      }
    }
  }
  (void)aoff;
  return FTHMS_OK;
}

extern "C" {

int fthms_problem_run_dev(fthms_problem *pb, int nk, const double *k_dev, fthms_c64 *U_dev,
                          fthms_c64 *alpha_tot_dev) {
  if (!pb || nk < 0 || (nk > 0 && !k_dev)) return fail(pb ? pb->ctx : nullptr, FTHMS_EINVAL,
                                                        "bad argument to fthms_problem_run_dev");
  if (nk == 0) return FTHMS_OK;
  fthms_ctx *ctx = pb->ctx;
  HIPCK(ctx, hipSetDevice(ctx->device));
  std::vector<double> k(nk);
  HIPCK(ctx, hipMemcpyAsync(k.data(), k_dev, sizeof(double) * nk, hipMemcpyDeviceToHost,
                            ctx->stream));
  HIPCK(ctx, hipStreamSynchronize(ctx->stream));
  double kmax = 0.0;
  for (double v : k) {
    if (!(v > 0.0) || !std::isfinite(v))
      return fail(ctx, FTHMS_EINVAL_DATA, "wavenumbers must be finite and > 0");
    kmax = std::max(kmax, v);
  }
  return problem_run_impl(pb, nk, k_dev, kmax, (double2 *)U_dev, (double2 *)alpha_tot_dev);
}

int fthms_problem_traces_dev(fthms_problem *pb, int nk, const double *k_dev,
                             const double *w_dev, int nt, const double *t_dev, double stop_tol,
                             fthms_c64 *traces_dev, int *steps) {
  if (!pb || nk < 1 || !k_dev || !w_dev || nt < 0 || (nt > 0 && (!t_dev || !traces_dev)))
    return fail(pb ? pb->ctx : nullptr, FTHMS_EINVAL, "bad argument to fthms_problem_traces_dev");
  fthms_ctx *ctx = pb->ctx;
  HIPCK(ctx, hipSetDevice(ctx->device));
  std::vector<double> k(nk);
  HIPCK(ctx, hipMemcpyAsync(k.data(), k_dev, sizeof(double) * nk, hipMemcpyDeviceToHost,
                            ctx->stream));
  HIPCK(ctx, hipStreamSynchronize(ctx->stream));
  double kmax = 0.0;
  for (double v : k) {
    if (!(v > 0.0) || !std::isfinite(v))
      return fail(ctx, FTHMS_EINVAL_DATA, "wavenumbers must be finite and > 0");
    kmax = std::max(kmax, v);
  }
  TraceReq tr{w_dev, nt, t_dev, stop_tol, (double2 *)traces_dev, steps};
  return problem_run_impl(pb, nk, k_dev, kmax, nullptr, nullptr, &tr);
}

int fthms_problem_traces(fthms_problem *pb, int nk, const double *k, const double *w, int nt,
                         const double *t, double stop_tol, fthms_c64 *traces, int *steps) {
  if (!pb || nk < 1 || !k || !w || nt < 0 || (nt > 0 && (!t || !traces)))
    return fail(pb ? pb->ctx : nullptr, FTHMS_EINVAL, "bad argument to fthms_problem_traces");
  fthms_ctx *ctx = pb->ctx;
  HIPCK(ctx, hipSetDevice(ctx->device));
  Staging st(ctx);
  double *dk, *dw, *dt = nullptr;
  double2 *du = nullptr;
  int rc;
  if ((rc = st.get(&dk, sizeof(double) * nk)) || (rc = st.get(&dw, sizeof(double) * nk)) ||
      (rc = st.get(&dt, sizeof(double) * std::max(nt, 1))) ||
      (rc = st.get(&du, sizeof(double2) * std::max(nt, 1) * std::max(pb->nobs, 1))))
    return rc;
  HIPCK(ctx, hipMemcpyAsync(dk, k, sizeof(double) * nk, hipMemcpyHostToDevice, ctx->stream));
  HIPCK(ctx, hipMemcpyAsync(dw, w, sizeof(double) * nk, hipMemcpyHostToDevice, ctx->stream));
  if (nt > 0)
    HIPCK(ctx, hipMemcpyAsync(dt, t, sizeof(double) * nt, hipMemcpyHostToDevice, ctx->stream));
  if ((rc = fthms_problem_traces_dev(pb, nk, dk, dw, nt, dt, stop_tol, (fthms_c64 *)du, steps)))
    return rc;
  if (nt > 0 && pb->nobs > 0)
    HIPCK(ctx, hipMemcpyAsync(traces, du, sizeof(double2) * (size_t)nt * pb->nobs,
                              hipMemcpyDeviceToHost, ctx->stream));
  HIPCK(ctx, hipStreamSynchronize(ctx->stream));
  return FTHMS_OK;
}

int fthms_problem_run(fthms_problem *pb, int nk, const double *k, fthms_c64 *U,
                      fthms_c64 *alpha_tot) {
  if (!pb || nk < 0 || (nk > 0 && !k)) return fail(pb ? pb->ctx : nullptr, FTHMS_EINVAL,
                                                    "bad argument to fthms_problem_run");
  if (nk == 0) return FTHMS_OK;
  fthms_ctx *ctx = pb->ctx;
  HIPCK(ctx, hipSetDevice(ctx->device));
  double kmax = 0.0;
  for (int i = 0; i < nk; ++i) {
    if (!(k[i] > 0.0) || !std::isfinite(k[i]))
      return fail(ctx, FTHMS_EINVAL_DATA, "wavenumbers must be finite and > 0");
    kmax = std::max(kmax, k[i]);
  }
  int nsum = 0;
  for (auto a : pb->arcs) nsum += a->n;
  Staging st(ctx);
  double *dk;
  double2 *dU = nullptr, *dA = nullptr;
  int rc;
  if ((rc = st.get(&dk, sizeof(double) * nk))) return rc;
  if (U && pb->nobs && (rc = st.get(&dU, sizeof(double2) * (size_t)nk * pb->nobs))) return rc;
  if (alpha_tot && (rc = st.get(&dA, sizeof(double2) * (size_t)nk * nsum))) return rc;
  HIPCK(ctx, hipMemcpyAsync(dk, k, sizeof(double) * nk, hipMemcpyHostToDevice, ctx->stream));
  if ((rc = problem_run_impl(pb, nk, dk, kmax, dU, dA))) return rc;
  if (dU)
    HIPCK(ctx, hipMemcpyAsync(U, dU, sizeof(double2) * (size_t)nk * pb->nobs,
                              hipMemcpyDeviceToHost, ctx->stream));
  if (dA)
    HIPCK(ctx, hipMemcpyAsync(alpha_tot, dA, sizeof(double2) * (size_t)nk * nsum,
                              hipMemcpyDeviceToHost, ctx->stream));
  HIPCK(ctx, hipStreamSynchronize(ctx->stream));
  return FTHMS_OK;
}

}  // extern "C"
