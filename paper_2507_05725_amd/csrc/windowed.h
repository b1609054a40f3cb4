// Windowing and time recentering of the multiple-scattering recursion
// (Section 2.1, eqs. windowing, Fourierk, TDsol; Algorithm 1 with Q windows;
// the window function of Section 5).
//
// Each step m works on boundary data g_{j,m}(y, t_n), t_n = n dt, at the
// nodes of every arc (time-major [nt][n]).  For every arc j and window q:
//   G(w_l) = sum_n dt P(t_n - s_q) g_j(t_n) exp(i w_l (t_n - s_q))      (eq. Fourierk)
//   Psi(w_l) = A_j(w_l)^{-1} G(w_l)       (factors of the first step reused)
//   V(w_l) at the other arcs' nodes and the observation points (near/far fields)
//   v(t_n) += (1/2pi) sum_l w_l V(w_l) exp(-i w_l (t_n - s_q))           (eq. TDsol)
// and after all arcs g_{k,m+1} = -chi_k sum_{j != k} v~_{j,k,m} (eqs.
// criterion_int2, vtilde: the fields skip the masked overlap nodes), while
// the observation fields accumulate into u_M.  Both transforms are the dense
// frequency/time kernel of the single-window path: the forward one with the
// roles of times and frequencies exchanged.  Window: s_q = 3/2 (q-1) H,
// P(s) = eta(s/H; 1/2, 1) on [-H/2, H], 1 - eta(s/H + 3/2; 1/2, 1) on
// (-H, -H/2), 0 elsewhere.  Signals are complex, frequencies positive.
// The initial data come from a train of Gaussian plane-wave pulses given in
// the time domain (u2 of Section 5 transformed back):
//   u(x, t) = sum_p f(t - p T - x.d),
//   f(tau) = sigma/(2 sqrt(pi)) exp(-i w0 (tau - tau0) - sigma^2 (tau - tau0)^2 / 4).
#pragma once

namespace fthms {

struct PulseTrainDev {
  double dx, dy, omega0, sigma, tau0, period;
  int npulse;
  // 1: the real pulses u3 of Section 5 (eq. planewave, t_lag = 2) instead,
  // u(x, t) = sum_p u3(x, t - p period) (eq. multi)
  int real_u3 = 0;
};

// out[n][i] = -chi[i] u(y_i, n dt)   (chi == nullptr: 1)
__global__ void pulse_train_kernel(PulseTrainDev in, const double2 *__restrict__ y,
                                   const double *__restrict__ chi, int n, int nt, double dt,
                                   double2 *__restrict__ out) {
  const long long nn = (long long)n * nt;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % n);
    const double tn = (double)(e / n) * dt;
    const double xd = y[i].x * in.dx + y[i].y * in.dy;
    double ar = 0.0, ai = 0.0;
    if (in.real_u3) {
      for (int p = 0; p < in.npulse; ++p) {
        const double l = tn - p * in.period - 2.0 - xd;
        ar += -sin(4.0 * l) * exp(-1.6 * (l - 3.0) * (l - 3.0));
      }
      const double sc = chi ? -chi[i] : -1.0;
      out[e] = make_double2(sc * ar, 0.0);
      continue;
    }
    for (int p = 0; p < in.npulse; ++p) {
      const double tau = tn - p * in.period - xd - in.tau0;
      const double a = in.sigma / (2.0 * sqrt(kPi)) * exp(-0.25 * in.sigma * in.sigma * tau * tau);
      double s, c;
      sincos(-in.omega0 * tau, &s, &c);
      ar += a * c;
      ai += a * s;
    }
    const double sc = chi ? -chi[i] : -1.0;
    out[e] = make_double2(sc * ar, sc * ai);
  }
}

// x[q][l][i] *= exp(i w_l s_q): the recentering phase of window q folded
// into its densities, so that all windows share one field evaluation and
// one inverse transform at unshifted times
__global__ void window_phase_kernel(double2 *__restrict__ x, int n, int nk, int Q,
                                    const double *__restrict__ k, const double *__restrict__ s) {
  const long long nn = (long long)n * nk * Q;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nn;
       e += (long long)gridDim.x * blockDim.x) {
    const long long b = e / n;
    const int l = (int)(b % nk), q = (int)(b / nk);
    double sn, cs;
    sincos(k[l] * s[q], &sn, &cs);
    const double2 v = x[e];
    x[e] = make_double2(v.x * cs - v.y * sn, v.x * sn + v.y * cs);
  }
}

// P(s) of the windowing partition of unity (host)
static double window_pou(double s, double H) {
  if (s >= -0.5 * H && s <= H) return eta_window(s / H, 0.5, 1.0);
  if (s > -H && s < -0.5 * H) return 1.0 - eta_window(s / H + 1.5, 0.5, 1.0);
  return 0.0;
}

// hfW (real signals, optional): the high-frequency transform's weights
// [nt][Q nk] at the shifted times t_n - s_q (column q nk + l), used for the
// way back instead of the trapezoid sum with the recentering phase.
static int problem_windowed_impl(fthms_problem *pb, int nk, const double *k_dev,
                                 const double *w_dev, const std::vector<double> &k_host,
                                 double kmax, int nt, double dt, int Q, double H,
                                 const PulseTrainDev &inc, double2 *traces,
                                 const double2 *hfW = nullptr) {
  fthms_ctx *ctx = pb->ctx;
  const int J = pb->narcs, P = pb->nobs;
  int rc = problem_plan(pb, kmax);
  if (rc) return rc;
  int nmax = std::max(P, 1);
  for (int j = 0; j < J; ++j) nmax = std::max(nmax, pb->arcs[j]->n);
  // workspace: per arc factors, permutations, status, right-hand sides and
  // densities for all frequencies, time series of data and cross fields;
  // shared frequency and time buffers, window tables
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t r = off;
    off += (bytes + 255) & ~(size_t)255;
    return r;
  };
  // refined form: FP64 matrices kept for the residuals beside FP32 factors
  const bool fp32 = pb->precision == FTHMS_FP32_REFINED;
  struct Ws {
    size_t A, A32, piv, swp, st, rr, G, psi, g, cr;
  };
  std::vector<Ws> o(J);
  for (int j = 0; j < J; ++j) {
    const size_t n = pb->arcs[j]->n;
    o[j].A = take(n * n * sizeof(double2) * nk);
    o[j].A32 = fp32 ? take(n * n * sizeof(float2) * nk) : 0;
    o[j].rr = take(sizeof(double) * nk);
    o[j].piv = take(n * sizeof(int) * nk);
    o[j].swp = take(kLuScratchBytes * nk);
    o[j].st = take(sizeof(int) * nk);
    o[j].G = take(n * sizeof(double2) * nk * Q);
    o[j].psi = take(n * sizeof(double2) * nk * Q);
    o[j].g = take(n * sizeof(double2) * nt);
    o[j].cr = take(n * sizeof(double2) * nt);
  }
  const size_t oV = take((size_t)nmax * sizeof(double2) * nk * Q);
  const size_t oT = take((size_t)nmax * sizeof(double2) * nt);
  const size_t oTq = take(sizeof(double) * (size_t)Q * nt);  // t_n - s_q
  const size_t oWq = take(sizeof(double) * (size_t)Q * nt);  // 2pi dt P(t_n - s_q)
  const size_t oNk = take(sizeof(double) * nk);              // -w_l
  const size_t oKq = take(sizeof(double) * nk * Q);          // w_l, tiled per window
  const size_t oWt = take(sizeof(double) * nk * Q);          // quadrature weights, tiled
  const size_t oSq = take(sizeof(double) * Q);               // s_q
  const size_t oT0 = take(sizeof(double) * nt);              // t_n
  if (ctx->budget && off > ctx->budget)
    return fail(ctx, FTHMS_ENOMEM, "windowed run: the factors and time series of all "
                                   "frequencies do not fit the budget");
  if ((rc = ensure_ws(ctx, off))) return rc;
  char *base = (char *)ctx->ws;
  auto at = [&](size_t o_) { return (void *)(base + o_); };
  double2 *V = (double2 *)at(oV), *T = (double2 *)at(oT);
  double *tq = (double *)at(oTq), *wq = (double *)at(oWq), *nkv = (double *)at(oNk);
  double *kq = (double *)at(oKq), *wt = (double *)at(oWt), *sqv = (double *)at(oSq);
  double *t0v = (double *)at(oT0);
  {
    std::vector<double> htq((size_t)Q * nt), hwq((size_t)Q * nt), hnk(nk), hsq(Q), ht0(nt);
    for (int q = 0; q < Q; ++q) {
      hsq[q] = 1.5 * H * q;
      for (int n = 0; n < nt; ++n) {
        const double s = n * dt - hsq[q];
        htq[(size_t)q * nt + n] = s;
        hwq[(size_t)q * nt + n] = 2.0 * kPi * dt * window_pou(s, H);
      }
    }
    for (int n = 0; n < nt; ++n) ht0[n] = n * dt;
    for (int l = 0; l < nk; ++l) hnk[l] = -k_host[l];
    // on the context stream: k_dev and w_dev were written there
    hipStream_t st = ctx->stream;
    HIPCK(ctx, hipMemcpyAsync(tq, htq.data(), sizeof(double) * htq.size(), hipMemcpyHostToDevice, st));
    HIPCK(ctx, hipMemcpyAsync(wq, hwq.data(), sizeof(double) * hwq.size(), hipMemcpyHostToDevice, st));
    HIPCK(ctx, hipMemcpyAsync(nkv, hnk.data(), sizeof(double) * nk, hipMemcpyHostToDevice, st));
    HIPCK(ctx, hipMemcpyAsync(sqv, hsq.data(), sizeof(double) * Q, hipMemcpyHostToDevice, st));
    HIPCK(ctx, hipMemcpyAsync(t0v, ht0.data(), sizeof(double) * nt, hipMemcpyHostToDevice, st));
    for (int q = 0; q < Q; ++q) {
      HIPCK(ctx, hipMemcpyAsync(kq + (size_t)q * nk, k_dev, sizeof(double) * nk,
                                hipMemcpyDeviceToDevice, st));
      HIPCK(ctx, hipMemcpyAsync(wt + (size_t)q * nk, w_dev, sizeof(double) * nk,
                                hipMemcpyDeviceToDevice, st));
    }
    HIPCK(ctx, hipStreamSynchronize(st));  // the host tables go out of scope
  }
  const int nkq = nk * Q;
  // factor every (arc, frequency) matrix once; initial data in time
  for (int j = 0; j < J; ++j) {
    const fthms_arc *a = pb->arcs[j];
    const int n = a->n;
    double2 *A = (double2 *)at(o[j].A);
    float2 *A32 = fp32 ? (float2 *)at(o[j].A32) : nullptr;
    const bool sym = use_sym_form(fp32, a);
    tbeg(ctx, "assemble");
    rc = assemble_launch(ctx, a, k_dev, nk, A, A32, sym);
    tend(ctx);
    if (rc) return rc;
    tbeg(ctx, "lu");
    LuOpts lo;
    lo.sym = sym;
    rc = launch_lu(ctx, fp32, fp32 ? (void *)A32 : (void *)A, n, (long long)n * n,
                   (int *)at(o[j].piv), at(o[j].swp), (int *)at(o[j].st), nk, 0, lo);
    tend(ctx);
    if (rc) return rc;
    const long long nn = (long long)nt * n;
    pulse_train_kernel<<<grid1d(nn), 256, 0, ctx->stream>>>(
        inc, a->d_y, J > 1 ? pb->d_chi[j] : nullptr, n, nt, dt, (double2 *)at(o[j].g));
    if ((rc = check_launch(ctx, "pulse_train_kernel"))) return rc;
  }
  const long long ntr = (long long)nt * P;
  if (ntr) zero_kernel<<<grid1d(ntr), 256, 0, ctx->stream>>>(traces, ntr);
  // all windows at once: (window, frequency) pairs with the phase folded in
  auto to_time = [&](int np, const double2 *Vf, double2 *out) -> int {
    if (hfW) {
      dim3 g2((np + 63) / 64, (nt + 63) / 64);
      hf_apply_kernel<false><<<g2, 256, 0, ctx->stream>>>(hfW, nt, nkq, Vf, np, out, 0);
      return check_launch(ctx, "hf_apply_kernel");
    }
    return launch_freq_to_time(ctx, nkq, kq, wt, np, Vf, nt, t0v, out);
  };
  for (int m = 0; m < pb->M; ++m) {
    for (int k = 0; k < J; ++k) {
      const long long nn = (long long)nt * pb->arcs[k]->n;
      zero_kernel<<<grid1d(nn), 256, 0, ctx->stream>>>((double2 *)at(o[k].cr), nn);
    }
    for (int j = 0; j < J; ++j) {
      const fthms_arc *a = pb->arcs[j];
      const int n = a->n;
      double2 *G = (double2 *)at(o[j].G), *psi = (double2 *)at(o[j].psi);
      for (int q = 0; q < Q; ++q) {
        // slow transform about s_q: sum over time samples with the window weights
        double2 *Gq = G + (size_t)q * nk * n, *pq = psi + (size_t)q * nk * n;
        tbeg(ctx, "window_transform");
        rc = launch_freq_to_time(ctx, nt, tq + (size_t)q * nt, wq + (size_t)q * nt, n,
                                 (const double2 *)at(o[j].g), nk, nkv, Gq);
        tend(ctx);
        if (rc) return rc;
        if (!fp32) {
          tbeg(ctx, "solve");
          lu_solve64_kernel<<<nk, kLuThreads, 0, ctx->stream>>>(
              (double2 *)at(o[j].A), lu_perm(at(o[j].swp), nk), n, (long long)n * n, Gq, pq, n);
          tend(ctx);
          if ((rc = check_launch(ctx, "lu_solve64_kernel"))) return rc;
        } else {
          // the first solve of each matrix uses fresh factors; every later
          // one (other windows, later steps) reuses them
          const bool later = m > 0 || q > 0;
          const bool sym = use_sym_form(fp32, pb->arcs[j]);
          tbeg(ctx, "solve");
          launch_refine(ctx->stream, sym, nk, (const float2 *)at(o[j].A32),
                        lu_perm(at(o[j].swp), nk), (const double2 *)at(o[j].A), n,
                        (long long)n * n, Gq, pq, n, pb->tol, 10, (int *)at(o[j].st),
                        (double *)at(o[j].rr), later ? 1 : 0);
          tend(ctx);
          if ((rc = check_launch(ctx, "refine_kernel"))) return rc;
          tbeg(ctx, "fallback");
          rc = launch_fallback(ctx, (double2 *)at(o[j].A), n, (long long)n * n,
                               (int *)at(o[j].piv), at(o[j].swp), Gq, pq, (int *)at(o[j].st), nk,
                               later ? kRedoLate : kRedoFailed, sym);
          tend(ctx);
          if (rc) return rc;
        }
      }
      if (!hfW) {
        window_phase_kernel<<<grid1d((long long)n * nkq), 256, 0, ctx->stream>>>(psi, n, nk, Q,
                                                                                 k_dev, sqv);
        if ((rc = check_launch(ctx, "window_phase_kernel"))) return rc;
      }
      // fields of all windows at the other arcs' nodes, back to time
      for (int k = 0; k < J && J > 1; ++k) {
        if (k == j) continue;
        const fthms_arc *b = pb->arcs[k];
        const long long nv = (long long)nkq * b->n;
        zero_kernel<<<grid1d(nv), 256, 0, ctx->stream>>>(V, nv);
        tbeg(ctx, "field");
        rc = field_dev_impl(ctx, a, nkq, kq, psi, n, b->n, b->d_y,
                            pb->pair_plan[(size_t)j * J + k], V, b->n, 0);
        tend(ctx);
        if (rc) return rc;
        tbeg(ctx, "freq_to_time");
        rc = to_time(b->n, V, T);
        tend(ctx);
        if (rc) return rc;
        axpy_kernel<<<grid1d((long long)nt * b->n), 256, 0, ctx->stream>>>(
            (double2 *)at(o[k].cr), T, (long long)nt * b->n);
      }
      if (P) {
        const long long nv = (long long)nkq * P;
        zero_kernel<<<grid1d(nv), 256, 0, ctx->stream>>>(V, nv);
        tbeg(ctx, "field");
        rc = field_dev_impl(ctx, a, nkq, kq, psi, n, P, pb->d_obs, pb->obs_plan[j], V, P, 0);
        tend(ctx);
        if (rc) return rc;
        tbeg(ctx, "freq_to_time");
        rc = to_time(P, V, T);
        tend(ctx);
        if (rc) return rc;
        axpy_kernel<<<grid1d(ntr), 256, 0, ctx->stream>>>(traces, T, ntr);
      }
    }
    // next step's data: g_k = -chi_k * (masked sum of the other arcs' fields)
    if (m + 1 < pb->M)
      for (int k = 0; k < J; ++k) {
        const int n = pb->arcs[k]->n;
        const long long nn = (long long)nt * n;
        chi_scale_kernel<<<grid1d(nn), 256, 0, ctx->stream>>>((const double2 *)at(o[k].cr),
                                                              pb->d_chi[k], n, nn,
                                                              (double2 *)at(o[k].g));
      }
    if ((rc = check_launch(ctx, "windowed step"))) return rc;
  }
  return FTHMS_OK;
}

}  // namespace fthms

extern "C" {

int fthms_problem_traces_windowed(fthms_problem *pb, int nk, const double *k, const double *w,
                                  int nt, double dt, int Q, double H,
                                  const fthms_pulse_train *inc, fthms_c64 *traces) {
  if (!pb || nk < 1 || !k || !w || nt < 1 || !(dt > 0.0) || Q < 1 || !(H > 0.0) || !inc ||
      !traces || inc->npulse < 1 || !(inc->sigma > 0.0))
    return fail(pb ? pb->ctx : nullptr, FTHMS_EINVAL,
                "bad argument to fthms_problem_traces_windowed");
  fthms_ctx *ctx = pb->ctx;
  double kmax = 0.0;
  for (int l = 0; l < nk; ++l) {
    if (!(k[l] > 0.0) || !std::isfinite(k[l]) || !std::isfinite(w[l]))
      return fail(ctx, FTHMS_EINVAL_DATA, "wavenumbers must be finite and > 0");
    kmax = std::max(kmax, k[l]);
  }
  HIPCK(ctx, hipSetDevice(ctx->device));
  Staging st(ctx);
  double *dk, *dw;
  double2 *du;
  int rc;
  const int P = std::max(pb->nobs, 1);
  if ((rc = st.get(&dk, sizeof(double) * nk)) || (rc = st.get(&dw, sizeof(double) * nk)) ||
      (rc = st.get(&du, sizeof(double2) * (size_t)nt * P)))
    return rc;
  HIPCK(ctx, hipMemcpyAsync(dk, k, sizeof(double) * nk, hipMemcpyHostToDevice, ctx->stream));
  HIPCK(ctx, hipMemcpyAsync(dw, w, sizeof(double) * nk, hipMemcpyHostToDevice, ctx->stream));
  PulseTrainDev d;
  d.dx = std::cos(inc->theta);
  d.dy = std::sin(inc->theta);
  d.omega0 = inc->omega0;
  d.sigma = inc->sigma;
  d.tau0 = inc->tau0;
  d.period = inc->period;
  d.npulse = inc->npulse;
  std::vector<double> kh(k, k + nk);
  if ((rc = problem_windowed_impl(pb, nk, dk, dw, kh, kmax, nt, dt, Q, H, d, du))) return rc;
  if (pb->nobs)
    HIPCK(ctx, hipMemcpyAsync(traces, du, sizeof(double2) * (size_t)nt * pb->nobs,
                              hipMemcpyDeviceToHost, ctx->stream));
  HIPCK(ctx, hipStreamSynchronize(ctx->stream));
  return FTHMS_OK;
}

int fthms_problem_traces_windowed_real(fthms_problem *pb, const fthms_hf_grid *grid, int nt,
                                       double dt, int Q, double H, const fthms_pulse3 *inc,
                                       double *traces) {
  HfSet hs;
  if (!pb || !hf_set_from(grid, hs) || nt < 1 || !(dt > 0.0) || Q < 1 || !(H > 0.0) || !inc ||
      !traces || inc->npulse < 1 || !std::isfinite(inc->theta) || !std::isfinite(inc->period))
    return fail(pb ? pb->ctx : nullptr, FTHMS_EINVAL,
                "bad argument to fthms_problem_traces_windowed_real");
  fthms_ctx *ctx = pb->ctx;
  const int nk = (int)hs.omega.size();
  const int nt_out = nt;
  // the recursion's time mesh covers [0, s_Q + H], the whole support of the
  // last window (the time mesh of Section 5): a window cut short would give
  // its data a jump that no band-limited transform reproduces; these
  // transforms have no period in time, so the mesh may extend past the
  // traces asked for
  nt = std::max(nt, (int)std::ceil((1.5 * (Q - 1) * H + H) / dt - 1e-9) + 1);
  HIPCK(ctx, hipSetDevice(ctx->device));
  // the transform's weights at the shifted times t_n - s_q, one row per
  // distinct time (the shifts are usually whole numbers of steps)
  HfFc fc;
  hf_fc_factor(fc, hs.L, hs.W - hs.wc, hs.wc);
  std::vector<zd> Wall((size_t)nt * Q * nk);
  std::map<long long, std::vector<zd>> rows;
  std::vector<zd> row(nk);
  for (int q = 0; q < Q; ++q)
    for (int n = 0; n < nt; ++n) {
      const double tt = n * dt - 1.5 * H * q;
      const long long key = std::llround(tt * 1e9);
      auto it = rows.find(key);
      if (it == rows.end()) {
        hf_weight_rows(hs, fc, &tt, 1, row.data());
        it = rows.emplace(key, row).first;
      }
      std::copy(it->second.begin(), it->second.end(),
                Wall.begin() + (size_t)n * Q * nk + (size_t)q * nk);
    }
  Staging st(ctx);
  double *dk, *dw;
  double2 *du, *dW;
  int rc;
  const int P = std::max(pb->nobs, 1);
  if ((rc = st.get(&dk, sizeof(double) * nk)) || (rc = st.get(&dw, sizeof(double) * nk)) ||
      (rc = st.get(&du, sizeof(double2) * (size_t)nt * P)) ||
      (rc = st.get(&dW, sizeof(double2) * Wall.size())))
    return rc;
  std::vector<double> zeros(nk, 0.0);
  HIPCK(ctx, hipMemcpyAsync(dk, hs.omega.data(), sizeof(double) * nk, hipMemcpyHostToDevice,
                            ctx->stream));
  HIPCK(ctx, hipMemcpyAsync(dw, zeros.data(), sizeof(double) * nk, hipMemcpyHostToDevice,
                            ctx->stream));
  HIPCK(ctx, hipMemcpyAsync(dW, Wall.data(), sizeof(double2) * Wall.size(), hipMemcpyHostToDevice,
                            ctx->stream));
  PulseTrainDev d{};
  d.dx = std::cos(inc->theta);
  d.dy = std::sin(inc->theta);
  d.period = inc->period;
  d.npulse = inc->npulse;
  d.real_u3 = 1;
  if ((rc = problem_windowed_impl(pb, nk, dk, dw, hs.omega, hs.W, nt, dt, Q, H, d, du, dW)))
    return rc;
  if (pb->nobs) {
    std::vector<double2> h((size_t)nt_out * pb->nobs);  // the first rows
    HIPCK(ctx, hipMemcpyAsync(h.data(), du, sizeof(double2) * h.size(), hipMemcpyDeviceToHost,
                              ctx->stream));
    HIPCK(ctx, hipStreamSynchronize(ctx->stream));
    for (size_t e = 0; e < h.size(); ++e) traces[e] = h[e].x;
  }
  HIPCK(ctx, hipStreamSynchronize(ctx->stream));
  return FTHMS_OK;
}

}  // extern "C"
