// Serving: a request loop over scattering jobs of different sizes.
//
// A request is a whole multiple-scattering problem -- arcs of one or more
// obstacles (node samples), frequencies with quadrature weights, incident
// field, observation points and times -- answered with its time traces.
// The server keeps a FIFO queue and W worker threads, each with its own
// context (own stream and workspace) on the same GPU.  A request is
// admitted when a worker is free and its HBM estimate fits next to the
// requests already running; admitted requests run concurrently, so their
// kernels overlap on the device while new ones keep arriving (continuous
// batching at the request level).  Each request runs alone in its context
// with a budget-independent chunking, so its result does not depend on
// what else is resident.  Latency is taken from submission to the traces
// being in host memory.
#pragma once

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>

struct fthms_server {
  struct Job {
    // copy of the request
    int narcs = 0, n = 0, nk = 0, nobs = 0, nt = 0, max_steps = 1;
    int closed = 0, precision = FTHMS_FP64;
    double period = 0.0, stop_tol = 0.0;
    std::vector<double> xy, dxy, ddxy, interval, k, w, obs, t;
    std::vector<int> group;
    fthms_incident inc{};
    // bookkeeping
    int state = FTHMS_JOB_QUEUED;
    int rc = FTHMS_OK;
    std::string err;
    size_t est = 0;
    bool cancel = false;
    std::chrono::steady_clock::time_point t_submit, t_start, t_done;
    // result
    std::vector<double2> traces;
    int steps = 0;
  };
  int device = 0;
  size_t budget = 0;
  size_t in_use = 0;
  int nworkers = 0;
  uint64_t next = 1;
  bool stop = false;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> queue;
  std::map<uint64_t, Job> jobs;
  std::vector<std::thread> workers;
  std::string err;
};

namespace {

// Device memory a request needs: every (arc, frequency) matrix resident at
// once (the time-domain stop rule keeps all frequencies in flight), factors,
// vectors and scratch, plus traces.
size_t request_bytes(const fthms_request *r) {
  const size_t n = (size_t)r->n;
  const size_t per = n * n * sizeof(double2) +
                     (r->precision == FTHMS_FP32_REFINED ? n * n * sizeof(float2) : 0) +
                     n * sizeof(int) + kLuScratchBytes + 4 * n * sizeof(double2) + sizeof(int) +
                     sizeof(double) + 2048;
  // closed obstacles: the stored cross operators of all patches ([S][S] per
  // frequency, S = narcs n) when they fit beside the rest
  const size_t S = n * (size_t)r->narcs;
  const size_t ops = (r->closed && r->narcs > 1 && S <= (size_t)kCrossMaxS)
                         ? (S * S + 2 * S) * sizeof(double2) * (size_t)r->nk
                         : 0;
  return per * (size_t)r->narcs * (size_t)r->nk + ops +
         2 * sizeof(double2) * (size_t)std::max(1, r->nt) * std::max(1, r->nobs) +
         sizeof(double2) * (size_t)r->nk * std::max(1, r->nobs) + ((size_t)64 << 20);
}

// Run one admitted request in the worker's context.
int serve_run(fthms_ctx *ctx, fthms_server::Job &jb) {
  const int J = jb.narcs, n = jb.n;
  std::vector<fthms_arc *> arcs(J, nullptr);
  int rc = FTHMS_OK;
  for (int j = 0; j < J && rc == FTHMS_OK; ++j)
    rc = jb.closed ? fthms_closed_create(ctx, n, jb.xy.data() + (size_t)2 * n * j,
                                         jb.dxy.data() + (size_t)2 * n * j,
                                         jb.ddxy.data() + (size_t)2 * n * j, &arcs[j])
                   : fthms_arc_create(ctx, n, jb.xy.data() + (size_t)2 * n * j,
                                      jb.dxy.data() + (size_t)2 * n * j, &arcs[j]);
  fthms_problem *pb = nullptr;
  if (rc == FTHMS_OK) {
    fthms_problem_desc d{};
    d.narcs = J;
    d.arcs = (const fthms_arc *const *)arcs.data();
    d.interval = jb.interval.data();
    d.period = jb.period;
    d.c0 = 1.0 / 3.0;
    d.c1 = 2.0 / 3.0;
    d.M = jb.max_steps;
    d.precision = jb.precision;
    d.tol = 1e-12;
    d.incident = jb.inc;
    d.nobs = jb.nobs;
    d.obs_xy = jb.obs.data();
    d.group = jb.group.data();
    rc = fthms_problem_create(ctx, &d, &pb);
  }
  if (rc == FTHMS_OK) {
    jb.traces.resize((size_t)jb.nt * jb.nobs);
    rc = fthms_problem_traces(pb, jb.nk, jb.k.data(), jb.w.data(), jb.nt, jb.t.data(),
                              jb.stop_tol, (fthms_c64 *)jb.traces.data(), &jb.steps);
  }
  if (rc) jb.err = fthms_last_error(ctx);
  if (pb) fthms_problem_destroy(pb);
  for (auto a : arcs)
    if (a) fthms_arc_destroy(a);
  // give the request's workspace back before the next one is admitted
  (void)hipStreamSynchronize(ctx->stream);
  dev_free(ctx, ctx->ws, ctx->ws_bytes);
  ctx->ws = nullptr;
  ctx->ws_bytes = 0;
  dev_free(ctx, ctx->ws2, ctx->ws2_bytes);
  ctx->ws2 = nullptr;
  ctx->ws2_bytes = 0;
  dev_free(ctx, ctx->ft, ctx->ft_bytes);
  ctx->ft = nullptr;
  ctx->ft_bytes = 0;
  return rc;
}

void serve_worker(fthms_server *sv) {
  fthms_ctx *ctx = nullptr;
  // a private stream per worker, so that requests run side by side
  const int rc0 = fthms_create(&ctx, sv->device, 0, FTHMS_OWN_STREAM);
  if (ctx) ctx->async_alloc = true;
  for (;;) {
    uint64_t id = 0;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      // strict FIFO: the oldest request waits for room, later ones behind it
      sv->cv.wait(lk, [&] {
        if (sv->stop) return true;
        if (sv->queue.empty()) return false;
        const auto &jb = sv->jobs[sv->queue.front()];
        return sv->in_use == 0 || sv->in_use + jb.est <= sv->budget;
      });
      if (sv->stop && sv->queue.empty()) break;
      if (sv->stop) break;
      id = sv->queue.front();
      sv->queue.pop_front();
      auto &jb = sv->jobs[id];
      jb.state = FTHMS_JOB_RUNNING;
      jb.t_start = std::chrono::steady_clock::now();
      sv->in_use += jb.est;
    }
    fthms_server::Job *jp;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      jp = &sv->jobs[id];  // std::map nodes are stable
    }
    int rc = rc0 ? rc0 : serve_run(ctx, *jp);
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      jp->t_done = std::chrono::steady_clock::now();
      jp->rc = rc;
      if (rc0) jp->err = "worker context: " + std::string(fthms_last_error(nullptr));
      jp->state = jp->cancel ? FTHMS_JOB_CANCELLED : rc ? FTHMS_JOB_FAILED : FTHMS_JOB_DONE;
      if (jp->cancel) std::vector<double2>().swap(jp->traces);
      sv->in_use -= jp->est;
    }
    sv->cv.notify_all();
  }
  if (ctx) fthms_destroy(ctx);
}

}  // namespace

extern "C" {

int fthms_server_create(int device, size_t hbm_budget, int workers, fthms_server **out) {
  if (!out || workers < 1 || workers > 64)
    return fail(nullptr, FTHMS_EINVAL, "workers must be in [1, 64]");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return fail(nullptr, FTHMS_EDEVICE, "no such HIP device");
  size_t freeb = 0, total = 0;
  if (hipSetDevice(device) != hipSuccess || hipMemGetInfo(&freeb, &total) != hipSuccess)
    return fail(nullptr, FTHMS_EDEVICE, "hipMemGetInfo failed");
  fthms_server *sv = new (std::nothrow) fthms_server;
  if (!sv) return fail(nullptr, FTHMS_ENOMEM, "host allocation failed");
  sv->device = device;
  sv->budget = hbm_budget ? hbm_budget : freeb / 10 * 9;
  // the workers allocate from the device's stream-ordered pool: keep freed
  // blocks in the pool for the next request instead of returning them at
  // every synchronisation
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess && pool) {
    uint64_t thr = (uint64_t)sv->budget;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  sv->nworkers = workers;
  for (int i = 0; i < workers; ++i) sv->workers.emplace_back(serve_worker, sv);
  *out = sv;
  return FTHMS_OK;
}

int fthms_server_destroy(fthms_server *sv) {
  if (!sv) return FTHMS_EINVAL;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    for (uint64_t id : sv->queue) sv->jobs[id].state = FTHMS_JOB_CANCELLED;
    sv->queue.clear();
  }
  sv->cv.notify_all();
  for (auto &t : sv->workers) t.join();
  delete sv;
  return FTHMS_OK;
}

const char *fthms_server_error(const fthms_server *sv) {
  if (!sv) return g_create_err.c_str();
  // a copy per calling thread: workers and other callers may replace sv->err
  static thread_local std::string copy;
  std::lock_guard<std::mutex> lk(const_cast<fthms_server *>(sv)->mu);
  copy = sv->err;
  return copy.c_str();
}

int fthms_submit(fthms_server *sv, const fthms_request *r, uint64_t *ticket) {
  if (!sv || !r || !ticket) return FTHMS_EINVAL;
  auto bad = [&](int code, const std::string &m) {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->err = m;
    return code;
  };
  if (r->narcs < 1 || r->n < 2 || r->n > kMaxN || !r->xy || !r->dxy ||
      (!r->closed && (!r->interval || !(r->period > 0.0))) ||
      (r->closed && (!r->ddxy || (r->n & 1))) || (r->closed != 0 && r->closed != 1) ||
      (r->precision != FTHMS_FP64 && r->precision != FTHMS_FP32_REFINED) || r->nk < 1 ||
      !r->k || !r->w || r->nobs < 1 || !r->obs_xy || r->nt < 1 || !r->t || r->max_steps < 1)
    return bad(FTHMS_EINVAL, "incomplete request");
  fthms_server::Job jb;
  jb.narcs = r->narcs;
  jb.n = r->n;
  jb.nk = r->nk;
  jb.nobs = r->nobs;
  jb.nt = r->nt;
  jb.max_steps = r->max_steps;
  jb.stop_tol = r->stop_tol;
  jb.closed = r->closed;
  jb.precision = r->precision;
  const size_t pts = (size_t)2 * r->n * r->narcs;
  jb.xy.assign(r->xy, r->xy + pts);
  jb.dxy.assign(r->dxy, r->dxy + pts);
  if (r->closed) {
    // every obstacle alone in its group; intervals are not used
    jb.ddxy.assign(r->ddxy, r->ddxy + pts);
    jb.period = 2.0 * kPi;
    jb.interval.resize(2 * (size_t)r->narcs);
    jb.group.resize(r->narcs);
    for (int j = 0; j < r->narcs; ++j) {
      jb.interval[2 * j] = 0.0;
      jb.interval[2 * j + 1] = 2.0 * kPi;
      jb.group[j] = j;
    }
  } else {
    jb.period = r->period;
    jb.interval.assign(r->interval, r->interval + 2 * (size_t)r->narcs);
    jb.group.assign(r->narcs, 0);
    if (r->group) jb.group.assign(r->group, r->group + r->narcs);
  }
  jb.k.assign(r->k, r->k + r->nk);
  jb.w.assign(r->w, r->w + r->nk);
  jb.obs.assign(r->obs_xy, r->obs_xy + 2 * (size_t)r->nobs);
  jb.t.assign(r->t, r->t + r->nt);
  jb.inc = r->incident;
  if (!finite_all(jb.xy.data(), jb.xy.size()) || !finite_all(jb.dxy.data(), jb.dxy.size()) ||
      !finite_all(jb.ddxy.data(), jb.ddxy.size()) || !finite_all(jb.k.data(), jb.k.size()) ||
      !finite_all(jb.w.data(), jb.w.size()) || !finite_all(jb.t.data(), jb.t.size()))
    return bad(FTHMS_EINVAL_DATA, "non-finite request data");
  for (double v : jb.k)
    if (!(v > 0.0)) return bad(FTHMS_EINVAL_DATA, "wavenumbers must be > 0");
  jb.est = request_bytes(r);
  if (jb.est > sv->budget)
    return bad(FTHMS_ENOMEM, "request needs ~" + std::to_string(jb.est >> 20) +
                                 " MiB, more than the server budget");
  jb.t_submit = std::chrono::steady_clock::now();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) {
      sv->err = "server is shutting down";
      return FTHMS_EINVAL;
    }
    *ticket = sv->next++;
    sv->jobs.emplace(*ticket, std::move(jb));
    sv->queue.push_back(*ticket);
  }
  sv->cv.notify_all();
  return FTHMS_OK;
}

int fthms_poll(fthms_server *sv, uint64_t ticket, int *state) {
  if (!sv || !state) return FTHMS_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->jobs.find(ticket);
  if (it == sv->jobs.end()) {
    sv->err = "unknown ticket";
    return FTHMS_EINVAL;
  }
  *state = it->second.state;
  return FTHMS_OK;
}

int fthms_fetch(fthms_server *sv, uint64_t ticket, fthms_c64 *traces, int *steps,
                double *latency_s) {
  if (!sv) return FTHMS_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->jobs.find(ticket);
  if (it == sv->jobs.end()) {
    sv->err = "unknown ticket";
    return FTHMS_EINVAL;
  }
  auto &jb = it->second;
  if (jb.state == FTHMS_JOB_QUEUED || jb.state == FTHMS_JOB_RUNNING) {
    sv->err = "request not finished";
    return FTHMS_EAGAIN;
  }
  int rc = FTHMS_OK;
  if (jb.state == FTHMS_JOB_DONE) {
    if (traces) std::memcpy(traces, jb.traces.data(), sizeof(double2) * jb.traces.size());
    if (steps) *steps = jb.steps;
    if (latency_s)
      *latency_s = std::chrono::duration<double>(jb.t_done - jb.t_submit).count();
  } else if (jb.state == FTHMS_JOB_FAILED) {
    sv->err = jb.err;
    rc = jb.rc;
  } else {
    sv->err = "request was cancelled";
    rc = FTHMS_ECANCELLED;
  }
  sv->jobs.erase(it);
  return rc;
}

int fthms_cancel(fthms_server *sv, uint64_t ticket) {
  if (!sv) return FTHMS_EINVAL;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(ticket);
    if (it == sv->jobs.end()) {
      sv->err = "unknown ticket";
      return FTHMS_EINVAL;
    }
    auto &jb = it->second;
    if (jb.state == FTHMS_JOB_QUEUED) {
      sv->queue.erase(std::find(sv->queue.begin(), sv->queue.end(), ticket));
      jb.state = FTHMS_JOB_CANCELLED;
    } else if (jb.state == FTHMS_JOB_RUNNING) {
      jb.cancel = true;  // the running request completes; its result is dropped
    }
  }
  sv->cv.notify_all();
  return FTHMS_OK;
}

}  // extern "C"
