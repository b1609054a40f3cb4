// libfthms: C-ABI entry points (declared in include/fthms.h) and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <functional>
#include <mutex>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "fthms.h"
#include "assemble.h"
#include "field.h"
#include "lu.h"
#include "nearfield.h"
#include "panel.h"
#include "panels.h"
#include "closed.h"
#include "gmres.h"
#include "hftransform.h"

using namespace fthms;

struct fthms_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // second stream (default priority) for the other half of a batched LU,
  // forked from and joined back into `stream` inside each call
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_lead = nullptr, ev_join = nullptr;
  // per-step events and a small pinned host buffer (device-decided stop rule)
  hipEvent_t ev_step[2] = {nullptr, nullptr};
  int *pinned = nullptr;
  size_t budget = 0;
  size_t held = 0;
  // serving workers allocate stream-ordered (hipMallocAsync / hipFreeAsync),
  // so that one request's frees do not wait for the other workers' kernels
  bool async_alloc = false;
  std::string err;
  // solve workspace and a second scratch area (both grown on demand)
  void *ws = nullptr;
  size_t ws_bytes = 0;
  void *ws2 = nullptr;
  // partial sums of the split frequency-to-time transform (optional)
  void *ft = nullptr;
  size_t ft_bytes = 0;
  size_t ws2_bytes = 0;
  // kernel timing with HIP events on `stream` (off while a graph is captured)
  bool timing = false;
  bool capturing = false;
  struct Pending {
    std::string name;
    hipEvent_t a, b;
    hipStream_t st;
  };
  std::vector<Pending> pending;
  std::vector<size_t> open;  // indices into `pending` of unfinished ranges
  std::map<std::string, std::pair<double, int>> times;
};

// An arc: one weighted Chebyshev panel (npan = 1, nper = n), or a
// composite-panel arc (npan panels of nper nodes, per-node weights w / d_w).
// theta: node angles within the panel; t: arc parameter of each node; s:
// speed |dx/dt| (one panel) or |dx/ds| (panels); cgx, cgy: Chebyshev
// coefficients of the geometry, [npan][nper].
struct fthms_arc {
  fthms_ctx *ctx = nullptr;
  int n = 0;
  int npan = 1, nper = 0;
  std::vector<double> theta, t, xy, dxy, s;
  std::vector<double> cgx, cgy;
  std::vector<double> breaks, w;
  std::vector<int> kinds;
  double hmax = 0.0;
  double2 *d_y = nullptr;
  // [2][n][n]: the frequency-independent log table G of the assembly, then
  // Gl = G + c_j log r_ij off the diagonal (c_j = 1/(2n); w_j/(2 pi) on
  // composite panels), the table of the large-argument form (assemble.h)
  double *d_G = nullptr;
  double *d_cos = nullptr;  // [nper][nper] cos(m theta_j), row j
  double *d_w = nullptr;    // composite-panel arcs: Fejer weights
  // closed patches (combined-field equation): tangents, log-quadrature
  // weights R_d and log(4 sin^2(pi d / N)), diagonal of K2
  bool closed = false;
  double2 *d_dy = nullptr;
  double *d_R = nullptr, *d_L = nullptr, *d_kd = nullptr;
  size_t bytes = 0;
};

static thread_local std::string g_create_err;

// G followed by Gl = G + c_j log r_ij (i != j) for an arc with nodes xy[n][2]:
// c_j = 1/(2n) on a single-panel arc, w_j/(2 pi) with column weights w.
static std::vector<double> with_log_shift(const std::vector<double> &G, const double *xy, int n,
                                          const double *w) {
  const size_t nn = (size_t)n * n;
  std::vector<double> out(2 * nn);
  std::copy(G.begin(), G.end(), out.begin());
  for (int j = 0; j < n; ++j) {
    const double c = w ? w[j] / (2.0 * kPi) : 0.5 / n;
    for (int i = 0; i < n; ++i) {
      const size_t e = (size_t)i + (size_t)j * n;
      double v = G[e];
      if (i != j) {
        const double dx = xy[2 * i] - xy[2 * j], dy = xy[2 * i + 1] - xy[2 * j + 1];
        v += c * std::log(std::sqrt(dx * dx + dy * dy));
      }
      out[nn + e] = v;
    }
  }
  return out;
}

// ---- fixed device scratch for the allocation-free entry point ------------
// The gather permutations of fthms_lu_solve_noalloc_dev live in this array:
// kNoAllocMatrices slots of kMaxN ints (16 MiB), one copy per device for the
// life of the process.  Host code never uses the array's name as an address:
// fthms_create looks up each device's copy with hipGetSymbolAddress (with
// that device current) and keeps the pointer in g_scratch_ptr.
constexpr int kNoAllocMatrices = 4096;
constexpr int kMaxDevices = 64;
__device__ __align__(256) int scratch[(size_t)kNoAllocMatrices * kMaxN];
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

static int fail(fthms_ctx *ctx, int code, const std::string &msg) {
  if (ctx) ctx->err = msg;
  else g_create_err = msg;
  return code;
}

#define HIPCK(ctx, call)                                                         \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess)                                                       \
      return fail((ctx), FTHMS_EDEVICE,                                          \
                  std::string(#call) + ": " + hipGetErrorString(e_));            \
  } while (0)

static int dev_alloc(fthms_ctx *ctx, void **p, size_t bytes) {
  if (ctx->budget && ctx->held + bytes > ctx->budget)
    return fail(ctx, FTHMS_ENOMEM,
                "device memory budget exceeded (" + std::to_string(ctx->held + bytes) +
                    " > " + std::to_string(ctx->budget) + " bytes)");
  if (ctx->async_alloc) {
    // stream-ordered: no device-wide synchronisation; the memory is ready
    // once this context's stream has reached the allocation
    HIPCK(ctx, hipMallocAsync(p, bytes ? bytes : 1, ctx->stream));
    HIPCK(ctx, hipStreamSynchronize(ctx->stream));
  } else {
    HIPCK(ctx, hipMalloc(p, bytes ? bytes : 1));
  }
  ctx->held += bytes;
  return FTHMS_OK;
}

static void dev_free(fthms_ctx *ctx, void *p, size_t bytes) {
  if (p) {
    if (ctx->async_alloc) (void)hipFreeAsync(p, ctx->stream);
    else (void)hipFree(p);
    ctx->held -= std::min(ctx->held, bytes);
  }
}

static int ensure_ws(fthms_ctx *ctx, size_t bytes) {
  if (ctx->ws_bytes >= bytes) return FTHMS_OK;
  (void)hipStreamSynchronize(ctx->stream);
  dev_free(ctx, ctx->ws, ctx->ws_bytes);
  ctx->ws = nullptr;
  ctx->ws_bytes = 0;
  int rc = dev_alloc(ctx, &ctx->ws, bytes);
  if (rc) return rc;
  ctx->ws_bytes = bytes;
  return FTHMS_OK;
}

// The context's pinned host buffer (16 ints, allocated on first use).
static int ctx_pinned(fthms_ctx *ctx, int **out) {
  if (!ctx->pinned) HIPCK(ctx, hipHostMalloc((void **)&ctx->pinned, 16 * sizeof(int)));
  *out = ctx->pinned;
  return FTHMS_OK;
}

static int ensure_ws2(fthms_ctx *ctx, size_t bytes) {
  if (ctx->ws2_bytes >= bytes) return FTHMS_OK;
  (void)hipStreamSynchronize(ctx->stream);
  dev_free(ctx, ctx->ws2, ctx->ws2_bytes);
  ctx->ws2 = nullptr;
  ctx->ws2_bytes = 0;
  int rc = dev_alloc(ctx, &ctx->ws2, bytes);
  if (rc) return rc;
  ctx->ws2_bytes = bytes;
  return FTHMS_OK;
}

// Scratch for the split transform if it can be had (budget, memory);
// false leaves the transform unsplit, and no error is recorded.
static bool try_ft_scratch(fthms_ctx *ctx, size_t bytes) {
  if (ctx->ft_bytes >= bytes) return true;
  if (ctx->budget && ctx->held - std::min(ctx->held, ctx->ft_bytes) + bytes > ctx->budget)
    return false;
  (void)hipStreamSynchronize(ctx->stream);
  dev_free(ctx, ctx->ft, ctx->ft_bytes);
  ctx->ft = nullptr;
  ctx->ft_bytes = 0;
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  ctx->ft = p;
  ctx->ft_bytes = bytes;
  ctx->held += bytes;
  return true;
}

static void tbeg(fthms_ctx *ctx, const char *name, hipStream_t st = nullptr) {
  if (!ctx->timing || ctx->capturing) return;
  if (!st) st = ctx->stream;
  fthms_ctx::Pending p;
  p.name = name;
  if (hipEventCreate(&p.a) != hipSuccess) {
    ctx->open.push_back(SIZE_MAX);  // keeps tbeg/tend paired
    return;
  }
  if (hipEventCreate(&p.b) != hipSuccess) {
    (void)hipEventDestroy(p.a);
    ctx->open.push_back(SIZE_MAX);
    return;
  }
  (void)hipEventRecord(p.a, st);
  p.st = st;
  ctx->open.push_back(ctx->pending.size());
  ctx->pending.push_back(p);
}

// closes the innermost range opened by tbeg (ranges nest)
static void tend(fthms_ctx *ctx) {
  if (!ctx->timing || ctx->capturing || ctx->open.empty()) return;
  const size_t i = ctx->open.back();
  ctx->open.pop_back();
  if (i != SIZE_MAX) (void)hipEventRecord(ctx->pending[i].b, ctx->pending[i].st);
}

static void timing_collect(fthms_ctx *ctx) {
  if (ctx->pending.empty()) return;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto &p : ctx->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      auto &t = ctx->times[p.name];
      t.first += ms;
      t.second += 1;
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  ctx->pending.clear();
}

static int check_launch(fthms_ctx *ctx, const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(ctx, FTHMS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return FTHMS_OK;
}

extern "C" {

int fthms_abi_version(void) { return FTHMS_ABI_VERSION; }

int fthms_create(fthms_ctx **out, int device, size_t hbm_budget_bytes, void *hip_stream) {
  if (!out) return fail(nullptr, FTHMS_EINVAL, "out is NULL");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
    return fail(nullptr, FTHMS_EDEVICE, "no HIP device available");
  if (device < 0 || device >= count)
    return fail(nullptr, FTHMS_EINVAL, "device index out of range");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess)
    return fail(nullptr, FTHMS_EDEVICE, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, FTHMS_EDEVICE,
                std::string("libfthms is built for gfx950, device is ") + prop.gcnArchName);
  fthms_ctx *ctx = new (std::nothrow) fthms_ctx;
  if (!ctx) return fail(nullptr, FTHMS_ENOMEM, "host allocation failed");
  ctx->device = device;
  ctx->budget = hbm_budget_bytes;
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return fail(nullptr, FTHMS_EDEVICE, "hipSetDevice failed");
  }
  if (device >= kMaxDevices) {
    delete ctx;
    return fail(nullptr, FTHMS_EINVAL, "device index beyond the library's device table");
  }
  {
    // this device's copy of the fixed scratch array, looked up once
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
      void *p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        delete ctx;
        return fail(nullptr, FTHMS_EDEVICE,
                    std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      }
      g_scratch_ptr[device] = p;
    }
  }
  if (hip_stream != FTHMS_OWN_STREAM) {
    ctx->stream = (hipStream_t)hip_stream;  // NULL: the null stream
  } else {
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
      delete ctx;
      return fail(nullptr, FTHMS_EDEVICE, "hipStreamCreate failed");
    }
    ctx->own_stream = true;
  }
  if (hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_lead, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_step[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_step[1], hipEventDisableTiming) != hipSuccess) {
    fthms_destroy(ctx);
    return fail(nullptr, FTHMS_EDEVICE, "hipStreamCreate/hipEventCreate failed");
  }
  *out = ctx;
  return FTHMS_OK;
}

int fthms_destroy(fthms_ctx *ctx) {
  if (!ctx) return FTHMS_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  timing_collect(ctx);
  dev_free(ctx, ctx->ws, ctx->ws_bytes);
  dev_free(ctx, ctx->ws2, ctx->ws2_bytes);
  dev_free(ctx, ctx->ft, ctx->ft_bytes);
  if (ctx->aux) {
    (void)hipStreamSynchronize(ctx->aux);
    (void)hipStreamDestroy(ctx->aux);
  }
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_lead) (void)hipEventDestroy(ctx->ev_lead);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  for (auto &e : ctx->ev_step)
    if (e) (void)hipEventDestroy(e);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return FTHMS_OK;
}

const char *fthms_last_error(const fthms_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

int fthms_sync(fthms_ctx *ctx) {
  if (!ctx) return FTHMS_EINVAL;
  HIPCK(ctx, hipStreamSynchronize(ctx->stream));
  return FTHMS_OK;
}

int fthms_timing_enable(fthms_ctx *ctx, int enable) {
  if (!ctx) return FTHMS_EINVAL;
  timing_collect(ctx);
  ctx->timing = enable != 0;
  return FTHMS_OK;
}

int fthms_timing_reset(fthms_ctx *ctx) {
  if (!ctx) return FTHMS_EINVAL;
  timing_collect(ctx);
  ctx->times.clear();
  return FTHMS_OK;
}

int fthms_timing_read(fthms_ctx *ctx, const char *name, double *total_ms, int *launches) {
  if (!ctx || !name) return FTHMS_EINVAL;
  timing_collect(ctx);
  auto it = ctx->times.find(name);
  if (total_ms) *total_ms = it == ctx->times.end() ? 0.0 : it->second.first;
  if (launches) *launches = it == ctx->times.end() ? 0 : it->second.second;
  return FTHMS_OK;
}

int fthms_cheb_nodes(int n, double *t_out) {
  if (n < 2 || !t_out) return FTHMS_EINVAL;
  for (int i = 1; i <= n; ++i) t_out[i - 1] = std::cos((2.0 * i - 1.0) * kPi / (2.0 * n));
  return FTHMS_OK;
}

// ---------------------------------------------------------------------------
// arcs: frequency-independent tables
// ---------------------------------------------------------------------------
int fthms_arc_create(fthms_ctx *ctx, int n, const double *xy, const double *dxy,
                     fthms_arc **out) {
  if (!ctx || !xy || !dxy || !out) return fail(ctx, FTHMS_EINVAL, "NULL argument");
  *out = nullptr;
  if (n < 2 || n > kMaxN) return fail(ctx, FTHMS_EINVAL, "arc size must be in [2, 1024]");
  for (int i = 0; i < 2 * n; ++i)
    if (!std::isfinite(xy[i]) || !std::isfinite(dxy[i]))
      return fail(ctx, FTHMS_EINVAL_DATA, "non-finite arc sample");
  fthms_arc *arc = new (std::nothrow) fthms_arc;
  if (!arc) return fail(ctx, FTHMS_ENOMEM, "host allocation failed");
  arc->ctx = ctx;
  arc->n = n;
  arc->nper = n;
  arc->theta.resize(n);
  arc->t.resize(n);
  arc->s.resize(n);
  arc->xy.assign(xy, xy + 2 * n);
  arc->dxy.assign(dxy, dxy + 2 * n);
  for (int i = 0; i < n; ++i) {
    arc->theta[i] = (2.0 * (i + 1) - 1.0) * kPi / (2.0 * n);
    arc->t[i] = std::cos(arc->theta[i]);
    arc->s[i] = std::hypot(dxy[2 * i], dxy[2 * i + 1]);
    if (!(arc->s[i] > 0.0)) {
      delete arc;
      return fail(ctx, FTHMS_EINVAL_DATA, "vanishing speed |x'(t)| at a node");
    }
  }
  double hmax = 0.0;
  for (int i = 0; i + 1 < n; ++i) {
    const double h = std::hypot(xy[2 * i + 2] - xy[2 * i], xy[2 * i + 3] - xy[2 * i + 1]);
    if (!(h > 0.0)) {
      delete arc;
      return fail(ctx, FTHMS_EINVAL_DATA, "coincident consecutive nodes");
    }
    hmax = std::max(hmax, h);
  }
  arc->hmax = hmax;
  // S(q pi / n) = sum_{m=1}^{n-1} cos(m q pi / n) / m, q = 0..2n-1, from an
  // exact-index cosine table; W_ij = -(pi/n)[log 2 + S(i-j) + S(i+j-1)]
  // (product-to-sum form of the Symm-identity weights).
  std::vector<double> ct(2 * n), S(2 * n, 0.0);
  for (int r = 0; r < 2 * n; ++r) ct[r] = std::cos(r * kPi / n);
  for (int q = 0; q < 2 * n; ++q) {
    double acc = 0.0;
    for (int m = n - 1; m >= 1; --m) acc += ct[(long long)m * q % (2 * n)] / m;
    S[q] = acc;
  }
  std::vector<double> G((size_t)n * n);
  const double ln2 = std::log(2.0);
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i) {
      const int qm = std::abs(i - j), qp = (i + 1) + (j + 1) - 1;
      const double W = -(kPi / n) * (ln2 + S[qm % (2 * n)] + S[qp % (2 * n)]);
      double g;
      if (i == j) {
        g = (-W - (kPi / n) * std::log(arc->s[i])) / (2.0 * kPi);
      } else {
        const double r = std::hypot(xy[2 * i] - xy[2 * j], xy[2 * i + 1] - xy[2 * j + 1]);
        if (!(r > 0.0)) {
          delete arc;
          return fail(ctx, FTHMS_EINVAL_DATA, "coincident nodes");
        }
        // |t_i - t_j| = 2 |sin((th_i + th_j)/2) sin((th_i - th_j)/2)|
        const double dt = 2.0 * std::fabs(std::sin(0.5 * (arc->theta[i] + arc->theta[j])) *
                                          std::sin(0.5 * (arc->theta[i] - arc->theta[j])));
        g = (-W - (kPi / n) * std::log(r / dt)) / (2.0 * kPi);
      }
      G[(size_t)i + (size_t)j * n] = g;
    }
  }
  // Chebyshev coefficients of the geometry (for near-field planning)
  arc->cgx.assign(n, 0.0);
  arc->cgy.assign(n, 0.0);
  for (int m = 0; m < n; ++m) {
    double ax = 0.0, ay = 0.0;
    for (int j = 0; j < n; ++j) {
      const double cc = std::cos(m * arc->theta[j]);
      ax += xy[2 * j] * cc;
      ay += xy[2 * j + 1] * cc;
    }
    const double f = (m == 0 ? 1.0 : 2.0) / n;
    arc->cgx[m] = f * ax;
    arc->cgy[m] = f * ay;
  }
  std::vector<double> cosT((size_t)n * n);  // [j][m] = cos(m theta_j)
  for (int j = 0; j < n; ++j)
    for (int m = 0; m < n; ++m) cosT[(size_t)j * n + m] = std::cos(m * arc->theta[j]);
  int rc;
  arc->bytes = sizeof(double2) * n + sizeof(double) * (size_t)n * n * 3;
  if ((rc = dev_alloc(ctx, (void **)&arc->d_y, sizeof(double2) * n)) ||
      (rc = dev_alloc(ctx, (void **)&arc->d_G, sizeof(double) * (size_t)n * n * 2)) ||
      (rc = dev_alloc(ctx, (void **)&arc->d_cos, sizeof(double) * (size_t)n * n))) {
    fthms_arc_destroy(arc);
    return rc;
  }
  const std::vector<double> G2 = with_log_shift(G, xy, n, nullptr);
  HIPCK(ctx, hipMemcpy(arc->d_y, xy, sizeof(double2) * n, hipMemcpyHostToDevice));
  HIPCK(ctx, hipMemcpy(arc->d_G, G2.data(), sizeof(double) * G2.size(), hipMemcpyHostToDevice));
  HIPCK(ctx, hipMemcpy(arc->d_cos, cosT.data(), sizeof(double) * (size_t)n * n,
                       hipMemcpyHostToDevice));
  *out = arc;
  return FTHMS_OK;
}

static bool panel_layout_ok(int npan, const double *breaks, const int *kinds, int n_per) {
  if (npan < 1 || npan > kMaxPanels || !breaks || !kinds || n_per < 2 ||
      (long long)npan * n_per > kMaxN)
    return false;
  if (breaks[0] != -1.0 || breaks[npan] != 1.0) return false;
  for (int p = 0; p < npan; ++p) {
    if (!(breaks[p + 1] > breaks[p])) return false;
    if (kinds[p] < kCovNone || kinds[p] > kCovRight) return false;
  }
  return true;
}

// arc parameter of node i of panel p: t_p + (t_{p+1} - t_p)(1 + theta(s_i))/2
static void panel_node_params(int npan, const double *breaks, const int *kinds, int n,
                              double *t, double *dtds) {
  for (int p = 0; p < npan; ++p)
    for (int i = 0; i < n; ++i) {
      const double si = std::cos((2.0 * i + 1.0) * kPi / (2.0 * n));
      double th, dth;
      cov_map(kinds[p], si, th, dth);
      const double h = 0.5 * (breaks[p + 1] - breaks[p]);
      t[p * n + i] = breaks[p] + h * (1.0 + th);
      if (dtds) dtds[p * n + i] = h * dth;
    }
}

int fthms_panel_nodes(int npan, const double *breaks, const int *kinds, int n_per,
                      double *t_out) {
  if (!t_out || !panel_layout_ok(npan, breaks, kinds, n_per)) return FTHMS_EINVAL;
  panel_node_params(npan, breaks, kinds, n_per, t_out, nullptr);
  return FTHMS_OK;
}

int fthms_arc_create_panels(fthms_ctx *ctx, int npan, const double *breaks, const int *kinds,
                            int n_per, const double *xy, const double *dxy, fthms_arc **out) {
  if (!ctx || !xy || !dxy || !out) return fail(ctx, FTHMS_EINVAL, "NULL argument");
  *out = nullptr;
  if (!panel_layout_ok(npan, breaks, kinds, n_per))
    return fail(ctx, FTHMS_EINVAL,
                "panels: need 1..16 panels, breaks -1 = t_0 < ... < t_P = 1, kinds 0..3, "
                "2 <= n_per and npan * n_per <= 1024");
  const int n = npan * n_per;
  for (int i = 0; i < 2 * n; ++i)
    if (!std::isfinite(xy[i]) || !std::isfinite(dxy[i]))
      return fail(ctx, FTHMS_EINVAL_DATA, "non-finite arc sample");
  fthms_arc *arc = new (std::nothrow) fthms_arc;
  if (!arc) return fail(ctx, FTHMS_ENOMEM, "host allocation failed");
  arc->ctx = ctx;
  arc->n = n;
  arc->npan = npan;
  arc->nper = n_per;
  arc->breaks.assign(breaks, breaks + npan + 1);
  arc->kinds.assign(kinds, kinds + npan);
  arc->xy.assign(xy, xy + 2 * n);
  arc->dxy.assign(dxy, dxy + 2 * n);
  arc->theta.resize(n);
  arc->t.resize(n);
  arc->s.resize(n);
  std::vector<double> dtds(n), w1;
  panel_node_params(npan, breaks, kinds, n_per, arc->t.data(), dtds.data());
  fejer_weights(n_per, w1);
  arc->w.resize(n);
  for (int i = 0; i < n; ++i) {
    arc->theta[i] = (2.0 * (i % n_per) + 1.0) * kPi / (2.0 * n_per);
    arc->s[i] = std::hypot(dxy[2 * i], dxy[2 * i + 1]) * std::fabs(dtds[i]);
    arc->w[i] = w1[i % n_per];
    if (!(std::hypot(dxy[2 * i], dxy[2 * i + 1]) > 0.0)) {
      delete arc;
      return fail(ctx, FTHMS_EINVAL_DATA, "vanishing speed |x'(t)| at a node");
    }
  }
  // largest distance between nodes adjacent along the arc (order of t)
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return arc->t[a] < arc->t[b]; });
  double hmax = 0.0;
  for (int q = 0; q + 1 < n; ++q) {
    const int i = ord[q], j = ord[q + 1];
    const double h = std::hypot(xy[2 * j] - xy[2 * i], xy[2 * j + 1] - xy[2 * i + 1]);
    if (!(h > 0.0)) {
      delete arc;
      return fail(ctx, FTHMS_EINVAL_DATA, "coincident nodes");
    }
    hmax = std::max(hmax, h);
  }
  arc->hmax = hmax;
  // per-panel Chebyshev coefficients of the geometry in s
  const PanelGeom geom = panel_geom_from_samples(npan, n_per, xy, dxy, breaks, kinds);
  arc->cgx = geom.cx;
  arc->cgy = geom.cy;
  std::vector<double> G;
  panel_log_table(geom, arc->xy, G);
  for (double g : G)
    if (!std::isfinite(g)) {
      delete arc;
      return fail(ctx, FTHMS_EINVAL_DATA, "log table: non-finite entry (degenerate geometry)");
    }
  std::vector<double> cosT((size_t)n_per * n_per);
  for (int j = 0; j < n_per; ++j)
    for (int m = 0; m < n_per; ++m) cosT[(size_t)j * n_per + m] = std::cos(m * arc->theta[j]);
  int rc;
  arc->bytes =
      sizeof(double2) * n + sizeof(double) * (2 * (size_t)n * n + (size_t)n_per * n_per + n);
  const std::vector<double> G2 = with_log_shift(G, arc->xy.data(), n, arc->w.data());
  if ((rc = dev_alloc(ctx, (void **)&arc->d_y, sizeof(double2) * n)) ||
      (rc = dev_alloc(ctx, (void **)&arc->d_G, sizeof(double) * G2.size())) ||
      (rc = dev_alloc(ctx, (void **)&arc->d_cos, sizeof(double) * (size_t)n_per * n_per)) ||
      (rc = dev_alloc(ctx, (void **)&arc->d_w, sizeof(double) * n))) {
    fthms_arc_destroy(arc);
    return rc;
  }
  if (hipMemcpy(arc->d_y, xy, sizeof(double2) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(arc->d_G, G2.data(), sizeof(double) * G2.size(), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(arc->d_cos, cosT.data(), sizeof(double) * (size_t)n_per * n_per,
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(arc->d_w, arc->w.data(), sizeof(double) * n, hipMemcpyHostToDevice) !=
          hipSuccess) {
    fthms_arc_destroy(arc);
    return fail(ctx, FTHMS_EDEVICE, "hipMemcpy of the arc tables failed");
  }
  *out = arc;
  return FTHMS_OK;
}

int fthms_tov_breaks(int narcs, const double *interval, const int *group, double period,
                     double *breaks, int *npan) {
  if (narcs < 1 || !interval || !(period > 0.0) || !breaks || !npan) return FTHMS_EINVAL;
  for (int j = 0; j < narcs; ++j) {
    if (!(interval[2 * j + 1] > interval[2 * j])) return FTHMS_EINVAL;
    // cyclic neighbours within the arc's group, in list order
    const int gj = group ? group[j] : 0;
    std::vector<int> mem;
    for (int i = 0; i < narcs; ++i)
      if ((group ? group[i] : 0) == gj) mem.push_back(i);
    std::vector<double> br = {-1.0, 1.0};
    if (mem.size() > 1) {
      const int q = (int)(std::find(mem.begin(), mem.end(), j) - mem.begin());
      const int m = (int)mem.size();
      const int prv = mem[(q + m - 1) % m], nxt = mem[(q + 1) % m];
      const double a = interval[2 * j], b = interval[2 * j + 1];
      // the truncated overlap ends where the previous arc ends and the next begins
      for (double e : {interval[2 * prv + 1], interval[2 * nxt]}) {
        double u = std::fmod(e - a, period);
        if (u < 0.0) u += period;
        if (u > 0.0 && u < b - a) br.push_back(-1.0 + 2.0 * u / (b - a));
      }
    }
    std::sort(br.begin(), br.end());
    npan[j] = (int)br.size() - 1;
    for (int e = 0; e < 4; ++e) breaks[4 * j + e] = e < (int)br.size() ? br[e] : 1.0;
  }
  return FTHMS_OK;
}

int fthms_arc_panel_table(const fthms_arc *arc, double *W, double *w) {
  if (!arc || !arc->d_w) return FTHMS_EINVAL;
  fthms_ctx *ctx = arc->ctx;
  const int n = arc->n;
  if (W) {
    std::vector<double> G((size_t)n * n);
    HIPCK(ctx, hipMemcpy(G.data(), arc->d_G, sizeof(double) * G.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) W[(size_t)i * n + j] = -2.0 * kPi * G[(size_t)i + (size_t)j * n];
  }
  if (w) std::memcpy(w, arc->w.data(), sizeof(double) * n);
  return FTHMS_OK;
}

int fthms_closed_create(fthms_ctx *ctx, int n, const double *xy, const double *dxy,
                        const double *ddxy, fthms_arc **out) {
  if (!ctx || !xy || !dxy || !ddxy || !out) return fail(ctx, FTHMS_EINVAL, "NULL argument");
  *out = nullptr;
  if (n < 4 || n > kMaxN || (n & 1))
    return fail(ctx, FTHMS_EINVAL, "closed patch: node count must be even, in [4, 1024]");
  for (int i = 0; i < 2 * n; ++i)
    if (!std::isfinite(xy[i]) || !std::isfinite(dxy[i]) || !std::isfinite(ddxy[i]))
      return fail(ctx, FTHMS_EINVAL_DATA, "non-finite closed-curve sample");
  fthms_arc *arc = new (std::nothrow) fthms_arc;
  if (!arc) return fail(ctx, FTHMS_ENOMEM, "host allocation failed");
  arc->ctx = ctx;
  arc->n = n;
  arc->nper = n;
  arc->closed = true;
  arc->xy.assign(xy, xy + 2 * n);
  arc->dxy.assign(dxy, dxy + 2 * n);
  arc->theta.resize(n);
  arc->t.resize(n);
  arc->s.resize(n);
  std::vector<double> kd(n), R(n), L(n, 0.0);
  double hmax = 0.0;
  for (int i = 0; i < n; ++i) {
    arc->theta[i] = 2.0 * kPi * i / n;
    arc->t[i] = -1.0 + (2.0 * i + 1.0) / n;  // parameter position, for bookkeeping only
    const double d1 = dxy[2 * i], d2 = dxy[2 * i + 1];
    const double s2 = d1 * d1 + d2 * d2;
    arc->s[i] = std::sqrt(s2);
    if (!(s2 > 0.0)) {
      delete arc;
      return fail(ctx, FTHMS_EINVAL_DATA, "vanishing speed |x'| at a node");
    }
    kd[i] = (d2 * ddxy[2 * i] - d1 * ddxy[2 * i + 1]) / (4.0 * kPi * s2);
    const int nx = (i + 1) % n;
    const double h = std::hypot(xy[2 * nx] - xy[2 * i], xy[2 * nx + 1] - xy[2 * i + 1]);
    if (!(h > 0.0)) {
      delete arc;
      return fail(ctx, FTHMS_EINVAL_DATA, "coincident consecutive nodes");
    }
    hmax = std::max(hmax, h);
  }
  arc->hmax = hmax;
  // R_d = -(2pi/m) sum_{l=1}^{m-1} cos(l d pi/m)/l - (pi/m^2) cos(d pi), m = n/2
  const int m = n / 2;
  for (int d = 0; d < n; ++d) {
    double acc = 0.0;
    for (int l = m - 1; l >= 1; --l) acc += std::cos(kPi * (double)((long long)l * d % n) / m) / l;
    R[d] = -(2.0 * kPi / m) * acc - (kPi / ((double)m * m)) * ((d & 1) ? -1.0 : 1.0);
    if (d) L[d] = std::log(4.0 * std::pow(std::sin(kPi * d / n), 2));
  }
  int rc;
  arc->bytes = sizeof(double2) * 2 * n + sizeof(double) * 3 * n;
  if ((rc = dev_alloc(ctx, (void **)&arc->d_y, sizeof(double2) * n)) ||
      (rc = dev_alloc(ctx, (void **)&arc->d_dy, sizeof(double2) * n)) ||
      (rc = dev_alloc(ctx, (void **)&arc->d_R, sizeof(double) * n)) ||
      (rc = dev_alloc(ctx, (void **)&arc->d_L, sizeof(double) * n)) ||
      (rc = dev_alloc(ctx, (void **)&arc->d_kd, sizeof(double) * n))) {
    fthms_arc_destroy(arc);
    return rc;
  }
  if (hipMemcpy(arc->d_y, xy, sizeof(double2) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(arc->d_dy, dxy, sizeof(double2) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(arc->d_R, R.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(arc->d_L, L.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(arc->d_kd, kd.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess) {
    fthms_arc_destroy(arc);
    return fail(ctx, FTHMS_EDEVICE, "hipMemcpy of the closed-patch tables failed");
  }
  *out = arc;
  return FTHMS_OK;
}

int fthms_arc_destroy(fthms_arc *arc) {
  if (!arc) return FTHMS_EINVAL;
  fthms_ctx *ctx = arc->ctx;
  if (ctx) {
    dev_free(ctx, arc->d_y, sizeof(double2) * arc->n);
    dev_free(ctx, arc->d_G, sizeof(double) * (size_t)arc->n * arc->n * 2);
    dev_free(ctx, arc->d_cos, sizeof(double) * (size_t)arc->nper * arc->nper);
    dev_free(ctx, arc->d_w, sizeof(double) * arc->n);
    dev_free(ctx, arc->d_dy, sizeof(double2) * arc->n);
    dev_free(ctx, arc->d_R, sizeof(double) * arc->n);
    dev_free(ctx, arc->d_L, sizeof(double) * arc->n);
    dev_free(ctx, arc->d_kd, sizeof(double) * arc->n);
  }
  delete arc;
  return FTHMS_OK;
}

int fthms_arc_size(const fthms_arc *arc) { return arc ? arc->n : FTHMS_EINVAL; }

}  // extern "C"

// ---------------------------------------------------------------------------
// batched solve
// ---------------------------------------------------------------------------
// Blocked LU of `count` matrices: per block of 64 columns one panel launch
// (one workgroup per matrix) and one strip launch (XCD-aware, one workgroup
// per 64-column strip per matrix).  only_failed: factor only the matrices
// whose status is negative (the FP64 redo of refined solves).
// Per-matrix LU scratch: the block row permutation and the inverse of the
// block's unit-lower diagonal part (sized for complex128).
// Regions, each `count` matrices long: [block permutation pairs][L11^{-1}]
// [row permutation of the finished factorisation (kMaxN ints)].
constexpr size_t kLuScratchHead = sizeof(int) * kSwapStride + sizeof(double2) * kLuNB * kLuNB;
constexpr size_t kLuScratchBytes = kLuScratchHead + sizeof(int) * kMaxN;

// Gather form of the factorisation's row interchanges in LU scratch `scr`
// of `count` matrices.
static int *lu_perm(void *scr, int count) {
  return (int *)((char *)scr + kLuScratchHead * (size_t)count);
}

static void launch_perm(hipStream_t st, const int *piv, int N, int *perm, const int *status,
                        int count, int only_failed) {
  const int S = (N + 63) / 64;
  if (S <= 1)
    perm_from_piv_kernel<1><<<count, 64, 0, st>>>(piv, N, perm, status, only_failed);
  else if (S <= 2)
    perm_from_piv_kernel<2><<<count, 64, 0, st>>>(piv, N, perm, status, only_failed);
  else if (S <= 4)
    perm_from_piv_kernel<4><<<count, 64, 0, st>>>(piv, N, perm, status, only_failed);
  else if (S <= 8)
    perm_from_piv_kernel<8><<<count, 64, 0, st>>>(piv, N, perm, status, only_failed);
  else
    perm_from_piv_kernel<16><<<count, 64, 0, st>>>(piv, N, perm, status, only_failed);
}

// Launch choices of the batched LU (the batch autotuner picks them per
// matrix size; every other caller uses the defaults).
struct LuOpts {
  bool split = true;      // two half batches on two streams (large batches)
  bool reg_panel = true;  // register-resident panel where the block fits
  // complex symmetric matrices: the symmetric form (no row interchanges,
  // checked against partial pivoting; lu.h), FP32 with N <= 512 only -- the
  // refined solve redoes a flagged matrix in FP64 from its FP64 copy
  bool sym = false;
  // FP32 only: trailing-update products on the FP16 matrix cores (the
  // low-precision factorisation of GMRES-IR)
  bool h16 = false;
};

// The symmetric form applies: FP32 factors (an FP64 copy stays for the
// redo) and every block within the register panel.  FTHMS_LU_SYM=0 in the
// environment turns it off (every matrix then takes the pivoting form).
static bool lu_sym_fits(bool fp32, int N) {
  static const bool allowed = [] {
    const char *e = getenv("FTHMS_LU_SYM");
    return !(e && e[0] == '0' && e[1] == '\0');
  }();
  return allowed && fp32 && N <= 512;
}

// Arc matrices that are complex symmetric: the single-panel scheme's
// (A_ij = A_ji exactly, the assembly writes each pair once and mirrors it);
// composite-panel and closed-patch matrices are not.
static bool arc_symmetric(const fthms_arc *arc) { return !arc->closed && !arc->d_w; }

// Refined solves of a symmetric arc's matrices take the symmetric form
// throughout: the lower block triangle assembled, the symmetric LU, the
// symmetric residual in the refinement (and the upper part completed before
// an FP64 redo).  One predicate for all of them.
static bool use_sym_form(bool fp32, const fthms_arc *arc) {
  return fp32 && arc_symmetric(arc) && lu_sym_fits(true, arc->n);
}

// Panel of the block at k0: register-resident kernel when the block fits
// (m = N - k0 <= 512 in FP32, <= 320 in FP64), else the LDS/global kernel.
// Symmetric form (FP32, m <= 512): the register panel without row interchanges.
// FTHMS_SYM_PANEL=reg in the environment selects the one-launch register
// panel over the whole column block for the symmetric form (a comparison
// switch); by default the diagonal block and the rows below it take a
// launch each.
static bool sym_panel_split() {
  static const bool split = [] {
    const char *e = getenv("FTHMS_SYM_PANEL");
    return !(e && std::string(e) == "reg");
  }();
  return split;
}

// The diagonal blocks of the two-launch form: one wave per matrix
// (lu_diag_sym_kernel) for launches of kDiagWaveMin matrices or more, the
// 1024-thread register panel below that (one matrix: 22 against 57 us, the
// 64 column steps shared by 16 waves; 4096 matrices: 237 against 198 us).
// The two take the same operations in the same order.  FTHMS_SYM_DIAG=reg
// in the environment takes the register panel always (a comparison switch).
constexpr int kDiagWaveMin = 1024;
static bool sym_diag_wave() {
  static const bool wave = [] {
    const char *e = getenv("FTHMS_SYM_DIAG");
    return !(e && std::string(e) == "reg");
  }();
  return wave;
}

static void launch_panel_sym(hipStream_t st, float2 *A, int N, long long ms, int k0, int *piv,
                             int *swp, float2 *linv, int *status, int count) {
  if (sym_panel_split()) {
    if (sym_diag_wave() && count >= kDiagWaveMin)
      lu_diag_sym_kernel<<<(count + kDiagWaves - 1) / kDiagWaves, 64 * kDiagWaves, 0, st>>>(
          A, N, ms, k0, piv, swp, status, count);
    else
      lu_panel_reg_kernel<float, 1, false><<<count, kPrThreads, 0, st>>>(
          A, N, ms, k0, piv, swp, linv, status, 0, kLuNB);
    const int rows = N - k0 - kLuNB;
    const int nt = std::min(256, (rows + 63) / 64 * 64);
    for (int b0 = 0; rows > 0 && b0 < count; b0 += 65535) {
      const int c = std::min(65535, count - b0);
      lu_rows_sym_kernel<float><<<dim3((rows + nt - 1) / nt, c), nt, 0, st>>>(
          A + (long long)b0 * ms, N, ms, k0, status + b0, 0);
    }
    return;
  }
  const int rl = (N - k0 + 63) / 64;
#define FTHMS_PANEL_SYM(RL)                                                         \
  lu_panel_reg_kernel<float, RL, false><<<count, kPrThreads, 0, st>>>(A, N, ms, k0, piv, swp, \
                                                                      linv, status, 0)
  switch (rl) {
    case 1: FTHMS_PANEL_SYM(1); break;
    case 2: FTHMS_PANEL_SYM(2); break;
    case 3: FTHMS_PANEL_SYM(3); break;
    case 4: FTHMS_PANEL_SYM(4); break;
    case 5: FTHMS_PANEL_SYM(5); break;
    case 6: FTHMS_PANEL_SYM(6); break;
    case 7: FTHMS_PANEL_SYM(7); break;
    default: FTHMS_PANEL_SYM(8); break;
  }
#undef FTHMS_PANEL_SYM
}

template <typename T, int R>
static void launch_panel(hipStream_t st, cplx_t<T> *A, int N, long long ms, int k0, int *piv,
                         int *swp, cplx_t<T> *linv, int *status, int count, int only_failed,
                         bool reg_panel) {
  const int m = N - k0;
  const int rl = (m + 63) / 64;
  const int rl_max = !reg_panel ? 0 : sizeof(T) == 4 ? 8 : 5;
#define FTHMS_PANEL_REG(RL)                                                            \
  lu_panel_reg_kernel<T, RL><<<count, kPrThreads, 0, st>>>(A, N, ms, k0, piv, swp, linv, \
                                                           status, only_failed)
  if (rl <= rl_max) {
    switch (rl) {
      case 1: FTHMS_PANEL_REG(1); return;
      case 2: FTHMS_PANEL_REG(2); return;
      case 3: FTHMS_PANEL_REG(3); return;
      case 4: FTHMS_PANEL_REG(4); return;
      default: break;
    }
    if (rl == 5) {
      FTHMS_PANEL_REG(5);
      return;
    }
    if constexpr (sizeof(T) == 4) {
      switch (rl) {
        case 6: FTHMS_PANEL_REG(6); return;
        case 7: FTHMS_PANEL_REG(7); return;
        default: FTHMS_PANEL_REG(8); return;
      }
    }
  }
#undef FTHMS_PANEL_REG
  lu_panel_kernel<T, R><<<count, kLuThreads, 0, st>>>(A, N, ms, k0, piv, swp, linv, status,
                                                      only_failed);
}

// One block step (panel, then strips) of `count` matrices on stream `st`.
template <typename T, int R>
static void lu_step(fthms_ctx *ctx, hipStream_t st, cplx_t<T> *A, int N, long long ms, int k0,
                    int *piv, int *swp, cplx_t<T> *linv, int *status, int count,
                    int only_failed, const LuOpts &o, hipEvent_t after_panel = nullptr) {
  // per-kernel timing ranges, except in the redo pass (timed as a whole)
  const bool tk = !only_failed;
  const int nb = std::min(kLuNB, N - k0);
  bool sym = false;
  if constexpr (sizeof(T) == 4) sym = o.sym && !only_failed && lu_sym_fits(true, N);
  if (tk) tbeg(ctx, "lu_panel", st);
  if constexpr (sizeof(T) == 4) {
    if (sym) launch_panel_sym(st, A, N, ms, k0, piv, swp, linv, status, count);
    else
      launch_panel<T, R>(st, A, N, ms, k0, piv, swp, linv, status, count, only_failed,
                         o.reg_panel);
  } else {
    launch_panel<T, R>(st, A, N, ms, k0, piv, swp, linv, status, count, only_failed,
                       o.reg_panel);
  }
  if (tk) tend(ctx);
  if (after_panel) (void)hipEventRecord(after_panel, st);
  // the symmetric form has no row interchanges: strips left of the block
  // have nothing to do
  const int nleft = sym ? 0 : (k0 + kStripW - 1) / kStripW;
  const int nright = (N - k0 - nb + kStripW - 1) / kStripW;
  if (nleft + nright > 0) {
    const long long blocks = 8LL * ((count + 7) / 8) * (nleft + nright);
    if (tk) tbeg(ctx, "lu_strip", st);
    bool done = false;
    if constexpr (sizeof(T) == 4) {
      const bool h16 = o.h16 && !only_failed;
      if (sym && h16)
        lu_strip_kernel<T, true, true><<<(unsigned)blocks, kLuThreads, 0, st>>>(
            A, N, ms, k0, swp, linv, count, nleft, nright, status, only_failed);
      else if (sym)
        lu_strip_kernel<T, true><<<(unsigned)blocks, kLuThreads, 0, st>>>(
            A, N, ms, k0, swp, linv, count, nleft, nright, status, only_failed);
      else if (h16)
        lu_strip_kernel<T, false, true><<<(unsigned)blocks, kLuThreads, 0, st>>>(
            A, N, ms, k0, swp, linv, count, nleft, nright, status, only_failed);
      done = sym || h16;
    }
    if (!done)
      lu_strip_kernel<T, false><<<(unsigned)blocks, kLuThreads, 0, st>>>(
          A, N, ms, k0, swp, linv, count, nleft, nright, status, only_failed);
    if (tk) tend(ctx);
  }
}

// Batches of at least this many matrices are factored as two halves on two
// streams, the second half one panel behind the first, so that the
// latency-bound panel kernel of one half runs beside the MFMA-bound strip
// kernel of the other.
constexpr int kLuSplitMin = 256;

// FTHMS_LU_SPLIT=0 in the environment keeps every batched LU on one stream
// (a kernel then runs with nothing beside it, e.g. to time it alone).
static bool lu_split_allowed() {
  const char *e = getenv("FTHMS_LU_SPLIT");
  return !(e && e[0] == '0' && e[1] == '\0');
}

template <typename T, int R>
static void lu_blocks(fthms_ctx *ctx, cplx_t<T> *A, int N, long long ms, int *piv, void *scr,
                      int *status, int count, int only_failed, const LuOpts &o) {
  int *swp = (int *)scr;
  cplx_t<T> *linv = (cplx_t<T> *)((char *)scr + sizeof(int) * kSwapStride * (size_t)count);
  if (only_failed || count < kLuSplitMin || !o.split || !lu_split_allowed()) {
    for (int k0 = 0; k0 < N; k0 += kLuNB)
      lu_step<T, R>(ctx, ctx->stream, A, N, ms, k0, piv, swp, linv, status, count, only_failed,
                    o);
    return;
  }
  // halves aligned to 8 so the XCD placement of every matrix is unchanged
  const int h = ((count / 2) + 7) & ~7;
  const int c2 = count - h;
  cplx_t<T> *A2 = A + (long long)h * ms;
  int *piv2 = piv + (long long)h * N;
  int *swp2 = swp + (long long)h * kSwapStride;
  cplx_t<T> *linv2 = linv + (long long)h * kLuNB * kLuNB;
  int *status2 = status + h;
  (void)hipEventRecord(ctx->ev_fork, ctx->stream);
  (void)hipStreamWaitEvent(ctx->aux, ctx->ev_fork, 0);
  for (int k0 = 0; k0 < N; k0 += kLuNB) {
    // the second half starts once the first half's first panel is done, so
    // that its panel runs beside the first half's first strip launch
    lu_step<T, R>(ctx, ctx->stream, A, N, ms, k0, piv, swp, linv, status, h, 0, o,
                  k0 == 0 ? ctx->ev_lead : nullptr);
    if (k0 == 0) (void)hipStreamWaitEvent(ctx->aux, ctx->ev_lead, 0);
  }
  for (int k0 = 0; k0 < N; k0 += kLuNB)
    lu_step<T, R>(ctx, ctx->aux, A2, N, ms, k0, piv2, swp2, linv2, status2, c2, 0, o);
  (void)hipEventRecord(ctx->ev_join, ctx->aux);
  (void)hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0);
}

// scr: count * kLuScratchBytes of device scratch
static int launch_lu(fthms_ctx *ctx, bool fp32, void *A, int N, long long ms, int *piv,
                     void *scr, int *status, int count, int only_failed = 0,
                     const LuOpts &o = LuOpts()) {
  const int R = (N + kLuThreads - 1) / kLuThreads;
  if (fp32) {
    float2 *a = (float2 *)A;
    switch (R) {
      case 1: lu_blocks<float, 1>(ctx, a, N, ms, piv, scr, status, count, only_failed, o); break;
      case 2: lu_blocks<float, 2>(ctx, a, N, ms, piv, scr, status, count, only_failed, o); break;
      case 3: lu_blocks<float, 3>(ctx, a, N, ms, piv, scr, status, count, only_failed, o); break;
      default: lu_blocks<float, 4>(ctx, a, N, ms, piv, scr, status, count, only_failed, o); break;
    }
  } else {
    double2 *a = (double2 *)A;
    switch (R) {
      case 1: lu_blocks<double, 1>(ctx, a, N, ms, piv, scr, status, count, only_failed, o); break;
      case 2: lu_blocks<double, 2>(ctx, a, N, ms, piv, scr, status, count, only_failed, o); break;
      case 3: lu_blocks<double, 3>(ctx, a, N, ms, piv, scr, status, count, only_failed, o); break;
      default: lu_blocks<double, 4>(ctx, a, N, ms, piv, scr, status, count, only_failed, o); break;
    }
  }
  launch_perm(ctx->stream, piv, N, lu_perm(scr, count), status, count, only_failed);
  return check_launch(ctx, "lu kernels");
}

// FP64 redo of refined solves: factor A64 in place for the matrices the
// redo mode selects (kRedoFailed: status < 0 after a first solve; kRedoLate:
// refinement failed at a later solve) and solve every matrix whose status
// is negative with its FP64 factors (those redone now and, at later solves,
// those redone before).
// lower: A holds its lower block triangle only (the symmetric form); the
// upper part of the selected matrices is completed first.
static int launch_fallback(fthms_ctx *ctx, double2 *A, int N, long long ms, int *piv, void *swp,
                           const double2 *b, double2 *x, int *status, int count,
                           int mode = kRedoFailed, bool lower = false) {
  const int nbk = (N + 63) / 64;
  if (lower && nbk > 1) {
    symmetrize_kernel<<<dim3(nbk * (nbk - 1) / 2, count), 256, 0, ctx->stream>>>(A, N, ms, status,
                                                                                mode);
    int rc = check_launch(ctx, "symmetrize_kernel");
    if (rc) return rc;
  }
  int rc = launch_lu(ctx, false, A, N, ms, piv, swp, status, count, mode);
  if (rc) return rc;
  if (mode == kRedoLate) {
    late_redo_done_kernel<<<(count + 255) / 256, 256, 0, ctx->stream>>>(status, count);
    if ((rc = check_launch(ctx, "late_redo_done_kernel"))) return rc;
  }
  solve_failed64_kernel<<<count, kLuThreads, 0, ctx->stream>>>(A, lu_perm(swp, count), N, ms, b,
                                                               x, N, status);
  return check_launch(ctx, "solve_failed64_kernel");
}

struct SolveWs {
  double2 *A64;
  float2 *A32;
  int *piv;
  void *swp;
  int *status;
  double *relres;
  int chunk;
};

static size_t per_matrix_bytes(int N, bool fp32) {
  const size_t nn = (size_t)N * N;
  return nn * sizeof(double2) + (fp32 ? nn * sizeof(float2) : 0) + sizeof(int) * N +
         kLuScratchBytes + sizeof(int) + sizeof(double) + 256;
}

static int solve_ws(fthms_ctx *ctx, int N, bool fp32, int nk, SolveWs &w) {
  const size_t per = per_matrix_bytes(N, fp32);
  size_t cap = kChunkBytes;
  if (ctx->budget) {
    const size_t avail = ctx->budget > ctx->held ? ctx->budget - ctx->held + ctx->ws_bytes : 0;
    cap = std::min(cap, avail);
  }
  int chunk = (int)std::min<size_t>((size_t)nk, std::max<size_t>(1, cap / per));
  chunk = std::min(chunk, 4096);
  const int nchunks = (nk + chunk - 1) / chunk;  // even split of the batch
  chunk = (nk + nchunks - 1) / nchunks;
  if ((size_t)chunk * per > cap) return fail(ctx, FTHMS_ENOMEM, "no room for one matrix");
  const size_t nn = (size_t)N * N;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  const size_t oA64 = take(nn * sizeof(double2) * chunk);
  const size_t oA32 = fp32 ? take(nn * sizeof(float2) * chunk) : 0;
  const size_t oP = take(sizeof(int) * (size_t)N * chunk);
  const size_t oW = take(kLuScratchBytes * chunk);
  const size_t oS = take(sizeof(int) * chunk);
  const size_t oR = take(sizeof(double) * chunk);
  int rc = ensure_ws(ctx, off);
  if (rc) return rc;
  char *base = (char *)ctx->ws;
  w.A64 = (double2 *)(base + oA64);
  w.A32 = fp32 ? (float2 *)(base + oA32) : nullptr;
  w.piv = (int *)(base + oP);
  w.swp = (void *)(base + oW);
  w.status = (int *)(base + oS);
  w.relres = (double *)(base + oR);
  w.chunk = chunk;
  return FTHMS_OK;
}

// lower: the lower block triangle only (symmetric arcs, the symmetric form)
static int assemble_launch(fthms_ctx *ctx, const fthms_arc *arc, const double *k_dev,
                           int count, double2 *A64, float2 *A32, bool lower = false) {
  const int N = arc->n;
  const int T = (N + 31) / 32;
  dim3 g(T * (T + 1) / 2, count), b(256);
  const long long ms = (long long)N * N;
  if (arc->closed) {
    dim3 gc(T, T, count);
    if (A32)
      cfie_assemble_kernel<true><<<gc, b, 0, ctx->stream>>>(arc->d_y, arc->d_dy, arc->d_R,
                                                            arc->d_L, arc->d_kd, N, k_dev, A64,
                                                            A32, ms);
    else
      cfie_assemble_kernel<false><<<gc, b, 0, ctx->stream>>>(arc->d_y, arc->d_dy, arc->d_R,
                                                             arc->d_L, arc->d_kd, N, k_dev, A64,
                                                             nullptr, ms);
    return check_launch(ctx, "cfie_assemble_kernel");
  }
  if (arc->d_w) {
    if (A32)
      assemble_kernel<true, true><<<g, b, 0, ctx->stream>>>(arc->d_y, arc->d_G, N, k_dev, A64,
                                                            A32, ms, nullptr, nullptr, arc->d_w);
    else
      assemble_kernel<false, true><<<g, b, 0, ctx->stream>>>(
          arc->d_y, arc->d_G, N, k_dev, A64, nullptr, ms, nullptr, nullptr, arc->d_w);
  } else {
    // Chebyshev arcs: kAsmF wavenumbers per block
    dim3 gm(T * (T + 1) / 2, (count + kAsmF - 1) / kAsmF);
    if (A32)
      assemble_mf_kernel<true><<<gm, b, 0, ctx->stream>>>(arc->d_y, arc->d_G, N, k_dev, count,
                                                          A64, A32, ms, lower ? 1 : 0);
    else
      assemble_mf_kernel<false><<<gm, b, 0, ctx->stream>>>(arc->d_y, arc->d_G, N, k_dev, count,
                                                           A64, nullptr, ms, lower ? 1 : 0);
    return check_launch(ctx, "assemble_mf_kernel");
  }
  return check_launch(ctx, "assemble_kernel");
}

// GMRES workspace per system: the basis [maxit + 1][N] and the triangular
// factor [maxit][maxit + 1] (double2 units)
static long long gmres_wstride(int N, int maxit) {
  return (long long)(maxit + 1) * N + (long long)maxit * (maxit + 1);
}

static int gmres_launch(fthms_ctx *ctx, const double2 *A, long long mstride, int N, int nb,
                        const double2 *b, long long bstride, double2 *x, long long xstride,
                        int maxit, double tol, double2 *work, int *iters, double *relres) {
  gmres_kernel<false><<<nb, kGmresThreads, 0, ctx->stream>>>(A, mstride, N, b, bstride, x,
                                                              xstride, maxit, tol, work,
                                                              gmres_wstride(N, maxit), iters,
                                                              relres);
  return check_launch(ctx, "gmres_kernel");
}

// Assembly + GMRES (FP64) for nk wavenumbers, chunked to the budget.
static int gmres_solve_impl(fthms_ctx *ctx, const fthms_arc *arc, int nk, const double *k_dev,
                            const double2 *rhs, double2 *alpha, double tol, int *iters_dev,
                            double *relres_dev) {
  const int N = arc->n;
  const int maxit = std::min(N, kGmresMaxIt);
  const size_t per = sizeof(double2) * ((size_t)N * N + (size_t)gmres_wstride(N, maxit)) +
                     sizeof(int) + sizeof(double) + 1024;
  size_t cap = kChunkBytes;
  if (ctx->budget) {
    const size_t avail = ctx->budget > ctx->held ? ctx->budget - ctx->held + ctx->ws_bytes : 0;
    cap = std::min(cap, avail);
  }
  int chunk = (int)std::min<size_t>((size_t)nk, std::max<size_t>(1, cap / per));
  chunk = std::min(chunk, 4096);
  const int nchunks = (nk + chunk - 1) / chunk;
  chunk = (nk + nchunks - 1) / nchunks;
  if ((size_t)chunk * per > cap) return fail(ctx, FTHMS_ENOMEM, "no room for one matrix");
  const size_t oA = 0;
  const size_t oW = (sizeof(double2) * (size_t)N * N * chunk + 255) & ~(size_t)255;
  const size_t oI = oW + ((sizeof(double2) * (size_t)gmres_wstride(N, maxit) * chunk + 255) &
                          ~(size_t)255);
  const size_t oR = oI + ((sizeof(int) * chunk + 255) & ~(size_t)255);
  const size_t total = oR + sizeof(double) * chunk;
  int rc = ensure_ws(ctx, total);
  if (rc) return rc;
  char *base = (char *)ctx->ws;
  double2 *A64 = (double2 *)(base + oA);
  double2 *work = (double2 *)(base + oW);
  int *it = (int *)(base + oI);
  double *rr = (double *)(base + oR);
  for (int f0 = 0; f0 < nk; f0 += chunk) {
    const int c = std::min(chunk, nk - f0);
    tbeg(ctx, "assemble");
    rc = assemble_launch(ctx, arc, k_dev + f0, c, A64, nullptr);
    tend(ctx);
    if (rc) return rc;
    tbeg(ctx, "gmres");
    rc = gmres_launch(ctx, A64, (long long)N * N, N, c, rhs + (long long)f0 * N, N,
                      alpha + (long long)f0 * N, N, maxit, tol, work,
                      iters_dev ? iters_dev + f0 : it, relres_dev ? relres_dev + f0 : rr);
    tend(ctx);
    if (rc) return rc;
  }
  return FTHMS_OK;
}

// GMRES-IR iterations per system at most (each applies the FP16-MFMA
// factors once): well-conditioned arcs need a handful.
constexpr int kGmresIrMaxIt = 30;

// Assembly, FP16-MFMA LU (FP32 storage; symmetric form where it applies)
// and FP64 GMRES right-preconditioned by it, for nk wavenumbers; systems whose
// factors are unusable (status -2) or whose GMRES misses tol are solved by
// the FP64 LU instead (iters -1).  iters: GMRES iterations.
static int gmres_ir_impl(fthms_ctx *ctx, const fthms_arc *arc, int nk, const double *k_dev,
                         const double2 *rhs, double2 *alpha, double tol, int *iters_dev,
                         double *relres_dev) {
  const int N = arc->n;
  const int maxit = std::min(N, kGmresIrMaxIt);
  const long long ws = gmres_wstride(N, maxit);
  const size_t nn = (size_t)N * N;
  const size_t per = nn * (sizeof(double2) + sizeof(float2)) + sizeof(int) * N + kLuScratchBytes +
                     sizeof(double2) * (size_t)ws + sizeof(int) + sizeof(double) + 2048;
  size_t cap = kChunkBytes;
  if (ctx->budget) {
    const size_t avail = ctx->budget > ctx->held ? ctx->budget - ctx->held + ctx->ws_bytes : 0;
    cap = std::min(cap, avail);
  }
  int chunk = (int)std::min<size_t>((size_t)nk, std::max<size_t>(1, cap / per));
  chunk = std::min(chunk, 4096);
  const int nchunks = (nk + chunk - 1) / chunk;
  chunk = (nk + nchunks - 1) / nchunks;
  if ((size_t)chunk * per > cap) return fail(ctx, FTHMS_ENOMEM, "no room for one matrix");
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t r = off;
    off += (bytes + 255) & ~(size_t)255;
    return r;
  };
  const size_t oA = take(sizeof(double2) * nn * chunk), oA32 = take(sizeof(float2) * nn * chunk);
  const size_t oP = take(sizeof(int) * (size_t)N * chunk), oS = take(kLuScratchBytes * chunk);
  const size_t oW = take(sizeof(double2) * (size_t)ws * chunk);
  const size_t oSt = take(sizeof(int) * chunk), oR = take(sizeof(double) * chunk);
  int rc = ensure_ws(ctx, off);
  if (rc) return rc;
  char *base = (char *)ctx->ws;
  double2 *A64 = (double2 *)(base + oA), *work = (double2 *)(base + oW);
  float2 *A32 = (float2 *)(base + oA32);
  int *piv = (int *)(base + oP), *status = (int *)(base + oSt);
  void *swp = base + oS;
  double *rr = (double *)(base + oR);
  const long long ms = (long long)nn;
  for (int f0 = 0; f0 < nk; f0 += chunk) {
    const int c = std::min(chunk, nk - f0);
    const double2 *b = rhs + (long long)f0 * N;
    double2 *x = alpha + (long long)f0 * N;
    tbeg(ctx, "assemble");
    rc = assemble_launch(ctx, arc, k_dev + f0, c, A64, A32);
    tend(ctx);
    if (rc) return rc;
    tbeg(ctx, "lu");
    LuOpts lo;
    lo.sym = arc_symmetric(arc) && lu_sym_fits(true, N);
    lo.h16 = true;
    rc = launch_lu(ctx, true, A32, N, ms, piv, swp, status, c, 0, lo);
    tend(ctx);
    if (rc) return rc;
    tbeg(ctx, "gmres");
    gmres_kernel<true><<<c, kGmresThreads, 0, ctx->stream>>>(
        A64, ms, N, b, N, x, N, maxit, tol, work, ws, iters_dev ? iters_dev + f0 : status, rr,
        A32, lu_perm(swp, c), status);
    tend(ctx);
    if ((rc = check_launch(ctx, "gmres_kernel (GMRES-IR)"))) return rc;
    tbeg(ctx, "fallback");
    rc = launch_fallback(ctx, A64, N, ms, piv, swp, b, x, status, c);
    tend(ctx);
    if (rc) return rc;
    if (iters_dev)
      HIPCK(ctx, hipMemcpyAsync(iters_dev + f0, status, sizeof(int) * c, hipMemcpyDeviceToDevice,
                                ctx->stream));
    if (relres_dev)
      HIPCK(ctx, hipMemcpyAsync(relres_dev + f0, rr, sizeof(double) * c, hipMemcpyDeviceToDevice,
                                ctx->stream));
  }
  return FTHMS_OK;
}

// Internal: solve for nk wavenumbers, device pointers, on ctx->stream.
static int solve_dev_impl(fthms_ctx *ctx, const fthms_arc *arc, int nk, const double *k_dev,
                          const double2 *rhs, double2 *alpha, int precision, double tol,
                          int *iters_dev, double *relres_dev) {
  const int N = arc->n;
  const bool fp32 = precision == FTHMS_FP32_REFINED;
  if (tol <= 0.0) tol = 1e-12;
  if (precision == FTHMS_GMRES)
    return gmres_solve_impl(ctx, arc, nk, k_dev, rhs, alpha, tol, iters_dev, relres_dev);
  if (precision == FTHMS_FP16_GMRES_IR)
    return gmres_ir_impl(ctx, arc, nk, k_dev, rhs, alpha, tol, iters_dev, relres_dev);
  SolveWs w;
  int rc = solve_ws(ctx, N, fp32, nk, w);
  if (rc) return rc;
  const long long ms = (long long)N * N;
  for (int f0 = 0; f0 < nk; f0 += w.chunk) {
    const int c = std::min(w.chunk, nk - f0);
    const double2 *b = rhs + (long long)f0 * N;
    double2 *x = alpha + (long long)f0 * N;
    const bool sym = use_sym_form(fp32, arc);
    tbeg(ctx, "assemble");
    rc = assemble_launch(ctx, arc, k_dev + f0, c, w.A64, fp32 ? w.A32 : nullptr, sym);
    tend(ctx);
    if (rc) return rc;
    tbeg(ctx, "lu");
    LuOpts lo;
    lo.sym = sym;
    rc = launch_lu(ctx, fp32, fp32 ? (void *)w.A32 : (void *)w.A64, N, ms, w.piv, w.swp, w.status,
                   c, 0, lo);
    tend(ctx);
    if (rc) return rc;
    if (!fp32) {
      tbeg(ctx, "solve");
      lu_solve64_kernel<<<c, kLuThreads, 0, ctx->stream>>>(w.A64, lu_perm(w.swp, c), N, ms, b, x,
                                                           N);
      tend(ctx);
      if ((rc = check_launch(ctx, "lu_solve64_kernel"))) return rc;
    } else {
      tbeg(ctx, "solve");
      launch_refine(ctx->stream, sym, c, w.A32, lu_perm(w.swp, c), w.A64, N, ms, b, x, N, tol, 10,
                    w.status, w.relres, 0);
      tend(ctx);
      if ((rc = check_launch(ctx, "refine_kernel"))) return rc;
      tbeg(ctx, "fallback");
      rc = launch_fallback(ctx, w.A64, N, ms, w.piv, w.swp, b, x, w.status, c, kRedoFailed, sym);
      tend(ctx);
      if (rc) return rc;
    }
    if (iters_dev)
      HIPCK(ctx, hipMemcpyAsync(iters_dev + f0, w.status, sizeof(int) * c,
                                hipMemcpyDeviceToDevice, ctx->stream));
    if (relres_dev) {
      if (fp32)
        HIPCK(ctx, hipMemcpyAsync(relres_dev + f0, w.relres, sizeof(double) * c,
                                  hipMemcpyDeviceToDevice, ctx->stream));
      else
        HIPCK(ctx, hipMemsetAsync(relres_dev + f0, 0, sizeof(double) * c, ctx->stream));
    }
  }
  return FTHMS_OK;
}

// Host-staging helper: device buffers freed on scope exit.
struct Staging {
  fthms_ctx *ctx;
  std::vector<std::pair<void *, size_t>> bufs;
  explicit Staging(fthms_ctx *c) : ctx(c) {}
  ~Staging() {
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &b : bufs) dev_free(ctx, b.first, b.second);
  }
  template <typename P> int get(P **p, size_t bytes) {
    void *q = nullptr;
    int rc = dev_alloc(ctx, &q, bytes);
    if (rc) return rc;
    bufs.push_back({q, bytes});
    *p = (P *)q;
    return FTHMS_OK;
  }
};

static bool finite_all(const double *p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

extern "C" {

int fthms_solve_dev(fthms_ctx *ctx, const fthms_arc *arc, int nk, const double *k_dev,
                    const fthms_c64 *rhs_dev, fthms_c64 *alpha_dev, int precision,
                    double tol, int *iters_dev, double *relres_dev) {
  if (!ctx || !arc || !k_dev || !rhs_dev || !alpha_dev || nk < 0)
    return fail(ctx, FTHMS_EINVAL, "bad argument to fthms_solve_dev");
  if (precision != FTHMS_FP64 && precision != FTHMS_FP32_REFINED && precision != FTHMS_GMRES &&
      precision != FTHMS_FP16_GMRES_IR)
    return fail(ctx, FTHMS_EINVAL, "unknown precision");
  if (nk == 0) return FTHMS_OK;
  HIPCK(ctx, hipSetDevice(ctx->device));
  return solve_dev_impl(ctx, arc, nk, k_dev, (const double2 *)rhs_dev, (double2 *)alpha_dev,
                        precision, tol, iters_dev, relres_dev);
}

int fthms_solve(fthms_ctx *ctx, const fthms_arc *arc, int nk, const double *k,
                const fthms_c64 *rhs, fthms_c64 *alpha, int precision, double tol, int *iters,
                double *relres) {
  if (!ctx || !arc || !k || !rhs || !alpha || nk < 0)
    return fail(ctx, FTHMS_EINVAL, "bad argument to fthms_solve");
  if (nk == 0) return FTHMS_OK;
  const int N = arc->n;
  for (int i = 0; i < nk; ++i)
    if (!(k[i] > 0.0) || !std::isfinite(k[i]))
      return fail(ctx, FTHMS_EINVAL_DATA, "wavenumbers must be finite and > 0");
  if (!finite_all((const double *)rhs, (size_t)2 * nk * N))
    return fail(ctx, FTHMS_EINVAL_DATA, "non-finite right-hand side");
  HIPCK(ctx, hipSetDevice(ctx->device));
  Staging st(ctx);
  double *dk;
  double2 *drhs, *dal;
  int *dit;
  double *drr;
  int rc;
  if ((rc = st.get(&dk, sizeof(double) * nk)) || (rc = st.get(&drhs, sizeof(double2) * nk * N)) ||
      (rc = st.get(&dal, sizeof(double2) * nk * N)) || (rc = st.get(&dit, sizeof(int) * nk)) ||
      (rc = st.get(&drr, sizeof(double) * nk)))
    return rc;
  HIPCK(ctx, hipMemcpyAsync(dk, k, sizeof(double) * nk, hipMemcpyHostToDevice, ctx->stream));
  HIPCK(ctx, hipMemcpyAsync(drhs, rhs, sizeof(double2) * nk * N, hipMemcpyHostToDevice,
                            ctx->stream));
  if ((rc = fthms_solve_dev(ctx, arc, nk, dk, (const fthms_c64 *)drhs, (fthms_c64 *)dal,
                            precision, tol, dit, drr)))
    return rc;
  std::vector<int> it(nk);
  HIPCK(ctx, hipMemcpyAsync(alpha, dal, sizeof(double2) * nk * N, hipMemcpyDeviceToHost,
                            ctx->stream));
  HIPCK(ctx, hipMemcpyAsync(it.data(), dit, sizeof(int) * nk, hipMemcpyDeviceToHost, ctx->stream));
  if (relres)
    HIPCK(ctx, hipMemcpyAsync(relres, drr, sizeof(double) * nk, hipMemcpyDeviceToHost,
                              ctx->stream));
  std::vector<double> rr(nk);
  HIPCK(ctx, hipMemcpyAsync(rr.data(), drr, sizeof(double) * nk, hipMemcpyDeviceToHost,
                            ctx->stream));
  HIPCK(ctx, hipStreamSynchronize(ctx->stream));
  if (iters) std::copy(it.begin(), it.end(), iters);
  if (precision == FTHMS_GMRES) {
    const double t = tol > 0.0 ? tol : 1e-12;
    for (int i = 0; i < nk; ++i)
      if (!(rr[i] <= t))
        return fail(ctx, FTHMS_ENOCONV, "GMRES did not reach the tolerance at wavenumber index " +
                                            std::to_string(i) + " within " +
                                            std::to_string(std::min(N, kGmresMaxIt)) +
                                            " iterations");
    return FTHMS_OK;
  }
  for (int i = 0; i < nk; ++i)
    if (it[i] == -2) return fail(ctx, FTHMS_ESINGULAR, "zero pivot at wavenumber index " +
                                                           std::to_string(i));
  return FTHMS_OK;
}

int fthms_gmres_dev(fthms_ctx *ctx, int n, int nb, const fthms_c64 *A_dev,
                    const fthms_c64 *b_dev, fthms_c64 *x_dev, double tol, int maxit,
                    int *iters_dev, double *relres_dev) {
  if (!ctx || n < 1 || n > kMaxN || nb < 0 ||
      (nb > 0 && (!A_dev || !b_dev || !x_dev || !iters_dev || !relres_dev)))
    return fail(ctx, FTHMS_EINVAL, "bad argument to fthms_gmres_dev");
  if (maxit < 1 || maxit > std::min(n, kGmresMaxIt))
    return fail(ctx, FTHMS_EINVAL, "maxit must be in [1, min(n, 256)]");
  if (nb == 0) return FTHMS_OK;
  HIPCK(ctx, hipSetDevice(ctx->device));
  int rc = ensure_ws2(ctx, sizeof(double2) * (size_t)gmres_wstride(n, maxit) * nb);
  if (rc) return rc;
  tbeg(ctx, "gmres");
  rc = gmres_launch(ctx, (const double2 *)A_dev, (long long)n * n, n, nb, (const double2 *)b_dev,
                    n, (double2 *)x_dev, n, maxit, tol > 0.0 ? tol : 1e-12,
                    (double2 *)ctx->ws2, iters_dev, relres_dev);
  tend(ctx);
  return rc;
}

static int to_incident(fthms_ctx *ctx, const fthms_incident *inc, IncidentDev &d) {
  if (!inc) return fail(ctx, FTHMS_EINVAL, "incident is NULL");
  if (inc->kind < 0 || inc->kind > 2) return fail(ctx, FTHMS_EINVAL, "unknown incident kind");
  d.kind = inc->kind;
  d.dx = std::cos(inc->theta);
  d.dy = std::sin(inc->theta);
  d.z0x = inc->z0[0];
  d.z0y = inc->z0[1];
  d.omega0 = inc->omega0;
  d.sigma = inc->kind == FTHMS_INC_PLANE ? 0.0 : inc->sigma;
  d.tau0 = inc->tau0;
  return FTHMS_OK;
}

int fthms_rhs_dev(fthms_ctx *ctx, const fthms_arc *arc, int nk, const double *k_dev,
                  const fthms_incident *inc, fthms_c64 *rhs_dev) {
  if (!ctx || !arc || !k_dev || !rhs_dev || nk < 0)
    return fail(ctx, FTHMS_EINVAL, "bad argument to fthms_rhs_dev");
  IncidentDev d;
  int rc = to_incident(ctx, inc, d);
  if (rc) return rc;
  if (nk == 0) return FTHMS_OK;
  HIPCK(ctx, hipSetDevice(ctx->device));
  dim3 g((arc->n + 255) / 256, nk);
  tbeg(ctx, "rhs");
  incident_kernel<<<g, 256, 0, ctx->stream>>>(d, arc->d_y, nullptr, arc->n, k_dev, -1.0,
                                               (double2 *)rhs_dev, arc->n);
  tend(ctx);
  return check_launch(ctx, "incident_kernel");
}

int fthms_rhs(fthms_ctx *ctx, const fthms_arc *arc, int nk, const double *k,
              const fthms_incident *inc, fthms_c64 *rhs) {
  if (!ctx || !arc || !k || !rhs || nk < 0) return fail(ctx, FTHMS_EINVAL, "bad argument");
  if (nk == 0) return FTHMS_OK;
  HIPCK(ctx, hipSetDevice(ctx->device));
  Staging st(ctx);
  double *dk;
  double2 *dr;
  int rc;
  if ((rc = st.get(&dk, sizeof(double) * nk)) || (rc = st.get(&dr, sizeof(double2) * nk * arc->n)))
    return rc;
  HIPCK(ctx, hipMemcpyAsync(dk, k, sizeof(double) * nk, hipMemcpyHostToDevice, ctx->stream));
  if ((rc = fthms_rhs_dev(ctx, arc, nk, dk, inc, (fthms_c64 *)dr))) return rc;
  HIPCK(ctx, hipMemcpyAsync(rhs, dr, sizeof(double2) * nk * arc->n, hipMemcpyDeviceToHost,
                            ctx->stream));
  HIPCK(ctx, hipStreamSynchronize(ctx->stream));
  return FTHMS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// fields
// ---------------------------------------------------------------------------
void near_plan_free(fthms_ctx *ctx, NearPlan &p);
int near_plan_build(fthms_ctx *ctx, const fthms_arc *arc, int np, const double *xy,
                    NearPlan &plan, const unsigned char *skip, double kmax);

// Field of arc `arc` with densities alpha[nk][astride] at points pts_dev
// classified by `plan`; U[nk][ustride] is written or accumulated.
int field_dev_impl(fthms_ctx *ctx, const fthms_arc *arc, int nk, const double *k_dev,
                   const double2 *alpha, long long astride, int np, const double2 *pts_dev,
                   const NearPlan &plan, double2 *U, long long ustride, int accumulate) {
  if (nk == 0 || np == 0) return FTHMS_OK;
  const int split = field_target_split(np), tpb = kFieldThreads / split;
  dim3 gf((np + tpb - 1) / tpb, nk);
  if (arc->closed) {
    closed_field_kernel<<<gf, kFieldThreads, 0, ctx->stream>>>(
        arc->d_y, arc->d_dy, arc->n, k_dev, alpha, astride, pts_dev, np, plan.d_cls, U, ustride,
        accumulate, split);
    int rc = check_launch(ctx, "closed_field_kernel");
    if (rc || plan.ntgt == 0) return rc;
    // near targets, level by level: density upsampled into ws2 (wavenumbers
    // in chunks that keep it within 64 MB), then the fine trapezoid rule
    for (int l = 0; l < kClosedLevels; ++l) {
      const int t0 = plan.lev_first[l], ntg = plan.lev_first[l + 1] - t0;
      if (ntg == 0) continue;
      const int M = plan.lev_kappa[l] * arc->n;
      const int chunk = std::max(1, std::min(nk, (int)((64ll << 20) / (sizeof(double2) * M))));
      if ((rc = ensure_ws2(ctx, sizeof(double2) * (size_t)chunk * M))) return rc;
      double2 *psif = (double2 *)ctx->ws2;
      for (int b0 = 0; b0 < nk; b0 += chunk) {
        const int c = std::min(chunk, nk - b0);
        closed_upsample_kernel<<<dim3((M + 255) / 256, c), 256, 0, ctx->stream>>>(
            alpha + (long long)b0 * astride, astride, arc->n, plan.lev_kappa[l], plan.d_Tf[l], psif);
        if ((rc = check_launch(ctx, "closed_upsample_kernel"))) return rc;
        closed_near_kernel<<<dim3(ntg, c), 256, 0, ctx->stream>>>(
            plan.d_yf[l], plan.d_dyf[l], M, k_dev + b0, psif, plan.d_tgt + t0, pts_dev,
            U + (long long)b0 * ustride, ustride, accumulate);
        if ((rc = check_launch(ctx, "closed_near_kernel"))) return rc;
      }
    }
    return FTHMS_OK;
  }
  {
    dim3 gm(gf.x, (nk + kFieldF - 1) / kFieldF);
    field_far_mf_kernel<<<gm, kFieldThreads, field_mf_lds_bytes(arc->n), ctx->stream>>>(
        arc->d_y, arc->n, arc->d_w, k_dev, nk, alpha, astride, pts_dev, np, plan.d_cls, U,
        ustride, accumulate, split);
  }
  int rc = check_launch(ctx, "field_far_mf_kernel");
  if (rc) return rc;
  if (plan.ntgt > 0) {
    if ((rc = ensure_ws2(ctx, sizeof(double2) * (size_t)nk * arc->n))) return rc;
    double2 *coef = (double2 *)ctx->ws2;
    cheb_coeff_kernel<<<nk, kFieldThreads, 0, ctx->stream>>>(arc->d_cos, arc->n, arc->nper,
                                                             alpha, astride, coef);
    if ((rc = check_launch(ctx, "cheb_coeff_kernel"))) return rc;
    dim3 gn(plan.ntgt, nk);
    field_near_kernel<<<gn, kFieldThreads, 0, ctx->stream>>>(
        plan.d_tgt, plan.d_qoff, plan.d_xq, plan.d_wq, plan.d_cq, plan.d_pq, arc->n, arc->nper,
        coef, k_dev, pts_dev, U, ustride, accumulate);
    rc = check_launch(ctx, "field_near_kernel");
  }
  return rc;
}

extern "C" {

int fthms_eval_field_dev(fthms_ctx *ctx, const fthms_arc *arc, int nk, const double *k_dev,
                         const fthms_c64 *alpha_dev, int np, const double *xy_dev,
                         fthms_c64 *U_dev) {
  if (!ctx || !arc || !k_dev || !alpha_dev || !xy_dev || !U_dev || nk < 0 || np < 0)
    return fail(ctx, FTHMS_EINVAL, "bad argument to fthms_eval_field_dev");
  if (nk == 0 || np == 0) return FTHMS_OK;
  HIPCK(ctx, hipSetDevice(ctx->device));
  // the near/far split and the near rule are planned on the host
  std::vector<double> xy(2 * (size_t)np), kh(nk);
  HIPCK(ctx, hipMemcpyAsync(xy.data(), xy_dev, sizeof(double) * 2 * np, hipMemcpyDeviceToHost,
                            ctx->stream));
  HIPCK(ctx, hipMemcpyAsync(kh.data(), k_dev, sizeof(double) * nk, hipMemcpyDeviceToHost,
                            ctx->stream));
  HIPCK(ctx, hipStreamSynchronize(ctx->stream));
  double kmax = 0.0;
  for (double v : kh) kmax = std::max(kmax, std::fabs(v));
  NearPlan plan;
  int rc = near_plan_build(ctx, arc, np, xy.data(), plan, nullptr, kmax);
  if (rc) return rc;
  tbeg(ctx, "field");
  rc = field_dev_impl(ctx, arc, nk, k_dev, (const double2 *)alpha_dev, arc->n, np,
                      (const double2 *)xy_dev, plan, (double2 *)U_dev, np, 0);
  tend(ctx);
  HIPCK(ctx, hipStreamSynchronize(ctx->stream));
  near_plan_free(ctx, plan);
  return rc;
}

int fthms_eval_field(fthms_ctx *ctx, const fthms_arc *arc, int nk, const double *k,
                     const fthms_c64 *alpha, int np, const double *xy, fthms_c64 *U) {
  if (!ctx || !arc || !k || !alpha || !xy || !U || nk < 0 || np < 0)
    return fail(ctx, FTHMS_EINVAL, "bad argument to fthms_eval_field");
  if (nk == 0 || np == 0) return FTHMS_OK;
  if (!finite_all(xy, 2 * (size_t)np)) return fail(ctx, FTHMS_EINVAL_DATA, "non-finite point");
  HIPCK(ctx, hipSetDevice(ctx->device));
  const int N = arc->n;
  Staging st(ctx);
  double *dk, *dxy;
  double2 *dal, *dU;
  int rc;
  if ((rc = st.get(&dk, sizeof(double) * nk)) || (rc = st.get(&dal, sizeof(double2) * nk * N)) ||
      (rc = st.get(&dxy, sizeof(double) * 2 * np)) || (rc = st.get(&dU, sizeof(double2) * nk * np)))
    return rc;
  HIPCK(ctx, hipMemcpyAsync(dk, k, sizeof(double) * nk, hipMemcpyHostToDevice, ctx->stream));
  HIPCK(ctx, hipMemcpyAsync(dal, alpha, sizeof(double2) * nk * N, hipMemcpyHostToDevice,
                            ctx->stream));
  HIPCK(ctx, hipMemcpyAsync(dxy, xy, sizeof(double) * 2 * np, hipMemcpyHostToDevice, ctx->stream));
  double kmax = 0.0;
  for (int i = 0; i < nk; ++i) kmax = std::max(kmax, std::fabs(k[i]));
  NearPlan plan;
  if ((rc = near_plan_build(ctx, arc, np, xy, plan, nullptr, kmax))) return rc;
  rc = field_dev_impl(ctx, arc, nk, dk, dal, N, np, (const double2 *)dxy, plan, dU, np, 0);
  if (rc == FTHMS_OK)
    rc = hipMemcpyAsync(U, dU, sizeof(double2) * nk * np, hipMemcpyDeviceToHost, ctx->stream) ==
                 hipSuccess
             ? FTHMS_OK
             : fail(ctx, FTHMS_EDEVICE, "copy of U failed");
  if (hipStreamSynchronize(ctx->stream) != hipSuccess && rc == FTHMS_OK)
    rc = fail(ctx, FTHMS_EDEVICE, "stream synchronisation failed");
  near_plan_free(ctx, plan);
  return rc;
}

// u[n][p] = (1/2pi) sum_l w_l U[l][p] exp(-i om_l t_n) on the context's stream.
// When the (time, point) tiles alone give few workgroups, the frequency sum
// is split over blockIdx.z (about 512 workgroups in all) into partial sums
// that a second kernel adds in a fixed order.
static int launch_freq_to_time(fthms_ctx *ctx, int nk, const double *om, const double *w, int np,
                               const double2 *U, int nt, const double *t, double2 *u) {
  if (np == 0 || nt == 0) return FTHMS_OK;
  const int gx = (np + kFtTile - 1) / kFtTile, gy = (nt + kFtTile - 1) / kFtTile;
  const int tiles = gx * gy;
  const int nchunk = std::max(1, (nk + kFtChunk - 1) / kFtChunk);
  int S = tiles >= 256 ? 1 : std::min(nchunk, (512 + tiles - 1) / tiles);
  int lsplit = ((nchunk + S - 1) / S) * kFtChunk;
  S = std::max(1, (nk + lsplit - 1) / lsplit);
  const long long nn = (long long)nt * np;
  if (S > 1 && !try_ft_scratch(ctx, sizeof(double2) * (size_t)S * (size_t)nn)) S = 1;
  if (S == 1) {
    freq_to_time_kernel<<<dim3(gx, gy, 1), 256, 0, ctx->stream>>>(nk, om, w, np, U, nt, t, u,
                                                                  std::max(nk, 1), nullptr);
    return check_launch(ctx, "freq_to_time_kernel");
  }
  double2 *part = (double2 *)ctx->ft;
  freq_to_time_kernel<<<dim3(gx, gy, S), 256, 0, ctx->stream>>>(nk, om, w, np, U, nt, t, u, lsplit,
                                                                 part);
  int rc = check_launch(ctx, "freq_to_time_kernel");
  if (rc) return rc;
  freq_to_time_sum_kernel<<<(unsigned)((nn + 255) / 256), 256, 0, ctx->stream>>>(S, nn, part, u);
  return check_launch(ctx, "freq_to_time_sum_kernel");
}

int fthms_freq_to_time_dev(fthms_ctx *ctx, int nk, const double *omega_dev, const double *w_dev,
                           int np, const fthms_c64 *U_dev, int nt, const double *t_dev,
                           fthms_c64 *u_dev) {
  if (!ctx || !omega_dev || !w_dev || !U_dev || !t_dev || !u_dev || nk < 0 || np < 0 || nt < 0)
    return fail(ctx, FTHMS_EINVAL, "bad argument to fthms_freq_to_time_dev");
  if (np == 0 || nt == 0) return FTHMS_OK;
  HIPCK(ctx, hipSetDevice(ctx->device));
  tbeg(ctx, "freq_to_time");
  const int rc = launch_freq_to_time(ctx, nk, omega_dev, w_dev, np, (const double2 *)U_dev, nt,
                                     t_dev, (double2 *)u_dev);
  tend(ctx);
  return rc;
}

int fthms_freq_to_time(fthms_ctx *ctx, int nk, const double *omega, const double *w, int np,
                       const fthms_c64 *U, int nt, const double *t, fthms_c64 *u) {
  if (!ctx || !omega || !w || !U || !t || !u || nk < 0 || np < 0 || nt < 0)
    return fail(ctx, FTHMS_EINVAL, "bad argument to fthms_freq_to_time");
  if (np == 0 || nt == 0) return FTHMS_OK;
  HIPCK(ctx, hipSetDevice(ctx->device));
  Staging st(ctx);
  double *dom, *dw, *dt;
  double2 *dU, *du;
  int rc;
  if ((rc = st.get(&dom, sizeof(double) * std::max(nk, 1))) ||
      (rc = st.get(&dw, sizeof(double) * std::max(nk, 1))) ||
      (rc = st.get(&dt, sizeof(double) * nt)) ||
      (rc = st.get(&dU, sizeof(double2) * std::max(nk, 1) * np)) ||
      (rc = st.get(&du, sizeof(double2) * nt * np)))
    return rc;
  if (nk > 0) {
    HIPCK(ctx, hipMemcpyAsync(dom, omega, sizeof(double) * nk, hipMemcpyHostToDevice, ctx->stream));
    HIPCK(ctx, hipMemcpyAsync(dw, w, sizeof(double) * nk, hipMemcpyHostToDevice, ctx->stream));
    HIPCK(ctx, hipMemcpyAsync(dU, U, sizeof(double2) * nk * np, hipMemcpyHostToDevice, ctx->stream));
  }
  HIPCK(ctx, hipMemcpyAsync(dt, t, sizeof(double) * nt, hipMemcpyHostToDevice, ctx->stream));
  if ((rc = fthms_freq_to_time_dev(ctx, nk, dom, dw, np, (const fthms_c64 *)dU, nt, dt,
                                   (fthms_c64 *)du)))
    return rc;
  HIPCK(ctx, hipMemcpyAsync(u, du, sizeof(double2) * nt * np, hipMemcpyDeviceToHost, ctx->stream));
  HIPCK(ctx, hipStreamSynchronize(ctx->stream));
  return FTHMS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// single stages
// ---------------------------------------------------------------------------
namespace fthms {
__global__ void bessel_kernel(int nz, const double *z, double *j0, double *y0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nz) return;
  double a, b;
  bessel_j0_y0(z[i], a, b);
  j0[i] = a;
  y0[i] = b;
}
}  // namespace fthms

extern "C" {

int fthms_assemble_dev(fthms_ctx *ctx, const fthms_arc *arc, int nk, const double *k_dev,
                       fthms_c64 *A_dev) {
  if (!ctx || !arc || nk < 0 || (nk > 0 && (!k_dev || !A_dev)))
    return fail(ctx, FTHMS_EINVAL, "bad argument to fthms_assemble_dev");
  if (nk == 0) return FTHMS_OK;
  HIPCK(ctx, hipSetDevice(ctx->device));
  tbeg(ctx, "assemble");
  int rc = assemble_launch(ctx, arc, k_dev, nk, (double2 *)A_dev, nullptr);
  tend(ctx);
  return rc;
}

int fthms_lu_dev(fthms_ctx *ctx, int n, int nb, int precision, void *A_dev, int *piv_dev,
                 int *info_dev) {
  if (!ctx || n < 1 || n > kMaxN || nb < 0 || (nb > 0 && (!A_dev || !piv_dev)))
    return fail(ctx, FTHMS_EINVAL, "bad argument to fthms_lu_dev");
  if (precision != FTHMS_FP64 && precision != FTHMS_FP32_REFINED && precision != FTHMS_FP32_SYM)
    return fail(ctx, FTHMS_EINVAL, "unknown precision");
  if (precision == FTHMS_FP32_SYM && !lu_sym_fits(true, n))
    return fail(ctx, FTHMS_EINVAL, "the symmetric form takes n <= 512");
  if (nb == 0) return FTHMS_OK;
  HIPCK(ctx, hipSetDevice(ctx->device));
  int rc = ensure_ws2(ctx, (kLuScratchBytes + sizeof(int)) * (size_t)nb + 256);
  if (rc) return rc;
  void *swp = ctx->ws2;
  int *status = (int *)((char *)ctx->ws2 + kLuScratchBytes * (size_t)nb);
  LuOpts lo;
  lo.sym = precision == FTHMS_FP32_SYM;
  tbeg(ctx, "lu");
  rc = launch_lu(ctx, precision != FTHMS_FP64, A_dev, n, (long long)n * n, piv_dev, swp, status,
                 nb, 0, lo);
  tend(ctx);
  if (rc == FTHMS_OK && info_dev)
    HIPCK(ctx, hipMemcpyAsync(info_dev, status, sizeof(int) * nb, hipMemcpyDeviceToDevice,
                              ctx->stream));
  return rc;
}

int fthms_lu_solve_dev(fthms_ctx *ctx, int n, int nb, const fthms_c64 *LU_dev, const int *piv_dev,
                       const fthms_c64 *b_dev, fthms_c64 *x_dev) {
  if (!ctx || n < 1 || n > kMaxN || nb < 0 ||
      (nb > 0 && (!LU_dev || !piv_dev || !b_dev || !x_dev)))
    return fail(ctx, FTHMS_EINVAL, "bad argument to fthms_lu_solve_dev");
  if (nb == 0) return FTHMS_OK;
  HIPCK(ctx, hipSetDevice(ctx->device));
  int rc = ensure_ws2(ctx, sizeof(int) * kMaxN * (size_t)nb + 256);
  if (rc) return rc;
  int *perm = (int *)ctx->ws2;
  tbeg(ctx, "solve");
  launch_perm(ctx->stream, piv_dev, n, perm, nullptr, nb, 0);
  lu_solve64_kernel<<<nb, kLuThreads, 0, ctx->stream>>>((const double2 *)LU_dev, perm, n,
                                                        (long long)n * n, (const double2 *)b_dev,
                                                        (double2 *)x_dev, n);
  tend(ctx);
  return check_launch(ctx, "lu_solve64_kernel");
}

int fthms_lu_solve_noalloc_dev(fthms_ctx *ctx, int n, int nb, const fthms_c64 *LU_dev,
                               const int *piv_dev, const fthms_c64 *b_dev, fthms_c64 *x_dev) {
  if (!ctx || n < 1 || n > kMaxN || nb < 0 ||
      (nb > 0 && (!LU_dev || !piv_dev || !b_dev || !x_dev)))
    return fail(ctx, FTHMS_EINVAL, "bad argument to fthms_lu_solve_noalloc_dev");
  if (nb > kNoAllocMatrices)
    return fail(ctx, FTHMS_EINVAL,
                "fthms_lu_solve_noalloc_dev: nb = " + std::to_string(nb) +
                    " exceeds the fixed scratch of " + std::to_string(kNoAllocMatrices) +
                    " matrices");
  if (nb == 0) return FTHMS_OK;
  HIPCK(ctx, hipSetDevice(ctx->device));
  int *perm = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    perm = (int *)g_scratch_ptr[ctx->device];
  }
  if (!perm) return fail(ctx, FTHMS_EDEVICE, "fixed scratch not set up for this device");
  // every entry the solve reads is written by the permutation kernel first,
  // so nothing needs clearing; no timing events either (they allocate)
  launch_perm(ctx->stream, piv_dev, n, perm, nullptr, nb, 0);
  lu_solve64_kernel<<<nb, kLuThreads, 0, ctx->stream>>>((const double2 *)LU_dev, perm, n,
                                                        (long long)n * n, (const double2 *)b_dev,
                                                        (double2 *)x_dev, n);
  return check_launch(ctx, "lu_solve64_kernel (no-alloc)");
}

int fthms_lu_refine_dev(fthms_ctx *ctx, int n, int nb, const fthms_c64 *A_dev,
                        const void *LU32_dev, const int *piv_dev, const fthms_c64 *b_dev,
                        fthms_c64 *x_dev, double tol, int max_iter, int *iters_dev,
                        double *relres_dev) {
  if (!ctx || n < 1 || n > kMaxN || nb < 0 || max_iter < 1 || max_iter > 100 ||
      !(tol > 0.0) ||
      (nb > 0 && (!A_dev || !LU32_dev || !piv_dev || !b_dev || !x_dev)))
    return fail(ctx, FTHMS_EINVAL, "bad argument to fthms_lu_refine_dev");
  if (nb == 0) return FTHMS_OK;
  HIPCK(ctx, hipSetDevice(ctx->device));
  // scratch: gather permutations [nb][kMaxN], then the status words [nb]
  const size_t perm_bytes = sizeof(int) * kMaxN * (size_t)nb;
  int rc = ensure_ws2(ctx, perm_bytes + sizeof(int) * (size_t)nb + 256);
  if (rc) return rc;
  int *perm = (int *)ctx->ws2;
  int *status = (int *)((char *)ctx->ws2 + perm_bytes);
  HIPCK(ctx, hipMemsetAsync(status, 0, sizeof(int) * (size_t)nb, ctx->stream));
  tbeg(ctx, "solve");
  launch_perm(ctx->stream, piv_dev, n, perm, nullptr, nb, 0);
  launch_refine(ctx->stream, false, nb, (const float2 *)LU32_dev, perm, (const double2 *)A_dev, n,
                (long long)n * n, (const double2 *)b_dev, (double2 *)x_dev, n, tol, max_iter,
                status, relres_dev, 0);
  tend(ctx);
  if ((rc = check_launch(ctx, "refine_kernel"))) return rc;
  if (iters_dev)
    HIPCK(ctx, hipMemcpyAsync(iters_dev, status, sizeof(int) * (size_t)nb,
                              hipMemcpyDeviceToDevice, ctx->stream));
  return FTHMS_OK;
}

static bool hf_set_from(const fthms_hf_grid *g, HfSet &s) {
  if (!g) return false;
  s.wc = g->wc;
  s.W = g->W;
  s.p = g->p;
  s.P = g->P;
  s.ncc = g->ncc;
  s.L = g->L;
  return hf_set_build(s);
}

int fthms_hf_frequencies(const fthms_hf_grid *g, double *omega, int *nk) {
  HfSet s;
  if (!nk || !hf_set_from(g, s)) return FTHMS_EINVAL;
  *nk = (int)s.omega.size();
  if (omega) std::copy(s.omega.begin(), s.omega.end(), omega);
  return FTHMS_OK;
}

int fthms_hf_to_time_dev(fthms_ctx *ctx, const fthms_hf_grid *g, int np, const fthms_c64 *U_dev,
                         double t0, double dt, int nt, double *u_dev) {
  HfSet s;
  if (!ctx || !hf_set_from(g, s) || np < 0 || nt < 0 || !std::isfinite(t0) ||
      !std::isfinite(dt) || (np > 0 && nt > 0 && (!U_dev || !u_dev)))
    return fail(ctx, FTHMS_EINVAL, "bad argument to fthms_hf_to_time_dev");
  if (np == 0 || nt == 0) return FTHMS_OK;
  HIPCK(ctx, hipSetDevice(ctx->device));
  const int nk = (int)s.omega.size();
  HfFc fc;
  hf_fc_factor(fc, s.L, s.W - s.wc, s.wc);
  std::vector<double> t(nt);
  for (int n = 0; n < nt; ++n) t[n] = t0 + n * dt;
  std::vector<zd> Wt((size_t)nt * nk);
  hf_weight_rows(s, fc, t.data(), nt, Wt.data());
  Staging st(ctx);
  double2 *dW;
  int rc;
  if ((rc = st.get(&dW, sizeof(double2) * Wt.size()))) return rc;
  HIPCK(ctx, hipMemcpyAsync(dW, Wt.data(), sizeof(double2) * Wt.size(), hipMemcpyHostToDevice,
                            ctx->stream));
  dim3 g2((np + 63) / 64, (nt + 63) / 64);
  tbeg(ctx, "freq_to_time");
  hf_apply_kernel<true><<<g2, 256, 0, ctx->stream>>>(dW, nt, nk, (const double2 *)U_dev, np,
                                                      u_dev, 0);
  tend(ctx);
  rc = check_launch(ctx, "hf_apply_kernel");
  // the host weights are freed on return: wait for the copy
  HIPCK(ctx, hipStreamSynchronize(ctx->stream));
  return rc;
}

int fthms_hf_to_time(fthms_ctx *ctx, const fthms_hf_grid *g, int np, const fthms_c64 *U,
                     double t0, double dt, int nt, double *u) {
  int nk = 0;
  if (!ctx || fthms_hf_frequencies(g, nullptr, &nk) != FTHMS_OK || np < 0 || nt < 0 ||
      (np > 0 && nt > 0 && (!U || !u)))
    return fail(ctx, FTHMS_EINVAL, "bad argument to fthms_hf_to_time");
  if (np == 0 || nt == 0) return FTHMS_OK;
  if (!finite_all((const double *)U, (size_t)2 * nk * np))
    return fail(ctx, FTHMS_EINVAL_DATA, "non-finite samples");
  HIPCK(ctx, hipSetDevice(ctx->device));
  Staging st(ctx);
  double2 *dU;
  double *du;
  int rc;
  if ((rc = st.get(&dU, sizeof(double2) * (size_t)nk * np)) ||
      (rc = st.get(&du, sizeof(double) * (size_t)nt * np)))
    return rc;
  HIPCK(ctx, hipMemcpyAsync(dU, U, sizeof(double2) * (size_t)nk * np, hipMemcpyHostToDevice,
                            ctx->stream));
  if ((rc = fthms_hf_to_time_dev(ctx, g, np, (const fthms_c64 *)dU, t0, dt, nt, du))) return rc;
  HIPCK(ctx, hipMemcpyAsync(u, du, sizeof(double) * (size_t)nt * np, hipMemcpyDeviceToHost,
                            ctx->stream));
  HIPCK(ctx, hipStreamSynchronize(ctx->stream));
  return FTHMS_OK;
}

int fthms_bessel_dev(fthms_ctx *ctx, int nz, const double *z_dev, double *j0_dev, double *y0_dev) {
  if (!ctx || nz < 0 || (nz > 0 && (!z_dev || !j0_dev || !y0_dev)))
    return fail(ctx, FTHMS_EINVAL, "bad argument to fthms_bessel_dev");
  if (nz == 0) return FTHMS_OK;
  HIPCK(ctx, hipSetDevice(ctx->device));
  bessel_kernel<<<(nz + 255) / 256, 256, 0, ctx->stream>>>(nz, z_dev, j0_dev, y0_dev);
  return check_launch(ctx, "bessel_kernel");
}

}  // extern "C"

#include "problem.h"
#include "windowed.h"
#include "batch.h"
#include "serve.h"
