/*
 * libfthms -- open-arc Helmholtz solves for the multi-patch / multiple-
 * scattering frequency-time hybrid (FTH-MS) method, on AMD MI355X (gfx950).
 *
 * What the library computes (paper: Pan, Bao, Yin, Bruno, "Multi-patch/
 * multiple-scattering frequency-time hybrid solver for interior and exterior
 * wave equation problems"):
 *
 *   * the first-kind open-arc integral equation V_Gamma[psi] = G and the
 *     single-layer potential S_Gamma[psi] (Section 3.2, eqs. FDBIEk-interior
 *     and FDsolk-interior) with Phi_k = (i/4) H0^(1)(k|x - y|) (Section 2.1),
 *     discretised with the endpoint-weighted Chebyshev density
 *     psi |x'| = alpha / sqrt(1 - t^2) (Section 4.3, eq. singularity);
 *   * one dense solve per (arc, wavenumber), batched over wavenumbers;
 *   * the frequency-domain multiple-scattering recursion over a cyclic set of
 *     overlapping arcs (Section 3.1, Definition inductive_int, eqs.
 *     criterion_int1/2, vtilde, POU1, mult-scatt-int);
 *   * the inverse Fourier transform of the fields to time traces (Section
 *     2.1, eq. backwardFT; eq. TDsol-interior with one time window).
 *
 * Conventions
 *   - Speed of propagation c = 1, so wavenumber k equals angular frequency.
 *   - Complex numbers are interleaved (re, im) doubles: fthms_c64, layout-
 *     identical to C99 double _Complex and to a complex128 tensor element.
 *   - Arrays are row-major: [freq][node], [freq][point], [time][point];
 *     points are [n][2] (x, y).
 *   - Arcs are given by samples of a parametrisation x(t), t in [-1, 1], at
 *     the first-kind Chebyshev nodes that fthms_cheb_nodes() returns.
 *
 * Ownership
 *   - Every *_create has a matching *_destroy.  The library owns contexts,
 *     arcs, problems and all device memory it allocates; it never frees
 *     caller memory.
 *   - Functions without the _dev suffix take host pointers, copy in and out,
 *     and return after the results are in host memory.
 *   - Functions with the _dev suffix take device pointers (e.g. from a torch
 *     tensor on the same device) and are stream-ordered on the context's
 *     stream: they return once the work is enqueued.
 *
 * Errors
 *   - Every function returns an int: FTHMS_OK (0) or a negative code.  No
 *     function throws or aborts across the ABI.  fthms_last_error() returns
 *     a description of the last failure on that context.
 *
 * Threading
 *   - A context is used by one host thread at a time.  Contexts are
 *     independent; several contexts may share a device.
 */
#ifndef FTHMS_H
#define FTHMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FTHMS_ABI_VERSION 2

enum {
  FTHMS_OK = 0,
  FTHMS_EINVAL = -1,      /* bad size, NULL pointer or unknown option   */
  FTHMS_EINVAL_DATA = -2, /* NaN/Inf or otherwise unusable input values  */
  FTHMS_ENOMEM = -3,      /* request exceeds the context's HBM budget    */
  FTHMS_ESINGULAR = -4,   /* exactly zero pivot in a factorisation       */
  FTHMS_ENOCONV = -5,     /* refinement hit its cap; results still valid */
  FTHMS_EDEVICE = -6,     /* HIP runtime error (text in last_error)      */
  FTHMS_EAGAIN = -7,      /* served request not finished yet             */
  FTHMS_ECANCELLED = -8   /* served request was cancelled                */
};

enum {
  FTHMS_FP64 = 0,
  FTHMS_FP32_REFINED = 1,
  FTHMS_GMRES = 2,
  FTHMS_FP32_SYM = 3,
  FTHMS_FP16_GMRES_IR = 4
};

enum { FTHMS_INC_PLANE = 0, FTHMS_INC_GPLANE = 1, FTHMS_INC_POINT = 2 };

typedef struct {
  double re, im;
} fthms_c64;

typedef struct fthms_ctx fthms_ctx;
typedef struct fthms_arc fthms_arc;
typedef struct fthms_problem fthms_problem;

/* Incident field (Section 5, eqs. pointsource and planewave2):
 *   PLANE : U = exp(i k x.d),  d = (cos theta, sin theta)
 *   GPLANE: U = exp(i k x.d) g(k)
 *   POINT : U = (5i/2) H0^(1)(k |x - z0|) g(k)   (g = 1 when sigma == 0)
 * with g(k) = exp(-(k - omega0)^2 / sigma^2) exp(i k tau0). */
typedef struct {
  int kind;
  double theta;
  double z0[2];
  double omega0, sigma, tau0;
} fthms_incident;

/* ---- library and context ---------------------------------------------- */

int fthms_abi_version(void);

/* Passed as `hip_stream` to fthms_create: the context creates and owns a
 * non-blocking stream of its own (default priority), unordered with every
 * other stream; the caller orders its own work with fthms_sync. */
#define FTHMS_OWN_STREAM ((void *)(intptr_t)-1)

/* Create a context on HIP device `device`.  `hbm_budget_bytes` caps the
 * device memory the context may hold (0 = no cap).  `hip_stream` is the
 * hipStream_t that _dev calls are ordered on: NULL is HIP's null (default)
 * stream, as everywhere in HIP -- the stream PyTorch uses by default, so
 * _dev calls on torch tensors follow torch's earlier work on it without a
 * synchronisation; FTHMS_OWN_STREAM asks for a private stream.  Fails with
 * FTHMS_EDEVICE when no gfx950 device is usable. */
int fthms_create(fthms_ctx **out, int device, size_t hbm_budget_bytes,
                 void *hip_stream);
int fthms_destroy(fthms_ctx *ctx);
/* Description of the last error on ctx (valid until the next call on ctx);
 * with ctx == NULL, the last error of fthms_create on this thread. */
const char *fthms_last_error(const fthms_ctx *ctx);
/* Block until all work enqueued on the context's stream has finished. */
int fthms_sync(fthms_ctx *ctx);

/* Kernel timing: while enabled, every kernel launch of the library is
 * bracketed by a pair of HIP events on the context's stream.  _read returns
 * the summed elapsed milliseconds and the launch count for one kernel class
 * ("assemble", "lu", "solve", "fallback", "rhs", "field", "field_cross",
 * "freq_to_time"); it synchronises the stream.  Timing adds a few
 * microseconds per launch. */
int fthms_timing_enable(fthms_ctx *ctx, int enable);
int fthms_timing_reset(fthms_ctx *ctx);
int fthms_timing_read(fthms_ctx *ctx, const char *name, double *total_ms,
                      int *launches);

/* ---- discretisation ---------------------------------------------------- */

/* First-kind Chebyshev nodes t_i = cos((2i - 1) pi / (2n)), i = 1..n
 * (n >= 2), written to t_out[n] in that order (t decreasing): the
 * collocation points of the endpoint-weighted density discretisation
 * (Section 4.3, eq. singularity: psi |x'| = alpha / sqrt(1 - t^2), alpha
 * expanded in Chebyshev polynomials). */
int fthms_cheb_nodes(int n, double *t_out);

/* Register one arc from samples at the Chebyshev nodes: xy[n][2] = x(t_i),
 * dxy[n][2] = dx/dt(t_i); 2 <= n <= 1024.  Builds the frequency-independent
 * tables of the Nystrom matrix (Section 4.2, frequency-independent kernel
 * decomposition) on the device.  Fails with FTHMS_EINVAL_DATA for
 * non-finite samples, coincident nodes or a vanishing speed |x'(t_i)|. */
int fthms_arc_create(fthms_ctx *ctx, int n, const double *xy,
                     const double *dxy, fthms_arc **out);
int fthms_arc_destroy(fthms_arc *arc);
/* Number of unknowns of the arc (n, or npan * n_per for panel arcs). */
int fthms_arc_size(const fthms_arc *arc);

/* ---- composite-panel arcs (Section 4.3, eqs. cov and psi-tilde) ----------
 *
 * The arc is cut at breaks[0] = -1 < breaks[1] < ... < breaks[npan] = 1 (in
 * its parameter t) into npan panels (1..16), so that no end of the arc or of
 * its truncated overlap lies inside a panel.  Panel p has a variable theta in
 * [-1, 1], t = breaks[p] + (breaks[p+1] - breaks[p]) (1 + theta) / 2, and
 * theta = theta(s) is the cosine change of variables of eq. cov given by
 * kinds[p]: FTHMS_COV_NONE (theta = s), FTHMS_COV_BOTH (singular ends at
 * both sides), FTHMS_COV_LEFT (at theta = -1), FTHMS_COV_RIGHT (at +1).
 * In s each panel has n_per first-kind Chebyshev nodes
 * s_i = cos((2i + 1) pi / (2 n_per)), i = 0..n_per-1, and the unknown is the
 * density per unit s, mu = psi |dx/ds| (the Jacobian-carrying density of
 * eq. psi-tilde): densities, right-hand sides and fields of such an arc are
 * [.][npan * n_per], panel by panel.  The matrix is
 * A_ij = -(1/2pi) J0(k r_ij) W_ij + w_j S_k(r_ij), where W is the
 * frequency-independent product-integration table of log|y_i - y(s)|
 * against each panel's interpolant, w the Fejer weights and S_k the smooth
 * part of the fundamental solution; fields use w for far targets and the
 * panel interpolants near the arc.  Composite-panel arcs work in
 * fthms_solve, fthms_eval_field, fthms_rhs, the stage entry points and
 * problems; batches (fthms_batch_create) take single-panel arcs only. */
enum { FTHMS_COV_NONE = 0, FTHMS_COV_BOTH = 1, FTHMS_COV_LEFT = 2, FTHMS_COV_RIGHT = 3 };

/* Arc parameters t at which to sample x(t) and dx/dt for a panel arc:
 * t_out[npan * n_per], panel by panel, nodes in the order above. */
int fthms_panel_nodes(int npan, const double *breaks, const int *kinds, int n_per,
                      double *t_out);

/* Register a composite-panel arc from samples xy, dxy [npan * n_per][2] of
 * x(t) and dx/dt at fthms_panel_nodes(); npan * n_per <= 1024.  Builds the
 * table W on the host (once per arc) and uploads it.  FTHMS_EINVAL for a bad
 * panel layout, FTHMS_EINVAL_DATA for non-finite samples, coincident nodes
 * or a vanishing speed. */
int fthms_arc_create_panels(fthms_ctx *ctx, int npan, const double *breaks, const int *kinds,
                            int n_per, const double *xy, const double *dxy, fthms_arc **out);

/* GMRES on nb dense systems A[nb][n][n] (column-major, complex128) with
 * right-hand sides b[nb][n] (device pointers, context stream): x[nb][n],
 * iterations iters[nb] and final relative residual estimates relres[nb];
 * the method of FTHMS_GMRES above, 1 <= maxit <= min(n, 256).  Stage entry
 * point for measurements on given matrices. */
int fthms_gmres_dev(fthms_ctx *ctx, int n, int nb, const fthms_c64 *A_dev,
                    const fthms_c64 *b_dev, fthms_c64 *x_dev, double tol, int maxit,
                    int *iters_dev, double *relres_dev);

/* ---- windowing and time recentering (Section 2.1, eqs. windowing,
 * Fourierk, TDsol; Algorithm 1 with Q windows) -----------------------------
 *
 * Time-domain incident field for windowed runs: a train of npulse Gaussian
 * plane-wave pulses (u2 of Section 5 in the time domain), direction theta,
 *   u(x, t) = sum_{p < npulse} f(t - p period - x.d),
 *   f(tau) = sigma/(2 sqrt(pi)) exp(-i omega0 (tau - tau0) - sigma^2 (tau - tau0)^2 / 4). */
typedef struct {
  double theta, omega0, sigma, tau0, period;
  int npulse;
} fthms_pulse_train;

/* Time traces u_M(x_p, t_n), t_n = n dt (n < nt), of the problem's M-step
 * recursion run through the time domain with Q windows (s_q = 3/2 (q-1) H,
 * the window function of Section 5): every step transforms each arc's
 * boundary data about each window centre over the nk frequencies k (with
 * quadrature weights w for the way back), solves with the factors of the
 * first step, evaluates the fields and transforms them back shifted by
 * s_q.  The data must fit inside sum_q window = 1, i.e. nt dt <= s_Q + H/2
 * for signals that last to the end.  Either precision (the refined form
 * keeps each matrix's FP32 factors for every window and step); traces [nt][nobs]
 * (host).  All frequencies and time series stay resident (FTHMS_ENOMEM if
 * they do not fit the budget). */
int fthms_problem_traces_windowed(fthms_problem *pb, int nk, const double *k, const double *w,
                                  int nt, double dt, int Q, double H,
                                  const fthms_pulse_train *inc, fthms_c64 *traces);

/* ---- high-frequency transforms of real signals (Section 4.1, eqs. ft_appr,
 * backwardFT1, int1, int2; the frequency set of Section 5) ------------------
 *
 * The frequency set: Clenshaw-Curtis points (ncc per interval, shared ends
 * once) on the graded intervals (mu_j, mu_{j+1}), mu_j = wc (j/P)^p,
 * j = 1..P-1 (mu_P = wc), then the uniform grid wc + l (W - wc)/L,
 * l = 0..L; sorted, each point once.  Requires 0 < wc < W, P >= 2, p >= 1,
 * 3 <= ncc <= 64, L >= 8. */
typedef struct {
  double wc, W, p;
  int P, ncc, L;
} fthms_hf_grid;

/* The set's frequencies (omega may be NULL: *nk receives the count). */
int fthms_hf_frequencies(const fthms_hf_grid *grid, double *omega, int *nk);

/* Inverse transform of a real signal from its samples on the set,
 * g(t) ~ (1/2pi) int_{-W}^{W} G e^{-iwt} dw = (1/pi) Re [int_0^{wc} + int_{wc}^{W}]
 * (G(-w) = conj G(w)): the part near 0 by Filon-Clenshaw-Curtis on the
 * graded intervals (the logarithmic singularity of 2D fields at w = 0; the
 * piece (0, mu_1) is left out), the rest by a least-squares Fourier
 * continuation of the uniform samples (period 2 (W - wc), modes |k| <= L/4)
 * integrated term by term.  U[nk][np] complex samples (device), times
 * t_n = t0 + n dt, u[nt][np] real (device).  The weights are built on the
 * host per call. */
int fthms_hf_to_time_dev(fthms_ctx *ctx, const fthms_hf_grid *grid, int np,
                         const fthms_c64 *U_dev, double t0, double dt, int nt, double *u_dev);
int fthms_hf_to_time(fthms_ctx *ctx, const fthms_hf_grid *grid, int np, const fthms_c64 *U,
                     double t0, double dt, int nt, double *u);

/* The real pulse incident field of Section 5: u3 (eq. planewave,
 * u3 = -sin(4 l) exp(-1.6 (l - 3)^2), l = t - 2 - x.d, d = (cos theta,
 * sin theta)) repeated npulse times, period apart (u4 of eq. multi: 5
 * pulses, 10 apart). */
typedef struct {
  double theta, period;
  int npulse;
} fthms_pulse3;

/* Real time traces u_M(x_p, t_n), t_n = n dt (n < nt), of the problem's
 * M-step recursion run through the time domain with Q windows (as
 * fthms_problem_traces_windowed) for the real pulse field inc: the slow
 * transforms are taken at the frequency set of `grid` and the way back is
 * the high-frequency transform of real signals above, at the shifted times
 * t_n - s_q.  traces[nt][nobs] (host, real).  The recursion itself runs on
 * the time mesh of Section 5, which covers [0, s_Q + H] (the last window's
 * whole support): max(nt, ceil((s_Q + H)/dt) + 1) samples; the traces are
 * the first nt, meaningful up to s_Q + H/2 where the windows sum to one.
 * Either precision; all frequencies and time series stay resident
 * (FTHMS_ENOMEM if they do not fit the budget).  The transform weights are
 * built on the host. */
int fthms_problem_traces_windowed_real(fthms_problem *pb, const fthms_hf_grid *grid, int nt,
                                       double dt, int Q, double H, const fthms_pulse3 *inc,
                                       double *traces);

/* ---- closed patches (Section 3.3, eqs. FDsolk-closed, FDBIEk-closed) -------
 *
 * A closed curve treated as one patch: its density solves the combined-field
 * equation (1/2 I + K - i eta V) Psi = G on the curve, with eta = k, and its
 * field is (D - i eta S) Psi outside (D, K double-layer potential/operator
 * with the outward normal).  Nystrom method for 2pi-periodic kernels with a
 * logarithmic singularity on n equispaced nodes (n even, 4..1024): sample a
 * counter-clockwise parametrisation x(tau) at tau_j = 2 pi j / n, giving
 * xy, dxy, ddxy [n][2] = x, x', x''.  Densities are per unit length at the
 * nodes.  Such an arc works in fthms_solve, fthms_rhs, fthms_eval_field and
 * problems (where it must be alone in its group: chi = 1, nothing masked);
 * fields are the trapezoid rule at targets 5 node spacings h (the largest)
 * or more from the nodes; nearer targets take the same rule on a grid kappa
 * = 2, 4, .., 128 times finer (the smallest with h / kappa <= d / 5.2, d
 * the target's distance to the curve), with the density's and the
 * geometry's trigonometric interpolants there; targets nearer than h / 25
 * are refused (FTHMS_EINVAL_DATA).  Not for batches. */
int fthms_closed_create(fthms_ctx *ctx, int n, const double *xy, const double *dxy,
                        const double *ddxy, fthms_arc **out);

/* Panel breakpoints of the arcs of cyclic partitions (the layout of
 * fthms_problem_desc: interval [narcs][2] on the parent curve of period
 * `period`, group [narcs] or NULL for one curve): arc j is cut where the
 * overlaps with its neighbours on the same curve end, i.e. at the ends of
 * its truncated overlap (Section 4.3).  breaks [narcs][4] receives
 * -1 = t_0 < ... < t_npan = 1 (unused entries 1), npan [narcs] the panel
 * count (3, or 1 for an arc alone on its curve). */
int fthms_tov_breaks(int narcs, const double *interval, const int *group, double period,
                     double *breaks, int *npan);

/* Copy out a panel arc's table W [n][n] (row i = target node, row-major)
 * and weights w [n] (either may be NULL).  FTHMS_EINVAL for other arcs. */
int fthms_arc_panel_table(const fthms_arc *arc, double *W, double *w);

/* ---- the per-(arc, k) solve --------------------------------------------- */

/* The open-arc first-kind equation V_Gamma[psi] = G (Section 3.2, eq.
 * FDBIEk-interior; Phi_k of Section 2.1; discretised per Section 4.3, eq.
 * singularity).  For each of nk wavenumbers k[i] > 0: assemble the Nystrom
 * matrix of V_Gamma on `arc`, factor it (LU with partial pivoting) and solve
 * A alpha = rhs[i].  rhs, alpha: [nk][n].  precision FTHMS_FP64 factors in
 * complex FP64; FTHMS_FP32_REFINED factors in complex FP32 (MFMA trailing
 * updates, pivots chosen on FP64 magnitudes) and refines with FP64
 * residuals until the predicted relative error of alpha is below tol
 * (tol <= 0: 1e-12; the prediction is |d_k|^2 / |d_{k-1}| for successive
 * corrections d, the initial solve counting as d_0), at most 10
 * iterations; solves that do not converge are redone in FP64.
 * iters[nk] (optional) receives the refinement steps per solve (0 for
 * FP64, -1 for a solve redone in FP64); relres[nk] (optional) the last
 * relative correction |delta|/|alpha|.  FTHMS_ESINGULAR if a pivot is
 * exactly zero (alpha is then not meaningful for that k).
 * Batches of at least 256 matrices are factored as two half batches on two
 * streams (same results as one); FTHMS_LU_SPLIT=0 in the environment keeps
 * them on one stream.
 * precision FTHMS_GMRES solves each assembled system with GMRES in FP64
 * instead (x0 = 0, modified Gram-Schmidt Arnoldi, Givens rotations, no
 * restart; the iterative solver the paper names beside direct ones, §5
 * Geometries 5) until the residual estimate is below tol |rhs| (tol <= 0:
 * 1e-12) or min(n, 256) iterations; iters receives the GMRES iterations,
 * relres the final relative residual estimate; the host entry point
 * returns FTHMS_ENOCONV (results written) if a system did not converge.
 * precision FTHMS_FP16_GMRES_IR (GMRES-IR, for well-conditioned arcs): the
 * matrices are factored with the trailing-update products on the FP16
 * matrix cores (FP32 storage and accumulation; the symmetric form for
 * single-panel arcs of n <= 512), and FP64 GMRES right-preconditioned by
 * those factors solves each system to tol (tol <= 0: 1e-12), at most
 * min(n, 30) iterations; a system whose factors are unusable or whose GMRES
 * misses tol is solved with FP64 LU instead.  iters receives the GMRES
 * iterations (-1 for an FP64 solve), relres the final relative residual
 * estimate. */
int fthms_solve(fthms_ctx *ctx, const fthms_arc *arc, int nk, const double *k,
                const fthms_c64 *rhs, fthms_c64 *alpha, int precision,
                double tol, int *iters, double *relres);
int fthms_solve_dev(fthms_ctx *ctx, const fthms_arc *arc, int nk,
                    const double *k_dev, const fthms_c64 *rhs_dev,
                    fthms_c64 *alpha_dev, int precision, double tol,
                    int *iters_dev, double *relres_dev);

/* Right-hand side of the sound-soft single-arc problem, b = -U^inc at the
 * arc's nodes (G = -u^i), for nk wavenumbers: rhs[nk][n]. */
int fthms_rhs(fthms_ctx *ctx, const fthms_arc *arc, int nk, const double *k,
              const fthms_incident *inc, fthms_c64 *rhs);
int fthms_rhs_dev(fthms_ctx *ctx, const fthms_arc *arc, int nk,
                  const double *k_dev, const fthms_incident *inc,
                  fthms_c64 *rhs_dev);

/* Single-layer potential U(z_p) = S_Gamma[psi](z_p) of the density alpha
 * at np points xy[np][2] (Section 3.2, eq. FDsolk-interior): U[nk][np].  Points farther than ten node spacings
 * from every node use the Gauss-Chebyshev rule; nearer points use a graded
 * composite Gauss-Legendre rule on the Chebyshev interpolant of alpha.  The
 * _dev form copies the points and wavenumbers to the host to plan the near
 * rule, so it synchronises the stream before enqueuing. */
int fthms_eval_field(fthms_ctx *ctx, const fthms_arc *arc, int nk,
                     const double *k, const fthms_c64 *alpha, int np,
                     const double *xy, fthms_c64 *U);
int fthms_eval_field_dev(fthms_ctx *ctx, const fthms_arc *arc, int nk,
                         const double *k_dev, const fthms_c64 *alpha_dev,
                         int np, const double *xy_dev, fthms_c64 *U_dev);

/* The inverse Fourier transform of Section 2.1 (eq. backwardFT, applied
 * as in eq. TDsol-interior with one window) by a quadrature over the given
 * frequencies:
 * u(x_p, t_n) = (1/2pi) sum_l w[l] U[l][p] exp(-i omega[l] t_n):
 * U[nk][np] -> u[nt][np]. */
int fthms_freq_to_time(fthms_ctx *ctx, int nk, const double *omega,
                       const double *w, int np, const fthms_c64 *U, int nt,
                       const double *t, fthms_c64 *u);
int fthms_freq_to_time_dev(fthms_ctx *ctx, int nk, const double *omega_dev,
                           const double *w_dev, int np,
                           const fthms_c64 *U_dev, int nt, const double *t_dev,
                           fthms_c64 *u_dev);

/* ---- single stages (per-kernel access) -------------------------------- */

/* Nystrom matrices of V_Gamma on `arc` for nk wavenumbers (the assembly
 * stage of fthms_solve): A[nk] of n x n complex128, column-major per matrix
 * (element (i, j) of matrix b at A[b n^2 + j n + i]). */
int fthms_assemble_dev(fthms_ctx *ctx, const fthms_arc *arc, int nk,
                       const double *k_dev, fthms_c64 *A_dev);

/* In-place LU with partial pivoting of nb column-major n x n complex
 * matrices, 1 <= n <= 1024.  precision FTHMS_FP64: A is complex128;
 * FTHMS_FP32_REFINED: A is complex64 (interleaved float re, im), factored
 * with FP32 MFMA updates and FP64 pivoting.  piv[nb][n] receives 0-based
 * pivot rows in LAPACK order (row i was swapped with piv[i]); info[nb]
 * (optional) 0, or -2 for an exactly zero pivot.
 * FTHMS_FP32_SYM (this stage only; the solves take it by themselves for
 * the complex symmetric matrices of single-panel arcs, n <= 512): A is
 * complex64 and complex symmetric (A = A^T, read from its lower triangle
 * and diagonal blocks), n <= 512, factored without row interchanges, the
 * trailing updates on and below the diagonal only.  The factors take the
 * same form as FTHMS_FP32_REFINED's (unit lower L, U above, piv[i] = i);
 * info is -2 where partial pivoting would have interchanged rows at some
 * column (a row below the diagonal with larger |re| + |im| in the reduced
 * matrix) or a pivot is exactly zero: those factors are not to be used. */
int fthms_lu_dev(fthms_ctx *ctx, int n, int nb, int precision, void *A_dev,
                 int *piv_dev, int *info_dev);

/* x = A^{-1} b from complex128 factors of fthms_lu_dev (FTHMS_FP64):
 * b, x: [nb][n]; b and x may alias. */
int fthms_lu_solve_dev(fthms_ctx *ctx, int n, int nb, const fthms_c64 *LU_dev,
                       const int *piv_dev, const fthms_c64 *b_dev,
                       fthms_c64 *x_dev);

/* The refinement stage of the FTHMS_FP32_REFINED solve (the direct solve of
 * Section 3.2, eq. FDBIEk-interior, factored in FP32 and corrected in FP64),
 * on caller-given matrices: A[nb] n x n complex128 (column-major, read
 * only), LU32[nb] its complex64 factors and piv[nb][n] the pivots, both as
 * fthms_lu_dev(FTHMS_FP32_REFINED) writes them, b[nb][n] right-hand sides
 * (device pointers, context stream).  x0 = LU32^{-1} P b, then repeatedly
 * r = b - A x in FP64, d = LU32^{-1} P r, x += d, until the predicted
 * relative error |d_k| (|d_k| / |d_{k-1}|) falls below tol (> 0), at most
 * max_iter (1..100) steps.  x[nb][n] receives the result; iters[nb]
 * (optional) the steps taken, or -1 when the corrections stopped
 * contracting or the cap was hit -- there is no FP64 redo here, x then
 * holds the last iterate; relres[nb] (optional) the last |d| / |x|.
 * b and x must not alias. */
int fthms_lu_refine_dev(fthms_ctx *ctx, int n, int nb, const fthms_c64 *A_dev,
                        const void *LU32_dev, const int *piv_dev, const fthms_c64 *b_dev,
                        fthms_c64 *x_dev, double tol, int max_iter, int *iters_dev,
                        double *relres_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * solve as fthms_lu_solve_dev, with its scratch (the gather permutations)
 * in a fixed device array of the library instead of the context's
 * workspace.  The array holds 4096 matrices of up to 1024 rows (16 MiB per
 * device, held until the process ends); nb > 4096 fails with FTHMS_EINVAL.
 * No device or host memory is allocated and no timing events are recorded.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (other streams, other threads, other contexts) race and must
 * be ordered by the caller. */
int fthms_lu_solve_noalloc_dev(fthms_ctx *ctx, int n, int nb, const fthms_c64 *LU_dev,
                               const int *piv_dev, const fthms_c64 *b_dev,
                               fthms_c64 *x_dev);

/* Device Bessel functions used by the kernels: J0(z) and Y0(z) for nz
 * arguments z > 0 (FP64). */
int fthms_bessel_dev(fthms_ctx *ctx, int nz, const double *z_dev,
                     double *j0_dev, double *y0_dev);

/* ---- multiple scattering over a cyclic partition ---------------------- */

/* A closed curve covered by narcs >= 2 overlapping arcs, cyclically ordered
 * (arc j overlaps arcs j-1 and j+1 only) -- or several closed curves
 * (obstacles of an exterior problem, Section 3.3): group[j] (optional;
 * NULL: one curve) names the curve of arc j, the arcs of one curve are
 * cyclic in the order given, and an arc alone in its group is a plain open
 * arc (chi = 1).  Every arc scatters onto every other one; the overlap
 * masking applies to neighbours on the same curve.  interval[2j], interval[2j+1] are
 * the parameter bounds of arc j on the parent closed curve of period
 * `period` (arc j's local t = -1 maps to interval[2j]); they decide overlap
 * membership.  c0, c1 are the POU constants of eq. POU1 (the paper uses
 * 1/3, 2/3); the window distances are chords.  M >= 1 multiple-scattering
 * steps.  precision FTHMS_FP64 or FTHMS_FP32_REFINED (FP32 factors kept
 * for all M steps and refined to tol at every solve; a matrix whose
 * refinement fails is refactored in FP64 once and solved with those
 * factors from then on).  narcs == 1 is allowed and
 * runs the plain sound-soft single-arc problem (G = -U^inc, no recursion,
 * either precision).  The field u_M is evaluated at nobs observation
 * points obs_xy[nobs][2] (copied at creation). */
typedef struct {
  int narcs;
  const fthms_arc *const *arcs;
  const double *interval;
  double period;
  double c0, c1;
  int M;
  int precision;
  double tol;
  fthms_incident incident;
  int nobs;
  const double *obs_xy;
  const int *group;
} fthms_problem_desc;

int fthms_problem_create(fthms_ctx *ctx, const fthms_problem_desc *desc,
                         fthms_problem **out);
int fthms_problem_destroy(fthms_problem *pb);

/* Run the multiple-scattering recursion (Section 3.1, Definition
 * inductive_int, eqs. criterion_int1, criterion_int2 and vtilde; the loop of
 * Algorithm 1 taken per frequency) at nk wavenumbers and evaluate
 * u_M = sum_m sum_j v_{j,m} (eq. mult-scatt-int) at the observation points:
 * U[nk][nobs] (optional).  alpha_tot (optional)
 * receives sum_m alpha_{j,m} as [nk][sum_j n_j] in arc order.  The _dev form
 * takes device pointers; it copies k to the host (to size the near-target
 * rules) and then enqueues everything on the context's stream. */
int fthms_problem_run_dev(fthms_problem *pb, int nk, const double *k_dev,
                          fthms_c64 *U_dev, fthms_c64 *alpha_tot_dev);
int fthms_problem_run(fthms_problem *pb, int nk, const double *k, fthms_c64 *U,
                      fthms_c64 *alpha_tot);

/* The recursion with time-domain output (eq. TDsol-interior with one
 * window): after each step m the traces u_m(x_p, t_n) = (1/2pi) sum_l w_l
 * U_m(x_p, k_l) e^{-i k_l t_n} at the observation points are updated, and the
 * run stops once |u_m - u_{m-1}| <= stop_tol |u_m| (L2 over all points and
 * times) or after the problem's M steps (stop_tol <= 0: always M).  w[nk]:
 * quadrature weights of the frequencies (e.g. trapezoid); traces[nt][nobs];
 * *steps (host, optional): steps taken.  All nk frequencies must fit the
 * workspace at once (FTHMS_ENOMEM otherwise). */
int fthms_problem_traces_dev(fthms_problem *pb, int nk, const double *k_dev,
                             const double *w_dev, int nt, const double *t_dev,
                             double stop_tol, fthms_c64 *traces_dev, int *steps);
int fthms_problem_traces(fthms_problem *pb, int nk, const double *k,
                         const double *w, int nt, const double *t,
                         double stop_tol, fthms_c64 *traces, int *steps);

/* ---- uneven batches ------------------------------------------------------ */

/* nb independent solves of the sound-soft single-arc problem (Section 3.2,
 * eq. FDBIEk-interior with G = -u^i): solve i on arcs[i] at wavenumber
 * k[i] > 0 with incident field inc[i].  The arcs may have different node
 * counts -- the uneven (arc, frequency) batches of multi-arc, many-frequency
 * workloads, where n follows the wavenumber.  Solves of equal n form groups
 * that are assembled, factored and solved together; the whole batch runs as
 * one HIP graph, captured at the first run and replayed afterwards.  The
 * batch copies its tables to the device and owns a workspace for its largest
 * group (groups are cut to fit 32 GiB or half the context's free budget;
 * FTHMS_ENOMEM if one matrix does not fit).  The arcs must outlive the batch.
 * Densities are packed: solve i occupies alpha[off_i, off_i + n_i) with
 * off_i = n_0 + ... + n_{i-1}.  precision and tol as in fthms_solve. */
typedef struct fthms_batch fthms_batch;
int fthms_batch_create(fthms_ctx *ctx, int nb, const fthms_arc *const *arcs,
                       const double *k, const fthms_incident *inc,
                       int precision, double tol, fthms_batch **out);
int fthms_batch_destroy(fthms_batch *batch);

/* total = sum of n_i; offsets[nb] (optional) = off_i. */
int fthms_batch_layout(const fthms_batch *batch, long long *total,
                       long long *offsets);

/* Enqueue the batch on the context's stream: alpha_dev[total] (device),
 * iters_dev[nb] (optional, device) as fthms_solve's iters, -2 for an
 * exactly zero pivot. */
int fthms_batch_run_dev(fthms_batch *batch, fthms_c64 *alpha_dev,
                        int *iters_dev);
/* Host form (synchronous); FTHMS_ESINGULAR if a pivot is exactly zero. */
int fthms_batch_run(fthms_batch *batch, fthms_c64 *alpha, int *iters);

/* Autotuner: for every group, time each launch variant of the batched LU on
 * the batch's own matrices (two half batches on two streams or one launch
 * sequence; register-resident or LDS panel where both apply), reps times
 * each (reps < 1: 2), keep the fastest, and capture a new graph at the next
 * run.  Only the launches change; the register and LDS panels may pick
 * different pivots among exactly tied candidates and round differently. */
int fthms_batch_tune(fthms_batch *batch, int reps);

/* Group structure: *ngroups and, per group (arrays of ngroups entries,
 * optional), its n, number of solves and chosen variant (split: two
 * streams; reg_panel: register-resident panel). */
int fthms_batch_buckets(const fthms_batch *batch, int *ngroups, int *n,
                        int *count, int *split, int *reg_panel);

/* ---- serving -------------------------------------------------------------- */

/* A request: one multiple-scattering problem answered with its time traces
 * (the arguments of fthms_problem_create + fthms_problem_traces in one
 * self-contained record; everything is copied at submission).  narcs
 * patches of n nodes each.  closed == 0: open arcs, xy, dxy [narcs][n][2]
 * samples of x(t), x'(t) at fthms_cheb_nodes(n), interval [narcs][2] and
 * group [narcs] (NULL: one curve) as in fthms_problem_desc.  closed == 1:
 * every patch is a closed obstacle solved as one combined-field patch
 * (Section 3.3, the paper's treatment of closed curves), xy, dxy, ddxy
 * [narcs][n][2] samples of x, x', x'' at tau_j = 2 pi j / n (n even) as in
 * fthms_closed_create; interval and group are ignored.  k, w [nk]
 * frequencies and quadrature weights; obs_xy [nobs][2]; t [nt]; at most
 * max_steps steps with the time-domain stop tolerance stop_tol (decided on
 * the device); precision FTHMS_FP64 or FTHMS_FP32_REFINED (refined to
 * 1e-12). */
typedef struct {
  int narcs;
  int n;
  const double *xy;
  const double *dxy;
  const double *interval;
  const int *group;
  double period;
  int nk;
  const double *k;
  const double *w;
  fthms_incident incident;
  int nobs;
  const double *obs_xy;
  int nt;
  const double *t;
  int max_steps;
  double stop_tol;
  int closed;
  const double *ddxy;
  int precision;
} fthms_request;

enum {
  FTHMS_JOB_QUEUED = 0,
  FTHMS_JOB_RUNNING = 1,
  FTHMS_JOB_DONE = 2,
  FTHMS_JOB_FAILED = 3,
  FTHMS_JOB_CANCELLED = 4
};

/* A server on one GPU: `workers` (1..64) worker threads, each with its own
 * context and stream; requests are admitted first come first served when a
 * worker is free and their device-memory estimate fits beside the running
 * ones within hbm_budget (0: 90% of the free memory).  Admitted requests
 * run concurrently and their kernels overlap on the device; each request's
 * result is independent of the others'. */
typedef struct fthms_server fthms_server;
int fthms_server_create(int device, size_t hbm_budget, int workers,
                        fthms_server **out);
/* Waits for running requests; queued ones are cancelled. */
int fthms_server_destroy(fthms_server *server);
/* Text of the last error on this server (NULL: of the last failed
 * fthms_server_create on this thread); the pointer stays valid until the
 * calling thread's next call of this function. */
const char *fthms_server_error(const fthms_server *server);

/* Queue a request; *ticket identifies it.  FTHMS_ENOMEM if its estimate
 * exceeds the server budget (refused outright), FTHMS_EINVAL(_DATA) for a
 * malformed request. */
int fthms_submit(fthms_server *server, const fthms_request *req,
                 uint64_t *ticket);
/* *state: one of FTHMS_JOB_*. */
int fthms_poll(fthms_server *server, uint64_t ticket, int *state);
/* For a finished request: traces [nt][nobs] (host), steps taken and the
 * latency from submission to the traces being in host memory (seconds);
 * releases the ticket.  FTHMS_EAGAIN while queued or running, the
 * request's error code if it failed, FTHMS_ECANCELLED if cancelled. */
int fthms_fetch(fthms_server *server, uint64_t ticket, fthms_c64 *traces,
                int *steps, double *latency_s);
/* Cancel: a queued request leaves the queue; a running one completes and
 * its result is dropped. */
int fthms_cancel(fthms_server *server, uint64_t ticket);

#ifdef __cplusplus
}
#endif

#endif /* FTHMS_H */
