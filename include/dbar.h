/*
 * dbar.h -- C ABI of the MI355X (gfx950) solver for complex-geometrical-optics (CGO) solutions of D-bar problems,
 * after Klein & McLaughlin, "Spectral approach to D-bar problems" (arXiv 1508.02363).
 *
 * Problem (Section 1, equations eq:038 and eq:039): for a Schwartz potential Q on R^2 and k in C, find m with
 *     dbar m = (1/2) e^{conj(kz) - kz} Q (conj(m) + 1),   m -> 0 as |z| -> infinity,
 * written in Fourier space for S(xi) = xi m^(xi) (equations eq:042 and MainEQa):
 *     A(S) := S + i F( q_k conj(h(S)) ) = -i F(q_k) =: b,      q_k = Q e^{conj(kz) - kz},
 * where h(S) = F^{-1}(S/xi) is evaluated with the regularisation of Section 4.2 (equations Sreg, Gchoice, fourreeg4,
 * fourreg5, fourreg5a, S0Taylor) and A is solved matrix-free by GMRES (Section 4.1) on the real vector
 * [Re S, Im S] (A is real-linear, not complex-linear).  At convergence m = h(S) and m^(1) = i S(0) (equation m1def).
 *
 * Grids (Section 4.1, equations 'domain' and 'xidomain'): N x N points, x_j = y_j = L(-pi + 2 pi j / N), and wave
 * numbers xi = m / L with m in [-N/2+1, N/2].  The transform F is the continuous one of Section 1,
 * F(f)(xi) = (1/2pi) int f e^{-i xi.x}, approximated on the grid by (dx^2/2pi) (-1)^(m1+m2) FFT2 (dx = 2 pi L / N).
 *
 * Array conventions (all complex arrays interleaved re, im, complex128 unless stated):
 *   x-space arrays (Q, m, h): row-major a[iy * N + ix] at (x_ix, y_iy).
 *   xi-space arrays (S):      row-major A[p2 * N + p1] in FFT order: index p means m = p (p <= N/2) or m = p - N,
 *                             xi1 = m(p1)/L, xi2 = m(p2)/L.  Values approximate the continuous S(xi).
 *   Per-k outputs are stacked: entry j of an nk-batch starts at element j * N * N.
 *   k values: interleaved (re, im) pairs, nk of them.
 *
 * Ownership: the caller owns every buffer it passes; the library never keeps a caller pointer after a call returns
 * (the serving queue copies its inputs).  The library owns its device workspace (kept between calls for reuse and
 * released by dbar_release()).  Device pointers must be device memory on the current HIP device.
 *
 * Errors: every entry point returns DBAR_OK (0) or a negative code; dbar_last_error() gives a message (per thread).
 * Calls are not re-entrant on one device from several threads (the workspace is shared); serialise them.
 */
#ifndef DBAR_H
#define DBAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DBAR_OK 0
#define DBAR_EINVAL (-1)   /* bad argument: N not a power of two in [8, 4096], L <= 0, M outside [0, 15], NaN/Inf
                              in Q or k, nk < 1, tol <= 0, NULL where a buffer is required */
#define DBAR_ENOMEM (-2)   /* device memory (or the serving HBM budget) exhausted */
#define DBAR_ENOCONV (-3)  /* GMRES stopped at max_iter before tol for at least one k; outputs are still written and
                              info[j].status tells which */
#define DBAR_EDEVICE (-4)  /* HIP runtime error (no device, launch failure, ...) */
#define DBAR_EAGAIN (-5)   /* serving: result not ready yet */
#define DBAR_ENOTFOUND (-6)/* serving: unknown ticket */

/* Discretisation (Section 4.1 and equation Gchoice): N x N grid on L[-pi, pi)^2, Taylor order M (n = 0..M). */
typedef struct {
  int32_t n;   /* grid points per axis, power of two, 8 <= n <= 4096 */
  int32_t M;   /* Taylor terms n = 0..M of G (the paper uses M = 11); 0 <= M <= 15 */
  double L;    /* domain scale: x, y in L[-pi, pi) */
} dbar_grid;

enum {
  DBAR_FP64 = 0,  /* everything in FP64 */
  DBAR_MIXED = 1, /* FP32 transforms and Krylov basis inside, FP64 residuals, moments, phases, Hessenberg (solve) */
  DBAR_FP32 = 2   /* FP32 transforms (dbar_apply / dbar_transform / dbar_dbar_inverse only) */
};
enum {
  DBAR_MODE_BATCHED = 0, /* many k per launch, device-side convergence flags, HIP graphs */
  DBAR_MODE_PLAIN = 1    /* one k per launch, the host reads the residual after every iteration */
};

typedef struct {
  int32_t restart;     /* Krylov vectors per cycle; default 40 (FP64), 20 (inner FP32 solves); max 64 */
  int32_t max_iter;    /* cap on GMRES iterations per k, all cycles together; default 1000 */
  int32_t precision;   /* DBAR_FP64 or DBAR_MIXED */
  int32_t mode;        /* DBAR_MODE_BATCHED or DBAR_MODE_PLAIN */
  int32_t batch;       /* k values per launch in batched mode; 0 = the tuner's choice for this grid size, else 64, or
                          on grids below N = 512 about 2^24 / N^2 (N = 128: 1024); capped by free device memory */
  int32_t use_graph;   /* batched mode: replay Krylov iterations from captured HIP graphs (1 = on) */
  int32_t reorth;      /* Gram-Schmidt passes: 1 = classical (default), 2 = classical twice.  One pass loses
                          orthogonality to ~1e-3 on this operator but GMRES reaches the same residual in the same
                          number of iterations; the FP64 residual is recomputed at every cycle end regardless. */
  int32_t check_every; /* batched mode: host reads convergence flags every this many iterations (default 4) */
  int32_t method;      /* DBAR_METHOD_PLAIN (Section 4, default) or DBAR_METHOD_ITERATED (Section 5.3: the once-iterated
                          equation eqh2 for h with the regularisation about xi = 2i conj(k), for large |k|; needs
                          2 L Re k and 2 L Im k to be integers, i.e. 2k on the xi grid, else DBAR_EINVAL) */
  int32_t space;       /* the vector GMRES iterates on.  DBAR_SPACE_X (default): s = F^{-1} S (iterated method:
                          F^{-1} h), on which the plain operator is s + i q_k conj(h) and the moments of equation
                          fourreeg4 are plain sums over the grid (three line-transform launches per application
                          instead of five; six instead of ten for the iterated method's B); F is unitary up to a
                          constant, so the Krylov steps and the residual ratio are those of S up to rounding.
                          DBAR_SPACE_XI: S (or h) itself, as written in Sections 4 and 5.3.  With DBAR_MIXED the
                          FP32 rounding of S (relative to S's size) becomes, through the inverse transform, an error
                          floor over the whole x grid, which the moments weight by |z|^n: the xi-space FP32 operator
                          loses accuracy beyond L of about 16 (more cycles from L = 32, no convergence at L = 64); in
                          x-space s itself is rounded, relative to each value, and there is no such limit. */
  double inner_tol;    /* DBAR_MIXED: residual reduction asked of each FP32 inner solve; 0 (default) = 1e-6 in
                          x-space, 1e-5 in xi-space */
  int32_t orth_window; /* plain method in x-space with one Gram-Schmidt pass: each new basis vector is orthogonalised
                          against the last orth_window vectors only (the Hessenberg matrix is then banded above the
                          window and the residual estimate a quasi-residual, which the FP64 residual recomputed at
                          every cycle end checks).  0 = against all of them (classical GMRES).  An entry that a
                          windowed cycle leaves unconverged at the restart length (strong potentials can stall under
                          the window) orthogonalises fully in its later cycles; the other entries of the batch keep
                          the window, so every entry's iterates do not depend on the rest of the batch.  Default set by
                          dbar_default_opts; negative or above the restart length: DBAR_EINVAL.  Other methods and
                          spaces always orthogonalise fully. */
  int32_t lanes;       /* batched mode: batches solved concurrently, each on a stream and workspace of its own (host
                          threads drive them), so that one lane's launches fill the GPU while another waits for its
                          convergence reads or ends a cycle with few entries still active.  With batch > 0 the
                          caller's batch is split into `lanes` equal parts; with batch = 0 each lane takes the
                          library's choice of entries per launch.  0 (default) = 2 when batch >= 16, or, with
                          batch = 0, when there are more k than one batch; else 1.  At most 2 (larger values are
                          taken as 2, negative ones as 0).  With more than one lane the Krylov iterations are
                          launched directly, not from captured graphs (use_graph applies to one lane); the plain
                          mode and, while it is on, the stage timer run one lane.  Every entry's result is the same
                          for any number of lanes. */
} dbar_opts;

enum { DBAR_METHOD_PLAIN = 0, DBAR_METHOD_ITERATED = 1 };
enum { DBAR_SPACE_X = 0, DBAR_SPACE_XI = 1 };

/* Per-k result. */
typedef struct {
  int32_t status;       /* DBAR_OK, or DBAR_ENOCONV (max_iter reached, or a residual that is not finite) */
  int32_t iters;        /* GMRES iterations (operator applications inside Krylov cycles) */
  int32_t outer;        /* FP64 residual evaluations (refinement steps in DBAR_MIXED; restarts + 1 in FP64) */
  int32_t reserved;
  double rel_residual;  /* ||b - A(S)||_2 / ||b||_2, recomputed in FP64 with the FP64 operator at the end */
  double m1_re, m1_im;  /* m^(1) = i S(0), the 1/z coefficient of m (equation m1def); 0 from dbar_reflection and
                           dbar_reconstruct, which do not form S */
  double cond_estimate; /* estimate of the condition number of A from the Krylov iteration: sigma_max / sigma_min of
                           the (upper-triangular factor of the) Hessenberg matrix of the solve's first GMRES cycle
                           (Section 4.1; the cycle from S = 0, normally the longest; serving requests: their longest
                           cycle).  Its singular values lie inside A's, so it estimates cond(A) from below; 0 when no
                           cycle ran (b = 0) */
  double err_estimate;  /* cond_estimate * rel_residual: an estimate (not a bound) of the relative 2-norm error of S
                           against the exact solution of the discrete system, i.e. against an FP64 solve to a tighter
                           tolerance.  Since cond_estimate can fall short of cond(A), so can this */
} dbar_info;
/* With DBAR_METHOD_ITERATED, iters and rel_residual refer to the equation for h (eqh2); S = f + h o (xi + 2i conj k)
 * (equation Sform) and m = F^{-1}(S/xi) is evaluated through the shift theorem. */

/* Fill *opts with the defaults listed above. */
void dbar_default_opts(dbar_opts* opts);

/*
 * Solve A(S) = b for each of nk values of k (host buffers).  Q: N*N complex128 (x-space).  k: nk pairs.
 * tol: stop when ||b - A(S)|| <= tol ||b|| (FP64 residual).  opts may be NULL (defaults).
 * S_out, m_out: nk*N*N complex128 each, or NULL if not wanted.  info: nk entries, or NULL.
 * Q = 0 gives S = 0 and m = 0 without iterating.  Returns DBAR_OK, DBAR_ENOCONV or an error.
 */
int dbar_solve(const dbar_grid* grid, const double* Q, int64_t nk, const double* k, double tol, const dbar_opts* opts,
               double* S_out, double* m_out, dbar_info* info);

/*
 * As dbar_solve, with Q, S_out and m_out in device memory (complex128, same layouts) and all work queued on
 * `stream` (a hipStream_t, NULL = the default stream).  k and info stay host memory.  Returns after the results are
 * complete on the device.
 */
int dbar_solve_device(const dbar_grid* grid, const void* Q_dev, int64_t nk, const double* k, double tol,
                      const dbar_opts* opts, void* S_dev, void* m_dev, dbar_info* info, void* stream);

/*
 * One application of the operator, A(S) = S + i F(q_k conj(h(S))) (Section 4, algorithm step 4, with Q replaced by
 * q_k = Q e^{conj(kz)-kz}, Section 5.1), on host buffers: Q and S_in N*N complex128, k one (re, im) pair,
 * AS_out N*N complex128.  precision: DBAR_FP64 or DBAR_FP32 (inputs rounded to FP32, moments and the closed-form
 * tail in FP64, result widened to FP64).
 */
int dbar_apply(const dbar_grid* grid, const double* Q, const double* k, const double* S_in, double* AS_out,
               int32_t precision);

/*
 * For callers that cannot allocate device memory (work under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): dbar_apply on device buffers, allocating nothing.  Q_dev and S_dev: N*N complex128 device
 * arrays (read only), AS_dev: N*N complex128 device array (written; must not overlap S_dev); k: one (re, im) pair on
 * the host; precision DBAR_FP64 or DBAR_FP32 (as dbar_apply); stream: a hipStream_t (NULL = the default stream).
 * Every intermediate array lives in one static device array of 34 MiB per GPU (held until the process ends), which
 * limits the grid to N <= 1024 (larger N: DBAR_EINVAL); the twiddle tables are a second static array, filled when
 * the library is loaded.  The first call on a device looks up the two arrays' device addresses; every call only
 * queues kernels on `stream` and returns without waiting (no host copies: the calls can be captured into a HIP
 * graph, and a captured graph replays correctly whatever other calls left in the array).  All calls on one GPU share
 * its array, so calls that overlap on one GPU (on
 * different streams, or while an earlier call's work is still running elsewhere) race: serialise them on one stream.
 */
int dbar_apply_noalloc(const dbar_grid* grid, const void* Q_dev, const double* k, const void* S_dev, void* AS_dev,
                       int32_t precision, void* stream);

/*
 * The grid transform consistent with the continuous F of Section 1: inverse = 0 gives
 * out = (dx^2/2pi) (-1)^(m1+m2) FFT2(in) (x-space in, xi-space out); inverse = 1 gives
 * out = (1/(2 pi L^2)) sum_m (-1)^(m1+m2) in_m e^{+2 pi i m.j/N} (xi-space in, x-space out).  Host buffers,
 * N*N complex128 each; precision DBAR_FP64 or DBAR_FP32.
 */
int dbar_transform(const dbar_grid* grid, int32_t inverse, const double* in, double* out, int32_t precision);

/*
 * The regularised inverse h(S) = F^{-1}(S/xi) of Section 4.2 (equations Sreg, Gchoice, fourreeg4, S0Taylor):
 * h = F^{-1}((S - G)/xi) + sum_n c_n W_n with the value at xi = 0 taken as the limit dS/dxi(0).  Since
 * F(dbar u) = (i/2) xi F(u), this is (i/2) dbar^{-1} F^{-1}(S).  Host buffers, N*N complex128 each.
 */
int dbar_dbar_inverse(const dbar_grid* grid, const double* S_in, double* h_out, int32_t precision);

/* ------------------------------------------------------------------------------------------------------------
 * Tuning.  Not in the paper: the column passes of the 2D transforms (the y-direction lines of the three FFTs of
 * the Section 4 algorithm) run on tiles of adjacent columns whose best width depends on the grid size and
 * precision, and the batched solver's entries per launch trade throughput against memory.  The choices are kept
 * per process and device-independent; they apply to every later solve, apply and session launch.  Do not call
 * these while another thread is inside a solve or while a serving session is running.
 * ------------------------------------------------------------------------------------------------------------ */
typedef struct {
  int32_t n_variants[2];    /* [0]: FP64 operator, [1]: FP32 operator; 0 if that operator was not tuned */
  int32_t chosen[2];        /* the variant kept */
  int32_t columns[2][4];    /* columns per tile of each variant */
  double ms[2][4];          /* one operator application over `batch` entries, per variant (milliseconds) */
  int32_t batch;            /* entries per launch kept for solves with opts->batch = 0 */
  int32_t batch_candidates[4];
  int32_t reserved;
  double per_entry_ms[4];   /* operator time per entry at each candidate batch size */
} dbar_tune_result;

/*
 * Time one operator application (A(S), FP64 and/or FP32 as `precision` says: DBAR_FP64, DBAR_MIXED (both) or
 * DBAR_FP32) over `batch` entries (1..1024) for every column-tile width valid at this grid size, keep the fastest,
 * then keep the smallest batch size (of batch, batch/2, batch/4, batch/8) whose per-entry time is within 5% of
 * the best.  out may be NULL.  Uses the library's workspace (device memory for `batch` entries).
 */
int dbar_autotune(const dbar_grid* grid, int32_t precision, int32_t batch, dbar_tune_result* out);
/* Force the column-tile variant of grid size n for the FP64 or FP32 operator (precision DBAR_FP64 / DBAR_FP32). */
int dbar_set_tile(int32_t n, int32_t precision, int32_t variant);
/* Current variant, its columns per tile and the number of variants for grid size n (any output may be NULL). */
int dbar_get_tile(int32_t n, int32_t precision, int32_t* variant, int32_t* columns, int32_t* variants);

/* ------------------------------------------------------------------------------------------------------------
 * DS II scattering transforms (Section 6).  Both run the iterated solver (Section 5.3) in FP64 or DBAR_MIXED as
 * opts->precision says (opts->method is ignored), batched over their many independent solves.
 * ------------------------------------------------------------------------------------------------------------ */

/*
 * Reflection coefficient r(k) = i h(i conj k) (equation rviah) of the potential q, in the Section 6 convention
 * (k replaced by k/2, so that k and xi are dual variables on the same grid): h solves the iterated equation for q
 * with spectral parameter k/2, and h(i conj k) is its value at the shift offset (L Im k, L Re k).  Equivalently
 * r = (M1^(1) - M2^(1))/2 for the CGO solutions M1, M2 of equations eq:021 and eq:022 (equation eq:023).
 * q: host N*N complex128 (x-space).  k: nk (re, im) pairs, each on the xi grid (L Re k and L Im k integers, else
 * DBAR_EINVAL).  r_out: nk complex128.  info: nk entries or NULL (iters and rel_residual of each solve for h).
 * Returns DBAR_OK, DBAR_ENOCONV (r_out still written) or an error.
 */
int dbar_reflection(const dbar_grid* grid, const double* q, int64_t nk, const double* k, double tol,
                    const dbar_opts* opts, double* r_out, dbar_info* info);

/*
 * Reconstruction of the potential q(x, y, t) from the reflection coefficient at t = 0 (equations dbarrecA,
 * dbarrecB, qRec, with r(k, t) = r(k, 0) exp(-i t Re(k^2)/2), equation rt in the Section 6 convention): the D-bar
 * problem of dbar_reflection with z and k interchanged and q replaced by conj(r(k, t)).  r: host N*N complex128 on
 * the xi grid of `grid`, laid out like S (r[p2 * N + p1] = r(k), k = xi of that index; the row and column of the
 * Nyquist wave number N/(2L) are taken as their periodic images at -N/(2L)).  q_out: host N*N complex128 on the x
 * grid of `grid`.  The problem is solved on the dual grid (N, M, L' = N/(2 pi L)), whose xi grid holds the x grid
 * of `grid`; it takes N*N solves (one per z).  info: N*N entries (row-major over z) or NULL.
 * Returns DBAR_OK, DBAR_ENOCONV (q_out still written) or an error.
 */
int dbar_reconstruct(const dbar_grid* grid, const double* r, double t, double tol, const dbar_opts* opts,
                     double* q_out, dbar_info* info);

/* ------------------------------------------------------------------------------------------------------------
 * Serving: a request queue with continuous batching.  Requests (one k, one Q, one grid each) are admitted into
 * device-resident slots when the HBM budget allows, advance together in per-grid-size batches of Krylov
 * iterations, and leave as soon as they converge; new requests take the freed slots at the next iteration
 * boundary.  A worker thread per grid class drives the device.  All solves use DBAR_MIXED precision to the
 * requested tolerance (FP64 residual), or DBAR_FP64 if asked.
 * Admission by HBM footprint (dbar_request_footprint): a grid class reserves up to max_slots footprints of the
 * budget when its first request arrives.  A request whose class cannot be reserved yet waits (first in, first out,
 * with every later request behind it); a class that runs idle while requests wait releases its workspace.  Only a
 * request whose footprint exceeds the whole budget is rejected (DBAR_ENOMEM from dbar_submit).  A result does not
 * depend on which other requests share its batch.
 * ------------------------------------------------------------------------------------------------------------ */
typedef struct dbar_session dbar_session;

typedef struct {
  size_t hbm_budget_bytes;  /* admission limit on the sum of request footprints (0 = 80% of free device memory) */
  int32_t max_slots;        /* max requests in flight per grid size (default 64) */
  int32_t precision;        /* DBAR_MIXED (default) or DBAR_FP64 */
  int32_t restart;          /* inner Krylov vectors (default 20) */
  int32_t reserved;
} dbar_session_opts;

typedef struct {
  uint64_t submitted, completed, rejected;  /* rejected: footprint above the whole budget */
  uint64_t in_flight, queued;                /* queued: submitted, not yet in a slot (pending included) */
  size_t bytes_in_use;                       /* footprints of the requests in flight */
  size_t bytes_reserved;                     /* workspaces reserved by the grid classes alive */
  uint64_t classes_created, classes_released;
} dbar_session_stats;

/* Create a session (opts may be NULL). */
int dbar_session_create(const dbar_session_opts* opts, dbar_session** out);
/* Queue one solve.  Q: host N*N complex128 (copied before return), k one (re, im) pair.  *ticket identifies it. */
int dbar_submit(dbar_session* s, const dbar_grid* grid, const double* Q, const double* k, double tol,
                uint64_t* ticket);
/* Fetch a finished solve: S_out / m_out host N*N complex128 (or NULL), info, and latency_s = seconds from
 * dbar_submit to the result being on the host (or NULL).  DBAR_EAGAIN while it runs.  A ticket can be fetched
 * once; afterwards it is unknown (DBAR_ENOTFOUND).  Returns DBAR_OK, DBAR_ENOCONV (max_iter reached) or an error. */
int dbar_poll(dbar_session* s, uint64_t ticket, double* S_out, double* m_out, dbar_info* info, double* latency_s);
/* As dbar_poll but blocks until the result is ready. */
int dbar_wait(dbar_session* s, uint64_t ticket, double* S_out, double* m_out, dbar_info* info, double* latency_s);
int dbar_session_get_stats(dbar_session* s, dbar_session_stats* st);
/* Bytes of device memory a request of this grid would hold while in flight. */
size_t dbar_request_footprint(const dbar_grid* grid, int32_t precision, int32_t restart);
/* Stop the worker (pending requests are abandoned) and free everything. */
void dbar_session_destroy(dbar_session* s);

/* ------------------------------------------------------------------------------------------------------------
 * Measurement.  The paper puts the cost of the method in the 2D FFTs of the GMRES iterations (remark after the
 * Section 4 algorithm: three 2D transforms per iteration).  These calls time every kernel launch of the library with
 * HIP events on the stream it is launched on, grouped by stage, and add up the algorithmic HBM bytes of each launch
 * (every array the stage must read or write counted once, for the batch entries active in that launch).
 * ------------------------------------------------------------------------------------------------------------ */
/* on = 1: clear and start recording; on = 0: stop (waits for the device and folds the records into the totals). */
int dbar_timer_enable(int32_t on);
/* Number of stage slots (valid stage indices are 0 .. n-1; unused ones report zero launches). */
int dbar_timer_num_stages(void);
/* Totals of one stage: its name (NUL-terminated, truncated to name_len), summed launch time in milliseconds,
 * number of launches and algorithmic bytes.  Any output pointer may be NULL. */
int dbar_timer_stage(int32_t stage, char* name, int32_t name_len, double* total_ms, int64_t* launches, double* bytes);

/* ------------------------------------------------------------------------------------------------------------ */
/* Message of the last error on this thread ("" if none). */
const char* dbar_last_error(void);
/* Free the cached device workspace of the one-shot calls (the solvers' workspaces and streams, and the twiddle
 * tables); it waits for a one-shot call running in another thread to return.  Serving sessions hold workspaces and
 * tables of their own and keep running; the allocation-free entry point keeps its static arrays. */
void dbar_release(void);
/* Library version, e.g. 100 for 0.1.0. */
int dbar_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DBAR_H */
