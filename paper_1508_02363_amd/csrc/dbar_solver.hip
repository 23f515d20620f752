// Host side of the D-bar solver: plans, workspace, the operator pipeline, device-resident GMRES and the C ABI.
//
// GMRES (Saad & Schultz) on the real 2N^2 form, restarted, x0 = 0, classical Gram-Schmidt (optionally twice),
// Givens rotations.  The Krylov basis is kept unnormalised: v_{j+1} is the orthogonalised A v_j written in place and
// q_j = sigma_j v_j with sigma_j = 1/||v_j|| (so no separate normalisation pass over memory).  All bookkeeping
// (Hessenberg, rotations, residual estimate, convergence flags) lives on the device, one record per batch entry;
// entries advance in lockstep and converged ones are masked out of every kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <cstring>
#include <map>
#include <memory>
#include <atomic>
#include <mutex>
#include <new>
#include <thread>
#include <string>
#include <vector>

#include "dbar.h"
#include "dbar_launch.h"
#include "dbar_solver.h"

namespace dbar {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// ------------------------------------------------------------------------------------------------------------
// Control kernels (one thread per batch entry)
// ------------------------------------------------------------------------------------------------------------
static __constant__ double kInvFactC[kMaxM + 2] = {
    1.0, 1.0, 5.0e-1, 1.6666666666666666e-1, 4.1666666666666664e-2, 8.3333333333333332e-3,
    1.3888888888888889e-3, 1.9841269841269841e-4, 2.4801587301587302e-5, 2.7557319223985893e-6,
    2.7557319223985888e-7, 2.5052108385441720e-8, 2.0876756987868100e-9, 1.6059043836821613e-10,
    1.1470745597729725e-11, 7.6471637318198164e-13, 4.7794773323873853e-14};

DBAR_D double wsum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}


// Deterministic block reduction of one entry's partials: red[v] = sum_blk part[v * nblk + blk] for v < nval
// (wave w sums the values v = w, w + NW, ...; lanes stride over the partials).  1024 threads.
constexpr int kCtlThreads = 1024;
// Values v >= nv1 come from part2 (v - nv1 of it, same nblk) when part2 is given.
template <int NT = kCtlThreads>
DBAR_D void reduce_entry(const double* __restrict__ part, int nval, int nblk, double* red,
                         const double* __restrict__ part2 = nullptr, int nv1 = 0) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int v = wave; v < nval; v += NW) {
    const double* p = (part2 && v >= nv1) ? part2 + (size_t)(v - nv1) * nblk : part + (size_t)v * nblk;
    // eight independent partial sums per lane: the loads of a chunk are in flight together
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int i = lane;
    for (; i + 7 * 64 < nblk; i += 8 * 64) {
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] += p[i + u * 64];
    }
    for (; i < nblk; i += 64) a[0] += p[i];
    double acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    acc = wsum(acc);
    if (lane == 0) red[v] = acc;
  }
  __syncthreads();
}

// d_n = w sum_tiles part, c_n = (-i/2)^n d_n / n! (equation fourreeg4 with Gchoice), R(0) = (-i/2) dt, for entry b,
// from the reduced tile sums tot: thread n < kNMom forms slot n ((-i/2)^n = (-i)^n 2^-n exactly).
DBAR_D void moments_combine(int b, const double* tot, double wscale, int M, c64* coefG, c64* dmom, c32* dmom32) {
  const int n = threadIdx.x;
  if (n >= kNMom) return;
  const c64 d{wscale * tot[2 * n], wscale * tot[2 * n + 1]};
  c64* cg = coefG + (size_t)b * kNMom;
  c64* dm = dmom + (size_t)b * kNMom;
  c32* dm32 = dmom32 + (size_t)b * kNMom;
  if (n == kMaxM + 1) {  // the conj(z) moment: R(0) = (-i/2) dt
    cg[n] = c64{0.0, -0.5} * d;
    dm[n] = d;
    dm32[n] = cvt<float>(d);
    return;
  }
  const double s = ldexp(1.0, -n);
  const c64 p = (n & 3) == 0 ? c64{s, 0.0} : (n & 3) == 1 ? c64{0.0, -s} : (n & 3) == 2 ? c64{-s, 0.0} : c64{0.0, s};
  dm[n] = n <= M ? d : c64{0.0, 0.0};
  dm32[n] = cvt<float>(dm[n]);
  cg[n] = n <= M ? kInvFactC[n] * (p * d) : c64{0.0, 0.0};
}

// All kCtlThreads threads of the block.
DBAR_D void moments_entry(int b, const double* part, int ntiles, double wscale, int M, c64* coefG, c64* dmom,
                          c32* dmom32) {
  constexpr int NV = 2 * kNMom;
  __shared__ double tot[NV];
  reduce_entry(part + (size_t)b * NV * ntiles, NV, ntiles, tot);
  moments_combine(b, tot, wscale, M, coefG, dmom, dmom32);
}

// One block of kCtlThreads per entry.
__global__ void __launch_bounds__(kCtlThreads) k_moments(const double* part, int ntiles, const int* act,
                                                         double wscale, int M, c64* coefG, c64* dmom, c32* dmom32) {
  const int b = blockIdx.x;
  if (act && !act[b]) return;
  moments_entry(b, part, ntiles, wscale, M, coefG, dmom, dmom32);
}

// Column j of the Hessenberg matrix from hsum and beta = ||v_{j+1}|| (unnormalised basis: column j is sigma_j times the
// products of A v_j), the previous Givens rotations applied, the new rotation, g and the residual estimate |g_{j+1}|.
DBAR_D void givens_commit(Ctl& c, int j, double beta) {
  const double sj = c.sigma[j];
  double* col = c.H + (size_t)j * (kMaxRestart + 1);
  for (int i = 0; i <= j; ++i) col[i] = sj * c.hsum[i];
  col[j + 1] = sj * beta;
  c.sigma[j + 1] = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int i = 0; i < j; ++i) {
    const double t = c.cs[i] * col[i] + c.sn[i] * col[i + 1];
    col[i + 1] = -c.sn[i] * col[i] + c.cs[i] * col[i + 1];
    col[i] = t;
  }
  const double den = hypot(col[j], col[j + 1]);
  c.cs[j] = den > 0.0 ? col[j] / den : 1.0;
  c.sn[j] = den > 0.0 ? col[j + 1] / den : 0.0;
  col[j] = den;
  col[j + 1] = 0.0;
  c.g[j + 1] = -c.sn[j] * c.g[j];
  c.g[j] = c.cs[j] * c.g[j];
  c.resid = fabs(c.g[j + 1]);
  c.jn = j + 1;
  c.iters += 1;
}

// Gram-Schmidt pass `pass` of step j: h_i = <v_i, w> from the partials, coef_i = sigma_i^2 h_i (the basis is kept
// unnormalised, v_i / ||v_i|| = sigma_i v_i), hsum_i accumulates sigma_i h_i over the passes.  One block per entry.
// early (one pass, value j + 1 of the partials = ||w||^2): the step's convergence is decided here, before the update
// that forms v_{j+1} runs.  With one classical pass v_{j+1} = w - sum_i hsum_i q_i (q_i = sigma_i v_i orthonormal), so
// ||v_{j+1}||^2 = ||w||^2 - sum_i hsum_i^2; where that difference keeps at least 1e-4 of ||w||^2 (the FP64 sums of
// products then fix beta to about 1e-3 relative or better), the rotation it implies gives the residual estimate, and
// an entry that meets its threshold (or the restart length) takes its last Givens step with this beta and leaves the
// cycle: the update, transform and moments of a v_{j+1} no step would use are not run for it.  Otherwise the step
// waits for the exact norm from the update, as without `early`.
// The partials cover the vectors lo..j; an entry whose own window starts later (full[b] == 0 with skip > 0: the launch
// covers the whole basis for entries that orthogonalise fully) takes the vectors lo + skip..j only.
// NT threads per entry: 256 while the step has at most 4 values (a windowed step), 1024 otherwise (a smaller block
// starts sooner when another stream's line kernels hold most of every CU; the sums are the same either way)
template <int NT>
__global__ void __launch_bounds__(NT) k_ctl_coef(Ctl* ctl, const double* part, int nval, int nblk, int* act, int j,
                                                 int pass, int early, int m, int lo, int skip, const int* full) {
  const int b = blockIdx.x;
  if (!act[b]) return;
  __shared__ double red[kMaxRestart + 2];
  reduce_entry<NT>(part + (size_t)b * nval * nblk, nval, nblk, red);
  if (threadIdx.x == 0) {
    Ctl& c = ctl[b];
    double p2 = 0.0;
    const int lob = lo + ((full && !full[b]) ? skip : 0);
    for (int i = 0; i < lob; ++i) c.coef[i] = c.hsum[i] = 0.0;  // outside the window (one pass)
    for (int i = lob; i <= j; ++i) {
      const double h = red[i - lo];
      c.coef[i] = c.sigma[i] * c.sigma[i] * h;
      c.hsum[i] = (pass ? c.hsum[i] : 0.0) + c.sigma[i] * h;
      p2 += c.hsum[i] * c.hsum[i];
    }
    if (early) {
      const double wn2 = red[j - lo + 1], b2 = wn2 - p2;
      if (b2 > 1e-4 * wn2) {
        const double beta = sqrt(b2), sj = c.sigma[j];
        // column j's last entry after the previous rotations, without touching the record
        double top = sj * c.hsum[0];
        for (int i = 0; i < j; ++i) top = -c.sn[i] * top + c.cs[i] * (sj * c.hsum[i + 1]);
        const double sub = sj * beta, den = hypot(top, sub);
        const double resid = den > 0.0 ? fabs(sub / den * c.g[j]) : 0.0;
        if (resid <= c.thresh || j + 1 >= m) {
          givens_commit(c, j, beta);
          act[b] = 0;
          if (resid > c.thresh) act[gridDim.x + b] = 1;  // stopped by the restart length
        }
      }
    }
  }
}

// Column j of the Hessenberg matrix from hsum and beta = ||w_new|| (reduced from the update's partials), Givens
// rotation, residual estimate; the entry leaves the cycle when the estimate meets its threshold.  All kCtlThreads
// threads of entry b's block.
DBAR_D void givens_entry(int b, Ctl* ctl, const double* pnorm, int nblk, int* act, int j, int m) {
  __shared__ double red[1];
  reduce_entry(pnorm + (size_t)b * nblk, 1, nblk, red);
  if (threadIdx.x != 0) return;
  Ctl& c = ctl[b];
  const double beta = sqrt(fmax(red[0], 0.0));
  givens_commit(c, j, beta);
  if (c.resid <= c.thresh || j + 1 >= m || beta == 0.0) act[b] = 0;
  if (c.resid > c.thresh && j + 1 >= m && beta != 0.0) act[gridDim.x + b] = 1;  // stopped by the restart length
}

__global__ void __launch_bounds__(kCtlThreads) k_ctl_givens(Ctl* ctl, const double* pnorm, int nblk, int* act, int j,
                                                            int m) {
  const int b = blockIdx.x;
  if (!act[b]) return;
  givens_entry(b, ctl, pnorm, nblk, act, j, m);
}

// The moments of the next basis vector (whose update and transform just ran) and the Givens step of the Krylov step
// that produced it, in one launch: the moments are used only if the entry stays active.
// 512 threads (a windowed step's moment sums take three rounds of its eight waves): a block of half a CU starts sooner
// than one of kCtlThreads beside another stream's line kernels (same sums; measured 0.6% off the two-lane step)
constexpr int kMomGivensThreads = 512;
__global__ void __launch_bounds__(kMomGivensThreads) k_moments_givens(const double* part, int ntiles, double wscale,
                                                                      int M,
                                                                c64* coefG, c64* dmom, c32* dmom32, Ctl* ctl,
                                                                const double* pnorm, int nblk, int* act, int j,
                                                                int m) {
  const int b = blockIdx.x;
  if (!act[b]) return;
  constexpr int NV = 2 * kNMom;
  __shared__ double tot[NV + 1];  // the moment sums, then |v_{j+1}|^2
  reduce_entry<kMomGivensThreads>(part + (size_t)b * NV * ntiles, NV + 1, ntiles, tot, pnorm + (size_t)b * nblk, NV);
  moments_combine(b, tot, wscale, M, coefG, dmom, dmom32);  // wave 0
  if (threadIdx.x == 64) {                                   // wave 1
    Ctl& c = ctl[b];
    const double beta = sqrt(fmax(tot[NV], 0.0));
    givens_commit(c, j, beta);
    if (c.resid <= c.thresh || j + 1 >= m || beta == 0.0) act[b] = 0;
    if (c.resid > c.thresh && j + 1 >= m && beta != 0.0) act[gridDim.x + b] = 1;  // stopped by the restart length
  }
}

// y = H^{-1} g (upper triangular jn x jn), coef_i = y_i sigma_i, zero beyond jn
// One block of 64 threads per entry: the factor's columns and g are staged in LDS by all lanes (their loads in
// flight together), then one thread runs the substitution on LDS values (the serial chain no longer waits on global
// memory for each term; same operations in the same order), and the lanes write the coefficients out.
__global__ void __launch_bounds__(64) k_ctl_trisolve(Ctl* ctl, const int* live, int B) {
  const int b = blockIdx.x;
  if (b >= B || !live[b]) return;
  Ctl& c = ctl[b];
  const int n = c.jn;
  const int i0 = threadIdx.x;
  constexpr int LD = kMaxRestart + 1;
  __shared__ double Hs[kMaxRestart * LD];
  __shared__ double y[kMaxRestart + 1];
  const double* Hc = c.H;
#pragma unroll 8
  for (int t = i0; t < n * LD; t += 64) Hs[t] = Hc[t];
  for (int t = i0; t < n; t += 64) y[t] = c.g[t];
  __syncthreads();
  if (i0 == 0) {
    for (int i = n - 1; i >= 0; --i) {
      double s = y[i];
      for (int l = i + 1; l < n; ++l) s -= Hs[l * LD + i] * y[l];
      const double d = Hs[i * LD + i];
      y[i] = d != 0.0 ? s / d : 0.0;
    }
  }
  __syncthreads();
  for (int t = i0; t <= kMaxRestart; t += 64) c.coef[t] = t < n ? y[t] * c.sigma[t] : 0.0;
}

// Condition estimate of one entry (one wave per entry): the extreme singular values of the upper-triangular factor R
// (jn x jn, column j in H[j * (kMaxRestart + 1)]) that the Givens rotations leave of the cycle's Hessenberg matrix --
// the same singular values as the (jn + 1) x jn Hessenberg matrix, and those lie inside A's (sigma_max(H) <= sigma_max(A),
// sigma_min(H) >= sigma_min(A)), so the ratio estimates cond(A) from below.  Power iteration on R^T R for sigma_max and
// inverse iteration (a forward and a back substitution per step) for sigma_min, lane i holding component i.  Taken only
// when the cycle is longer than the one behind the current estimate (the longest cycle has seen most of the spectrum).
constexpr int kCondIters = 12;
__global__ void __launch_bounds__(64) k_cond_estimate(Ctl* ctl, const int* live) {
  const int b = blockIdx.x;
  if (live && !live[b]) return;
  Ctl& c = ctl[b];
  const int n = c.jn;
  if (n <= c.kappa_n || n < 1) return;
  const int i = threadIdx.x;
  constexpr int LD = kMaxRestart + 1;
  // the n x n factor staged in LDS once: the iterations below read it many times.  The columns' n LD values are read
  // as one flat range, eight loads per thread in flight at a time (column by column, each read waited for its own
  // load before the next was issued); the entries below the diagonal are never read.
  __shared__ double Rs[kMaxRestart * LD];
  const double* Hc = c.H;
#pragma unroll 8
  for (int t = i; t < n * LD; t += 64) Rs[t] = Hc[t];
  __syncthreads();
  auto R = [&](int row, int col) { return Rs[col * LD + row]; };
  for (int l = 0; l < n; ++l)
    if (!(R(l, l) != 0.0)) return;  // breakdown (exact solution reached): keep the previous estimate
  // reciprocals of the diagonal, once: the substitutions below multiply instead of dividing on their serial chain
  __shared__ double Dinv[kMaxRestart];
  if (i < n) Dinv[i] = 1.0 / R(i, i);
  __syncthreads();
  // sigma_max: x <- R^T R x, normalised
  double x = i < n ? 1.0 + 0.01 * i : 0.0;
  double nrm = sqrt(wsum(x * x));
  x /= nrm;
  double smax2 = 0.0;
  for (int it = 0; it < kCondIters; ++it) {
    double y = 0.0;  // (R x)_i = sum_{l >= i} R_il x_l
    for (int l = 0; l < n; ++l) {
      const double xl = __shfl(x, l, 64);
      if (i < n && l >= i) y += R(i, l) * xl;
    }
    double z = 0.0;  // (R^T y)_i = sum_{l <= i} R_li y_l
    for (int l = 0; l < n; ++l) {
      const double yl = __shfl(y, l, 64);
      if (i < n && l <= i) z += R(l, i) * yl;
    }
    smax2 = sqrt(wsum(z * z));  // |R^T R x| for |x| = 1
    x = smax2 > 0.0 ? z / smax2 : 0.0;
  }
  // sigma_min: x <- (R^T R)^{-1} x = R^{-1} R^{-T} x, normalised
  x = i < n ? 1.0 + 0.01 * i : 0.0;
  nrm = sqrt(wsum(x * x));
  x /= nrm;
  double inv2 = 0.0;
  for (int it = 0; it < kCondIters; ++it) {
    double r = x, u = 0.0;  // R^T u = x (forward substitution, column by column)
    for (int l = 0; l < n; ++l) {
      const double ul = __shfl(r, l, 64) * Dinv[l];
      if (i == l) u = ul;
      if (i > l && i < n) r -= R(l, i) * ul;
    }
    r = u;
    double v = 0.0;  // R v = u (back substitution)
    for (int l = n - 1; l >= 0; --l) {
      const double vl = __shfl(r, l, 64) * Dinv[l];
      if (i == l) v = vl;
      if (i < l) r -= R(i, l) * vl;
    }
    inv2 = sqrt(wsum(v * v));  // |(R^T R)^{-1} x| for |x| = 1
    x = inv2 > 0.0 ? v / inv2 : 0.0;
  }
  if (i == 0 && smax2 > 0.0 && inv2 > 0.0) {
    c.kappa = fmax(c.kappa, sqrt(smax2 * inv2));
    c.kappa_n = n;
  }
}

// start a Krylov cycle from the residual whose squared norm is nred[b] (already stored as v_0)
__global__ void k_ctl_start(Ctl* ctl, const double* nred, const int* live, int* act, double abs_tol, double rel_tol,
                            const double* tolv, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  Ctl& c = ctl[b];
  // an entry whose last cycle ended at the restart length orthogonalises fully from now on (read only by windowed
  // cycles); the flag is set by the Givens step when the restart length, not the threshold, ends the entry's cycle
  if (act[B + b]) act[2 * B + b] = 1;
  act[B + b] = 0;
  if (!live[b]) {
    act[b] = 0;
    return;
  }
  const double rn = sqrt(fmax(nred[b], 0.0));
  // abs_tol is a fraction of the entry's tolerance (tolv[b], or 1 when tolv is NULL and abs_tol carries it)
  const double at = tolv ? abs_tol * tolv[b] : abs_tol;
  c.rnorm = rn;
  c.sigma[0] = rn > 0.0 ? 1.0 / rn : 0.0;
  c.g[0] = rn;
  c.thresh = fmax(at * c.bnorm, rel_tol * rn);
  c.jn = 0;
  act[b] = rn > c.thresh ? 1 : 0;
}

// after a recomputed residual: done when ||r|| <= tol ||b||
__global__ void k_ctl_check(Ctl* ctl, const double* nred, int* live, int* act, double tol, int first,
                            const int* mask, const double* tolv, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B || (!first && !live[b]) || (mask && !mask[b])) return;
  Ctl& c = ctl[b];
  // (a sum of squares: no clamp, so that a residual that is not finite stays NaN and never counts as converged)
  const double rn = sqrt(nred[b]);
  if (first) {
    c.bnorm = rn;
    c.iters = 0;
    c.cycles = 0;
    c.jn = 0;
    c.kappa = 0.0;
    c.kappa_n = 0;
    act[B + b] = 0;
    act[2 * B + b] = 0;  // a new solve starts with the Gram-Schmidt window
  }
  c.rnorm = rn;
  c.cycles += 1;
  const double t = tolv ? tolv[b] : tol;
  if (rn <= t * c.bnorm) live[b] = 0;
}

// e^{conj(kz) - kz} = e^{-2i k2 x} e^{-2i k1 y} (eq:039) as two FP64 tables per entry, x_j = L(-pi + 2 pi j / N)
__global__ void k_phase_tables(const c64* kv, int N, double L, c64* ex, c64* ey, c32* ex32, c32* ey32, int B) {
  const int b = blockIdx.y;
  if (b >= B) return;
  const c64 k = kv[b];
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N; j += gridDim.x * blockDim.x) {
    const double x = L * (-kPi + (2.0 * kPi / N) * j);
    double s1, c1, s2, c2;
    sincos(-2.0 * k.im * x, &s1, &c1);
    sincos(-2.0 * k.re * x, &s2, &c2);
    ex[(size_t)b * N + j] = c64{c1, s1};
    ey[(size_t)b * N + j] = c64{c2, s2};
    ex32[(size_t)b * N + j] = c32{(float)c1, (float)s1};
    ey32[(size_t)b * N + j] = c32{(float)c2, (float)s2};
  }
}

// compact per-entry results: iterations, residual evaluations, ||b||, ||r||, S(0), and with shifts (iterated
// method) h at the shift offset (m1, m2) = (2 k2 L, 2 k1 L), i.e. h(xi = 2i conj k)
__global__ void k_gather_results(const Ctl* ctl, const c64* x, size_t n, const c64* h, const int* shv, int N,
                                 EntryResult* out, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const Ctl& c = ctl[b];
  c64 hs{0.0, 0.0};
  if (shv) {
    const int p1 = ((shv[2 * b] % N) + N) % N, p2 = ((shv[2 * b + 1] % N) + N) % N;
    hs = h[(size_t)b * n + (size_t)p2 * N + p1];
  }
  out[b] = EntryResult{c.iters, c.cycles, c.bnorm, c.rnorm, x[(size_t)b * n], hs, c.kappa};
}

void launch_phase_tables(const c64* kv_dev, int N, double L, c64* ex, c64* ey, c32* ex32, c32* ey32, int B,
                         hipStream_t s) {
  TimerScope ts(kStageControl, 0.0, B, nullptr, s);
  hipLaunchKernelGGL(k_phase_tables, dim3((N + 255) / 256, B), dim3(256), 0, s, kv_dev, N, L, ex, ey, ex32, ey32, B);
}

// ------------------------------------------------------------------------------------------------------------
// Plans and workspace
// ------------------------------------------------------------------------------------------------------------
DevBuf::~DevBuf() {
  if (p) (void)hipFree(p);
}
int DevBuf::ensure(size_t nbytes) {
  if (nbytes <= bytes) return DBAR_OK;
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
  if (nbytes == 0) return DBAR_OK;
  hipError_t e = hipMalloc(&p, nbytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
    return fail(DBAR_ENOMEM, "hipMalloc(" + std::to_string(nbytes) + " bytes) failed: " + hipGetErrorString(e));
  }
  bytes = nbytes;
  return DBAR_OK;
}

PinnedInts::~PinnedInts() {
  if (p) (void)hipHostFree(p);
}
int PinnedInts::ensure(size_t n) {
  if (n <= count) return DBAR_OK;
  if (p) (void)hipHostFree(p);
  p = nullptr;
  count = 0;
  if (hipHostMalloc(reinterpret_cast<void**>(&p), n * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
    return fail(DBAR_ENOMEM, "hipHostMalloc failed");
  }
  count = n;
  return DBAR_OK;
}

static std::mutex g_mutex;      // serialises the one-shot C-ABI calls (shared workspace)
static std::mutex g_tw_mutex;   // twiddle cache (also used by the serving workers)
static std::map<int, std::unique_ptr<Twiddles>> g_twiddles;

void host_twiddles(int N, c64* out64, c32* out32) {
  for (int j = 0; j < N; ++j) {
    const long double a = -2.0L * 3.14159265358979323846264338327950288L * j / N;
    out64[j] = c64{(double)cosl(a), (double)sinl(a)};
    out32[j] = c32{(float)cosl(a), (float)sinl(a)};
  }
}

// exp(-2 pi i j / N) in long double, rounded once
int get_twiddles(int N, const void** d64, const void** d32) {
  std::lock_guard<std::mutex> lock(g_tw_mutex);
  auto it = g_twiddles.find(N);
  if (it == g_twiddles.end()) {
    auto t = std::make_unique<Twiddles>();
    std::vector<c64> h64(N);
    std::vector<c32> h32(N);
    host_twiddles(N, h64.data(), h32.data());
    int rc = t->d64.ensure(N * sizeof(c64));
    if (rc) return rc;
    rc = t->d32.ensure(N * sizeof(c32));
    if (rc) return rc;
    if (hipMemcpy(t->d64.p, h64.data(), N * sizeof(c64), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(t->d32.p, h32.data(), N * sizeof(c32), hipMemcpyHostToDevice) != hipSuccess)
      return fail(DBAR_EDEVICE, "twiddle upload failed");
    it = g_twiddles.emplace(N, std::move(t)).first;
  }
  *d64 = it->second->d64.p;
  *d32 = it->second->d32.p;
  return DBAR_OK;
}

int validate_grid(const dbar_grid* g) {
  if (!g) return fail(DBAR_EINVAL, "grid is NULL");
  const int N = g->n;
  if (N < 8 || N > 4096 || (N & (N - 1)) != 0)
    return fail(DBAR_EINVAL, "grid n must be a power of two in [8, 4096], got " + std::to_string(N));
  if (!(g->L > 0.0) || !std::isfinite(g->L)) return fail(DBAR_EINVAL, "grid L must be finite and > 0");
  if (g->M < 0 || g->M > kMaxM) return fail(DBAR_EINVAL, "grid M must be in [0, 15]");
  return DBAR_OK;
}


void Work::drop_graphs() {
  for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
  graphs.clear();
}
Work::~Work() { drop_graphs(); }
Work& Work::operator=(Work&& o) noexcept {
  drop_graphs();
  N = o.N; B = o.B; m = o.m; prec = o.prec; n = o.n; Q_bs = o.Q_bs;
  x = std::move(o.x); bvec = std::move(o.bvec); T64 = std::move(o.T64); r64 = std::move(o.r64);
  T32 = std::move(o.T32); V = std::move(o.V); Q64 = std::move(o.Q64); Q32 = std::move(o.Q32);
  ex = std::move(o.ex); ey = std::move(o.ey); coefG = std::move(o.coefG); dmom = std::move(o.dmom);
  ex32 = std::move(o.ex32); ey32 = std::move(o.ey32); dmom32 = std::move(o.dmom32); unit32 = std::move(o.unit32);
  part_mom = std::move(o.part_mom); part_vec = std::move(o.part_vec); part_norm = std::move(o.part_norm);
  dred = std::move(o.dred); nred = std::move(o.nred); ctl = std::move(o.ctl); act = std::move(o.act);
  live = std::move(o.live); kvals = std::move(o.kvals); results = std::move(o.results);
  shv = std::move(o.shv); unit = std::move(o.unit); Hbuf = std::move(o.Hbuf);
  Sx = std::move(o.Sx); mx = std::move(o.mx); Fx = std::move(o.Fx); Ax = std::move(o.Ax);
  outS = o.outS; outm = o.outm; x_zero = o.x_zero;
  full_host = std::move(o.full_host);
  host_act = std::move(o.host_act); host_live = std::move(o.host_live);
  graphs = std::move(o.graphs);
  graph_epoch = o.graph_epoch;
  return *this;
}

size_t Work::vec_bytes(int prec) const { return (size_t)n * (prec == DBAR_FP64 ? sizeof(c64) : sizeof(c32)); }

int Work::setup(int N_, int B_, int m_, int prec_, bool shared_q) {
  // captured graphs hold raw pointers and sizes of this workspace: drop them if anything can change
  if (N_ != N || B_ != B || m_ != m || prec_ != prec || (shared_q ? 0 : (size_t)N_ * N_) != Q_bs) drop_graphs();
  const void* before[] = {x.p, V.p, T64.p, T32.p, ctl.p, act.p, part_vec.p, part_norm.p, part_mom.p, dred.p,
                          nred.p, Q32.p, Q64.p, ex.p, ey.p, coefG.p, dmom.p, shv.p, unit.p, Hbuf.p, ex32.p, ey32.p,
                          dmom32.p, unit32.p};
  N = N_;
  B = B_;
  m = m_;
  prec = prec_;
  n = (size_t)N * N;
  const size_t nb = (size_t)B * n;
  const bool mixed = prec == DBAR_MIXED;
  int rc;
  if ((rc = x.ensure(nb * sizeof(c64)))) return rc;
  if ((rc = bvec.ensure(nb * sizeof(c64)))) return rc;
  if ((rc = T64.ensure(nb * sizeof(c64)))) return rc;
  if ((rc = r64.ensure(mixed ? nb * sizeof(c64) : 0))) return rc;
  if ((rc = T32.ensure(mixed ? nb * sizeof(c32) : 0))) return rc;
  if ((rc = V.ensure(nb * (m + 1) * (mixed ? sizeof(c32) : sizeof(c64))))) return rc;
  const size_t nq = shared_q ? n : nb;
  if ((rc = Q64.ensure(nq * sizeof(c64)))) return rc;
  if ((rc = Q32.ensure(mixed ? nq * sizeof(c32) : 0))) return rc;
  Q_bs = shared_q ? 0 : n;
  if ((rc = ex.ensure((size_t)B * N * sizeof(c64)))) return rc;
  if ((rc = ey.ensure((size_t)B * N * sizeof(c64)))) return rc;
  if ((rc = coefG.ensure((size_t)B * kNMom * sizeof(c64)))) return rc;
  if ((rc = dmom.ensure((size_t)B * kNMom * sizeof(c64)))) return rc;
  if ((rc = dmom32.ensure((size_t)B * kNMom * sizeof(c32)))) return rc;
  if ((rc = ex32.ensure((size_t)B * N * sizeof(c32)))) return rc;
  if ((rc = ey32.ensure((size_t)B * N * sizeof(c32)))) return rc;
  // partial buffers for the narrowest column tiles (the most tiles), whatever the current choice
  const int tiles = std::max(line_tiles_max(N, true, true), line_tiles_max(N, true, false));
  const int rtiles = std::max(line_tiles(N, false, true), line_tiles(N, false, false));
  if ((rc = part_mom.ensure((size_t)B * 2 * kNMom * std::max(tiles, rtiles) * sizeof(double)))) return rc;
  if ((rc = part_vec.ensure((size_t)B * (kMaxRestart + 2) * std::max(vec_blocks(n), rtiles) * sizeof(double))))
    return rc;
  if ((rc = part_norm.ensure((size_t)B * std::max(vec_blocks(n), rtiles) * sizeof(double)))) return rc;
  if ((rc = dred.ensure((size_t)B * (kMaxRestart + 2) * sizeof(double)))) return rc;
  if ((rc = nred.ensure((size_t)B * sizeof(double)))) return rc;
  if ((rc = ctl.ensure((size_t)B * sizeof(Ctl)))) return rc;
  if ((rc = kvals.ensure((size_t)B * sizeof(c64)))) return rc;
  if ((rc = shv.ensure((size_t)B * 2 * sizeof(int)))) return rc;
  if (unit.bytes < (size_t)N * sizeof(c64) || unit32.bytes < (size_t)N * sizeof(c32)) {
    if ((rc = unit.ensure((size_t)N * sizeof(c64)))) return rc;
    if ((rc = unit32.ensure((size_t)N * sizeof(c32)))) return rc;
    std::vector<c64> ones(N, c64{1.0, 0.0});
    std::vector<c32> ones32(N, c32{1.0f, 0.0f});
    if (hipMemcpy(unit.p, ones.data(), N * sizeof(c64), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(unit32.p, ones32.data(), N * sizeof(c32), hipMemcpyHostToDevice) != hipSuccess)
      return fail(DBAR_EDEVICE, "upload of the unit phase table failed");
  }
  if ((rc = results.ensure((size_t)B * sizeof(EntryResult)))) return rc;
  // [B, 2B): left a cycle at the restart length; [2B, 3B): orthogonalises fully (see full_host)
  if ((rc = act.ensure((size_t)3 * B * sizeof(int)))) return rc;
  full_host.assign(B, 0);
  if ((rc = live.ensure((size_t)B * sizeof(int)))) return rc;
  if ((rc = host_act.ensure(2 * B))) return rc;
  if ((rc = host_live.ensure(B))) return rc;
  const void* after[] = {x.p, V.p, T64.p, T32.p, ctl.p, act.p, part_vec.p, part_norm.p, part_mom.p, dred.p,
                         nred.p, Q32.p, Q64.p, ex.p, ey.p, coefG.p, dmom.p, shv.p, unit.p, Hbuf.p, ex32.p, ey32.p,
                          dmom32.p, unit32.p};
  if (std::memcmp(before, after, sizeof(before)) != 0) drop_graphs();
  return DBAR_OK;
}

static Work g_work;

// ------------------------------------------------------------------------------------------------------------
// Operator pipeline
// ------------------------------------------------------------------------------------------------------------
LineArgs Pipeline::base(int B, const int* act, unsigned flags) const {
  LineArgs a;
  a.B = B;
  a.act = act;
  a.L = L;
  a.M = M;
  a.ci = 1.0 / (2.0 * kPi * L * L);
  const double dx = 2.0 * kPi * L / N;
  a.cf = dx * dx / (2.0 * kPi);
  if (flags & kUnitPhase) {  // k = 0: one shared table of ones
    a.ex = unit;
    a.ey = unit;
    a.ex32 = unit32;
    a.ey32 = unit32;
    a.e_bs = 0;
  } else {
    a.ex = ex;
    a.ey = ey;
    a.ex32 = ex32;
    a.ey32 = ey32;
    a.e_bs = (size_t)N;
  }
  a.shv = (flags & kShifted) ? shv : nullptr;
  a.coefG = coefG;
  a.dmom = dmom;
  a.dmom32 = dmom32;
  return a;
}

template <typename T>
static const void* tw_of(const Pipeline& p) {
  return sizeof(T) == sizeof(double) ? p.tw64 : p.tw32;
}

// Taylor data of `in` (xi-space): F^{-1} in, d_n, c_n, R(0) -- about xi = 0, or about xi = a with kShifted
template <typename T>
void Pipeline::moments(const void* in, size_t in_bs, void* Tbuf, int B, const int* act, unsigned flags,
                       hipStream_t s) const {
  LineArgs a = base(B, act, flags);
  a.tw = tw_of<T>(*this);
  a.in = in;
  a.in_bs = in_bs;
  a.out = Tbuf;
  a.out_bs = n;
  launch_lines_any<T>(N, LineOp::RowsInvScaled, a, s);
  a.in = Tbuf;
  a.in_bs = n;
  a.part = part_mom;
  launch_lines_any<T>(N, LineOp::ColsInvMoments, a, s);
  const double dx = 2.0 * kPi * L / N;
  TimerScope ts(kStageMoments, 0.0, B, act, s);
  hipLaunchKernelGGL(k_moments, dim3(B), dim3(kCtlThreads), 0, s, part_mom, line_tiles(N, true, sizeof(T) == 8), act,
                     dx * dx / (2.0 * kPi), M, coefG, dmom, dmom32);
}

// out = alpha S_ep + beta i F(q conj(hh(in))) + gamma Y, with hh the regularised inverse of in/xi (or of in/(xi - a)
// with kShifted) and q = Q e_k (Q alone with kShifted or kUnitPhase); S_ep defaults to in
template <typename T>
void Pipeline::apply_impl(const void* in, size_t in_bs, void* out, size_t out_bs, const void* Qp, size_t Q_bs,
                          void* Tbuf, int B, const int* act, double alpha, double beta, const void* Y, size_t Y_bs,
                          bool want_norm, unsigned flags, const void* S_ep, size_t S_ep_bs, hipStream_t s, const DotReq* dr) const {
  moments<T>(in, in_bs, Tbuf, B, act, flags, s);
  LineArgs a = base(B, act, flags);
  a.tw = tw_of<T>(*this);
  a.in = in;
  a.in_bs = in_bs;
  a.out = Tbuf;
  a.out_bs = n;
  launch_lines_any<T>(N, LineOp::RowsInvRegular, a, s);
  a.in = Tbuf;
  a.in_bs = n;
  a.Q = Qp;
  a.Q_bs = Q_bs;
  launch_lines_any<T>(N, LineOp::ColsInvTailFwd, a, s);
  a.out = out;
  a.out_bs = out_bs;
  a.S = S_ep ? S_ep : in;
  a.S_bs = S_ep ? S_ep_bs : in_bs;
  a.alpha = alpha;
  a.beta = c64{0.0, beta};
  a.Y = Y;
  a.Y_bs = Y_bs;
  a.gamma = Y ? 1.0 : 0.0;
  a.want_norm = want_norm ? 1 : 0;
  a.part = part_vec;
  if (dr) {
    a.dotV = dr->V;
    a.dotV_bs = dr->V_bs;
    a.dot_nv = dr->nv;
    a.dot_part = dr->part;
  }
  launch_lines_any<T>(N, LineOp::RowsFwdEpilogue, a, s);
}

template <typename T>
void Pipeline::apply(const void* in, size_t in_bs, void* out, size_t out_bs, const void* Qp, size_t Q_bs, void* Tbuf,
                     int B, const int* act, double alpha, double beta, const void* Y, size_t Y_bs, bool want_norm,
                     hipStream_t s, const DotReq* dr, const XOut* xo) const {
  if (xspace) {
    apply_x<T>(in, in_bs, out, out_bs, Qp, Q_bs, Tbuf, B, act, alpha, beta, Y, Y_bs, want_norm, s, dr, xo);
    return;
  }
  apply_impl<T>(in, in_bs, out, out_bs, Qp, Q_bs, Tbuf, B, act, alpha, beta, Y, Y_bs, want_norm, 0u, nullptr, 0, s,
                dr);
}

int Pipeline::apply_tiles(bool fp64) const { return line_tiles(N, false, fp64); }  // both forms end on rows
int Pipeline::rhs_blocks() const { return xspace ? vec_blocks(n) : line_tiles(N, false, true); }

// The operator on s = F^{-1} S.  With S = F s (F: cf phase FFT2, F^{-1}: ci phase IFFT2, F^{-1} F = identity),
// F^{-1} A(S) = alpha s + beta i q_k conj(h(S)) + gamma Y: the moments of s are read as s is loaded, F s runs as the
// row pass of the first launch and the column pass of the second, which divides by xi and starts F^{-1}, and the
// third launch finishes F^{-1} along rows, adds the closed-form tail and forms the result in x-space.
template <typename T>
void Pipeline::apply_x_first(const void* in, size_t in_bs, void* Tbuf, int B, const int* act, unsigned flags,
                             const UpdReq* u, hipStream_t s) const {
  LineArgs a = base(B, act, flags);
  a.tw = tw_of<T>(*this);
  a.in = in;
  a.in_bs = in_bs;
  a.out = Tbuf;
  a.out_bs = n;
  a.part = part_mom;
  if (u) {
    a.dotV = u->V;
    a.dotV_bs = u->V_bs;
    a.upd_nv = u->nv;
    a.upd_coef = u->coef;
    a.upd_coef_bs = u->coef_bs;
    a.upd_out = const_cast<void*>(in);
    a.upd_part = u->part;
    a.upd_sign = u->sign;
    a.upd_v32 = u->v32 ? 1 : 0;
    a.upd_zero = u->zero_in ? 1 : 0;
  }
  launch_lines_any<T>(N, LineOp::RowsFwdMoments, a, s);
  const double dx = 2.0 * kPi * L / N;
  const int tiles = line_tiles(N, false, sizeof(T) == 8);
  TimerScope ts(kStageMoments, 0.0, B, act, s);
  if (u && u->ctl)
    hipLaunchKernelGGL(k_moments_givens, dim3(B), dim3(kMomGivensThreads), 0, s, part_mom, tiles, dx * dx / (2.0 * kPi),
                       M, coefG, dmom, dmom32, u->ctl, u->part, tiles, const_cast<int*>(act), u->j, u->m);
  else
    hipLaunchKernelGGL(k_moments, dim3(B), dim3(kCtlThreads), 0, s, part_mom, tiles, act, dx * dx / (2.0 * kPi), M,
                       coefG, dmom, dmom32);
}

template <typename T>
void Pipeline::apply_x_rest(const void* in, size_t in_bs, void* out, size_t out_bs, const void* Qp, size_t Q_bs,
                            void* Tbuf, int B, const int* act, double alpha, double beta, const void* Y, size_t Y_bs,
                            bool want_norm, hipStream_t s, const DotReq* dr, const XOut* xo, unsigned flags,
                            const void* S_ep, size_t S_ep_bs) const {
  LineArgs a = base(B, act, flags);
  a.tw = tw_of<T>(*this);
  a.in = Tbuf;  // in place: a column tile is read whole before it is written
  a.in_bs = n;
  a.out = Tbuf;
  a.out_bs = n;
  a.sout = xo ? xo->S : nullptr;
  a.sout_bs = n;
  launch_lines_any<T>(N, LineOp::ColsFwdRegularInv, a, s);
  a.sout = nullptr;
  a.hout = xo ? xo->h : nullptr;
  a.hout_bs = n;
  a.out32 = xo ? xo->r32 : nullptr;
  a.out32_bs = xo ? xo->r32_bs : 0;
  a.Q = Qp;
  a.Q_bs = Q_bs;
  a.out = out;
  a.out_bs = out_bs;
  a.S = S_ep ? S_ep : in;
  a.S_bs = S_ep ? S_ep_bs : in_bs;
  a.alpha = alpha;
  a.beta = c64{0.0, beta};
  a.y_rhs = Y == kYRhs ? 1 : 0;
  a.Y = a.y_rhs ? nullptr : Y;
  a.Y_bs = Y_bs;
  a.gamma = Y ? 1.0 : 0.0;
  a.want_norm = want_norm ? 1 : 0;
  a.part = part_vec;
  if (dr) {
    a.dotV = dr->V;
    a.dotV_bs = dr->V_bs;
    a.dot_nv = dr->nv;
    a.dot_part = dr->part;
    a.dot_self = dr->self ? 1 : 0;
    a.dot_full = dr->full;
    a.dot_skip = dr->skip;
  }
  launch_lines_any<T>(N, LineOp::RowsInvTailEpilogue, a, s);
}

template <typename T>
void Pipeline::apply_x(const void* in, size_t in_bs, void* out, size_t out_bs, const void* Qp, size_t Q_bs,
                       void* Tbuf, int B, const int* act, double alpha, double beta, const void* Y, size_t Y_bs,
                       bool want_norm, hipStream_t s, const DotReq* dr, const XOut* xo, unsigned flags,
                       const void* S_ep, size_t S_ep_bs) const {
  apply_x_first<T>(in, in_bs, Tbuf, B, act, flags, nullptr, s);
  apply_x_rest<T>(in, in_bs, out, out_bs, Qp, Q_bs, Tbuf, B, act, alpha, beta, Y, Y_bs, want_norm, s, dr, xo, flags,
                  S_ep, S_ep_bs);
}

// x-space right-hand side F^{-1} b = -i q_k = -i Q e_k (b = -i F(q_k)), with |.|^2 partials per block
template <typename TO>
__global__ void __launch_bounds__(256) k_rhs_x(const c64* Q, size_t Q_bs, const c64* ex, const c64* ey, size_t e_bs,
                                               int N, cx<TO>* out, size_t out_bs, double* part, int B,
                                               const int* act) {
  const int b = blockIdx.y;
  if (b >= B || (act && !act[b])) return;
  const size_t n = (size_t)N * N;
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int pos = (int)(i / N), col = (int)(i % N);
    const c64 q = Q[(size_t)b * Q_bs + i] * (ex[(size_t)b * e_bs + col] * ey[(size_t)b * e_bs + pos]);
    const c64 v{q.im, -q.re};
    out[(size_t)b * out_bs + i] = cvt<TO>(v);
    acc += v.re * v.re + v.im * v.im;
  }
  __shared__ double red[4];
  acc = wsum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)b * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

void Pipeline::rhs_x(const void* Q64p, size_t Q_bs, void* out, size_t out_bs, bool out32, int B, const int* act,
                     unsigned flags, hipStream_t s) const {
  const LineArgs a = base(B, act, flags & kUnitPhase);
  // the potential counted once when the entries share it (Q_bs = 0)
  TimerScope ts(kStageConvert, (double)n * ((Q_bs ? sizeof(c64) : 0) + (out32 ? sizeof(c32) : sizeof(c64))), B, act, s,
                Q_bs ? 0.0 : (double)n * sizeof(c64));
  const dim3 grid(rhs_blocks(), B);
  const c64* Q = static_cast<const c64*>(Q64p);
  if (out32)
    hipLaunchKernelGGL(k_rhs_x<float>, grid, dim3(256), 0, s, Q, Q_bs, a.ex, a.ey, a.e_bs, N, static_cast<c32*>(out),
                       out_bs, part_vec, B, act);
  else
    hipLaunchKernelGGL(k_rhs_x<double>, grid, dim3(256), 0, s, Q, Q_bs, a.ex, a.ey, a.e_bs, N, static_cast<c64*>(out),
                       out_bs, part_vec, B, act);
}

// H(h) = -i F(Q conj(F^{-1}(h/(xi - a)))) (equation eqh2), into Hout
template <typename T>
void Pipeline::H_of(const void* in, size_t in_bs, void* Hout, size_t H_bs, const void* Qp, size_t Q_bs, void* Tbuf,
                    int B, const int* act, hipStream_t s) const {
  apply_impl<T>(in, in_bs, Hout, H_bs, Qp, Q_bs, Tbuf, B, act, 0.0, -1.0, nullptr, 0, false, kShifted, nullptr, 0, s);
}

// B(h) = h - K0(H(h)) = h + i F(Q conj(F^{-1}(H/xi))), written as alpha h + beta i F(...) + gamma Y
template <typename T>
void Pipeline::apply_B(const void* in, size_t in_bs, void* out, size_t out_bs, const void* Qp, size_t Q_bs,
                       void* Tbuf, void* Hbuf, int B, const int* act, double alpha, double beta, const void* Y,
                       size_t Y_bs, bool want_norm, hipStream_t s, const DotReq* dr, const XOutB* xb) const {
  if (xspace) {
    apply_B_first<T>(in, in_bs, Tbuf, B, act, nullptr, s);
    apply_B_rest<T>(in, in_bs, out, out_bs, Qp, Q_bs, Tbuf, Hbuf, B, act, alpha, beta, Y, Y_bs, want_norm, s, dr, xb);
    return;
  }
  H_of<T>(in, in_bs, Hbuf, n, Qp, Q_bs, Tbuf, B, act, s);
  apply_impl<T>(Hbuf, n, out, out_bs, Qp, Q_bs, Tbuf, B, act, alpha, beta, Y, Y_bs, want_norm, kUnitPhase, in,
                in_bs, s, dr);
}

// x-space B on eta: psi = F^{-1} H(F eta) = -i q conj(h_a(F eta)) (regularised about xi = a; q alone), the operator's
// three launches with the shifted regularisation and alpha = 0 (the first of them here) ...
template <typename T>
void Pipeline::apply_B_first(const void* in, size_t in_bs, void* Tbuf, int B, const int* act, const UpdReq* u,
                             hipStream_t s) const {
  apply_x_first<T>(in, in_bs, Tbuf, B, act, kShifted, u, s);
}

template <typename T>
void Pipeline::apply_B_rest(const void* in, size_t in_bs, void* out, size_t out_bs, const void* Qp, size_t Q_bs,
                            void* Tbuf, void* Hbuf, int B, const int* act, double alpha, double beta, const void* Y,
                            size_t Y_bs, bool want_norm, hipStream_t s, const DotReq* dr, const XOutB* xb) const {
  XOut xh;
  if (xb) {
    xh.S = xb->hxi;
    xh.h = xb->ha;
  }
  apply_x_rest<T>(in, in_bs, Hbuf, n, Qp, Q_bs, Tbuf, B, act, 0.0, -1.0, nullptr, 0, false, s, nullptr, &xh, kShifted,
                  nullptr, 0);
  // ... then eta + i q conj(h0(F psi)) (k = 0 phase, about xi = 0), the alpha term and the products taken with eta
  XOut x0;
  if (xb) {
    x0.S = xb->f;
    x0.h = xb->h0;
    x0.r32 = xb->r32;
    x0.r32_bs = xb->r32_bs;
  }
  apply_x<T>(Hbuf, n, out, out_bs, Qp, Q_bs, Tbuf, B, act, alpha, beta, Y, Y_bs, want_norm, s, dr, &x0, kUnitPhase,
             in, in_bs);
}

// b = -i F(Q e_k) (FP64; e_k = 1 with kUnitPhase), with |b|^2 partials (rhs_blocks() per entry); in x-space -i Q e_k
void Pipeline::rhs(const void* Q64p, size_t Q_bs, void* T64, c64* bout, int B, const int* act, unsigned flags,
                   hipStream_t s) const {
  if (xspace) {
    rhs_x(Q64p, Q_bs, bout, n, false, B, act, flags, s);
    return;
  }
  LineArgs a = base(B, act, flags & kUnitPhase);
  a.tw = tw_of<double>(*this);
  a.Q = Q64p;
  a.Q_bs = Q_bs;
  a.out = T64;
  a.out_bs = n;
  launch_lines_any<double>(N, LineOp::ColsFwdPotential, a, s);
  a.in = T64;
  a.in_bs = n;
  a.out = bout;
  a.out_bs = n;
  a.alpha = 0.0;
  a.beta = c64{0.0, -1.0};
  a.gamma = 0.0;
  a.want_norm = 1;
  a.part = part_vec;
  launch_lines_any<double>(N, LineOp::RowsFwdEpilogue, a, s);
}

// hout (=|+=) h(in): the regularised inverse of in/xi; with kShifted that of in/(xi - a), times e_k if phase_out
template <typename T>
void Pipeline::h_of(const void* in, size_t in_bs, void* hout, size_t hout_bs, void* Tbuf, int B, const int* act,
                    hipStream_t s, unsigned flags, bool phase_out, bool accumulate) const {
  moments<T>(in, in_bs, Tbuf, B, act, flags, s);
  LineArgs a = base(B, act, flags);
  a.tw = tw_of<T>(*this);
  a.in = in;
  a.in_bs = in_bs;
  a.out = Tbuf;
  a.out_bs = n;
  launch_lines_any<T>(N, LineOp::RowsInvRegular, a, s);
  a.in = Tbuf;
  a.in_bs = n;
  a.hout = hout;
  a.hout_bs = hout_bs;
  a.tail_phase_out = phase_out ? 1 : 0;
  a.accumulate = accumulate ? 1 : 0;
  launch_lines_any<T>(N, LineOp::ColsInvTail, a, s);
}

template <typename T>
void Pipeline::transform(bool inverse, const void* in, void* out, void* Tbuf, hipStream_t s) const {
  LineArgs a = base(1, nullptr, 0u);
  a.tw = tw_of<T>(*this);
  if (inverse) {
    a.in = in;
    a.out = Tbuf;
    launch_lines_any<T>(N, LineOp::RowsInvScaled, a, s);
    a.in = Tbuf;
    a.out = out;
    launch_lines_any<T>(N, LineOp::ColsInvPlain, a, s);
  } else {
    a.in = in;
    a.out = Tbuf;
    launch_lines_any<T>(N, LineOp::ColsFwdPlain, a, s);
    a.in = Tbuf;
    a.out = out;
    a.alpha = 0.0;
    a.beta = c64{1.0, 0.0};
    launch_lines_any<T>(N, LineOp::RowsFwdEpilogue, a, s);
  }
}

#define DBAR_PIPE_INST(T)                                                                                        \
  template void Pipeline::apply<T>(const void*, size_t, void*, size_t, const void*, size_t, void*, int,            \
                                   const int*, double, double, const void*, size_t, bool, hipStream_t,            \
                                   const DotReq*, const XOut*) const;                                             \
  template void Pipeline::apply_B<T>(const void*, size_t, void*, size_t, const void*, size_t, void*, void*, int,   \
                                     const int*, double, double, const void*, size_t, bool, hipStream_t,          \
                                     const DotReq*, const XOutB*) const;                                          \
  template void Pipeline::apply_B_first<T>(const void*, size_t, void*, int, const int*, const UpdReq*,             \
                                           hipStream_t) const;                                                    \
  template void Pipeline::apply_B_rest<T>(const void*, size_t, void*, size_t, const void*, size_t, void*, void*,   \
                                          int, const int*, double, double, const void*, size_t, bool,             \
                                          hipStream_t, const DotReq*, const XOutB*) const;                        \
  template void Pipeline::H_of<T>(const void*, size_t, void*, size_t, const void*, size_t, void*, int, const int*, \
                                  hipStream_t) const;                                                            \
  template void Pipeline::h_of<T>(const void*, size_t, void*, size_t, void*, int, const int*, hipStream_t,         \
                                  unsigned, bool, bool) const;                                                   \
  template void Pipeline::transform<T>(bool, const void*, void*, void*, hipStream_t) const;                      \
  template void Pipeline::apply_x<T>(const void*, size_t, void*, size_t, const void*, size_t, void*, int,          \
                                     const int*, double, double, const void*, size_t, bool, hipStream_t,          \
                                     const DotReq*, const XOut*, unsigned, const void*, size_t) const;            \
  template void Pipeline::apply_x_first<T>(const void*, size_t, void*, int, const int*, unsigned, const UpdReq*,  \
                                           hipStream_t) const;                                                    \
  template void Pipeline::apply_x_rest<T>(const void*, size_t, void*, size_t, const void*, size_t, void*, int,     \
                                          const int*, double, double, const void*, size_t, bool, hipStream_t,     \
                                          const DotReq*, const XOut*, unsigned, const void*, size_t) const;
DBAR_PIPE_INST(double)
DBAR_PIPE_INST(float)
#undef DBAR_PIPE_INST

// S = f + h o (xi + a): out[p] = f[p] + h[p + (m1, m2)] (periodic index roll, equation Sform)
__global__ void k_roll_add(const c64* f, const c64* h, const int* shv, int N, c64* out, int B) {
  const int b = blockIdx.y;
  if (b >= B) return;
  const size_t n = (size_t)N * N;
  const int o1 = shv[2 * b], o2 = shv[2 * b + 1];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int p2 = (int)(i / N), p1 = (int)(i % N);
    const size_t src = (size_t)((p2 + o2) & (N - 1)) * N + ((p1 + o1) & (N - 1));
    out[(size_t)b * n + i] = f[(size_t)b * n + i] + h[(size_t)b * n + src];
  }
}

// m += e_k h_a on the x grid (e_k = ex[x index] ey[y index]): the second term of m in the iterated method
__global__ void k_add_phase(c64* m, const c64* ha, const c64* ex, const c64* ey, int N, int B) {
  const int b = blockIdx.y;
  if (b >= B) return;
  const size_t n = (size_t)N * N;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int p2 = (int)(i / N), p1 = (int)(i % N);
    const size_t o = (size_t)b * n + i;
    m[o] = m[o] + (ex[(size_t)b * N + p1] * ey[(size_t)b * N + p2]) * ha[o];
  }
}

void launch_add_phase(c64* m, const c64* ha, const c64* ex, const c64* ey, int N, int B, hipStream_t s) {
  TimerScope ts(kStageConvert, 3.0 * (double)N * N * sizeof(c64), B, nullptr, s);
  hipLaunchKernelGGL(k_add_phase, dim3(std::min(4096, (N * N + 255) / 256), B), dim3(256), 0, s, m, ha, ex, ey, N, B);
}

void launch_roll_add(const c64* f, const c64* h, const int* shv, int N, c64* out, int B, hipStream_t s) {
  TimerScope ts(kStageConvert, 3.0 * (double)N * N * sizeof(c64), B, nullptr, s);
  hipLaunchKernelGGL(k_roll_add, dim3(std::min(4096, (N * N + 255) / 256), B), dim3(256), 0, s, f, h, shv, N, out, B);
}

int make_pipeline(const dbar_grid* g, Work& w, Pipeline* p) {
  int rc = get_twiddles(g->n, &p->tw64, &p->tw32);
  if (rc) return rc;
  p->N = g->n;
  p->M = g->M;
  p->L = g->L;
  p->n = (size_t)g->n * g->n;
  p->ex = static_cast<const c64*>(w.ex.p);
  p->ey = static_cast<const c64*>(w.ey.p);
  p->coefG = static_cast<c64*>(w.coefG.p);
  p->dmom = static_cast<c64*>(w.dmom.p);
  p->dmom32 = static_cast<c32*>(w.dmom32.p);
  p->ex32 = static_cast<const c32*>(w.ex32.p);
  p->ey32 = static_cast<const c32*>(w.ey32.p);
  p->unit32 = static_cast<const c32*>(w.unit32.p);
  p->part_mom = static_cast<double*>(w.part_mom.p);
  p->part_vec = static_cast<double*>(w.part_vec.p);
  p->unit = static_cast<const c64*>(w.unit.p);
  p->shv = static_cast<const int*>(w.shv.p);
  return DBAR_OK;
}

// ------------------------------------------------------------------------------------------------------------
// GMRES driver for one batch of entries
// ------------------------------------------------------------------------------------------------------------
int ctl_blocks(int B) { return (B + 63) / 64; }

template <class... A>
static void launch_ctl_coef(int nval, int B, hipStream_t s, A... args) {
  if (nval <= 4)
    hipLaunchKernelGGL(k_ctl_coef<256>, dim3(B), dim3(256), 0, s, args...);
  else
    hipLaunchKernelGGL(k_ctl_coef<kCtlThreads>, dim3(B), dim3(kCtlThreads), 0, s, args...);
}

// One Krylov cycle in lockstep; returns the number of iterations run (max over entries).
// With cfg.use_graph each group of iterations between two convergence reads is captured once into a HIP graph (per
// element size, method, space, group, passes and batch) and replayed on later cycles and calls; nothing in a
// captured group is a memset or a host transfer.
template <typename T>
int krylov_cycle(const Pipeline& P, Work& w, const BatchCfg& cfg, int it_budget, hipStream_t s) {
  const int B = w.B;
  const size_t n = w.n;
  const size_t V_bs = n * (w.m + 1);
  Ctl* ctl = static_cast<Ctl*>(w.ctl.p);
  int* act = static_cast<int*>(w.act.p);
  double* part = static_cast<double*>(w.part_vec.p);
  double* pnorm = static_cast<double*>(w.part_norm.p);
  const int nvb = vec_blocks(n);
  const void* Qp = sizeof(T) == 8 ? w.Q64.p : w.Q32.p;
  void* Tbuf = sizeof(T) == 8 ? w.T64.p : w.T32.p;
  char* V = static_cast<char*>(w.V.p);
  const int mlim = std::min(w.m, it_budget);

  // x-space, one Gram-Schmidt pass: the update of step j runs inside the first launch of step j + 1's operator (which
  // reads the new vector anyway; for the iterated method the first launch of B's shifted pass); step 0 starts the
  // operator on v_0 itself.  The step's convergence is decided from ||w||^2 and the products before that update
  // (k_ctl_coef), so an entry's last step runs no update, and its Givens step otherwise rides on the moment reduction
  // of v_{j+1}.  The Gram-Schmidt window applies to the plain method.
  const bool fused = P.xspace && cfg.reorth == 1;
  const int window = cfg.method == 0 ? cfg.orth_window : 0;
  // entries that stalled under the window in an earlier cycle orthogonalise fully: the launches then cover the whole
  // basis, and the other entries skip the vectors below their own window inside them
  bool any_full = false;
  if (fused && window > 0)
    for (int b = 0; b < B; ++b) any_full |= w.full_host[b] != 0;
  const int* full = any_full ? act + 2 * B : nullptr;
  auto enqueue = [&](int j) {
    void* vj = V + (size_t)j * n * sizeof(cx<T>);
    void* vj1 = V + (size_t)(j + 1) * n * sizeof(cx<T>);
    if (fused) {
      // the window of basis vectors this step orthogonalises against: v_lo_win .. v_j (all of them without a window);
      // the launch covers v_lo .. v_j
      const int lo_win = window > 0 ? std::max(0, j - window + 1) : 0;
      const int lo = any_full ? 0 : lo_win;
      char* Vlo = V + (size_t)lo * n * sizeof(cx<T>);
      DotReq dr;
      dr.V = Vlo;
      dr.V_bs = V_bs;
      dr.nv = j - lo + 1;
      dr.part = part;
      dr.self = true;  // ||w||^2 for the early convergence decision
      dr.full = full;
      dr.skip = lo_win - lo;
      if (cfg.method == 1) {
        if (j == 0) P.apply_B_first<T>(vj, V_bs, Tbuf, B, act, nullptr, s);
        P.apply_B_rest<T>(vj, V_bs, vj1, V_bs, Qp, w.Q_bs, Tbuf, w.Hbuf.p, B, act, 1.0, 1.0, nullptr, 0, false, s, &dr,
                          nullptr);
      } else {
        if (j == 0) P.apply_x_first<T>(vj, V_bs, Tbuf, B, act, 0u, nullptr, s);
        P.apply_x_rest<T>(vj, V_bs, vj1, V_bs, Qp, w.Q_bs, Tbuf, B, act, 1.0, 1.0, nullptr, 0, false, s, &dr, nullptr,
                          0u, nullptr, 0);
      }
      {
        TimerScope ts(kStageControl, 0.0, B, nullptr, s);
        launch_ctl_coef(j - lo + 2, B, s, ctl, part, j - lo + 2, P.apply_tiles(sizeof(T) == 8), act, j, 0, 1, w.m, lo,
                        lo_win - lo, full);
      }
      UpdReq u;
      u.V = Vlo;
      u.V_bs = V_bs;
      u.nv = j - lo + 1;
      u.coef = &ctl[0].coef[lo];
      u.coef_bs = sizeof(Ctl) / sizeof(double);
      u.part = pnorm;
      u.ctl = ctl;  // step j's Givens step rides on the moment reduction of v_{j+1}
      u.j = j;
      u.m = w.m;
      if (cfg.method == 1)
        P.apply_B_first<T>(vj1, V_bs, Tbuf, B, act, &u, s);
      else
        P.apply_x_first<T>(vj1, V_bs, Tbuf, B, act, 0u, &u, s);
      return;
    }
    // the first Gram-Schmidt pass's products Re<V_i, w>, i <= j, come out of the operator's last kernel
    DotReq dr;
    dr.V = V;
    dr.V_bs = V_bs;
    dr.nv = j + 1;
    dr.part = part;
    if (cfg.method == 1)
      P.apply_B<T>(vj, V_bs, vj1, V_bs, Qp, w.Q_bs, Tbuf, w.Hbuf.p, B, act, 1.0, 1.0, nullptr, 0, false, s, &dr);
    else
      P.apply<T>(vj, V_bs, vj1, V_bs, Qp, w.Q_bs, Tbuf, B, act, 1.0, 1.0, nullptr, 0, false, s, &dr);
    for (int pass = 0; pass < cfg.reorth; ++pass) {
      VecArgs va;
      va.B = B;
      va.act = act;
      va.n = n;
      va.V = V;
      va.V_bs = V_bs;
      va.nv = j + 1;
      va.w = vj1;
      va.w_bs = V_bs;
      va.part = part;
      va.want_self = 0;
      int nblk = P.apply_tiles(sizeof(T) == 8);  // pass 0: partials of the operator's last kernel
      if (pass > 0) {
        launch_dots<T>(va, s);
        nblk = nvb;
      }
      {
        TimerScope ts(kStageControl, 0.0, B, nullptr, s);
        launch_ctl_coef(j + 1, B, s, ctl, part, j + 1, nblk, act, j, pass, 0, w.m, 0, 0, nullptr);
      }
      va.coef = &ctl[0].coef[0];
      va.coef_bs = sizeof(Ctl) / sizeof(double);
      va.want_self = pass + 1 == cfg.reorth ? 1 : 0;
      va.part = pnorm;
      launch_update<T>(va, s);
    }
    TimerScope ts(kStageControl, 0.0, B, nullptr, s);
    hipLaunchKernelGGL(k_ctl_givens, dim3(B), dim3(kCtlThreads), 0, s, ctl, pnorm, nvb, act, j, w.m);
  };

  bool graphs = cfg.use_graph && !timer_on();
  if (w.graph_epoch != tuning_epoch()) {  // captured with another tile choice
    w.drop_graphs();
    w.graph_epoch = tuning_epoch();
  }
  // Steps run in groups that end where the host reads the convergence flags (every check_every steps and at the
  // restart length); with graphs each group is one captured graph, replayed on later cycles and calls.
  // Groups are check_every steps long; once at most a quarter of the batch is still active the cycle is near its end
  // and the groups halve, so that the steps launched after the last entry converged (which run empty) stay few.
  int j = 0, len = cfg.check_every;
  while (j < mlim) {
    const int j1 = std::min(mlim, j + len);
    bool done = false;
    if (graphs) {
      uint64_t Lbits = 0;
      std::memcpy(&Lbits, &P.L, sizeof(Lbits));
      const Work::GraphKey key((int)sizeof(T) + 16 * cfg.method + 64 * (P.xspace ? 1 : 0), j * 1024 + j1,
                               cfg.reorth + 16 * (fused ? window : 0) + 4096 * (any_full ? 1 : 0), B, P.N, P.M,
                               Lbits);
      auto it = w.graphs.find(key);
      if (it != w.graphs.end()) {
        done = hipGraphLaunch(it->second, s) == hipSuccess;
      } else if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        for (int jj = j; jj < j1; ++jj) enqueue(jj);
        hipGraph_t graph = nullptr;
        hipGraphExec_t ge = nullptr;
        if (hipStreamEndCapture(s, &graph) == hipSuccess && graph &&
            hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0) == hipSuccess) {
          w.graphs[key] = ge;
          done = hipGraphLaunch(ge, s) == hipSuccess;
        } else if (ge) {
          (void)hipGraphExecDestroy(ge);
        }
        if (graph) (void)hipGraphDestroy(graph);
      }
      if (!done) {
        (void)hipGetLastError();  // capture or replay unavailable: enqueue directly from now on
        graphs = false;
      }
    }
    if (!done)
      for (int jj = j; jj < j1; ++jj) enqueue(jj);
    j = j1;
    (void)hipMemcpyAsync(w.host_act.data(), act, 2 * B * sizeof(int), hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);
    int active = 0;
    for (int b = 0; b < B; ++b) {
      active += w.host_act[b] != 0;
      // an entry that left this cycle at the restart length orthogonalises fully from the next cycle on (the cycle
      // start sets its device flag from the same restart flag)
      if (w.host_act[B + b] != 0) w.full_host[b] = 1;
    }
    if (active == 0) return j;
    if (4 * active <= B) len = std::max(1, cfg.check_every / 2);
  }
  return j;
}

// x += sum coef_i V_i and the FP64 residual r = b - A(x) (into r_out), with squared norms in nred
template <typename T>
void end_cycle(const Pipeline& P, Work& w, int nv, void* r_out, hipStream_t s, int method, bool cond, bool outputs) {
  const int B = w.B;
  const size_t n = w.n;
  Ctl* ctl = static_cast<Ctl*>(w.ctl.p);
  int* live = static_cast<int*>(w.live.p);
  hipLaunchKernelGGL(k_ctl_trisolve, dim3(B), dim3(64), 0, s, ctl, live, B);
  if (cond) launch_cond_estimate(w, s);
  VecArgs va;
  va.B = B;
  va.act = live;
  va.n = n;
  va.V = w.V.p;
  va.V_bs = n * (w.m + 1);
  va.nv = nv;
  va.w = w.x.p;
  va.w_bs = n;
  va.coef = &ctl[0].coef[0];
  va.coef_bs = sizeof(Ctl) / sizeof(double);
  // the x-space residual's first launch reads x anyway: x += sum y_i V_i runs inside it
  const bool fuse_axpy = P.xspace;
  if (!fuse_axpy) launch_axpy_multi<double, T>(va, s);
  UpdReq u;  // the fused solution update
  u.V = w.V.p;
  u.V_bs = n * (w.m + 1);
  u.nv = nv;
  u.coef = &ctl[0].coef[0];
  u.coef_bs = sizeof(Ctl) / sizeof(double);
  u.sign = -1.0;
  u.v32 = sizeof(T) == 4;
  u.zero_in = fuse_axpy && w.x_zero;
  if (fuse_axpy) w.x_zero = false;
  const size_t r_bs = sizeof(T) == 8 ? n * (w.m + 1) : n;
  if (method == 1 && !P.xspace) {
    P.apply_B<double>(w.x.p, n, r_out, r_bs, w.Q64.p, w.Q_bs, w.T64.p, w.Hbuf.p, B, live, -1.0, -1.0, w.bvec.p, n,
                      true, s);
  } else if (method == 1) {
    // x-space iterated method: h = F eta, f = H(h), the shifted inverse of h and h(f) come along (S, m, m1 and r are
    // formed from the last evaluation's; with !outputs the caller knows this evaluation is not the last); the mixed
    // solver's residual goes straight to the next FP32 basis vector
    XOutB xb;
    xb.hxi = outputs ? w.Sx.p : nullptr;
    xb.f = outputs ? w.Fx.p : nullptr;
    xb.ha = outputs ? w.Ax.p : nullptr;
    xb.h0 = outputs ? w.m_dst() : nullptr;
    if (sizeof(T) == 4) {
      xb.r32 = w.V.p;
      xb.r32_bs = n * (w.m + 1);
    }
    P.apply_B_first<double>(w.x.p, n, w.T64.p, B, live, &u, s);
    P.apply_B_rest<double>(w.x.p, n, sizeof(T) == 4 ? nullptr : r_out, r_bs, w.Q64.p, w.Q_bs, w.T64.p, w.Hbuf.p, B,
                           live, -1.0, -1.0, kYRhs, 0, true, s, nullptr, &xb);
  } else if (!P.xspace)
    P.apply<double>(w.x.p, n, r_out, r_bs, w.Q64.p, w.Q_bs, w.T64.p, B, live, -1.0, -1.0, w.bvec.p, n, true, s);
  else {
    // x-space: S = F x and m = h(S) of this x come along (the last evaluation's are the outputs; with !outputs the
    // caller knows this evaluation is not the last); the mixed solver's residual goes straight to the next cycle's
    // first basis vector in FP32
    XOut xo;
    xo.S = outputs ? w.S_dst(0) : nullptr;
    xo.h = outputs ? w.m_dst() : nullptr;
    if (sizeof(T) == 4) {
      xo.r32 = w.V.p;
      xo.r32_bs = n * (w.m + 1);
    }
    P.apply_x_first<double>(w.x.p, n, w.T64.p, B, live, 0u, &u, s);
    P.apply_x_rest<double>(w.x.p, n, sizeof(T) == 4 ? nullptr : r_out, r_bs, w.Q64.p, w.Q_bs, w.T64.p, B, live, -1.0,
                           -1.0, kYRhs, 0, true, s, nullptr, &xo, 0u, nullptr, 0);
  }
  launch_reduce(static_cast<double*>(w.part_vec.p), 1, P.apply_tiles(true), static_cast<double*>(w.nred.p), B, live,
                s);
}

template int krylov_cycle<float>(const Pipeline&, Work&, const BatchCfg&, int, hipStream_t);
template int krylov_cycle<double>(const Pipeline&, Work&, const BatchCfg&, int, hipStream_t);
template void end_cycle<float>(const Pipeline&, Work&, int, void*, hipStream_t, int, bool, bool);
template void end_cycle<double>(const Pipeline&, Work&, int, void*, hipStream_t, int, bool, bool);

void launch_cond_estimate(Work& w, hipStream_t s) {
  TimerScope ts(kStageControl, 0.0, w.B, nullptr, s);
  hipLaunchKernelGGL(k_cond_estimate, dim3(w.B), dim3(64), 0, s, static_cast<Ctl*>(w.ctl.p),
                     static_cast<const int*>(w.live.p));
}

void launch_ctl_check(Work& w, double tol, int first, const int* mask, const double* tolv, hipStream_t s) {
  TimerScope ts(kStageControl, 0.0, w.B, nullptr, s);
  hipLaunchKernelGGL(k_ctl_check, dim3(ctl_blocks(w.B)), dim3(64), 0, s, static_cast<Ctl*>(w.ctl.p),
                     static_cast<const double*>(w.nred.p), static_cast<int*>(w.live.p), static_cast<int*>(w.act.p),
                     tol, first, mask, tolv, w.B);
}
void launch_ctl_start(Work& w, double abs_tol, double rel_tol, const double* tolv, hipStream_t s) {
  TimerScope ts(kStageControl, 0.0, w.B, nullptr, s);
  hipLaunchKernelGGL(k_ctl_start, dim3(ctl_blocks(w.B)), dim3(64), 0, s, static_cast<Ctl*>(w.ctl.p),
                     static_cast<const double*>(w.nred.p), static_cast<const int*>(w.live.p),
                     static_cast<int*>(w.act.p), abs_tol, rel_tol, tolv, w.B);
}

__global__ void k_zero_done(c64* a0, c64* a1, c64* a2, c64* a3, const int* live, const int* mask, size_t n) {
  const int b = blockIdx.y;
  if (live[b] || (mask && !mask[b])) return;
  c64* const arr[4] = {a0, a1, a2, a3};
  for (int k = 0; k < 4; ++k) {
    if (!arr[k]) continue;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
      arr[k][(size_t)b * n + i] = c64{0.0, 0.0};
  }
}

void launch_zero_done(Work& w, const int* mask, bool iterated, hipStream_t s) {
  // plain: S and m where they are left; iterated: h (Sx), f (Fx), the shifted inverse (Ax) and m, from which S is
  // formed
  hipLaunchKernelGGL(k_zero_done, dim3((unsigned)std::min<size_t>(1024, (w.n + 255) / 256), w.B), dim3(256), 0, s,
                     static_cast<c64*>(iterated ? w.Sx.p : w.S_dst(0)), static_cast<c64*>(w.m_dst()),
                     iterated ? static_cast<c64*>(w.Fx.p) : nullptr, iterated ? static_cast<c64*>(w.Ax.p) : nullptr,
                     static_cast<const int*>(w.live.p), mask, w.n);
}

int run_batch(const Pipeline& P, Work& w, const BatchCfg& cfg, hipStream_t s, std::vector<int>& iters_out) {
  const int B = w.B;
  const size_t n = w.n;
  const bool mixed = w.prec == DBAR_MIXED;
  Ctl* ctl = static_cast<Ctl*>(w.ctl.p);
  int* act = static_cast<int*>(w.act.p);
  int* live = static_cast<int*>(w.live.p);
  double* nred = static_cast<double*>(w.nred.p);
  // b = -i F(q_k), |b|
  // plain: b = -i F(Q e_k); iterated (equation eqh2): b = -i F(Q).  In x-space -i q_k goes straight to the first basis
  // vector (the residuals form it in their last launch: no b array)
  const unsigned rhs_flags = cfg.method == 1 ? kUnitPhase : 0u;
  if (P.xspace)
    P.rhs_x(w.Q64.p, w.Q_bs, w.V.p, n * (w.m + 1), mixed, B, nullptr, rhs_flags, s);
  else
    P.rhs(w.Q64.p, w.Q_bs, w.T64.p, static_cast<c64*>(w.bvec.p), B, nullptr, rhs_flags, s);
  launch_reduce(static_cast<double*>(w.part_vec.p), 1, P.rhs_blocks(), nred, B, nullptr, s);
  // x = 0: the x-space residual's first launch writes x = sum y_i V_i on the first update (no memset)
  w.x_zero = P.xspace;
  w.full_host.assign(B, 0);  // device flags: cleared by the first residual check below
  if (!w.x_zero && hipMemsetAsync(w.x.p, 0, (size_t)B * n * sizeof(c64), s) != hipSuccess)
    return fail(DBAR_EDEVICE, "hipMemsetAsync failed");
  for (int b = 0; b < B; ++b) w.host_live[b] = 1;
  if (hipMemcpyAsync(live, w.host_live.data(), B * sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(DBAR_EDEVICE, "hipMemcpyAsync failed");
  // r0 = b (x0 = 0); entries with b = 0 are done at once
  hipLaunchKernelGGL(k_ctl_check, dim3(ctl_blocks(B)), dim3(64), 0, s, ctl, nred, live, act, 0.0, 1, nullptr, nullptr,
                     B);
  if (P.xspace) {  // S = m = 0 for entries with b = 0 (no residual evaluation writes them)
    launch_zero_done(w, nullptr, cfg.method == 1, s);
  } else if (mixed) {
    launch_convert<float, double>(w.bvec.p, n, w.V.p, n * (w.m + 1), n, B, nullptr, 1.0, s);
  } else {
    launch_convert<double, double>(w.bvec.p, n, w.V.p, n * (w.m + 1), n, B, nullptr, 1.0, s);
  }
  int total = 0;
  iters_out.assign(B, 0);
  while (true) {
    (void)hipMemcpyAsync(w.host_live.data(), live, B * sizeof(int), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(DBAR_EDEVICE, "stream synchronize failed");
    bool any = false;
    for (int b = 0; b < B; ++b) any |= w.host_live[b] != 0;
    if (!any || total >= cfg.max_iter) break;
    const double rel = mixed ? cfg.inner_tol : 0.0;
    const double abs_tol = mixed ? 0.3 * cfg.tol : 0.5 * cfg.tol;
    hipLaunchKernelGGL(k_ctl_start, dim3(ctl_blocks(B)), dim3(64), 0, s, ctl, nred, live, act, abs_tol, rel, nullptr, B);
    int ran;
    // The first cycle of a mixed-precision x-space solve starts from |r| = |b| and asks its FP32 inner solve for
    // inner_tol of that, which FP32 arithmetic cannot better by many orders: with tol far below inner_tol its residual
    // evaluation is not the last one, and it leaves S and m unwritten (two N x N FP64 arrays per entry).  So that the
    // outputs always come from the last evaluation, an entry that would meet tol there anyway runs one more cycle
    // (whose evaluation writes them) instead of finishing.
    const bool outputs = !(mixed && P.xspace && total == 0 && cfg.tol < 1e-3 * cfg.inner_tol);
    // the condition estimate is taken from the first cycle (from x = 0: the longest, every entry in it)
    if (mixed) {
      ran = krylov_cycle<float>(P, w, cfg, cfg.max_iter - total, s);
      end_cycle<float>(P, w, ran, w.r64.p, s, cfg.method, total == 0, outputs);
    } else {
      ran = krylov_cycle<double>(P, w, cfg, cfg.max_iter - total, s);
      end_cycle<double>(P, w, ran, w.V.p, s, cfg.method, total == 0);
    }
    total += ran;
    hipLaunchKernelGGL(k_ctl_check, dim3(ctl_blocks(B)), dim3(64), 0, s, ctl, nred, live, act,
                       outputs ? cfg.tol : -1.0, 0, nullptr, nullptr, B);
    if (mixed && !P.xspace) launch_convert<float, double>(w.r64.p, n, w.V.p, n * (w.m + 1), n, B, live, 1.0, s);
    if (ran == 0) break;
  }
  if (hipStreamSynchronize(s) != hipSuccess) return fail(DBAR_EDEVICE, "stream synchronize failed");
  return DBAR_OK;
}

// ------------------------------------------------------------------------------------------------------------
// C ABI helpers
// ------------------------------------------------------------------------------------------------------------
static bool all_finite(const double* p, size_t cnt) {
  for (size_t i = 0; i < cnt; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// batch size chosen by the tuner per (N, precision); 0 = not tuned (the default below)
static std::atomic<int> g_batch[2][12];
static int batch_slot(int N) {
  int i = 0;
  for (int m = 8; m < N && i < 11; m <<= 1) ++i;
  return i;
}
static int tuned_batch(int N, bool fp64) { return g_batch[fp64 ? 1 : 0][batch_slot(N)].load(); }

static int check_device() {
  int cnt = 0;
  hipError_t e = hipGetDeviceCount(&cnt);
  if (e != hipSuccess || cnt < 1) {
    (void)hipGetLastError();
    return fail(DBAR_EDEVICE, "no HIP device available");
  }
  return DBAR_OK;
}

// The solver's own stream (default priority, non-blocking): graph capture needs a stream other than the legacy
// default one, and the caller's stream is joined through events.
static hipStream_t g_stream = nullptr;
static hipEvent_t g_join = nullptr;

static int solver_stream(hipStream_t caller, hipStream_t* out) {
  if (!g_stream) {
    if (hipStreamCreateWithFlags(&g_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&g_join, hipEventDisableTiming) != hipSuccess)
      return fail(DBAR_EDEVICE, "stream creation failed");
  }
  if (hipEventRecord(g_join, caller) != hipSuccess || hipStreamWaitEvent(g_stream, g_join, 0) != hipSuccess)
    return fail(DBAR_EDEVICE, "stream join failed");
  *out = g_stream;
  return DBAR_OK;
}

// Lanes of a batched solve (see solve_impl): lane 0 runs on the solver stream with g_work, lane l > 0 on a stream and
// workspace of its own, joined to the caller's stream through the same event.
constexpr int kMaxLanes = 2;
static Work g_lane_work[kMaxLanes - 1];
static hipStream_t g_lane_stream[kMaxLanes - 1];

static Work& lane_work(int l) { return l == 0 ? g_work : g_lane_work[l - 1]; }

// The host thread of lane l > 0, kept from one solve to the next: creating a thread per call, and the runtime's set-up
// of a new thread at its first HIP calls, cost hundreds of microseconds between back-to-back solves.  run() hands it
// one job and returns at once; wait() returns when the job has finished.  The thread waits on a condition variable
// between jobs and exits when the process ends (the destructor).
class LaneThread {
 public:
  ~LaneThread() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      quit_ = true;
    }
    cv_.notify_all();
    if (th_.joinable()) th_.join();
  }
  // false if no thread could be created (the caller then runs the job itself)
  bool run(std::function<void()> job) {
    if (!th_.joinable()) {
      try {
        th_ = std::thread([this] { loop(); });
      } catch (...) {
        return false;
      }
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      job_ = std::move(job);
      pending_ = true;
      done_ = false;
    }
    cv_.notify_all();
    return true;
  }
  void wait() {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [this] { return done_; });
  }

 private:
  void loop() {
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
      cv_.wait(lk, [this] { return pending_ || quit_; });
      if (!pending_) return;  // quit with no job
      std::function<void()> job = std::move(job_);
      pending_ = false;
      lk.unlock();
      job();
      lk.lock();
      done_ = true;
      cv_.notify_all();
    }
  }
  std::thread th_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::function<void()> job_;
  bool pending_ = false, done_ = false, quit_ = false;
};
static LaneThread g_lane_thread[kMaxLanes - 1];

// (lane 0 first: it records the join event on the caller's stream)
static int lane_stream(int l, hipStream_t caller, hipStream_t* out) {
  if (l == 0) return solver_stream(caller, out);
  hipStream_t& s = g_lane_stream[l - 1];
  if (!s && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
    s = nullptr;
    return fail(DBAR_EDEVICE, "stream creation failed");
  }
  if (hipStreamWaitEvent(s, g_join, 0) != hipSuccess) return fail(DBAR_EDEVICE, "stream join failed");
  *out = s;
  return DBAR_OK;
}

// grid offset of 2 k_c L (k_c a component of k), known to be an integer
static int shift_of(double kc, double L) { return (int)std::nearbyint(2.0 * kc * L); }

// r_out (host, nk complex, or NULL): with the iterated method, i h(2i conj k) per entry; when S and m are both NULL
// the S and m post-processing is skipped (the reflection-coefficient path)
int solve_impl(const dbar_grid* grid, const void* Q, bool q_on_device, int64_t nk, const double* k, double tol,
               const dbar_opts* opts_in, void* S, void* m, bool out_on_device, dbar_info* info, hipStream_t caller,
               double* r_out) {
  int rc = validate_grid(grid);
  if (rc) return rc;
  if (nk < 1) return fail(DBAR_EINVAL, "nk must be >= 1");
  if (!k || !Q) return fail(DBAR_EINVAL, "Q and k must not be NULL");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(DBAR_EINVAL, "tol must be finite and > 0");
  if (!all_finite(k, 2 * (size_t)nk)) return fail(DBAR_EINVAL, "k contains NaN or Inf");
  dbar_opts o;
  dbar_default_opts(&o);
  if (opts_in) o = *opts_in;
  if (o.precision != DBAR_FP64 && o.precision != DBAR_MIXED)
    return fail(DBAR_EINVAL, "precision must be DBAR_FP64 or DBAR_MIXED for a solve");
  if (o.restart <= 0) o.restart = o.precision == DBAR_MIXED ? 20 : 40;
  if (o.restart > kMaxRestart) return fail(DBAR_EINVAL, "restart must be <= 64");
  if (o.max_iter <= 0) o.max_iter = 1000;
  if (o.reorth < 1 || o.reorth > 2) o.reorth = 1;
  if (o.check_every <= 0) o.check_every = 4;
  if (o.orth_window < 0 || o.orth_window > o.restart)
    return fail(DBAR_EINVAL, "orth_window must be in [0, restart]");
  // default: the x-space FP32 operator keeps 1e-6 attainable per cycle (its moments are exact sums of the FP32
  // vector); the xi-space one forms them after an FP32 round trip and stalls near 1e-5
  const bool xspace_solve = o.space == DBAR_SPACE_X;
  if (!(o.inner_tol > 0.0) || o.inner_tol >= 1.0) o.inner_tol = xspace_solve ? 1e-6 : 1e-5;
  if (o.method != 0 && o.method != 1) return fail(DBAR_EINVAL, "method must be 0 (plain) or 1 (iterated)");
  if (o.space != DBAR_SPACE_X && o.space != DBAR_SPACE_XI)
    return fail(DBAR_EINVAL, "space must be DBAR_SPACE_X or DBAR_SPACE_XI");
  if (o.method == 1) {
    for (int64_t j = 0; j < 2 * nk; ++j) {
      const double m = 2.0 * k[j] * grid->L;
      if (std::fabs(m - std::nearbyint(m)) > 1e-9 * std::max(1.0, std::fabs(m)))
        return fail(DBAR_EINVAL, "the iterated method needs 2k on the xi grid: 2 L Re k and 2 L Im k integers");
    }
  }
  if ((rc = check_device())) return rc;
  const int N = grid->n;
  const size_t n = (size_t)N * N;
  std::lock_guard<std::mutex> lock(g_mutex);
  // Q on the host: check finiteness
  std::vector<double> hQ;
  if (!q_on_device) {
    if (!all_finite(static_cast<const double*>(Q), 2 * n)) return fail(DBAR_EINVAL, "Q contains NaN or Inf");
  }
  const int tuned = tuned_batch(N, o.precision == DBAR_FP64);
  // untuned default: 64 entries, or on small grids enough entries for about 2^24 grid points per launch (N = 128:
  // 1024), which a launch needs to fill the GPU
  const int dflt = (int)std::max<int64_t>(64, std::min<int64_t>(4096, (int64_t(1) << 24) / ((int64_t)N * N)));
  int B = o.mode == DBAR_MODE_PLAIN ? 1 : (o.batch > 0 ? o.batch : (int)std::min<int64_t>(nk, tuned > 0 ? tuned : dflt));
  B = (int)std::min<int64_t>(B, nk);
  // Lanes: the batch split into parts solved concurrently, each on a stream and workspace of its own; part c goes to
  // lane c % lanes.  A caller's batch of 16 or more is split in two; with the library's choice of batch (the tuned or
  // default entries per launch) each of two lanes takes that many entries when there are more k than one batch.  One
  // lane keeps the captured-graph path; with more, the launches are direct (a capture in one host thread interferes
  // with the other thread's calls).  The stage timer times one lane.
  int lanes = 1;
  if (o.mode != DBAR_MODE_PLAIN && !timer_on()) {
    if (o.lanes > 0) lanes = std::min(o.lanes, kMaxLanes);
    else if (o.batch > 0) lanes = B >= 16 ? 2 : 1;
    else lanes = nk > B ? 2 : 1;
    if (o.batch <= 0 && lanes > 1) B = (int)std::min<int64_t>(nk, (int64_t)lanes * B);
  }
  if (o.mode != DBAR_MODE_PLAIN && o.batch <= 0) {
    // fit the batch to free memory: basis + 6 vectors per entry
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) {
      const size_t per = n * ((o.restart + 1) * (o.precision == DBAR_MIXED ? 8 : 16) + 8 * 16) + 65536;
      const size_t cap = (size_t)(0.7 * (double)fr) / per;
      if (cap >= 1 && (size_t)B > cap) B = (int)cap;
    }
  }
  lanes = std::max(1, std::min(lanes, B));
  const int Bl = (B + lanes - 1) / lanes;
  BatchCfg cfg;
  cfg.tol = tol;
  cfg.max_iter = o.max_iter;
  cfg.reorth = o.reorth;
  cfg.use_graph = o.mode == DBAR_MODE_PLAIN || lanes > 1 ? 0 : o.use_graph;
  cfg.method = o.method;
  cfg.check_every = o.mode == DBAR_MODE_PLAIN ? 1 : o.check_every;
  cfg.inner_tol = o.inner_tol;
  cfg.orth_window = o.orth_window;
  cfg.xspace = o.space == DBAR_SPACE_X ? 1 : 0;
  struct Lane {
    Work* w = nullptr;
    hipStream_t s = nullptr;
    Pipeline P;
  };
  Lane ln[kMaxLanes];
  for (int l = 0; l < lanes; ++l) {
    if ((rc = lane_stream(l, caller, &ln[l].s))) return rc;
    Work& w = lane_work(l);
    ln[l].w = &w;
    const hipStream_t s = ln[l].s;
    if ((rc = w.setup(N, Bl, o.restart, o.precision, true))) return rc;
    if ((rc = make_pipeline(grid, w, &ln[l].P))) return rc;
    ln[l].P.xspace = cfg.xspace != 0;
    if (q_on_device) {
      if (hipMemcpyAsync(w.Q64.p, Q, n * sizeof(c64), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(DBAR_EDEVICE, "Q copy failed");
    } else {
      if (hipMemcpyAsync(w.Q64.p, Q, n * sizeof(c64), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(DBAR_EDEVICE, "Q upload failed");
    }
    if (o.precision == DBAR_MIXED) launch_convert<float, double>(w.Q64.p, 0, w.Q32.p, 0, n, 1, nullptr, 1.0, s);
    if (cfg.method == 1 && (rc = w.Hbuf.ensure((size_t)Bl * n * sizeof(c64)))) return rc;
    if (cfg.xspace &&
        ((rc = w.Sx.ensure((size_t)Bl * n * sizeof(c64))) || (rc = w.mx.ensure((size_t)Bl * n * sizeof(c64)))))
      return rc;
    if (cfg.xspace && cfg.method == 1 &&
        ((rc = w.Fx.ensure((size_t)Bl * n * sizeof(c64))) || (rc = w.Ax.ensure((size_t)Bl * n * sizeof(c64)))))
      return rc;
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  // one lane's parts, in order; returns DBAR_OK, DBAR_ENOCONV (some entry did not converge) or an error
  auto run_lane = [&](int l) -> int {
    Work& w = *ln[l].w;
    const hipStream_t s = ln[l].s;
    const Pipeline& P = ln[l].P;
    std::vector<EntryResult> hres(Bl);
    std::vector<int> shifts(2 * (size_t)Bl);
    int result = DBAR_OK;
    for (int64_t k0 = (int64_t)l * Bl; k0 < nk; k0 += (int64_t)lanes * Bl) {
      const int nb = (int)std::min<int64_t>(Bl, nk - k0);
      w.B = nb;
      w.outS = cfg.xspace && out_on_device && S ? static_cast<char*>(S) + (size_t)k0 * n * sizeof(c64) : nullptr;
      w.outm = cfg.xspace && out_on_device && m ? static_cast<char*>(m) + (size_t)k0 * n * sizeof(c64) : nullptr;
      if (hipMemcpyAsync(w.kvals.p, k + 2 * k0, (size_t)nb * sizeof(c64), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(DBAR_EDEVICE, "k upload failed");
      if (cfg.method == 1) {
        for (int b = 0; b < nb; ++b) {
          shifts[2 * b] = shift_of(k[2 * (k0 + b) + 1], grid->L);
          shifts[2 * b + 1] = shift_of(k[2 * (k0 + b)], grid->L);
        }
        if (hipMemcpyAsync(w.shv.p, shifts.data(), (size_t)nb * 2 * sizeof(int), hipMemcpyHostToDevice, s) !=
            hipSuccess)
          return fail(DBAR_EDEVICE, "shift upload failed");
      }
      launch_phase_tables(static_cast<const c64*>(w.kvals.p), N, grid->L, static_cast<c64*>(w.ex.p),
                          static_cast<c64*>(w.ey.p), static_cast<c32*>(w.ex32.p), static_cast<c32*>(w.ey32.p), nb, s);
      std::vector<int> its;
      if (const int brc = run_batch(P, w, cfg, s, its)) return brc;
      // outputs.  Plain on s: S and m from the last residual evaluation.  Iterated on s: S = f + h o (xi + a) (equation
      // Sform, formed in place in Fx) and m = h(f) + e_k F^{-1}(h/(xi - a)) (in place in mx) from that evaluation's
      // h, f and inverses.  On S: S = x and m = h(x) (plain), or formed from h below (iterated).  S0src holds S(0) for
      // m1, hsrc the iterated method's xi-space h (r = i h(a)).
      const bool form = cfg.method == 1 && (S || m || !r_out);  // dbar_reflection alone needs only h(a)
      const c64* S0src = static_cast<const c64*>(w.x.p);
      const c64* hsrc = static_cast<const c64*>(w.x.p);
      const void* Sout = nullptr;
      const void* mout = nullptr;
      // (x-space outputs the solve wrote straight into the caller's device arrays need no copy)
      if (cfg.xspace && cfg.method == 0) {
        S0src = static_cast<const c64*>(w.S_dst(0));
        Sout = w.outS ? nullptr : w.Sx.p;
        mout = w.outm ? nullptr : w.mx.p;
      } else if (cfg.xspace) {
        hsrc = static_cast<const c64*>(w.Sx.p);
        if (form) {
          launch_roll_add(static_cast<const c64*>(w.Fx.p), static_cast<const c64*>(w.Sx.p),
                          static_cast<const int*>(w.shv.p), N, static_cast<c64*>(w.S_dst(1)), nb, s);
          launch_add_phase(static_cast<c64*>(w.m_dst()), static_cast<const c64*>(w.Ax.p),
                           static_cast<const c64*>(w.ex.p), static_cast<const c64*>(w.ey.p), N, nb, s);
          S0src = static_cast<const c64*>(w.S_dst(1));
          Sout = w.outS ? nullptr : w.Fx.p;
          mout = w.outm ? nullptr : w.mx.p;
        }
      } else if (cfg.method == 0) {
        Sout = w.x.p;
        if (m) {
          P.h_of<double>(w.x.p, n, w.T64.p, n, w.bvec.p, nb, nullptr, s);  // bvec reused as scratch
          mout = w.T64.p;
        }
      } else if (form) {
        // f = H(h) (into Hbuf), S = f + h o (xi + a) (into bvec), m = h(f) + e_k F^{-1}(h/(xi - a)) (into T64)
        c64* Hb = static_cast<c64*>(w.Hbuf.p);
        c64* Sb = static_cast<c64*>(w.bvec.p);
        P.H_of<double>(w.x.p, n, Hb, n, w.Q64.p, w.Q_bs, Sb, nb, nullptr, s);
        P.h_of<double>(Hb, n, w.T64.p, n, Sb, nb, nullptr, s);
        P.h_of<double>(w.x.p, n, w.T64.p, n, Sb, nb, nullptr, s, kShifted, true, true);
        launch_roll_add(Hb, static_cast<const c64*>(w.x.p), static_cast<const int*>(w.shv.p), N, Sb, nb, s);
        S0src = Sb;
        Sout = Sb;
        mout = w.T64.p;
      }
      const hipMemcpyKind kind = out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
      if (S && Sout &&
          hipMemcpyAsync(static_cast<char*>(S) + (size_t)k0 * n * sizeof(c64), Sout, (size_t)nb * n * sizeof(c64), kind,
                         s) != hipSuccess)
        return fail(DBAR_EDEVICE, "S copy failed");
      if (m && mout &&
          hipMemcpyAsync(static_cast<char*>(m) + (size_t)k0 * n * sizeof(c64), mout, (size_t)nb * n * sizeof(c64), kind,
                         s) != hipSuccess)
        return fail(DBAR_EDEVICE, "m copy failed");
      hipLaunchKernelGGL(k_gather_results, dim3(ctl_blocks(nb)), dim3(64), 0, s, static_cast<const Ctl*>(w.ctl.p),
                         S0src, n, hsrc, cfg.method == 1 ? static_cast<const int*>(w.shv.p) : nullptr, N,
                         static_cast<EntryResult*>(w.results.p), nb);
      (void)hipMemcpyAsync(hres.data(), w.results.p, (size_t)nb * sizeof(EntryResult), hipMemcpyDeviceToHost, s);
      (void)hipMemcpyAsync(w.host_live.data(), w.live.p, nb * sizeof(int), hipMemcpyDeviceToHost, s);
      if (hipStreamSynchronize(s) != hipSuccess) return fail(DBAR_EDEVICE, "stream synchronize failed");
      for (int b = 0; b < nb; ++b) {
        const EntryResult& c = hres[b];
        const bool ok = w.host_live[b] == 0;
        if (!ok) result = DBAR_ENOCONV;
        if (info) {
          dbar_info& I = info[k0 + b];
          I.status = ok ? DBAR_OK : DBAR_ENOCONV;
          I.iters = c.iters;
          I.outer = c.cycles;
          I.reserved = 0;
          I.rel_residual = c.bnorm > 0.0 ? c.rnorm / c.bnorm : 0.0;
          I.cond_estimate = c.kappa;
          I.err_estimate = c.kappa * I.rel_residual;
          I.m1_re = form || cfg.method == 0 ? -c.s00.im : 0.0;  // m1 = i S(0); not formed on the r-only path
          I.m1_im = form || cfg.method == 0 ? c.s00.re : 0.0;
        }
        if (r_out) {  // r = i h(2i conj k)
          r_out[2 * (k0 + b)] = -c.hsh.im;
          r_out[2 * (k0 + b) + 1] = c.hsh.re;
        }
      }
    }
    w.outS = nullptr;
    w.outm = nullptr;
    return result;
  };
  int result = DBAR_OK;
  if (lanes == 1) {
    result = run_lane(0);
  } else {
    // lanes 1.. on their host threads (each with the device current), lane 0 on the calling thread; a lane whose
    // thread cannot be created runs on the calling thread after lane 0
    int rcs[kMaxLanes];
    std::string errs[kMaxLanes];
    // (host allocations inside a lane can throw; the lane then ends with an error code, not the process)
    auto lane_fn = [&](int l) {
      try {
        (void)hipSetDevice(dev);
        rcs[l] = run_lane(l);
        if (rcs[l] != DBAR_OK && rcs[l] != DBAR_ENOCONV) errs[l] = g_last_error;
      } catch (const std::bad_alloc&) {
        rcs[l] = DBAR_ENOMEM;
        errs[l] = "host memory exhausted in a lane's solve";
      } catch (...) {
        rcs[l] = DBAR_EDEVICE;
        errs[l] = "a lane's solve failed on its host thread";
      }
    };
    bool on_thread[kMaxLanes] = {};
    for (int l = 1; l < lanes; ++l) on_thread[l] = g_lane_thread[l - 1].run([&lane_fn, l] { lane_fn(l); });
    lane_fn(0);
    for (int l = 1; l < lanes; ++l) {
      if (on_thread[l]) g_lane_thread[l - 1].wait();
      else lane_fn(l);
    }
    if (rcs[0] != DBAR_OK && rcs[0] != DBAR_ENOCONV) return fail(rcs[0], errs[0]);
    for (int l = 1; l < lanes; ++l)
      if (rcs[l] != DBAR_OK && rcs[l] != DBAR_ENOCONV) return fail(rcs[l], errs[l]);
    for (int l = 0; l < lanes; ++l)
      if (rcs[l] == DBAR_ENOCONV) result = DBAR_ENOCONV;
  }
  if (result == DBAR_ENOCONV) fail(DBAR_ENOCONV, "GMRES reached max_iter before tol for some k");
  return result;
}

}  // namespace dbar

// ------------------------------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------------------------------
using namespace dbar;

extern "C" {

void dbar_default_opts(dbar_opts* o) {
  if (!o) return;
  o->restart = 0;
  o->max_iter = 1000;
  o->precision = DBAR_FP64;
  o->mode = DBAR_MODE_BATCHED;
  o->batch = 0;
  o->use_graph = 1;
  o->reorth = 1;
  o->check_every = 4;
  o->method = 0;
  o->space = DBAR_SPACE_X;
  o->inner_tol = 0.0;
  o->orth_window = kDefaultOrthWindow;
}

const char* dbar_last_error(void) { return g_last_error.c_str(); }

int dbar_version(void) { return 100; }

void dbar_release(void) {
  std::lock_guard<std::mutex> lock(g_mutex);
  g_work = Work();
  for (int l = 0; l + 1 < kMaxLanes; ++l) {
    g_lane_work[l] = Work();
    if (g_lane_stream[l]) (void)hipStreamDestroy(g_lane_stream[l]);
    g_lane_stream[l] = nullptr;
  }
  {
    std::lock_guard<std::mutex> tl(g_tw_mutex);
    g_twiddles.clear();
  }
  if (g_stream) (void)hipStreamDestroy(g_stream);
  if (g_join) (void)hipEventDestroy(g_join);
  g_stream = nullptr;
  g_join = nullptr;
}

int dbar_solve(const dbar_grid* grid, const double* Q, int64_t nk, const double* k, double tol, const dbar_opts* opts,
               double* S_out, double* m_out, dbar_info* info) {
  return solve_impl(grid, Q, false, nk, k, tol, opts, S_out, m_out, false, info, nullptr, nullptr);
}

int dbar_solve_device(const dbar_grid* grid, const void* Q_dev, int64_t nk, const double* k, double tol,
                      const dbar_opts* opts, void* S_dev, void* m_dev, dbar_info* info, void* stream) {
  return solve_impl(grid, Q_dev, true, nk, k, tol, opts, S_dev, m_dev, true, info,
                    static_cast<hipStream_t>(stream), nullptr);
}

// Tuner: times one operator application over `batch` entries for every column-tile width of the grid size, keeps the
// fastest, then times the operator at a few batch sizes and keeps the smallest within 5% of the best per-entry time.
int dbar_autotune(const dbar_grid* grid, int32_t precision, int32_t batch, dbar_tune_result* out) {
  int rc = validate_grid(grid);
  if (rc) return rc;
  if (precision != DBAR_FP64 && precision != DBAR_MIXED && precision != DBAR_FP32)
    return fail(DBAR_EINVAL, "precision must be DBAR_FP64, DBAR_MIXED or DBAR_FP32");
  if (batch < 1 || batch > 1024) return fail(DBAR_EINVAL, "batch must be in [1, 1024]");
  if ((rc = check_device())) return rc;
  std::lock_guard<std::mutex> lock(g_mutex);
  const int N = grid->n;
  const size_t n = (size_t)N * N;
  hipStream_t s = nullptr;
  if ((rc = solver_stream(nullptr, &s))) return rc;
  Work& w = g_work;
  // FP32 operator buffers come with the mixed layout; one Krylov vector pair serves as input and output
  if ((rc = w.setup(N, batch, 1, precision == DBAR_FP64 ? DBAR_FP64 : DBAR_MIXED, true))) return rc;
  Pipeline P;
  if ((rc = make_pipeline(grid, w, &P))) return rc;
  P.xspace = true;  // the operator as the plain method's solves apply it
  // zero inputs: the kernels' work does not depend on the data (k = 0, Q = 0, S = 0)
  const size_t vb = precision == DBAR_FP64 ? sizeof(c64) : sizeof(c32);
  if (hipMemsetAsync(w.x.p, 0, (size_t)batch * n * sizeof(c64), s) != hipSuccess ||
      hipMemsetAsync(w.V.p, 0, (size_t)batch * n * 2 * vb, s) != hipSuccess ||
      hipMemsetAsync(w.Q64.p, 0, n * sizeof(c64), s) != hipSuccess ||
      hipMemsetAsync(w.kvals.p, 0, (size_t)batch * sizeof(c64), s) != hipSuccess ||
      (precision != DBAR_FP64 && hipMemsetAsync(w.Q32.p, 0, n * sizeof(c32), s) != hipSuccess))
    return fail(DBAR_EDEVICE, "tuner buffer initialisation failed");
  w.B = batch;
  launch_phase_tables(static_cast<const c64*>(w.kvals.p), N, grid->L, static_cast<c64*>(w.ex.p),
                      static_cast<c64*>(w.ey.p), static_cast<c32*>(w.ex32.p), static_cast<c32*>(w.ey32.p), batch, s);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(DBAR_EDEVICE, "event creation failed");
  const size_t V_bs = n * 2;  // the workspace basis holds m + 1 = 2 vectors per entry
  auto time_apply = [&](bool fp64, int B, int reps) -> double {
    auto once = [&]() {
      if (fp64)
        P.apply<double>(w.x.p, n, w.bvec.p, n, w.Q64.p, 0, w.T64.p, B, nullptr, 1.0, 1.0, nullptr, 0, false, s);
      else
        P.apply<float>(w.V.p, V_bs, static_cast<char*>(w.V.p) + n * sizeof(c32), V_bs, w.Q32.p, 0, w.T32.p, B,
                       nullptr, 1.0, 1.0, nullptr, 0, false, s);
    };
    once();  // warm-up (first launch of each kernel)
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r) once();
    (void)hipEventRecord(e1, s);
    float ms = 0.f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
    return ms / reps;
  };
  dbar_tune_result res{};
  int result = DBAR_OK;
  for (int f = 0; f < 2 && result == DBAR_OK; ++f) {  // f = 0: FP64 operator, 1: FP32 operator
    const bool fp64 = f == 0;
    if (fp64 ? precision == DBAR_FP32 : precision == DBAR_FP64) continue;
    const int nv = tile_variants(N, fp64);
    res.n_variants[f] = nv;
    int best = 0;
    for (int v = 0; v < nv; ++v) {
      set_tile_variant(N, fp64, v);
      res.columns[f][v] = tile_columns(N, fp64, v);
      res.ms[f][v] = time_apply(fp64, batch, 5);
      if (res.ms[f][v] < 0.0) result = fail(DBAR_EDEVICE, "timing failed");
      if (res.ms[f][v] < res.ms[f][best]) best = v;
    }
    set_tile_variant(N, fp64, best);
    res.chosen[f] = best;
  }
  // batch size: per-entry time at batch, batch/2, batch/4, batch/8 with the operator that dominates the solves
  if (result == DBAR_OK) {
    const bool fp64 = precision == DBAR_FP64;
    double best_pe = 1e300;
    for (int c = 0; c < 4; ++c) {
      const int Bc = std::max(1, batch >> c);
      res.batch_candidates[c] = Bc;
      res.per_entry_ms[c] = time_apply(fp64, Bc, 3) / Bc;
      best_pe = std::min(best_pe, res.per_entry_ms[c]);
    }
    res.batch = batch;
    for (int c = 3; c >= 0; --c)
      if (res.per_entry_ms[c] <= 1.05 * best_pe) {
        res.batch = res.batch_candidates[c];
        break;
      }
    g_batch[fp64 ? 1 : 0][batch_slot(N)] = res.batch;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  w.drop_graphs();
  if (out) *out = res;
  return result;
}

int dbar_set_tile(int32_t n, int32_t precision, int32_t variant) {
  dbar_grid g{n, 11, 1.0};
  int rc = validate_grid(&g);
  if (rc) return rc;
  const bool fp64 = precision == DBAR_FP64;
  if (precision != DBAR_FP64 && precision != DBAR_FP32) return fail(DBAR_EINVAL, "precision must be FP64 or FP32");
  if (variant < 0 || variant >= tile_variants(n, fp64)) return fail(DBAR_EINVAL, "no such tile variant for this grid");
  std::lock_guard<std::mutex> lock(g_mutex);
  set_tile_variant(n, fp64, variant);
  return DBAR_OK;
}

int dbar_get_tile(int32_t n, int32_t precision, int32_t* variant, int32_t* columns, int32_t* variants) {
  dbar_grid g{n, 11, 1.0};
  int rc = validate_grid(&g);
  if (rc) return rc;
  if (precision != DBAR_FP64 && precision != DBAR_FP32) return fail(DBAR_EINVAL, "precision must be FP64 or FP32");
  const bool fp64 = precision == DBAR_FP64;
  const int v = tile_variant(n, fp64);
  if (variant) *variant = v;
  if (columns) *columns = tile_columns(n, fp64, v);
  if (variants) *variants = tile_variants(n, fp64);
  return DBAR_OK;
}

static int single_prep(const dbar_grid* grid, int precision, Work*& w, Pipeline& P) {
  int rc = validate_grid(grid);
  if (rc) return rc;
  if (precision != DBAR_FP64 && precision != DBAR_FP32) return fail(DBAR_EINVAL, "precision must be FP64 or FP32");
  if ((rc = check_device())) return rc;
  w = &g_work;
  if ((rc = w->setup(grid->n, 1, 1, precision == DBAR_FP32 ? DBAR_MIXED : DBAR_FP64, true))) return rc;
  w->B = 1;
  return make_pipeline(grid, *w, &P);
}

int dbar_apply(const dbar_grid* grid, const double* Q, const double* k, const double* S_in, double* AS_out,
               int32_t precision) {
  if (!Q || !k || !S_in || !AS_out) return fail(DBAR_EINVAL, "NULL buffer");
  std::lock_guard<std::mutex> lock(g_mutex);
  Work* w;
  Pipeline P;
  int rc = single_prep(grid, precision, w, P);
  if (rc) return rc;
  const int N = grid->n;
  const size_t n = (size_t)N * N;
  if (!all_finite(Q, 2 * n) || !all_finite(k, 2) || !all_finite(S_in, 2 * n))
    return fail(DBAR_EINVAL, "NaN or Inf in the inputs");
  hipStream_t s = nullptr;
  (void)hipMemcpy(w->kvals.p, k, sizeof(c64), hipMemcpyHostToDevice);
  launch_phase_tables(static_cast<const c64*>(w->kvals.p), N, grid->L, static_cast<c64*>(w->ex.p),
                      static_cast<c64*>(w->ey.p), static_cast<c32*>(w->ex32.p), static_cast<c32*>(w->ey32.p), 1, s);
  (void)hipMemcpy(w->Q64.p, Q, n * sizeof(c64), hipMemcpyHostToDevice);
  (void)hipMemcpy(w->x.p, S_in, n * sizeof(c64), hipMemcpyHostToDevice);
  if (precision == DBAR_FP64) {
    P.apply<double>(w->x.p, n, w->bvec.p, n, w->Q64.p, 0, w->T64.p, 1, nullptr, 1.0, 1.0, nullptr, 0, false, s);
    if (hipMemcpy(AS_out, w->bvec.p, n * sizeof(c64), hipMemcpyDeviceToHost) != hipSuccess)
      return fail(DBAR_EDEVICE, "copy back failed");
  } else {
    launch_convert<float, double>(w->Q64.p, 0, w->Q32.p, 0, n, 1, nullptr, 1.0, s);
    launch_convert<float, double>(w->x.p, 0, w->V.p, 0, n, 1, nullptr, 1.0, s);
    char* V1 = static_cast<char*>(w->V.p) + n * sizeof(c32);
    P.apply<float>(w->V.p, n, V1, n, w->Q32.p, 0, w->T32.p, 1, nullptr, 1.0, 1.0, nullptr, 0, false, s);
    launch_convert<double, float>(V1, 0, w->bvec.p, 0, n, 1, nullptr, 1.0, s);
    if (hipMemcpy(AS_out, w->bvec.p, n * sizeof(c64), hipMemcpyDeviceToHost) != hipSuccess)
      return fail(DBAR_EDEVICE, "copy back failed");
  }
  if (hipDeviceSynchronize() != hipSuccess) return fail(DBAR_EDEVICE, "kernel failure");
  return DBAR_OK;
}

int dbar_transform(const dbar_grid* grid, int32_t inverse, const double* in, double* out, int32_t precision) {
  if (!in || !out) return fail(DBAR_EINVAL, "NULL buffer");
  std::lock_guard<std::mutex> lock(g_mutex);
  Work* w;
  Pipeline P;
  int rc = single_prep(grid, precision, w, P);
  if (rc) return rc;
  const size_t n = (size_t)grid->n * grid->n;
  if (!all_finite(in, 2 * n)) return fail(DBAR_EINVAL, "NaN or Inf in the input");
  (void)hipMemcpy(w->x.p, in, n * sizeof(c64), hipMemcpyHostToDevice);
  if (precision == DBAR_FP64) {
    P.transform<double>(inverse != 0, w->x.p, w->bvec.p, w->T64.p, nullptr);
  } else {
    launch_convert<float, double>(w->x.p, 0, w->V.p, 0, n, 1, nullptr, 1.0, nullptr);
    char* V1 = static_cast<char*>(w->V.p) + n * sizeof(c32);
    P.transform<float>(inverse != 0, w->V.p, V1, w->T32.p, nullptr);
    launch_convert<double, float>(V1, 0, w->bvec.p, 0, n, 1, nullptr, 1.0, nullptr);
  }
  if (hipMemcpy(out, w->bvec.p, n * sizeof(c64), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(DBAR_EDEVICE, "copy back failed");
  return DBAR_OK;
}

int dbar_dbar_inverse(const dbar_grid* grid, const double* S_in, double* h_out, int32_t precision) {
  if (!S_in || !h_out) return fail(DBAR_EINVAL, "NULL buffer");
  std::lock_guard<std::mutex> lock(g_mutex);
  Work* w;
  Pipeline P;
  int rc = single_prep(grid, precision, w, P);
  if (rc) return rc;
  const size_t n = (size_t)grid->n * grid->n;
  if (!all_finite(S_in, 2 * n)) return fail(DBAR_EINVAL, "NaN or Inf in the input");
  (void)hipMemcpy(w->x.p, S_in, n * sizeof(c64), hipMemcpyHostToDevice);
  if (precision == DBAR_FP64) {
    P.h_of<double>(w->x.p, n, w->bvec.p, n, w->T64.p, 1, nullptr, nullptr);
  } else {
    launch_convert<float, double>(w->x.p, 0, w->V.p, 0, n, 1, nullptr, 1.0, nullptr);
    char* V1 = static_cast<char*>(w->V.p) + n * sizeof(c32);
    P.h_of<float>(w->V.p, n, V1, n, w->T32.p, 1, nullptr, nullptr);
    launch_convert<double, float>(V1, 0, w->bvec.p, 0, n, 1, nullptr, 1.0, nullptr);
  }
  if (hipMemcpy(h_out, w->bvec.p, n * sizeof(c64), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(DBAR_EDEVICE, "copy back failed");
  return DBAR_OK;
}

}  // extern "C"
