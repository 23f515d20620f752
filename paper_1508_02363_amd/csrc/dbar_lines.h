// Fused line-transform kernels of the D-bar operator (included only by the per-N translation units).
//
// One application of A(S) = S + i F(q_k conj(h(S))) (paper Section 4, algorithm step 4, with Q -> q_k of Section 5.1)
// runs as six launches:
//   RowsInvScaled   F^{-1} S, first pass
//   ColsInvMoments  F^{-1} S, second pass, fused with the Taylor moments d_n = F(z^n s)(0)   (equation fourreeg4)
//   (moment reduction: d_n, c_n = (-i/2)^n d_n / n!, R(0) = (-i/2) F(conj(z) s)(0))
//   RowsInvRegular  R = (S - G)/xi with G of equation Gchoice, first pass of F^{-1} R
//   ColsInvTailFwd  second pass of F^{-1} R, h = F^{-1} R + sum c_n W_n (equation S0Taylor), u = q_k conj(h),
//                   first pass of F u  -- all in registers between the two column transforms
//   RowsFwdEpilogue second pass of F u and A(S) = S + i F(u)
//
// The same operator on s = F^{-1} S (the form the Krylov solver iterates on: F is unitary up to a constant, so GMRES
// takes the same steps, and the moments are sums over the x grid that need no transform) runs as three launches plus
// the moment reduction:
//   RowsFwdMoments      moments d_n = F(z^n s)(0), dt = F(conj(z) s)(0) of the input, first pass of F s
//   ColsFwdRegularInv   second pass of F s (= S), R = (S - G)/xi, first pass of F^{-1} R
//   RowsInvTailEpilogue second pass of F^{-1} R, h, and F^{-1} A(S) = s + i q_k conj(h)
#pragma once

#include "dbar_fft.h"
#include "dbar_launch.h"

namespace dbar {

static __constant__ double kInvFact[40] = {
    1.0, 1.0, 5.0e-1, 1.6666666666666666e-1, 4.1666666666666664e-2, 8.3333333333333332e-3,
    1.3888888888888889e-3, 1.9841269841269841e-4, 2.4801587301587302e-5, 2.7557319223985893e-6,
    2.7557319223985888e-7, 2.5052108385441720e-8, 2.0876756987868100e-9, 1.6059043836821613e-10,
    1.1470745597729725e-11, 7.6471637318198164e-13, 4.7794773323873853e-14, 2.8114572543455206e-15,
    1.5619206968586225e-16, 8.2206352466243295e-18, 4.1103176233121648e-19, 1.9572941063391263e-20,
    8.8967913924505741e-22, 3.8681701706306835e-23, 1.6117375710961184e-24, 6.4469502843844736e-26,
    2.4795962632247972e-27, 9.1836898637955460e-29, 3.2798892370698378e-30, 1.1309962886447717e-31,
    3.7699876288159054e-33, 1.2161250415535179e-34, 3.8003907548547434e-36, 1.1516335620771951e-37,
    3.3871575355211620e-39, 9.6775929586318906e-41, 2.6882202662866363e-42, 7.2654601791530714e-44,
    1.9119632050402819e-45, 4.9024697565135435e-47};

// Smallest u beyond which e^{-u} sum_{k<=M} u^k/k! (times a safety factor 10) is below the rounding unit, so that
// P(n+1, u) = 1 exactly for every n <= M and omega_n = i / z^{n+1} (index M = 0..15).
static __constant__ float kTailOneF32[16] = {19.0f,  22.75f, 26.0f,  28.75f, 31.25f, 33.5f,  36.0f,  38.0f,
                                             40.25f, 42.25f, 44.25f, 46.25f, 48.0f,  50.0f,  51.75f, 53.75f};
static __constant__ double kTailOneF64[16] = {39.25, 43.75, 47.25, 50.5, 53.5, 56.25, 59.0, 61.5,
                                              64.0,  66.5,  68.75, 71.0, 73.25, 75.5, 77.5, 79.75};

// Exact binomial coefficients C(n, k), n, k <= kMaxM (Pascal's rule at compile time), and reciprocals 1/j of the
// integers (j < kNInv) for the tail recurrences, which would otherwise divide in every step.
struct BinomTable {
  double v[kMaxM + 1][kMaxM + 1];
};
constexpr BinomTable make_binom() {
  BinomTable t{};
  for (int n = 0; n <= kMaxM; ++n)
    for (int k = 0; k <= n; ++k) t.v[n][k] = (k == 0 || k == n) ? 1.0 : t.v[n - 1][k - 1] + t.v[n - 1][k];
  return t;
}
static __constant__ BinomTable kBinom = make_binom();

constexpr int kNInv = 256;
struct InvTable {
  double d[kNInv];
  float f[kNInv];
};
constexpr InvTable make_inv() {
  InvTable t{};
  for (int j = 1; j < kNInv; ++j) t.d[j] = 1.0 / j, t.f[j] = 1.0f / j;
  return t;
}
static __constant__ InvTable kInv = make_inv();
template <typename TT>
DBAR_D TT inv_int(int j) {
  if constexpr (sizeof(TT) == 8) return kInv.d[j];
  else return kInv.f[j];
}


// x_j = L(-pi + 2 pi j / N)
template <int N>
DBAR_D double xgrid(int j, double L) {
  return L * (-kPi + (2.0 * kPi / N) * j);
}
// the same in the arithmetic type TT (the FP32 operator evaluates its tail in FP32)
template <typename TT, int N>
DBAR_D TT xgrid_t(int j, double L) {
  if constexpr (sizeof(TT) == 8) return xgrid<N>(j, L);
  else return static_cast<float>(L) * (static_cast<float>(-kPi) + static_cast<float>(2.0 * kPi / N) * j);
}

// 1/r: FP64 division, or the hardware reciprocal (1 ulp) in FP32
template <typename TT>
DBAR_D TT recip(TT r) {
  if constexpr (sizeof(TT) == 8) return 1.0 / r;
  else return __builtin_amdgcn_rcpf(r);
}

// Coefficients c_k = prod_{j=1..k} (M+1)/(M+1+j) of F(u) = (M+1)! sum_k u^k/(M+1+k)! in powers of v = u/(M+1), and
// the number of terms after which the rest is below half a rounding unit of F for every v < 1 (FP32 or FP64), for
// the orders the tail is instantiated with (M = 11 and kMaxM).  Read from constant memory in a loop unrolled by four:
// fully unrolled, the compiler keeps every coefficient in a register; rolled, each step waits for its own read.
constexpr int kSerK32[2] = {25, 28}, kSerK64[2] = {40, 45};
struct SeriesTables {
  double d[2][45];
  float f[2][28];
};
constexpr SeriesTables make_series() {
  SeriesTables t{};
  for (int w = 0; w < 2; ++w) {
    const int M1 = (w == 0 ? 11 : kMaxM) + 1;
    double c = 1.0;
    for (int k = 0; k < 45; ++k) {
      if (k > 0) c = c * (double)M1 / (double)(M1 + k);
      t.d[w][k] = c;
      if (k < 28) t.f[w][k] = (float)c;
    }
  }
  return t;
}
static __constant__ SeriesTables kSeries = make_series();

// sum_{n=0}^{M} d_n omega_n(z),  omega_n = i P(n+1, u) / z^{n+1},  u = |z|^2/4  (c_n W_n = d_n omega_n).
// u <  M+1: omega_n = i E_n (conj(z)/4)^{n+1} with E_n = e^{-u} sum_k u^k/(n+1+k)!  (equation fourreg5a with the
//           factor e^{-u}); E_M by its series (a fixed-length polynomial), E_n = u E_{n+1} + e^{-u}/(n+1)! downwards
//           (positive terms only).
// u >= M+1: omega_n = i (1 - e^{-u} sum_{k<=n} u^k/k!) / z^{n+1}  (equation fourreg5); no cancellation there.
// TT is the arithmetic type: double in the FP64 operator, float in the FP32 one (whose data carry 24-bit mantissas).
// MM is the Taylor order the loops are unrolled for: the order M itself (M = 11, the paper's choice), or kMaxM for any
// M, which is exact too because d_n = 0 for M < n <= kMaxM.  d holds d_0..d_kMaxM in registers.
template <typename TT, int MM>
DBAR_D cx<TT> tail_sum(TT x, TT y, const cx<TT> (&d)[kMaxM + 1]) {
  const TT r2 = x * x + y * y;
  const TT u = TT(0.25) * r2;
  const TT one_from = sizeof(TT) == 8 ? TT(kTailOneF64[MM]) : TT(kTailOneF32[MM]);
  if (u >= one_from) {  // all P(n+1, u) = 1: i sum_n d_n / z^{n+1}
    const TT ir2 = recip(r2);
    const cx<TT> w{x * ir2, -y * ir2};
    cx<TT> acc = d[MM];
#pragma unroll
    for (int n = MM - 1; n >= 0; --n) acc = cfma(w, acc, d[n]);
    return mul_i(w * acc);
  }
  const TT eu = exp(-u);
  cx<TT> acc{TT(0), TT(0)};
  if (u < TT(MM + 1)) {
    // E_M = e^{-u} F(u) / (M+1)!, F(u) = sum_k c_k v^k with v = u/(M+1) < 1, c_k = prod_{j<=k} (M+1)/(M+1+j):
    // a fixed number of Horner steps (positive terms; the first omitted one is below half a rounding unit of F)
    static_assert(MM == 11 || MM == kMaxM, "series tables for M = 11 and kMaxM");
    constexpr int W = MM == 11 ? 0 : 1;
    constexpr int K = sizeof(TT) == 8 ? kSerK64[W] : kSerK32[W];
    const TT* c;
    if constexpr (sizeof(TT) == 8) c = kSeries.d[W];
    else c = kSeries.f[W];
    const TT v = u * TT(1.0 / (MM + 1));
    TT F = c[K - 1];
#pragma unroll 4
    for (int k = K - 2; k >= 0; --k) F = F * v + c[k];
    TT E = eu * F * TT(kInvFact[MM + 1]);
    const cx<TT> zeta{TT(0.25) * x, TT(-0.25) * y};
    acc = E * d[MM];
#pragma unroll
    for (int n = MM - 1; n >= 0; --n) {
      E = u * E + eu * TT(kInvFact[n + 1]);
      acc = cfma(zeta, acc, E * d[n]);
    }
    acc = zeta * acc;
  } else {
    TT P[MM + 1];
    TT t = eu, S = eu;
#pragma unroll
    for (int n = 0; n <= MM; ++n) {
      P[n] = TT(1) - S;
      t *= u * inv_int<TT>(n + 1);
      S += t;
    }
    const TT ir2 = recip(r2);
    const cx<TT> w{x * ir2, -y * ir2};  // 1/z
    acc = P[MM] * d[MM];
#pragma unroll
    for (int n = MM - 1; n >= 0; --n) acc = cfma(w, acc, P[n] * d[n]);
    acc = w * acc;
  }
  return mul_i(acc);
}

// ------------------------------------------------------------------------------------------------------------
// Block reduction of per-thread FP64 values into global partials dst[v * stride]
// ------------------------------------------------------------------------------------------------------------
DBAR_D double wsum64(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

template <int NT, int NV>
DBAR_D void block_reduce_store(const double (&vals)[NV], double* __restrict__ dst, size_t stride, double* scratch) {
  __syncthreads();  // scratch aliases the transform's LDS
  if constexpr (NT >= 64) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double x = vals[v];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
      if (lane == 0) scratch[wave * NV + v] = x;
    }
    __syncthreads();
    for (int v = threadIdx.x; v < NV; v += NT) {
      double s = 0.0;
      for (int w = 0; w < NT / 64; ++w) s += scratch[w * NV + v];
      dst[v * stride] = s;
    }
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) scratch[threadIdx.x * NV + v] = vals[v];
    __syncthreads();
    for (int v = threadIdx.x; v < NV; v += NT) {  // fewer threads than values in tiny blocks
      double s = 0.0;
      for (int t = 0; t < NT; ++t) s += scratch[t * NV + v];
      dst[v * stride] = s;
    }
  }
}

// ------------------------------------------------------------------------------------------------------------
// Tiling
// ------------------------------------------------------------------------------------------------------------
template <typename T, int N>
struct Tiling {
  using G = LineGeom<N>;
  static constexpr int cmin(int a, int b) { return a < b ? a : b; }
  static constexpr int cmax(int a, int b) { return a > b ? a : b; }
  static constexpr int kLdsBudget = 150 * 1024;
  static constexpr int fit(int lines) {
    while (lines > 1 && lines * G::LDS_LINE * (int)sizeof(cx<T>) > kLdsBudget) lines /= 2;
    return lines;
  }
  static constexpr int ROWS = fit(cmin(N, cmax(1, 128 / G::TPL)));
  // (FP32 at N = 4096: the LDS holds four full-height lines, but a four-line tile needs more than the 128 VGPRs of
  // four waves per SIMD and spills 72 bytes per lane; two lines fit without a spill and run faster)
  static constexpr int COLS = sizeof(T) == 4 && N >= 4096 ? 2
                                                          : fit(cmin(N, cmax(64 / (int)sizeof(cx<T>), cmax(1, 64 / G::TPL))));
  // Column-tile variants for the tuner: 0 = COLS (the default), then the wider tiles COLS << 1, COLS << 2 while the
  // block has at most 1024 threads and the tile's lines fit the LDS budget, then the narrower tile COLS / 2 (more
  // blocks per CU where one full-height tile fills most of the LDS, as at N = 4096).
  static constexpr bool wide_ok(int c) {
    return c <= N && c * G::TPL <= 1024 && c * G::LDS_LINE * (int)sizeof(cx<T>) <= kLdsBudget;
  }
  static constexpr int NWIDE = wide_ok(COLS << 1) ? (wide_ok(COLS << 2) ? 2 : 1) : 0;
  static constexpr bool NARROW = COLS >= 2;
  static constexpr int variants() { return 1 + NWIDE + (NARROW ? 1 : 0); }
  template <int V>
  static constexpr int cols_v() { return V == 0 ? COLS : V <= NWIDE ? (COLS << V) : COLS / 2; }
  template <int V>
  static constexpr bool cols_valid() { return V < variants(); }
  // Tile width of the FP32 transform array (t_index): the default column tile, but at least 8 columns, so that the
  // row launches move 64-byte pieces.  At N = 4096 the column tile is 2 columns (4 at most); 2- or 4-column pieces
  // cost the row launches more (they leave partial lines) than the narrow column tiles gain from whole pieces.
  static constexpr int LAYOUT_W = COLS < 8 && N >= 8 ? 8 : COLS;
};

// Index of element (row, col) of the x-space operator's transform array (the output of its first launch, rewritten in
// place by the column launch, read by the last).  FP32: column-tile-major with tiles of Tiling::LAYOUT_W columns, each
// tile one contiguous N x LAYOUT_W block, so that the column launch reads and writes whole or partial lines of it and
// the row launches whole LAYOUT_W-element pieces; the width is a compile-time constant, so the per-thread addresses
// keep constant strides.  FP64: row-major (the tiled FP64 array measured slower).
template <typename T, int N>
DBAR_D size_t t_index(int row, int col) {
  if constexpr (sizeof(T) == 8) {
    return (size_t)row * N + col;
  } else {
    constexpr int TW = Tiling<T, N>::LAYOUT_W;
    return ((size_t)(col / TW) * N + row) * TW + (col % TW);
  }
}

// LDS of one line-kernel block: the line data, or the scratch of its reductions, whichever is larger
template <typename T, int N, int LINES, bool COLS>
struct LdsSize {
  static constexpr int TPL = LineGeom<N>::TPL;
  static constexpr int NT = LINES * TPL;
  static constexpr int kData = LINES * LineGeom<N>::LDS_LINE * (int)sizeof(cx<T>);
  static constexpr int LN = LINES;
  static constexpr int kScratchReduce = (NT >= 64 ? NT / 64 : NT) * 2 * kNMom * (int)sizeof(double);
  // the moment reduction's groups (MomentsBase::finish_kk): runs of min(TPL, 64) lanes of a row; on a column tile
  // (wave, column) pairs when the block has whole waves and fewer than 64 columns, else single threads
  static constexpr int NG = COLS ? ((NT >= 64 && LN < 64) ? (NT / 64) * LN : NT) : NT / (TPL < 64 ? TPL : 64);
  static constexpr int kScratchMoments = (NG * 2 * (kMaxM + 1) + LN * 2 * kNMom + LN * 2 * (kMaxM + 1)) * 8;
  static constexpr int kScratch = kScratchReduce > kScratchMoments ? kScratchReduce : kScratchMoments;
  static constexpr int kElems = ((kData > kScratch ? kData : kScratch) + (int)sizeof(cx<T>) - 1) / (int)sizeof(cx<T>);
};

// ------------------------------------------------------------------------------------------------------------
// Operations
// ------------------------------------------------------------------------------------------------------------
struct NoAcc {};

template <typename T, int N>
struct OpBase {
  static constexpr bool ROLLED = false;  // heavy per-element epilogue: process through LDS in a rolled loop
  LineArgs a;
  // the blocks of one tile for every entry of the batch are dispatched together, on one XCD (k_lines): for stages
  // that read an array all entries share (the potential), whose rows then stay in that XCD's L2 while the entries pass
  static constexpr bool TILE_MAJOR = false;
  DBAR_D bool active(int b) const { return a.act == nullptr || a.act[b] != 0; }
  DBAR_D const cx<T>* inp(int b) const { return static_cast<const cx<T>*>(a.in) + (size_t)b * a.in_bs; }
  DBAR_D cx<T>* outp(int b) const { return static_cast<cx<T>*>(a.out) + (size_t)b * a.out_bs; }
  template <class Acc> DBAR_D void mid(int, int, int, cx<T>&) const {}
  template <int NT, class Acc> DBAR_D void finish(Acc&, int, int, int, double*) const {}
  // after the stores: dots over the values the stores left in the thread's registers (ops that define DOTS)
  static constexpr bool DOTS = false;
  // the op works on its loaded values before the first transform (loaded(acc, b, line, jt, v, tile, ntiles, scratch)
  // may change them; it must be called by all threads of the block)
  static constexpr bool LOADACC = false;
  // ROLLED stores: > 1: the op's store_all stores the thread's elements GROUP at a time, else store one at a time
  static constexpr int GROUP = 1;
  // per-block data read once at kernel start, before any store (ops that need it define PRE and a Pre type)
  static constexpr bool PRE = false;
  struct Pre {};
  DBAR_D void prologue(int, Pre&) const {}
};

// out = IFFT_rows(phase * ci * in)
template <typename T, int N>
struct OpRowsInvScaled : OpBase<T, N> {
  static constexpr int DIR1 = +1;
  static constexpr bool TWO = false;
  using Acc = NoAcc;
  DBAR_D cx<T> load(int b, int row, int pos) const {
    const T f = static_cast<T>(((row + pos) & 1) ? -this->a.ci : this->a.ci);
    return f * this->inp(b)[(size_t)row * N + pos];
  }
  DBAR_D void store(Acc&, int b, int row, int pos, cx<T> v) const { this->outp(b)[(size_t)row * N + pos] = v; }
};

// Moments sum z^n s (n <= M) and sum conj(z) s of x-space values s, reduced in FP64.  Along a line one coordinate
// is fixed (x on a column, y on a row); each thread accumulates mu_k = sum t^k s over its elements (t the varying
// coordinate: real weights, k <= M) and the line's share of d_n = sum_k C(n,k) (fixed part)^(n-k) (t part)^k is
// formed once at the end: on a column d_n = sum_k C(n,k) x^{n-k} i^k mu_k, conj moment x mu_0 - i mu_1; on a row
// d_n = sum_k C(n,k) (iy)^{n-k} mu_k, conj moment mu_1 - iy mu_0 (the binomial terms exceed |z|^n by at most
// 2^{n/2}, i.e. < 50x at n = 11: a few ulps of FP64).
// One step of a recursive-halving wave reduction: lanes with bit OFF clear keep the lower NV/2 of their values, the
// others the upper half, each summed with its partner's copy of the same half (lane ^ OFF).
template <typename T, int NV, int OFF>
DBAR_D void halve_exchange(T (&x)[32], int lane) {
  const bool hi = (lane & OFF) != 0;
#pragma unroll
  for (int i = 0; i < NV / 2; ++i) {
    const T keep = hi ? x[i + NV / 2] : x[i];
    const T send = hi ? x[i] : x[i + NV / 2];
    x[i] = keep + __shfl_xor(send, OFF, 64);
  }
}

template <typename T, int N, bool ALONG_X>
struct MomentsBase : OpBase<T, N> {
  static constexpr int NV = 2 * kNMom;
  static constexpr int NMU = 2 * (kMaxM + 1);  // mu_0 .. mu_kMaxM (re, im)
  // Per-thread moments are accumulated in the transform's precision (16 elements per thread; the FP32 operator's s
  // carries FP32 rounding anyway, and the regularisation is exact for any G coefficients); every reduction beyond
  // the thread and the binomial combination run in FP64.
  struct Acc {
    T v[NMU];  // mu_k = sum t^k s over this thread's elements
  };
  // the fixed coordinate of line `line`
  DBAR_D double fixed(int line) const { return xgrid<N>(line, this->a.L); }
  // s at position pos of line `line` into this thread's mu_k
  DBAR_D void add(Acc& acc, int b, int line, int pos, cx<T> v) const {
    cx<T> s = v;
    // shifted regularisation: Taylor coefficients at xi = a are moments of s e^{-i a.x} = s e_k (the varying
    // coordinate's factor here, the fixed one's in combine_one)
    if (this->a.shv) {
      const size_t o = (size_t)b * this->a.e_bs + pos;
      if constexpr (sizeof(T) == 8) s = s * (ALONG_X ? this->a.ex[o] : this->a.ey[o]);
      else s = s * (ALONG_X ? this->a.ex32[o] : this->a.ey32[o]);
    }
    (void)line;
    // mu_0..mu_KK with KK fixed at compile time: the order M = 11 itself, else kMaxM (the extra mu_k are unused);
    // mu_1 is always needed (conj moment)
    if (this->a.M == 11) accumulate<11>(acc, xgrid_t<T, N>(pos, this->a.L), s);
    else accumulate<kMaxM>(acc, xgrid_t<T, N>(pos, this->a.L), s);
  }
  template <int KK>
  DBAR_D static void accumulate(Acc& acc, T t, cx<T> s) {
    T tp = T(1);
#pragma unroll
    for (int k = 0; k <= KK; ++k) {
      acc.v[2 * k] += tp * s.re;
      acc.v[2 * k + 1] += tp * s.im;
      tp *= t;
    }
  }
  // all of the thread's loaded values v[s] (position jt + s TPL) into its mu_k, the order's branch taken once
  DBAR_D void add_loaded(Acc& acc, int b, int line, int jt, const cx<T>* v) const {
    if (this->a.M == 11) add_all<11>(acc, b, jt, v);
    else add_all<kMaxM>(acc, b, jt, v);
    (void)line;
  }
  template <int KK>
  DBAR_D void add_all(Acc& acc, int b, int jt, const cx<T>* v) const {
    using G = LineGeom<N>;
#pragma unroll
    for (int s = 0; s < G::RMAX; ++s) {
      const int pos = jt + s * G::TPL;
      cx<T> sv = v[s];
      if (this->a.shv) {
        const size_t o = (size_t)b * this->a.e_bs + pos;
        if constexpr (sizeof(T) == 8) sv = sv * (ALONG_X ? this->a.ex[o] : this->a.ey[o]);
        else sv = sv * (ALONG_X ? this->a.ex32[o] : this->a.ey32[o]);
      }
      accumulate<KK>(acc, xgrid_t<T, N>(pos, this->a.L), sv);
    }
  }
  // Moment q of one line from its mu_k (q <= M; 0 for M < q <= kMaxM; q = kMaxM+1: the conj moment), c its fixed
  // coordinate; with the shifted regularisation times the line's factor of e_k.  mu is (re, im) interleaved.
  DBAR_D c64 combine_one(const double* mu, double c, int q, int b, int line) const {
    double re = 0.0, im = 0.0;
    if (q == kMaxM + 1) {
      if constexpr (ALONG_X) {  // mu_1 - i y mu_0
        re = mu[2] + c * mu[1];
        im = mu[3] - c * mu[0];
      } else {  // x mu_0 - i mu_1
        re = c * mu[0] + mu[3];
        im = c * mu[1] - mu[2];
      }
    } else if (q <= this->a.M) {
      double cpow = 1.0;  // c^{q-k} for k = q, q-1, ..., 0
      for (int k = q; k >= 0; --k) {
        const double w = kBinom.v[q][k] * cpow;
        const double mr = mu[2 * k], mi = mu[2 * k + 1];
        switch ((ALONG_X ? q - k : k) & 3) {  // times i^k (column) or i^{q-k} (row)
          case 0: re += w * mr; im += w * mi; break;
          case 1: re -= w * mi; im += w * mr; break;
          case 2: re -= w * mr; im -= w * mi; break;
          default: re += w * mi; im -= w * mr; break;
        }
        cpow *= c;
      }
    }
    c64 d{re, im};
    if (this->a.shv) d = (ALONG_X ? this->a.ey : this->a.ex)[(size_t)b * this->a.e_bs + line] * d;
    return d;
  }

  template <int NT>
  DBAR_D void finish(Acc& acc, int b, int tile, int ntiles, double* scratch) const {
    if (this->a.M == 11) finish_kk<NT, 11>(acc, b, tile, ntiles, scratch);
    else finish_kk<NT, kMaxM>(acc, b, tile, ntiles, scratch);
  }
  // Block reduction: 1) each line's mu_k summed over its threads within a wave by shuffles (a column tile
  // interleaves its lines, so a column's lanes differ by multiples of LN; a row's lanes are contiguous), parked in
  // LDS per reduction group; 2) summed over the line's groups (one thread per line and value); 3) combined into the
  // moments (one thread per line and moment); 4) the tile's partials: sum over its lines.
  template <int NT, int KK>
  DBAR_D void finish_kk(Acc& acc, int b, int tile, int ntiles, double* scratch) const {
    constexpr int NU = 2 * (KK + 1);  // mu values in use
    double* dst = this->a.part + (size_t)b * NV * ntiles + tile;
    constexpr int TPL = LineGeom<N>::TPL;
    constexpr int LN = NT / TPL;  // lines per tile
    // reduction groups: runs of GS consecutive lanes on a row tile; (wave, column) pairs on a column tile of fewer
    // than 64 columns (SHFL), else single threads
    constexpr int GS = ALONG_X ? (TPL < 64 ? TPL : 64) : 1;
    constexpr bool SHFL = !ALONG_X && NT >= 64 && LN < 64;
    constexpr int NG = ALONG_X ? NT / GS : SHFL ? (NT / 64) * LN : NT;
    static_assert(NG == LdsSize<T, N, LN, !ALONG_X>::NG, "LDS scratch sized for another reduction layout");
    __syncthreads();  // scratch aliases the transform's LDS
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double* sc = scratch;                 // [NG][NMU]
    double* colv = scratch + NG * NMU;    // [LN][NV]
    double* mus = colv + LN * NV;         // [LN][NMU]
    if constexpr (ALONG_X && GS == 64) {
      // a whole wave per row: recursive halving over the NMU = 32 values (those beyond NU are zero), five exchanges
      // that each send half of a lane's values and keep the other half summed with the partner's, then one plain
      // exchange; lane l ends with value l >> 1 summed over the wave (32 shuffles per lane instead of 6 NU)
      static_assert(NMU == 32, "the halving below is laid out for 32 values");
      T x[NMU];
#pragma unroll
      for (int q = 0; q < NMU; ++q) x[q] = q < NU ? acc.v[q] : T(0);
      halve_exchange<T, 32, 32>(x, lane);
      halve_exchange<T, 16, 16>(x, lane);
      halve_exchange<T, 8, 8>(x, lane);
      halve_exchange<T, 4, 4>(x, lane);
      halve_exchange<T, 2, 2>(x, lane);
      x[0] += __shfl_xor(x[0], 1, 64);
      if ((lane & 1) == 0) sc[wave * NMU + (lane >> 1)] = static_cast<double>(x[0]);
    } else {
#pragma unroll
      for (int q = 0; q < NU; ++q) {
        T x = acc.v[q];
        if constexpr (ALONG_X) {
#pragma unroll
          for (int off = GS / 2; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
        } else if constexpr (SHFL) {
#pragma unroll
          for (int off = 32; off >= LN; off >>= 1) x += __shfl_xor(x, off, 64);
        }
        acc.v[q] = x;
      }
      int g = -1;
      if constexpr (ALONG_X) {
        if (threadIdx.x % GS == 0) g = threadIdx.x / GS;
      } else if constexpr (SHFL) {
        if (lane < LN) g = wave * LN + lane;
      } else {
        g = threadIdx.x;  // thread t serves column t % LN
      }
      if (g >= 0) {
#pragma unroll
        for (int q = 0; q < NMU; ++q) sc[g * NMU + q] = q < NU ? static_cast<double>(acc.v[q]) : 0.0;
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < LN * NMU; t += NT) {
      const int c = t / NMU, q = t % NMU;
      double v = 0.0;
      if constexpr (ALONG_X) {
        constexpr int GPL = TPL / GS;  // groups per row
        for (int k = 0; k < GPL; ++k) v += sc[(c * GPL + k) * NMU + q];
      } else if constexpr (SHFL) {
        for (int w = 0; w < NT / 64; ++w) v += sc[(w * LN + c) * NMU + q];
      } else {
        for (int k = c; k < NT; k += LN) v += sc[k * NMU + q];
      }
      mus[c * NMU + q] = v;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < LN * kNMom; t += NT) {
      const int c = t / kNMom, q = t % kNMom;
      const int line = tile * LN + c;
      const c64 d = combine_one(mus + c * NMU, fixed(line), q, b, line);
      colv[c * NV + 2 * q] = d.re;
      colv[c * NV + 2 * q + 1] = d.im;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < NV; q += NT) {
      double t = 0.0;
      for (int c = 0; c < LN; ++c) t += colv[c * NV + q];
      dst[(size_t)q * ntiles] = t;
    }
  }
};

// IFFT_cols(in) and the moments of the result (second pass of F^{-1} S; nothing is stored)
template <typename T, int N>
struct OpColsInvMoments : MomentsBase<T, N, false> {
  static constexpr int DIR1 = +1;
  static constexpr bool TWO = false;
  static constexpr bool ROLLED = true;
  using Acc = typename MomentsBase<T, N, false>::Acc;
  DBAR_D cx<T> load(int b, int col, int pos) const { return this->inp(b)[(size_t)pos * N + col]; }
  DBAR_D void store(Acc& acc, int b, int col, int pos, cx<T> v) const { this->add(acc, b, col, pos, v); }
};

// x-space operator, first launch: the moments of the input s as it is read, then out = FFT_rows(s) (first pass of
// F s).  With upd_coef set it first updates s by a combination of basis vectors, s -= upd_sign sum_i coef_i V_i over
// upd_nv of them (FP64 accumulation, as the vector kernels; V in FP32 if upd_v32), and stores s back in place: the
// Gram-Schmidt step that produced s (with its |s|^2 partials in upd_part[b][tile]), or the solution update
// x += sum y_i V_i of a cycle end (upd_sign -1) -- the operator's first launch reads s anyway.
template <typename T, int N>
struct OpRowsFwdMoments : MomentsBase<T, N, true> {
  static constexpr int DIR1 = -1;
  static constexpr bool TWO = false;
  static constexpr bool LOADACC = true;
  using Acc = typename MomentsBase<T, N, true>::Acc;
  DBAR_D cx<T> load(int b, int row, int pos) const { return this->inp(b)[(size_t)row * N + pos]; }
  template <int NT>
  DBAR_D void loaded(Acc& acc, int b, int row, int jt, cx<T>* v, int tile, int ntiles, double* scratch) const {
    using G = LineGeom<N>;
    const LineArgs& a = this->a;
    if (a.upd_coef) {
      const double* coef = a.upd_coef + (size_t)b * a.upd_coef_bs;
      const cx<T>* V = static_cast<const cx<T>*>(a.dotV) + (size_t)b * a.dotV_bs + (size_t)row * N;
      c64 w[G::RMAX];
#pragma unroll
      for (int s = 0; s < G::RMAX; ++s) w[s] = a.upd_zero ? c64{0.0, 0.0} : cvt<double>(v[s]);
#pragma unroll 1
      for (int i = 0; i < a.upd_nv; ++i) {
        const double c = a.upd_sign * coef[i];
        if (c == 0.0) continue;  // also keeps never-written basis slots (any bit pattern) out of the sum
        if (sizeof(T) == 8 && a.upd_v32) {
          const c32* Vi = static_cast<const c32*>(a.dotV) + (size_t)b * a.dotV_bs + (size_t)row * N + (size_t)i * N * N;
#pragma unroll
          for (int s = 0; s < G::RMAX; ++s) w[s] = w[s] - c * cvt<double>(Vi[jt + s * G::TPL]);
        } else {
          const cx<T>* Vi = V + (size_t)i * N * N;
#pragma unroll
          for (int s = 0; s < G::RMAX; ++s) w[s] = w[s] - c * cvt<double>(Vi[jt + s * G::TPL]);
        }
      }
      cx<T>* out = static_cast<cx<T>*>(a.upd_out) + (size_t)b * a.in_bs + (size_t)row * N;
      double nrm[1] = {0.0};
#pragma unroll
      for (int s = 0; s < G::RMAX; ++s) {
        v[s] = cvt<T>(w[s]);
        out[jt + s * G::TPL] = v[s];
        nrm[0] += rdot(v[s], v[s]);
      }
      if (a.upd_part) {
        block_reduce_store<NT, 1>(nrm, a.upd_part + (size_t)b * ntiles + tile, 0, scratch);
        __syncthreads();  // the scratch aliases the LDS the transform's first exchange writes
      }
    }
    this->add_loaded(acc, b, row, jt, v);
  }
  DBAR_D void store(Acc&, int b, int row, int pos, cx<T> v) const {
    this->outp(b)[t_index<T, N>(row, pos)] = v;
  }
};

// sum_{n <= MM} c_n w^n by Horner's rule
template <int MM>
DBAR_D c64 g_poly(const c64* __restrict__ c, c64 w) {
  c64 g = c[MM];
#pragma unroll
  for (int n = MM - 1; n >= 0; --n) g = cfma(w, g, c[n]);
  return g;
}
// the same in FP32, from the FP32 roundings of the coefficients
template <int MM>
DBAR_D c32 g_poly32(const c64* __restrict__ c, c32 w) {
  c32 g = cvt<float>(c[MM]);
#pragma unroll
  for (int n = MM - 1; n >= 0; --n) g = cfma(w, g, cvt<float>(c[n]));
  return g;
}

// Per-entry data of the regularised division: the grid offsets (o1, o2) of the regularisation point a and the entry's
// coefficients c_0..c_kMaxM of G (R(0) in slot kMaxM+1), read where they are used: only the points near a need them
// (|xi - a|^2 < 740: 5% of the grid at N = 1024, L = 5), so they are not held in registers across a block's loop.
struct RegPre {
  int o1, o2;
  const c64* c;
};
DBAR_D void regularised_pre(const LineArgs& a, int b, RegPre& p) {
  p.o1 = a.shv ? a.shv[2 * b] : 0;
  p.o2 = a.shv ? a.shv[2 * b + 1] : 0;
  p.c = a.coefG + (size_t)b * kNMom;
}

// R = (S - G)/xi (R(0) from coefG slot kMaxM+1), then out = IFFT_rows(phase * ci * R)
// phase * ci * (S - G)/xi at (row, pos) of entry b, S = sv there (R(0) = coefG slot kMaxM+1 at xi = a)
template <typename T, int N>
DBAR_D cx<T> regularised(const LineArgs& a, const RegPre& p, int row, int pos, cx<T> sv) {
  const c64* c = p.c;
  // xi - a with a = 2i conj(k) on the grid (not reduced modulo the period: the quotient only jumps at the edge),
  // as integer wave numbers: L^2 |xi - a|^2 = m1^2 + m2^2 exactly
  const int m1 = wavenum(pos, N) - p.o1, m2 = wavenum(row, N) - p.o2;
  const int q = m1 * m1 + m2 * m2;
  const double f = ((row + pos) & 1) ? -a.ci : a.ci;
  if (q == 0) return cvt<T>(f * c[kMaxM + 1]);
  const double invL = 1.0 / a.L;
  if constexpr (sizeof(T) == 8) {
    // G only where e^{-|xi|^2} has not underflowed
    const double xi1 = m1 * invL, xi2 = m2 * invL, r2 = xi1 * xi1 + xi2 * xi2;
    if (r2 < 740.0) {
      // unrolled for the order (c_n = 0 beyond M): the coefficient loads are issued together
      const c64 xib{xi1, -xi2};
      const c64 g = a.M == 11 ? g_poly<11>(c, xib) : g_poly<kMaxM>(c, xib);
      sv = sv - exp(-r2) * g;
    }
    const double ir2 = f / r2;
    return cx<T>{(sv.re * xi1 + sv.im * xi2) * ir2, (sv.im * xi1 - sv.re * xi2) * ir2};
  } else {
    // The FP32 operator (inner solves) forms G in FP32 too: S is already rounded to FP32, and G's rounding is of the
    // same size.  e^{-|xi|^2} is zero in FP32 from |xi|^2 = 104 on, so G is formed inside that disc only (|conj(xi)|^n
    // < 2e11 there, far from FP32 overflow).
    const float il = static_cast<float>(invL);
    const float t1 = static_cast<float>(m1) * il, t2 = static_cast<float>(m2) * il;
    const float r2 = t1 * t1 + t2 * t2;
    if (r2 < 104.0f) {
      const c32 w{t1, -t2};
      const c32 g = a.M == 11 ? g_poly32<11>(c, w) : g_poly32<kMaxM>(c, w);
      sv = sv - exp(-r2) * g;
    }
    const float ir2 = static_cast<float>(f) * recip(r2);
    return cx<T>{(sv.re * t1 + sv.im * t2) * ir2, (sv.im * t1 - sv.re * t2) * ir2};
  }
}

template <typename T, int N>
struct OpRowsInvRegular : OpBase<T, N> {
  static constexpr int DIR1 = +1;
  static constexpr bool TWO = false;
  using Acc = NoAcc;
  DBAR_D cx<T> load(int b, int row, int pos) const {
    RegPre p;
    regularised_pre(this->a, b, p);
    return regularised<T, N>(this->a, p, row, pos, this->inp(b)[(size_t)row * N + pos]);
  }
  DBAR_D void store(Acc&, int b, int row, int pos, cx<T> v) const { this->outp(b)[(size_t)row * N + pos] = v; }
};

// x-space operator, second launch: S = cf phase FFT_cols(in) (the second pass of F s; optionally stored to sout),
// R = (S - G)/xi, then out = IFFT_cols(phase ci R), between the two column transforms (rolled through LDS: the FP64
// G terms)
template <typename T, int N>
struct OpColsFwdRegInv : OpBase<T, N> {
  static constexpr int DIR1 = -1;
  static constexpr bool TWO = true;
  static constexpr bool ROLLED = true;
  using Acc = NoAcc;
  DBAR_D cx<T> load(int b, int col, int pos) const { return this->inp(b)[t_index<T, N>(pos, col)]; }
  static constexpr bool PRE = true;
  using Pre = RegPre;
  DBAR_D void prologue(int b, Pre& p) const { regularised_pre(this->a, b, p); }
  template <class A>
  DBAR_D void mid(int b, int col, int pos, cx<T>& v, const Pre& p) const {
    const T f = static_cast<T>(((col + pos) & 1) ? -this->a.cf : this->a.cf);
    const cx<T> S = f * v;
    if (this->a.sout) (static_cast<cx<T>*>(this->a.sout) + (size_t)b * this->a.sout_bs)[(size_t)pos * N + col] = S;
    v = regularised<T, N>(this->a, p, pos, col, S);  // row = xi2 index (pos), position = xi1 index (col)
  }
  DBAR_D void store(Acc&, int b, int col, int pos, cx<T> v, const Pre&) const {
    this->outp(b)[t_index<T, N>(pos, col)] = v;
  }
};

// r = IFFT_cols(in); h = r + tail; [hout = h]; u = q_k conj(h); out = FFT_cols(u)   (TAILONLY: stop after hout)
template <typename T, int N, bool TAILONLY>
struct OpColsInvTail : OpBase<T, N> {
  static constexpr int DIR1 = +1;
  static constexpr bool TWO = !TAILONLY;
  static constexpr bool ROLLED = true;
  using Acc = NoAcc;
  DBAR_D cx<T> load(int b, int col, int pos) const { return this->inp(b)[(size_t)pos * N + col]; }
  DBAR_D cx<T> phase(int b, int col, int pos) const {
    // tabulated in FP64 (arguments up to hundreds of radians; the FP32 operator reads their FP32 roundings); the
    // product is formed in T
    const size_t o = (size_t)b * this->a.e_bs;
    if constexpr (sizeof(T) == 8) return this->a.ex[o + col] * this->a.ey[o + pos];
    else return this->a.ex32[o + col] * this->a.ey32[o + pos];
  }
  // the moments d_0..d_kMaxM of this entry (zero beyond M) in registers, in the transform's precision
  static constexpr bool PRE = true;
  struct Pre {
    cx<T> d[kMaxM + 1];
  };
  DBAR_D void prologue(int b, Pre& p) const {
    const cx<T>* d;
    if constexpr (sizeof(T) == 8) d = this->a.dmom + (size_t)b * kNMom;
    else d = this->a.dmom32 + (size_t)b * kNMom;
#pragma unroll
    for (int n = 0; n <= kMaxM; ++n) p.d[n] = d[n];
  }
  // h = F^{-1}R + sum d_n omega_n; with the shifted regularisation the closed-form part is e^{i a.x} sum d_n omega_n
  DBAR_D cx<T> h_at(int b, int col, int pos, cx<T> v, const Pre& p) const {
    const T x = xgrid_t<T, N>(col, this->a.L), y = xgrid_t<T, N>(pos, this->a.L);
    const cx<T> t = this->a.M == 11 ? tail_sum<T, 11>(x, y, p.d) : tail_sum<T, kMaxM>(x, y, p.d);
    return this->a.shv ? v + conj(phase(b, col, pos)) * t : v + t;
  }
  template <class A>
  DBAR_D void mid(int b, int col, int pos, cx<T>& v, const Pre& p) const {
    const cx<T> h = h_at(b, col, pos, v, p);
    if (this->a.hout) (static_cast<cx<T>*>(this->a.hout) + (size_t)b * this->a.hout_bs)[(size_t)pos * N + col] = h;
    const cx<T> q = (static_cast<const cx<T>*>(this->a.Q) + (size_t)b * this->a.Q_bs)[(size_t)pos * N + col];
    // plain: q_k = Q e_k; shifted (the operator H of equation eqh2): Q alone
    v = (this->a.shv ? q : q * phase(b, col, pos)) * conj(h);
  }
  DBAR_D void store(Acc&, int b, int col, int pos, cx<T> v, const Pre& p) const {
    if constexpr (TAILONLY) {
      cx<T> h = h_at(b, col, pos, v, p);
      if (this->a.tail_phase_out) h = phase(b, col, pos) * h;
      cx<T>* dst = static_cast<cx<T>*>(this->a.hout) + (size_t)b * this->a.hout_bs + (size_t)pos * N + col;
      if (this->a.accumulate) h = h + *dst;
      *dst = h;
    } else {
      this->outp(b)[(size_t)pos * N + col] = v;
    }
  }
};

// X = FFT_rows(in); out = alpha S + beta cf phase X + gamma Y; optional |out|^2 partials
template <typename T, int N>
struct OpRowsFwdEpilogue : OpBase<T, N> {
  static constexpr int DIR1 = -1;
  static constexpr bool TWO = false;
  static constexpr bool DOTS = true;
  struct Acc {
    double v[1];
    double sdot;  // Re<S, out> over this thread's elements (S is the last vector of the fused products)
  };
  DBAR_D cx<T> load(int b, int row, int pos) const { return this->inp(b)[(size_t)row * N + pos]; }
  // X (the row transform's output) is replaced by the stored value, for the Gram-Schmidt products below
  DBAR_D void store(Acc& acc, int b, int row, int pos, cx<T>& X) const {
    const LineArgs& a = this->a;
    const size_t idx = (size_t)row * N + pos;
    const double f = ((row + pos) & 1) ? -a.cf : a.cf;
    c64 o = a.beta * (f * cvt<double>(X));
    c64 sv{0.0, 0.0};
    if (a.alpha != 0.0) {
      sv = cvt<double>((static_cast<const cx<T>*>(a.S) + (size_t)b * a.S_bs)[idx]);
      o = o + a.alpha * sv;
    }
    if (a.gamma != 0.0) o = o + a.gamma * cvt<double>((static_cast<const cx<T>*>(a.Y) + (size_t)b * a.Y_bs)[idx]);
    const cx<T> ot = cvt<T>(o);
    this->outp(b)[idx] = ot;
    X = ot;
    const c64 od = cvt<double>(ot);
    acc.v[0] += norm2(od);
    acc.sdot += sv.re * od.re + sv.im * od.im;
  }
  template <int NT>
  DBAR_D void finish(Acc& acc, int b, int tile, int ntiles, double* scratch) const {
    if (!this->a.want_norm) return;
    block_reduce_store<NT, 1>(acc.v, this->a.part + (size_t)b * ntiles + tile, 0, scratch);
  }
  // Re<V_i, out> over this tile for i < dot_nv, from the output values in registers (FP64 accumulation, the order
  // fixed): the multi-dot of the first classical Gram-Schmidt pass without reading the new vector back.  The last
  // vector, V_{dot_nv - 1}, is the epilogue's S (the operator's input) and was accumulated by the stores.
  template <int NT>
  DBAR_D void dots(const Acc& acc, const cx<T>* v, int b, int row, int jt, int tile, int ntiles,
                   double* scratch) const {
    using G = LineGeom<N>;
    const LineArgs& a = this->a;
    if (a.dot_nv <= 0) return;
    const cx<T>* V = static_cast<const cx<T>*>(a.dotV) + (size_t)b * a.dotV_bs + (size_t)row * N;
    double* dst = a.dot_part + (size_t)b * a.dot_nv * ntiles + tile;
    const double last[1] = {acc.sdot};
    block_reduce_store<NT, 1>(last, dst + (size_t)(a.dot_nv - 1) * ntiles, 0, scratch);
#pragma unroll 1
    for (int i = 0; i < a.dot_nv - 1; ++i) {
      const cx<T>* Vi = V + (size_t)i * N * N;
      double p4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < G::RMAX; ++s) {
        const c64 x = cvt<double>(Vi[jt + s * G::TPL]);
        const c64 w = cvt<double>(v[s]);
        p4[s & 3] += x.re * w.re + x.im * w.im;
      }
      const double val[1] = {(p4[0] + p4[1]) + (p4[2] + p4[3])};
      block_reduce_store<NT, 1>(val, dst + (size_t)i * ntiles, 0, scratch);
    }
  }
};

// x-space operator, third launch: r = IFFT_rows(in) (second pass of F^{-1} R), h = r + sum d_n omega_n, and the
// x-space form of A: out = alpha s + beta q_k conj(h) + gamma Y (F^{-1} of S + i F(q_k conj(h)) is s + i q_k conj(h));
// optional |out|^2 partials, h itself (hout) and the products Re<V_i, out> of the first Gram-Schmidt pass.
// Rows keep every global access of the epilogue and the products contiguous across a wave.
template <typename T, int N>
struct OpRowsInvTailEpi : OpColsInvTail<T, N, false> {
  static constexpr int DIR1 = +1;
  static constexpr bool TWO = false;
  static constexpr bool ROLLED = true;
  static constexpr bool DOTS = true;
  // q_k's potential is one array for the batch: tile-major at N = 4096, where the potential (134 MB in FP32) is
  // otherwise fetched again for most entries (measured 3-7% off the launch); at N = 1024 the tile-major order
  // measured 2-4% slower per launch, and the entry-major order stays
  static constexpr bool TILE_MAJOR = N >= 4096;
  using Pre = typename OpColsInvTail<T, N, false>::Pre;
  struct Acc {
    double v[1];
    double sdot;  // Re<S, out> over this thread's elements (S is the last vector of the fused products)
  };
  DBAR_D cx<T> load(int b, int row, int pos) const { return this->inp(b)[t_index<T, N>(row, pos)]; }
  // The stores run GROUP elements at a time: the group's global reads (q, the x factor of e_k, S, Y) are issued
  // together ahead of its tails.  The LDS slot of each element (the row transform's output r) is replaced by the
  // stored value, for the Gram-Schmidt products.
  // four at a time: wider groups hold more registers than the loads in flight repay (the FP32 launch drops to three
  // waves per SIMD at eight)
  static constexpr int GROUP_W = 4;
  static constexpr int GROUP = LineGeom<N>::RMAX < GROUP_W ? LineGeom<N>::RMAX : GROUP_W;
  struct GroupIn {
    cx<T> q[GROUP], s[GROUP], y[GROUP], ex[GROUP];
  };
  // the group's q (times the x factor of e_k on the plain operator), S and Y
  DBAR_D void group_load(GroupIn& g, int b, int row, int jt, int s0) const {
    using G = LineGeom<N>;
    const LineArgs& a = this->a;
    const size_t base = (size_t)row * N;
    const cx<T>* Qb = static_cast<const cx<T>*>(a.Q) + (size_t)b * a.Q_bs + base;
    const cx<T>* Sb = static_cast<const cx<T>*>(a.S) + (size_t)b * a.S_bs + base;
    const cx<T>* Yb = static_cast<const cx<T>*>(a.Y) + (size_t)b * a.Y_bs + base;
    const size_t eo = (size_t)b * a.e_bs;
#pragma unroll
    for (int u = 0; u < GROUP; ++u) {
      const int pos = jt + (s0 + u) * G::TPL;
      g.q[u] = Qb[pos];
      g.s[u] = a.alpha != 0.0 ? Sb[pos] : cx<T>{T(0), T(0)};
      g.y[u] = (a.gamma != 0.0 && !a.y_rhs) ? Yb[pos] : cx<T>{T(0), T(0)};
      if (a.shv) g.ex[u] = cx<T>{T(1), T(0)};
      else if constexpr (sizeof(T) == 8) g.ex[u] = a.ex[eo + pos];
      else g.ex[u] = a.ex32[eo + pos];
    }
  }
  template <int LS>
  DBAR_D void store_all(Acc& acc, int b, int row, int jt, cx<T>* my, const Pre& p) const {
    using G = LineGeom<N>;
    static_assert(G::RMAX % GROUP == 0, "whole groups");
    const LineArgs& a = this->a;
    const size_t base = (size_t)row * N;
    // the y factor of e_k is the row's (1 with the shifted regularisation, where q stands alone)
    cx<T> ey{T(1), T(0)};
    if (!a.shv) {
      if constexpr (sizeof(T) == 8) ey = a.ey[(size_t)b * a.e_bs + row];
      else ey = a.ey32[(size_t)b * a.e_bs + row];
    }
#pragma unroll 1
    for (int s0 = 0; s0 < G::RMAX; s0 += GROUP) {
      GroupIn cur;
      group_load(cur, b, row, jt, s0);
#pragma unroll
      for (int u = 0; u < GROUP; ++u) {
        const int pos = jt + (s0 + u) * G::TPL;
        cx<T>& slot = my[G::padded(pos) * LS];
        const cx<T> h = this->h_at(b, pos, row, slot, p);  // x index pos, y index row
        if (a.hout) (static_cast<cx<T>*>(a.hout) + (size_t)b * a.hout_bs)[base + pos] = h;
        const cx<T> qk = cur.q[u] * (cur.ex[u] * ey);
        const cx<T> w = qk * conj(h);
        const cx<T> yv = a.y_rhs ? mul_mi(qk) : cur.y[u];
        cx<T> ot;
        if constexpr (sizeof(T) == 8) {
          ot = a.beta * w + a.alpha * cur.s[u] + a.gamma * yv;
        } else {  // the FP32 operator's result is FP32: form it in FP32
          ot = cvt<T>(a.beta) * w + static_cast<T>(a.alpha) * cur.s[u] + static_cast<T>(a.gamma) * yv;
        }
        if (a.out) this->outp(b)[base + pos] = ot;
        if constexpr (sizeof(T) == 8) {
          if (a.out32) (static_cast<c32*>(a.out32) + (size_t)b * a.out32_bs)[base + pos] = cvt<float>(ot);
        }
        slot = ot;
        acc.v[0] += rdot(ot, ot);
        acc.sdot += rdot(cur.s[u], ot);
      }
    }
  }
  template <int NT>
  DBAR_D void finish(Acc& acc, int b, int tile, int ntiles, double* scratch) const {
    if (!this->a.want_norm) return;
    block_reduce_store<NT, 1>(acc.v, this->a.part + (size_t)b * ntiles + tile, 0, scratch);
  }
  // Re<V_i, out> over this tile for i < dot_nv (FP64 accumulation, the order fixed); V_{dot_nv - 1} is S, whose
  // products the stores accumulated, as they did |out|^2 (value dot_nv with dot_self).  Each wave reduces its
  // products by shuffles and parks them in LDS; one barrier
  // then serves all of them (the waves read their next V_i while others still compute).
  template <int NT>
  DBAR_D void dots(const Acc& acc, const cx<T>* v, int b, int row, int jt, int tile, int ntiles,
                   double* scratch) const {
    using G = LineGeom<N>;
    const LineArgs& a = this->a;
    const int nv = a.dot_nv;
    if (nv <= 0) return;
    const int nval = nv + (a.dot_self ? 1 : 0);
    // vectors below the entry's Gram-Schmidt window (never V_{nv - 1}, the input itself)
    const int skip = (a.dot_full && !a.dot_full[b]) ? a.dot_skip : 0;
    const cx<T>* V = static_cast<const cx<T>*>(a.dotV) + (size_t)b * a.dotV_bs + (size_t)row * N;
    double* dst = a.dot_part + (size_t)b * nval * ntiles + tile;
    auto partial = [&](int i) {
      const cx<T>* Vi = V + (size_t)i * N * N;
      double p4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < G::RMAX; ++s) p4[s & 3] += rdot(Vi[jt + s * G::TPL], v[s]);
      return (p4[0] + p4[1]) + (p4[2] + p4[3]);
    };
    if constexpr (NT >= 64) {
      constexpr int NW = NT / 64;
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
      __syncthreads();  // scratch aliases the LDS the stores and the norm reduction used
      double x = wsum64(acc.sdot);
      if (lane == 0) scratch[(nv - 1) * NW + wave] = x;
      if (a.dot_self) {
        x = wsum64(acc.v[0]);
        if (lane == 0) scratch[nv * NW + wave] = x;
      }
#pragma unroll 1
      for (int i = 0; i < nv - 1; ++i) {
        x = i < skip ? 0.0 : wsum64(partial(i));
        if (lane == 0) scratch[i * NW + wave] = x;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < nval; i += NT) {
        double t = 0.0;
        for (int q = 0; q < NW; ++q) t += scratch[i * NW + q];
        dst[(size_t)i * ntiles] = t;
      }
    } else {
      const double last[1] = {acc.sdot};
      block_reduce_store<NT, 1>(last, dst + (size_t)(nv - 1) * ntiles, 0, scratch);
      if (a.dot_self) block_reduce_store<NT, 1>(acc.v, dst + (size_t)nv * ntiles, 0, scratch);
#pragma unroll 1
      for (int i = 0; i < nv - 1; ++i) {
        const double val[1] = {i < skip ? 0.0 : partial(i)};
        block_reduce_store<NT, 1>(val, dst + (size_t)i * ntiles, 0, scratch);
      }
    }
  }
};

// out = FFT_cols(Q e_k)
template <typename T, int N>
struct OpColsFwdPotential : OpBase<T, N> {
  static constexpr int DIR1 = -1;
  static constexpr bool TWO = false;
  using Acc = NoAcc;
  DBAR_D cx<T> load(int b, int col, int pos) const {
    const c64 q = cvt<double>((static_cast<const cx<T>*>(this->a.Q) + (size_t)b * this->a.Q_bs)[(size_t)pos * N + col]);
    const c64 e = this->a.ex[(size_t)b * this->a.e_bs + col] * this->a.ey[(size_t)b * this->a.e_bs + pos];
    return cvt<T>(q * e);
  }
  DBAR_D void store(Acc&, int b, int col, int pos, cx<T> v) const { this->outp(b)[(size_t)pos * N + col] = v; }
};

// out = FFT_cols(in) (DIR -1) or IFFT_cols(in) (DIR +1)
template <typename T, int N, int DIR>
struct OpColsPlain : OpBase<T, N> {
  static constexpr int DIR1 = DIR;
  static constexpr bool TWO = false;
  using Acc = NoAcc;
  DBAR_D cx<T> load(int b, int col, int pos) const { return this->inp(b)[(size_t)pos * N + col]; }
  DBAR_D void store(Acc&, int b, int col, int pos, cx<T> v) const { this->outp(b)[(size_t)pos * N + col] = v; }
};

// ------------------------------------------------------------------------------------------------------------
// The generic line kernel
// ------------------------------------------------------------------------------------------------------------
DBAR_D int xcd_swizzle(int bid, int nblk) {
  // blocks are dispatched round-robin over the 8 XCDs; give each XCD a contiguous range of tiles so that tiles
  // sharing cache lines (narrow column tiles) meet in the same L2
  if ((nblk & 7) != 0) return bid;
  return (bid & 7) * (nblk >> 3) + (bid >> 3);
}


// Occupancy floor: at least 4 waves per SIMD (<= 128 VGPRs) for the wide column tiles, whose LDS allows two
// blocks per CU only if the registers do too.
template <int NT>
struct MinWaves {
  static constexpr int value = NT >= 256 ? 4 : 1;
};

template <typename T, int N, int LINES, bool COLS, class Op>
__global__ void __launch_bounds__(LINES * LineGeom<N>::TPL, MinWaves<LINES * LineGeom<N>::TPL>::value)
    k_lines(Op op) {
  using G = LineGeom<N>;
  constexpr int NT = LINES * G::TPL;
  __shared__ cx<T> lds[LdsSize<T, N, LINES, COLS>::kElems];
  // pass-1 twiddle table: column stages only (their element work makes them arithmetic-bound)
  __shared__ cx<T> lds_t1[COLS ? Pass1Table<N>::SIZE : 1];
  constexpr int NTILES = N / LINES;
  int b, tile;
  if constexpr (Op::TILE_MAJOR) {
    // one-dimensional grid of NTILES x B blocks; block i goes to XCD i mod 8, whose k-th block (k = i / 8) is entry
    // k mod B of tile k / B within the XCD's contiguous range of tiles
    const int i = blockIdx.x, nb = gridDim.x / NTILES;
    if constexpr ((NTILES & 7) == 0) {
      const int k = i >> 3;
      tile = (i & 7) * (NTILES >> 3) + k / nb;
      b = k % nb;
    } else {
      tile = i / nb;
      b = i % nb;
    }
  } else {
    b = blockIdx.y;
    tile = xcd_swizzle(blockIdx.x, gridDim.x);
  }
  if (!op.active(b)) return;
  typename Op::Pre pre;
  op.prologue(b, pre);
  const int tid = threadIdx.x;
  const int ln = COLS ? (tid % LINES) : (tid / G::TPL);
  const int jt = COLS ? (tid / LINES) : (tid % G::TPL);
  const int line = tile * LINES + ln;
  const cx<T>* tw = static_cast<const cx<T>*>(op.a.tw);
  if constexpr (COLS) fill_pass1_table<T, N>(lds_t1, tw, tid, NT);

  typename Op::Acc acc{};
  cx<T> v[G::RMAX];
#pragma unroll
  for (int s = 0; s < G::RMAX; ++s) v[s] = op.load(b, line, jt + s * G::TPL);
  if constexpr (Op::LOADACC) op.template loaded<NT>(acc, b, line, jt, v, tile, NTILES, reinterpret_cast<double*>(lds));
  // LDS: a row tile keeps each line contiguous (one line per wave or less); a column tile interleaves its lines
  // element by element, so that the lanes of a wave (consecutive columns) hit consecutive banks
  constexpr int LS = COLS ? LINES : 1;
  cx<T>* my = COLS ? lds + ln : lds + ln * G::LDS_LINE;
  line_fft<T, N, Op::DIR1, LS, COLS>(v, jt, my, tw, lds_t1);
  // Heavy per-element work (FP64 moments, the closed-form tail) runs in a rolled loop over values parked in LDS at
  // the thread's own positions: registers stay low (occupancy) and no barrier is needed until the next exchange.
  if constexpr (Op::TWO) {
    if constexpr (Op::ROLLED) {
#pragma unroll
      for (int s = 0; s < G::RMAX; ++s) my[G::padded(jt + s * G::TPL) * LS] = v[s];
#pragma unroll 1
      for (int s = 0; s < G::RMAX; ++s) {
        const int pos = jt + s * G::TPL;
        cx<T> t = my[G::padded(pos) * LS];
        if constexpr (Op::PRE) op.template mid<typename Op::Acc>(b, line, pos, t, pre);
        else op.template mid<typename Op::Acc>(b, line, pos, t);
        my[G::padded(pos) * LS] = t;
      }
#pragma unroll
      for (int s = 0; s < G::RMAX; ++s) v[s] = my[G::padded(jt + s * G::TPL) * LS];
      __syncthreads();  // the forward transform's first exchange writes other threads' positions
    } else {
#pragma unroll
      for (int s = 0; s < G::RMAX; ++s) {
        if constexpr (Op::PRE) op.template mid<typename Op::Acc>(b, line, jt + s * G::TPL, v[s], pre);
        else op.template mid<typename Op::Acc>(b, line, jt + s * G::TPL, v[s]);
      }
    }
    line_fft<T, N, -Op::DIR1, LS, COLS>(v, jt, my, tw, lds_t1);
  }
  if constexpr (Op::ROLLED && !Op::TWO) {
#pragma unroll
    for (int s = 0; s < G::RMAX; ++s) my[G::padded(jt + s * G::TPL) * LS] = v[s];
    if constexpr (Op::GROUP > 1) {
      op.template store_all<LS>(acc, b, line, jt, my, pre);
    } else {
#pragma unroll 1
      for (int s = 0; s < G::RMAX; ++s) {
        const int pos = jt + s * G::TPL;
        if constexpr (Op::PRE) op.store(acc, b, line, pos, my[G::padded(pos) * LS], pre);
        else op.store(acc, b, line, pos, my[G::padded(pos) * LS]);
      }
    }
    // the stored values (the stores may replace them) back to registers for the products below, before the
    // reductions reuse the LDS (the thread's own positions: no barrier)
    if constexpr (Op::DOTS) {
#pragma unroll
      for (int s = 0; s < G::RMAX; ++s) v[s] = my[G::padded(jt + s * G::TPL) * LS];
    }
  } else {
#pragma unroll
    for (int s = 0; s < G::RMAX; ++s) {
      if constexpr (Op::PRE) op.store(acc, b, line, jt + s * G::TPL, v[s], pre);
      else op.store(acc, b, line, jt + s * G::TPL, v[s]);
    }
  }
  op.template finish<NT>(acc, b, tile, NTILES, reinterpret_cast<double*>(lds));
  if constexpr (Op::DOTS) op.template dots<NT>(acc, v, b, line, jt, tile, NTILES, reinterpret_cast<double*>(lds));
}

template <typename T, int N, bool COLS, class Op, int V = 0>
void launch_op(const LineArgs& a, hipStream_t s) {
  constexpr int LINES = COLS ? Tiling<T, N>::template cols_v<V>() : Tiling<T, N>::ROWS;
  constexpr int NT = LINES * LineGeom<N>::TPL;
  Op op;
  op.a = a;
  const dim3 grid = Op::TILE_MAJOR ? dim3((N / LINES) * a.B) : dim3(N / LINES, a.B);
  hipLaunchKernelGGL((k_lines<T, N, LINES, COLS, Op>), grid, dim3(NT), 0, s, op);
}

// column stages at tile variant V (only the valid variants are instantiated)
template <typename T, int N, class Op>
void launch_cols(const LineArgs& a, hipStream_t s) {
  if constexpr (Tiling<T, N>::template cols_valid<3>()) {
    if (a.tile == 3) return launch_op<T, N, true, Op, 3>(a, s);
  }
  if constexpr (Tiling<T, N>::template cols_valid<2>()) {
    if (a.tile == 2) return launch_op<T, N, true, Op, 2>(a, s);
  }
  if constexpr (Tiling<T, N>::template cols_valid<1>()) {
    if (a.tile == 1) return launch_op<T, N, true, Op, 1>(a, s);
  }
  launch_op<T, N, true, Op, 0>(a, s);
}

template <typename T, int N>
void launch_lines(LineOp op, const LineArgs& a, hipStream_t s) {
  switch (op) {
    case LineOp::RowsInvScaled: launch_op<T, N, false, OpRowsInvScaled<T, N>>(a, s); break;
    case LineOp::ColsInvMoments: launch_cols<T, N, OpColsInvMoments<T, N>>(a, s); break;
    case LineOp::RowsInvRegular: launch_op<T, N, false, OpRowsInvRegular<T, N>>(a, s); break;
    case LineOp::ColsInvTailFwd: launch_cols<T, N, OpColsInvTail<T, N, false>>(a, s); break;
    case LineOp::ColsInvTail: launch_cols<T, N, OpColsInvTail<T, N, true>>(a, s); break;
    case LineOp::RowsFwdEpilogue: launch_op<T, N, false, OpRowsFwdEpilogue<T, N>>(a, s); break;
    case LineOp::ColsFwdPotential: launch_cols<T, N, OpColsFwdPotential<T, N>>(a, s); break;
    case LineOp::ColsFwdPlain: launch_cols<T, N, OpColsPlain<T, N, -1>>(a, s); break;
    case LineOp::ColsInvPlain: launch_cols<T, N, OpColsPlain<T, N, +1>>(a, s); break;
    case LineOp::RowsFwdMoments: launch_op<T, N, false, OpRowsFwdMoments<T, N>>(a, s); break;
    case LineOp::ColsFwdRegularInv: launch_cols<T, N, OpColsFwdRegInv<T, N>>(a, s); break;
    case LineOp::RowsInvTailEpilogue: launch_op<T, N, false, OpRowsInvTailEpi<T, N>>(a, s); break;
  }
}

#define DBAR_INSTANTIATE_N(NN)                                                  \
  template void launch_lines<double, NN>(LineOp, const LineArgs&, hipStream_t); \
  template void launch_lines<float, NN>(LineOp, const LineArgs&, hipStream_t);

}  // namespace dbar
