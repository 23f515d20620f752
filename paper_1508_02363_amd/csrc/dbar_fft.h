// Line FFTs for gfx950: Stockham autosort radix-16 passes with LDS exchanges.
//
// A "line" is one row or one column of an N x N complex array.  TPL = N / RMAX threads cooperate on a line
// (RMAX = 16, or N when N < 16).  Thread jt of a line always holds, in registers, the elements at positions
//     jt + s * TPL,   s = 0 .. RMAX-1
// before and after every pass.  Consequently the first pass loads straight from global memory and the last pass
// leaves the transformed line in registers in the same position pattern; only the exchanges between passes go
// through LDS.  An inverse transform that ends in registers can feed a forward transform directly (used to fuse the
// x-space pointwise step between the second and third 2D FFT of the operator).
//
// Pass (R, NS): butterfly j (0 <= j < N/R) reads positions j + r N/R, multiplies element r by W^{r (j mod NS)} with
// W = exp(DIR 2 pi i / (NS R)), does an R-point DFT and writes element r to (j / NS) NS R + (j mod NS) + r NS.
// Radix sequence: 16, 16, ..., then 2/4/8 for the remainder (N = 2^p, 8 <= N <= 4096).
// DIR = -1 is the forward transform sum_j x_j e^{-2 pi i jm/N}; DIR = +1 the unnormalised inverse.
#pragma once

#include "dbar_common.h"

namespace dbar {

// ------------------------------------------------------------------------------------------------------------
// Small DFTs in registers
// ------------------------------------------------------------------------------------------------------------

// cos / sin of 2 pi m / 16, m = 0..15
struct W16 {
  static constexpr double c[16] = {1.0,
                                   0.92387953251128675613,
                                   0.70710678118654752440,
                                   0.38268343236508977173,
                                   0.0,
                                   -0.38268343236508977173,
                                   -0.70710678118654752440,
                                   -0.92387953251128675613,
                                   -1.0,
                                   -0.92387953251128675613,
                                   -0.70710678118654752440,
                                   -0.38268343236508977173,
                                   0.0,
                                   0.38268343236508977173,
                                   0.70710678118654752440,
                                   0.92387953251128675613};
  static constexpr double s[16] = {0.0,
                                   0.38268343236508977173,
                                   0.70710678118654752440,
                                   0.92387953251128675613,
                                   1.0,
                                   0.92387953251128675613,
                                   0.70710678118654752440,
                                   0.38268343236508977173,
                                   0.0,
                                   -0.38268343236508977173,
                                   -0.70710678118654752440,
                                   -0.92387953251128675613,
                                   -1.0,
                                   -0.92387953251128675613,
                                   -0.70710678118654752440,
                                   -0.38268343236508977173};
};

// a * exp(DIR * 2 pi i * M / 16), with the trivial angles done exactly
template <int M, int DIR, typename T>
DBAR_D cx<T> mul_w16(cx<T> a) {
  constexpr int m = ((M % 16) + 16) % 16;
  if constexpr (m == 0) {
    return a;
  } else if constexpr (m == 4) {
    return DIR < 0 ? mul_mi(a) : mul_i(a);
  } else if constexpr (m == 8) {
    return -a;
  } else if constexpr (m == 12) {
    return DIR < 0 ? mul_i(a) : mul_mi(a);
  } else {
    const T c = static_cast<T>(W16::c[m]);
    const T s = static_cast<T>(DIR * W16::s[m]);
    return cx<T>{a.re * c - a.im * s, a.re * s + a.im * c};
  }
}

template <int DIR, typename T>
DBAR_D void dft2(cx<T>& x0, cx<T>& x1) {
  cx<T> a = x0 + x1;
  x1 = x0 - x1;
  x0 = a;
}

template <int DIR, typename T>
DBAR_D void dft4(cx<T>& x0, cx<T>& x1, cx<T>& x2, cx<T>& x3) {
  cx<T> a0 = x0 + x2, a1 = x0 - x2, a2 = x1 + x3;
  cx<T> d = x1 - x3;
  cx<T> a3 = DIR < 0 ? mul_mi(d) : mul_i(d);
  x0 = a0 + a2;
  x2 = a0 - a2;
  x1 = a1 + a3;
  x3 = a1 - a3;
}

template <int R, int DIR, typename T>
DBAR_D void dft(cx<T>* x) {
  if constexpr (R == 2) {
    dft2<DIR>(x[0], x[1]);
  } else if constexpr (R == 4) {
    dft4<DIR>(x[0], x[1], x[2], x[3]);
  } else if constexpr (R == 8) {
    // r = 2 r1 + r2: DFT4 over r1, twiddle W8^{r2 f1}, DFT2 over r2
    dft4<DIR>(x[0], x[2], x[4], x[6]);
    dft4<DIR>(x[1], x[3], x[5], x[7]);
    x[3] = mul_w16<2, DIR>(x[3]);
    x[5] = mul_w16<4, DIR>(x[5]);
    x[7] = mul_w16<6, DIR>(x[7]);
    cx<T> y[8];
#pragma unroll
    for (int f1 = 0; f1 < 4; ++f1) {
      y[f1] = x[2 * f1] + x[2 * f1 + 1];
      y[f1 + 4] = x[2 * f1] - x[2 * f1 + 1];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = y[i];
  } else if constexpr (R == 16) {
    // r = 4 r1 + r2: DFT4 over r1 (stride 4), twiddle W16^{r2 f1}, DFT4 over r2
    dft4<DIR>(x[0], x[4], x[8], x[12]);
    dft4<DIR>(x[1], x[5], x[9], x[13]);
    dft4<DIR>(x[2], x[6], x[10], x[14]);
    dft4<DIR>(x[3], x[7], x[11], x[15]);
    // x[r2 + 4 f1] now holds y[r2][f1]
    x[5] = mul_w16<1, DIR>(x[5]);
    x[9] = mul_w16<2, DIR>(x[9]);
    x[13] = mul_w16<3, DIR>(x[13]);
    x[6] = mul_w16<2, DIR>(x[6]);
    x[10] = mul_w16<4, DIR>(x[10]);
    x[14] = mul_w16<6, DIR>(x[14]);
    x[7] = mul_w16<3, DIR>(x[7]);
    x[11] = mul_w16<6, DIR>(x[11]);
    x[15] = mul_w16<9, DIR>(x[15]);
    dft4<DIR>(x[0], x[1], x[2], x[3]);
    dft4<DIR>(x[4], x[5], x[6], x[7]);
    dft4<DIR>(x[8], x[9], x[10], x[11]);
    dft4<DIR>(x[12], x[13], x[14], x[15]);
    // x[4 f1 + f2] holds X[f1 + 4 f2]
    cx<T> y[16];
#pragma unroll
    for (int f1 = 0; f1 < 4; ++f1)
#pragma unroll
      for (int f2 = 0; f2 < 4; ++f2) y[f1 + 4 * f2] = x[4 * f1 + f2];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = y[i];
  }
}

// ------------------------------------------------------------------------------------------------------------
// Line geometry
// ------------------------------------------------------------------------------------------------------------

template <int N>
struct LineGeom {
  static_assert(N >= 8 && N <= 4096 && (N & (N - 1)) == 0, "N must be a power of two in [8, 4096]");
  static constexpr int RMAX = N < 16 ? N : 16;
  static constexpr int TPL = N / RMAX;  // threads per line
  static constexpr int LOG = (N >= 4096)   ? 12
                             : (N >= 2048) ? 11
                             : (N >= 1024) ? 10
                             : (N >= 512)  ? 9
                             : (N >= 256)  ? 8
                             : (N >= 128)  ? 7
                             : (N >= 64)   ? 6
                             : (N >= 32)   ? 5
                             : (N >= 16)   ? 4
                                           : 3;
  static constexpr int P16 = N < 16 ? 0 : LOG / 4;             // number of radix-16 passes
  static constexpr int REM = N < 16 ? N : (1 << (LOG % 4));    // last radix (1 = none)
  static constexpr int NPASS = P16 + (REM > 1 ? 1 : 0);
  // LDS padding: one element every 16 keeps strided Stockham writes from piling onto the same banks
  static constexpr int padded(int n) { return n + (n >> 4); }
  static constexpr int LDS_LINE = padded(N);
};

// radix and NS of pass number `pass`
template <int N, int PASS>
struct PassInfo {
  using G = LineGeom<N>;
  static constexpr int R = (PASS < G::P16) ? 16 : G::REM;
  static constexpr int NS = [] {
    int ns = 1;
    for (int p = 0; p < PASS; ++p) ns *= (p < G::P16 ? 16 : G::REM);
    return ns;
  }();
};

// Twiddles of pass 1 (NS = 16, radix R1): W_N^{r k N/(16 R1)} = W_{16 R1}^{r k} for r < R1, k < 16, whatever N is.
// Kept in LDS as t1[(r - 1) * 16 + k] (r-major: the lanes of a wave, consecutive k, read consecutive banks).
template <int N>
struct Pass1Table {
  static constexpr bool USED = LineGeom<N>::NPASS > 1;
  static constexpr int R1 = USED ? PassInfo<N, 1>::R : 2;
  static constexpr int SIZE = (R1 - 1) * 16;
};

// Fill the pass-1 table from the global twiddle table exp(-2 pi i m / N) (all threads of the block; ordered before
// its first use by the barriers of pass 0's exchange).
template <typename T, int N>
DBAR_D void fill_pass1_table(cx<T>* __restrict__ t1, const cx<T>* __restrict__ tw, int tid, int nt) {
  using P1 = Pass1Table<N>;
  if constexpr (P1::USED) {
    for (int t = tid; t < P1::SIZE; t += nt) {
      const int r = t / 16 + 1, k = t % 16;
      t1[t] = tw[r * k * (N / (16 * P1::R1))];
    }
  }
}

// One Stockham pass in registers (twiddle + DFT).  v[s] holds position jt + s*TPL.  T1: pass 1 reads its twiddles
// from the LDS table t1 (kernels bound by arithmetic) instead of forming them from tw (kernels bound by memory).
template <typename T, int N, int PASS, int DIR, bool T1>
DBAR_D void fft_pass_regs(cx<T>* v, int jt, const cx<T>* __restrict__ tw, const cx<T>* __restrict__ t1) {
  using G = LineGeom<N>;
  constexpr int R = PassInfo<N, PASS>::R;
  constexpr int NS = PassInfo<N, PASS>::NS;
  constexpr int NB = G::RMAX / R;  // butterflies per thread
  constexpr int TS = N / (NS * R); // twiddle table stride
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int j = jt + q * G::TPL;
    cx<T> b[R];
#pragma unroll
    for (int r = 0; r < R; ++r) b[r] = v[q + r * NB];
    if constexpr (T1 && PASS == 1 && NS == 16) {
      const int k = j % 16;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const cx<T> t = t1[(r - 1) * 16 + k];
        b[r] = b[r] * (DIR < 0 ? t : conj(t));
      }
    } else if constexpr (NS > 1) {
      // W^r from the table entries for the powers of two in r (at most 3 products: r < 16), formed per element so
      // that only log2(R) twiddles are live at a time
      const int k = j % NS;
      constexpr int LR = R == 16 ? 4 : R == 8 ? 3 : R == 4 ? 2 : 1;
      cx<T> wp[LR];
#pragma unroll
      for (int q2 = 0; q2 < LR; ++q2) {
        const cx<T> t = tw[(1 << q2) * k * TS];  // table holds exp(-2 pi i m / N)
        wp[q2] = DIR < 0 ? t : conj(t);
      }
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cx<T> wr = wp[__builtin_ctz(r)];
#pragma unroll
        for (int q2 = __builtin_ctz(r) + 1; q2 < LR; ++q2)
          if (r & (1 << q2)) wr = wr * wp[q2];
        b[r] = b[r] * wr;
      }
    }
    dft<R, DIR>(b);
#pragma unroll
    for (int r = 0; r < R; ++r) v[q + r * NB] = b[r];
  }
}

// Write the output of pass PASS to LDS (its Stockham destination positions) ...  Element p of a line lives at
// line[padded(p) * LS]: LS = 1 for a line of its own, LS = lines per tile when the lines of a column tile are
// interleaved element by element (the threads of one wave then touch consecutive addresses across the tile's lines)
template <typename T, int N, int PASS, int LS>
DBAR_D void lds_store_pass(cx<T>* __restrict__ line, const cx<T>* v, int jt) {
  using G = LineGeom<N>;
  constexpr int R = PassInfo<N, PASS>::R;
  constexpr int NS = PassInfo<N, PASS>::NS;
  constexpr int NB = G::RMAX / R;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int j = jt + q * G::TPL;
    const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
    for (int r = 0; r < R; ++r) line[G::padded(base + r * NS) * LS] = v[q + r * NB];
  }
}

// ... and read the input pattern of the next pass.
template <typename T, int N, int LS>
DBAR_D void lds_load_line(const cx<T>* __restrict__ line, cx<T>* v, int jt) {
  using G = LineGeom<N>;
#pragma unroll
  for (int s = 0; s < G::RMAX; ++s) v[s] = line[G::padded(jt + s * G::TPL) * LS];
}

// Full line transform: registers in (positions jt + s*TPL), registers out (same positions, transformed).
// `line` is this line's LDS buffer (LDS_LINE elements at stride LS).  Must be called by all threads of the block
// (barriers).
template <typename T, int N, int DIR, int LS, bool T1>
DBAR_D void line_fft(cx<T>* v, int jt, cx<T>* __restrict__ line, const cx<T>* __restrict__ tw,
                     const cx<T>* __restrict__ t1) {
  using G = LineGeom<N>;
  fft_pass_regs<T, N, 0, DIR, T1>(v, jt, tw, t1);
  if constexpr (G::NPASS > 1) {
    lds_store_pass<T, N, 0, LS>(line, v, jt);
    __syncthreads();
    lds_load_line<T, N, LS>(line, v, jt);
    __syncthreads();
    fft_pass_regs<T, N, 1, DIR, T1>(v, jt, tw, t1);
  }
  if constexpr (G::NPASS > 2) {
    lds_store_pass<T, N, 1, LS>(line, v, jt);
    __syncthreads();
    lds_load_line<T, N, LS>(line, v, jt);
    __syncthreads();
    fft_pass_regs<T, N, 2, DIR, T1>(v, jt, tw, t1);
  }
  static_assert(G::NPASS <= 3, "N <= 4096 needs at most three passes");
}

}  // namespace dbar
