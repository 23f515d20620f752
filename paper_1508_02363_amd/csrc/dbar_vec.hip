// Krylov vector kernels for GMRES on the real 2N^2 form of the D-bar system.
//
// The operator A(S) = S + i F(q_k conj(h(S))) is real-linear but not complex-linear (the conjugation), so GMRES
// runs on v = [Re S, Im S] with the inner product <u, v> = sum Re(conj(u) v) (paper Section 4.1: the matrix is never
// stored, only its action).  Complex arrays are used as they are: the real view is just the interleaved storage.
// Every sum is accumulated in FP64, per block, and reduced in a fixed order (results do not depend on the batch).
#include "dbar_launch.h"

namespace dbar {

int vec_blocks(size_t n) { return static_cast<int>((n + kVecChunk - 1) / kVecChunk); }

template <typename T>
DBAR_D cx<T> ld(const void* p, size_t i) {
  return static_cast<const cx<T>*>(p)[i];
}

DBAR_D double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// part[b][i][blk] = sum over the block's chunk of Re(conj(V_i) w), i < nv; optionally part[b][nv][blk] = |w|^2
template <typename T>
__global__ void __launch_bounds__(kVecBlock) k_dots(VecArgs a) {
  const int b = blockIdx.y;
  if (a.act && !a.act[b]) return;
  __shared__ double red[kVecBlock / 64][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const size_t base = (size_t)blockIdx.x * kVecChunk + threadIdx.x;
  const cx<T>* w = static_cast<const cx<T>*>(a.w) + (size_t)b * a.w_bs;
  const cx<T>* V = static_cast<const cx<T>*>(a.V) + (size_t)b * a.V_bs;
  c64 wv[kVecEPT];
#pragma unroll
  for (int e = 0; e < kVecEPT; ++e) {
    const size_t idx = base + (size_t)e * kVecBlock;
    wv[e] = idx < a.n ? cvt<double>(w[idx]) : c64{0.0, 0.0};
  }
  const int nval = a.nv + (a.want_self ? 1 : 0);
  double* out = a.part + (size_t)b * nval * gridDim.x + blockIdx.x;
  for (int i0 = 0; i0 < nval; i0 += 64) {
    const int cnt = nval - i0 < 64 ? nval - i0 : 64;
    for (int ii = 0; ii < cnt; ++ii) {
      const int i = i0 + ii;
      double acc = 0.0;
      if (i < a.nv) {
        const cx<T>* Vi = V + (size_t)i * a.n;
#pragma unroll
        for (int e = 0; e < kVecEPT; ++e) {
          const size_t idx = base + (size_t)e * kVecBlock;
          if (idx < a.n) {
            const c64 x = cvt<double>(Vi[idx]);
            acc += x.re * wv[e].re + x.im * wv[e].im;
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < kVecEPT; ++e) acc += norm2(wv[e]);
      }
      acc = wave_sum(acc);
      if (lane == 0) red[wave][ii] = acc;
    }
    __syncthreads();
    if (threadIdx.x < cnt) {
      double s = 0.0;
#pragma unroll
      for (int wv2 = 0; wv2 < kVecBlock / 64; ++wv2) s += red[wv2][threadIdx.x];
      out[(size_t)(i0 + threadIdx.x) * gridDim.x] = s;
    }
    __syncthreads();
  }
}

// w -= sum_i coef[b][i] V_i ; optional part[b][0][blk] = |w_new|^2
template <typename T>
__global__ void __launch_bounds__(kVecBlock) k_update(VecArgs a) {
  const int b = blockIdx.y;
  if (a.act && !a.act[b]) return;
  __shared__ double red[kVecBlock / 64];
  const size_t base = (size_t)blockIdx.x * kVecChunk + threadIdx.x;
  cx<T>* w = static_cast<cx<T>*>(a.w) + (size_t)b * a.w_bs;
  const cx<T>* V = static_cast<const cx<T>*>(a.V) + (size_t)b * a.V_bs;
  const double* coef = a.coef + (size_t)b * a.coef_bs;
  c64 acc[kVecEPT];
#pragma unroll
  for (int e = 0; e < kVecEPT; ++e) {
    const size_t idx = base + (size_t)e * kVecBlock;
    acc[e] = idx < a.n ? cvt<double>(w[idx]) : c64{0.0, 0.0};
  }
  for (int i = 0; i < a.nv; ++i) {
    const double c = coef[i];
    if (c == 0.0) continue;  // also keeps never-written basis slots (any bit pattern) out of the sum
    const cx<T>* Vi = V + (size_t)i * a.n;
#pragma unroll
    for (int e = 0; e < kVecEPT; ++e) {
      const size_t idx = base + (size_t)e * kVecBlock;
      if (idx < a.n) acc[e] = acc[e] - c * cvt<double>(Vi[idx]);
    }
  }
  double nrm = 0.0;
#pragma unroll
  for (int e = 0; e < kVecEPT; ++e) {
    const size_t idx = base + (size_t)e * kVecBlock;
    if (idx < a.n) {
      const cx<T> o = cvt<T>(acc[e]);
      w[idx] = o;
      nrm += norm2(cvt<double>(o));
    }
  }
  if (a.want_self) {
    nrm = wave_sum(nrm);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < kVecBlock / 64; ++k) s += red[k];
      a.part[(size_t)b * gridDim.x + blockIdx.x] = s;
    }
  }
}

// w (TX) += sum_i coef[b][i] V_i (TV)
template <typename TX, typename TV>
__global__ void __launch_bounds__(kVecBlock) k_axpy_multi(VecArgs a) {
  const int b = blockIdx.y;
  if (a.act && !a.act[b]) return;
  const size_t base = (size_t)blockIdx.x * kVecChunk + threadIdx.x;
  cx<TX>* w = static_cast<cx<TX>*>(a.w) + (size_t)b * a.w_bs;
  const cx<TV>* V = static_cast<const cx<TV>*>(a.V) + (size_t)b * a.V_bs;
  const double* coef = a.coef + (size_t)b * a.coef_bs;
  c64 acc[kVecEPT];
#pragma unroll
  for (int e = 0; e < kVecEPT; ++e) {
    const size_t idx = base + (size_t)e * kVecBlock;
    acc[e] = idx < a.n ? cvt<double>(w[idx]) : c64{0.0, 0.0};
  }
  for (int i = 0; i < a.nv; ++i) {
    const double c = coef[i];
    if (c == 0.0) continue;  // entries that stopped early have zero coefficients beyond their own iterations
    const cx<TV>* Vi = V + (size_t)i * a.n;
#pragma unroll
    for (int e = 0; e < kVecEPT; ++e) {
      const size_t idx = base + (size_t)e * kVecBlock;
      if (idx < a.n) acc[e] = acc[e] + c * cvt<double>(Vi[idx]);
    }
  }
#pragma unroll
  for (int e = 0; e < kVecEPT; ++e) {
    const size_t idx = base + (size_t)e * kVecBlock;
    if (idx < a.n) w[idx] = cvt<TX>(acc[e]);
  }
}

template <typename TO, typename TI>
__global__ void __launch_bounds__(kVecBlock) k_convert(const TI* in, size_t in_bs, TO* out, size_t out_bs, size_t n,
                                                        const int* act, double scale) {
  const int b = blockIdx.y;
  if (act && !act[b]) return;
  const cx<TI>* x = reinterpret_cast<const cx<TI>*>(in) + (size_t)b * in_bs;
  cx<TO>* y = reinterpret_cast<cx<TO>*>(out) + (size_t)b * out_bs;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = cvt<TO>(scale * cvt<double>(x[i]));
}

// out[b][v] = sum_blk part[b][v][blk], fixed order
__global__ void __launch_bounds__(256) k_reduce(const double* part, int nval, int nblk, double* out, const int* act) {
  const int b = blockIdx.y, v = blockIdx.x;
  if (act && !act[b]) return;
  __shared__ double red[4];
  const double* p = part + ((size_t)b * nval + v) * nblk;
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) s += p[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[(size_t)b * nval + v] = red[0] + red[1] + red[2] + red[3];
}

template <typename T>
void launch_dots(const VecArgs& a, hipStream_t s) {
  TimerScope ts(kStageDots + (sizeof(T) == 4), (double)(a.nv + 1) * a.n * sizeof(cx<T>), a.B, a.act, s);
  hipLaunchKernelGGL(k_dots<T>, dim3(vec_blocks(a.n), a.B), dim3(kVecBlock), 0, s, a);
}
template <typename T>
void launch_update(const VecArgs& a, hipStream_t s) {
  TimerScope ts(kStageUpdate + (sizeof(T) == 4), (double)(a.nv + 2) * a.n * sizeof(cx<T>), a.B, a.act, s);
  hipLaunchKernelGGL(k_update<T>, dim3(vec_blocks(a.n), a.B), dim3(kVecBlock), 0, s, a);
}
template <typename TX, typename TV>
void launch_axpy_multi(const VecArgs& a, hipStream_t s) {
  const int st = sizeof(TX) == 4 ? 2 : (sizeof(TV) == 4 ? 1 : 0);
  TimerScope ts(kStageAxpy + st, (double)a.nv * a.n * sizeof(cx<TV>) + 2.0 * a.n * sizeof(cx<TX>), a.B, a.act, s);
  hipLaunchKernelGGL((k_axpy_multi<TX, TV>), dim3(vec_blocks(a.n), a.B), dim3(kVecBlock), 0, s, a);
}
template <typename TO, typename TI>
void launch_convert(const void* in, size_t in_bs, void* out, size_t out_bs, size_t n, int B, const int* act,
                    double scale, hipStream_t s) {
  TimerScope ts(kStageConvert, (double)n * (sizeof(cx<TO>) + sizeof(cx<TI>)), B, act, s);
  int blocks = static_cast<int>((n + 1023) / 1024);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((k_convert<TO, TI>), dim3(blocks, B), dim3(kVecBlock), 0, s, static_cast<const TI*>(in), in_bs,
                     static_cast<TO*>(out), out_bs, n, act, scale);
}
void launch_reduce(const double* part, int nval, int nblk, double* out, int B, const int* act, hipStream_t s) {
  TimerScope ts(kStageReduce, (double)nval * nblk * sizeof(double), B, act, s);
  hipLaunchKernelGGL(k_reduce, dim3(nval, B), dim3(256), 0, s, part, nval, nblk, out, act);
}

template void launch_dots<double>(const VecArgs&, hipStream_t);
template void launch_dots<float>(const VecArgs&, hipStream_t);
template void launch_update<double>(const VecArgs&, hipStream_t);
template void launch_update<float>(const VecArgs&, hipStream_t);
template void launch_axpy_multi<double, double>(const VecArgs&, hipStream_t);
template void launch_axpy_multi<double, float>(const VecArgs&, hipStream_t);
template void launch_axpy_multi<float, float>(const VecArgs&, hipStream_t);
template void launch_convert<float, double>(const void*, size_t, void*, size_t, size_t, int, const int*, double,
                                            hipStream_t);
template void launch_convert<double, float>(const void*, size_t, void*, size_t, size_t, int, const int*, double,
                                            hipStream_t);
template void launch_convert<double, double>(const void*, size_t, void*, size_t, size_t, int, const int*, double,
                                             hipStream_t);

}  // namespace dbar
