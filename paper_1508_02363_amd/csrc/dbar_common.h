// Common device/host definitions for the D-bar GPU library (gfx950).
//
// Complex numbers are stored interleaved (re, im) in 8- or 16-byte aligned pairs.  All arrays on an N x N grid are
// row-major: x-space arrays a[iy][ix] with x_j = L(-pi + 2 pi j/N); xi-space arrays A[p2][p1] in FFT order, where
// the index p stands for the wave number m = p (p <= N/2) or m = p - N (p > N/2) and xi = m / L (paper Section 4.1,
// equations 'domain' and 'xidomain': the Nyquist wave number is +N/(2L)).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define DBAR_HD __host__ __device__ __forceinline__
#define DBAR_D __device__ __forceinline__

namespace dbar {

constexpr int kMaxM = 15;          // largest Taylor order M supported (the paper uses M = 11, at most about 20)
constexpr int kNMom = kMaxM + 2;   // moments d_0..d_M plus the conj(z) moment
constexpr double kPi = 3.14159265358979323846;

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};
using c64 = cx<double>;
using c32 = cx<float>;

template <typename T> DBAR_HD cx<T> mk(T a, T b) { return cx<T>{a, b}; }
template <typename T> DBAR_HD cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> DBAR_HD cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> DBAR_HD cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <typename T> DBAR_HD cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> DBAR_HD cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> DBAR_HD cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
template <typename T> DBAR_HD cx<T> mul_i(cx<T> a) { return {-a.im, a.re}; }     // i * a
template <typename T> DBAR_HD cx<T> mul_mi(cx<T> a) { return {a.im, -a.re}; }    // -i * a
template <typename T> DBAR_HD T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }

DBAR_HD float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
DBAR_HD double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
// a * b + c as four fused multiply-adds (the operators above take six instructions for it: the addition of c cannot
// be contracted into the product's last step)
template <typename T> DBAR_HD cx<T> cfma(cx<T> a, cx<T> b, cx<T> c) {
  return {fmar(a.re, b.re, fmar(-a.im, b.im, c.re)), fmar(a.re, b.im, fmar(a.im, b.re, c.im))};
}
// Re(conj(a) b) as a double, for FP64 accumulation.  FP32 data: the product is formed in FP32 (one fused rounding);
// its error, relative to |a||b| per element and of random sign, is below what the FP32 data carry themselves.
template <typename T> DBAR_HD double rdot(cx<T> a, cx<T> b) {
  if constexpr (sizeof(T) == 4) return static_cast<double>(fmar(a.im, b.im, a.re * b.re));
  else return a.re * b.re + a.im * b.im;
}

template <typename To, typename From> DBAR_HD cx<To> cvt(cx<From> a) {
  return cx<To>{static_cast<To>(a.re), static_cast<To>(a.im)};
}

DBAR_HD int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// Wave number index p -> signed wave number m in [-N/2+1, N/2].
DBAR_HD int wavenum(int p, int N) { return p <= N / 2 ? p : p - N; }

}  // namespace dbar
