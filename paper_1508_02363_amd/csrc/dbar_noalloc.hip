// Allocation-free variant of the one-operator-application entry point: A(S) = S + i F(q_k conj(h(S))) on device
// buffers with every intermediate array in one file-scope device array, for callers that cannot allocate device
// memory (work under graph capture, tight serving loops, harnesses that forbid allocation).
//
// The scratch array holds, for grids up to N = kNoAllocMaxN:
//   * the transform scratch of the operator (FP64: one N x N complex128 array; FP32: the transform array and the
//     FP32 roundings of Q, S and the result, N x N complex64 each -- 32 N^2 bytes either way);
//   * the per-k phase tables e^{-2i k2 x_j}, e^{-2i k1 y_j} (FP64 and FP32), k itself, the Taylor data (d_n, c_n,
//     R(0)) and the per-tile partial sums of the moment reduction.
// Nothing in it has to start at zero: every call writes each part it reads before reading it.  All calls on one GPU
// share that GPU's copy (it keeps the last call's contents), so calls that overlap on one GPU race: serialise them on
// one stream.  The twiddle tables exp(-2 pi i j / N) of every power of two 8 <= N <= kNoAllocMaxN sit in a second
// file-scope device array that is initialised when the code object loads (values computed at compile time), so no
// call, the first included, copies anything from the host: the entry point can be captured into a HIP graph from its
// first call on.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "dbar.h"
#include "dbar_launch.h"
#include "dbar_solver.h"

namespace dbar {

namespace {
constexpr int kNoAllocMaxN = 1024;
constexpr size_t kNMax = (size_t)kNoAllocMaxN * kNoAllocMaxN;
constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
// sum of N over the powers of two 8 .. kNoAllocMaxN; the tables of grid size N start at entry N - 8
constexpr size_t kTwEntries = 2 * (size_t)kNoAllocMaxN - 8;
constexpr size_t kOffBig = 0;                                        // 32 N^2 bytes (see above)
constexpr size_t kOffPhase = align256(kOffBig + 32 * kNMax);         // ex, ey (FP64), ex32, ey32 (FP32)
constexpr size_t kOffK = align256(kOffPhase + (size_t)kNoAllocMaxN * 2 * (sizeof(c64) + sizeof(c32)));
constexpr size_t kOffMom = align256(kOffK + sizeof(c64));            // coefG, dmom (FP64), dmom32
constexpr size_t kOffPartMom = align256(kOffMom + (size_t)kNMom * (2 * sizeof(c64) + sizeof(c32)));
// moment partials: 2 kNMom values per tile, at most N tiles per entry (one line per tile)
constexpr size_t kOffPartVec = align256(kOffPartMom + 2 * (size_t)kNMom * kNoAllocMaxN * sizeof(double));
constexpr size_t kScratchBytes = align256(kOffPartVec + (size_t)kNoAllocMaxN * sizeof(double));
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// exp(-2 pi i j / N), j < N, for every power of two 8 <= N <= kNoAllocMaxN (grid size N at entry N - 8), evaluated at
// compile time in long double: the angle 2 pi j / N reduced to the first octant by the symmetries of the circle (exact:
// j and N are integers), then the Taylor series of sin and cos there, rounded once to FP64 and to FP32.
constexpr long double kPiL = 3.14159265358979323846264338327950288L;
constexpr long double series_sin(long double x) {  // |x| <= pi/4: 16 terms leave < 1e-30
  long double term = x, sum = x;
  for (int k = 1; k < 16; ++k) {
    term *= -x * x / ((long double)(2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr long double series_cos(long double x) {
  long double term = 1.0L, sum = 1.0L;
  for (int k = 1; k < 16; ++k) {
    term *= -x * x / ((long double)(2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
struct TwTables {
  c64 d[kTwEntries];
  c32 f[kTwEntries];
};
constexpr TwTables make_tw_tables() {
  TwTables t{};
  for (int N = 8; N <= kNoAllocMaxN; N <<= 1)
    for (int j = 0; j < N; ++j) {
      // 2 pi j / N = (o + rem / N) pi / 4 with octant o; phi = rem / N pi / 4, psi = pi / 4 - phi
      const long oct = 8L * j;
      const int o = static_cast<int>(oct / N), rem = static_cast<int>(oct % N);
      const long double phi = (long double)rem / N * (kPiL / 4), psi = (long double)(N - rem) / N * (kPiL / 4);
      const long double cp = series_cos(phi), sp = series_sin(phi), cq = series_cos(psi), sq = series_sin(psi);
      long double c = 0.0L, s = 0.0L;  // cos and sin of 2 pi j / N
      switch (o) {
        case 0: c = cp; s = sp; break;
        case 1: c = sq; s = cq; break;
        case 2: c = -sp; s = cp; break;
        case 3: c = -cq; s = sq; break;
        case 4: c = -cp; s = -sp; break;
        case 5: c = -sq; s = -cq; break;
        case 6: c = sp; s = -cp; break;
        default: c = cq; s = -sq; break;
      }
      t.d[N - 8 + j] = c64{(double)c, (double)-s};
      t.f[N - 8 + j] = c32{(float)c, (float)-s};
    }
  return t;
}
static __device__ __align__(256) TwTables tw_tables = make_tw_tables();

static std::mutex g_na_mutex;
static unsigned char* g_na_ptr[kMaxDevices];  // the device address of `scratch` on each device (null: not set up)
static TwTables* g_na_tw[kMaxDevices];        // the device address of `tw_tables` on each device

// Set-up on device dev (with dev current, under g_na_mutex): the device addresses of the scratch array and of the
// twiddle tables.
static int noalloc_setup(int dev, unsigned char** out, const TwTables** tw) {
  if (g_na_ptr[dev]) {
    *out = g_na_ptr[dev];
    *tw = g_na_tw[dev];
    return DBAR_OK;
  }
  void* p = nullptr;
  void* q = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess && p) e = hipGetSymbolAddress(&q, HIP_SYMBOL(tw_tables));
  if (e != hipSuccess || !p || !q) {
    (void)hipGetLastError();
    return fail(DBAR_EDEVICE, std::string("hipGetSymbolAddress of the scratch arrays failed: ") + hipGetErrorString(e));
  }
  g_na_ptr[dev] = static_cast<unsigned char*>(p);
  g_na_tw[dev] = static_cast<TwTables*>(q);
  *out = g_na_ptr[dev];
  *tw = g_na_tw[dev];
  return DBAR_OK;
}

__global__ void k_store_k(c64* kv, double kre, double kim) { *kv = c64{kre, kim}; }

}  // namespace dbar

using namespace dbar;

extern "C" {

int dbar_apply_noalloc(const dbar_grid* grid, const void* Q_dev, const double* k, const void* S_dev, void* AS_dev,
                       int32_t precision, void* stream) {
  int rc = validate_grid(grid);
  if (rc) return rc;
  if (grid->n > kNoAllocMaxN)
    return fail(DBAR_EINVAL, "dbar_apply_noalloc: grid size " + std::to_string(grid->n) +
                                 " exceeds the allocation-free maximum N = " + std::to_string(kNoAllocMaxN));
  if (!Q_dev || !k || !S_dev || !AS_dev) return fail(DBAR_EINVAL, "NULL buffer");
  if (precision != DBAR_FP64 && precision != DBAR_FP32) return fail(DBAR_EINVAL, "precision must be FP64 or FP32");
  if (!std::isfinite(k[0]) || !std::isfinite(k[1])) return fail(DBAR_EINVAL, "k contains NaN or Inf");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return fail(DBAR_EDEVICE, "no usable HIP device");
  }
  std::lock_guard<std::mutex> lock(g_na_mutex);
  unsigned char* base = nullptr;
  const TwTables* tw = nullptr;
  if ((rc = noalloc_setup(dev, &base, &tw))) return rc;
  const int N = grid->n;
  const size_t n = (size_t)N * N;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the moment partials of the column pass: one value pair per Taylor term and tile (at most N tiles)
  if (line_tiles(N, true, precision == DBAR_FP64) > kNoAllocMaxN) return fail(DBAR_EINVAL, "tile layout too large");
  Pipeline P;
  P.N = N;
  P.M = grid->M;
  P.L = grid->L;
  P.n = n;
  P.tw64 = tw->d + (N - 8);
  P.tw32 = tw->f + (N - 8);
  c64* ex = reinterpret_cast<c64*>(base + kOffPhase);
  c64* ey = ex + N;
  c32* ex32 = reinterpret_cast<c32*>(ey + N);
  c32* ey32 = ex32 + N;
  P.ex = ex;
  P.ey = ey;
  P.ex32 = ex32;
  P.ey32 = ey32;
  c64* coefG = reinterpret_cast<c64*>(base + kOffMom);
  P.coefG = coefG;
  P.dmom = coefG + kNMom;
  P.dmom32 = reinterpret_cast<c32*>(coefG + 2 * kNMom);
  P.part_mom = reinterpret_cast<double*>(base + kOffPartMom);
  P.part_vec = reinterpret_cast<double*>(base + kOffPartVec);
  P.xspace = false;  // the operator as written on S (Section 4 algorithm, step 4)
  c64* kv = reinterpret_cast<c64*>(base + kOffK);
  hipLaunchKernelGGL(k_store_k, dim3(1), dim3(1), 0, s, kv, k[0], k[1]);
  launch_phase_tables(kv, N, grid->L, ex, ey, ex32, ey32, 1, s);
  if (precision == DBAR_FP64) {
    void* T = base + kOffBig;
    P.apply<double>(S_dev, n, AS_dev, n, Q_dev, 0, T, 1, nullptr, 1.0, 1.0, nullptr, 0, false, s);
  } else {
    c32* T32 = reinterpret_cast<c32*>(base + kOffBig);
    c32* Q32 = T32 + n;
    c32* S32 = Q32 + n;
    c32* out32 = S32 + n;
    launch_convert<float, double>(Q_dev, 0, Q32, 0, n, 1, nullptr, 1.0, s);
    launch_convert<float, double>(S_dev, 0, S32, 0, n, 1, nullptr, 1.0, s);
    P.apply<float>(S32, n, out32, n, Q32, 0, T32, 1, nullptr, 1.0, 1.0, nullptr, 0, false, s);
    launch_convert<double, float>(out32, 0, AS_dev, 0, n, 1, nullptr, 1.0, s);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(DBAR_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return DBAR_OK;
}

}  // extern "C"
