// Allocation-free variant of the one-operator-application entry point: A(S) = S + i F(q_k conj(h(S))) on device
// buffers with every intermediate array in one file-scope device array, for callers that cannot allocate device
// memory (work under graph capture, tight serving loops, harnesses that forbid allocation).
//
// The scratch array holds, for grids up to N = kNoAllocMaxN:
//   * the transform scratch of the operator (FP64: one N x N complex128 array; FP32: the transform array and the
//     FP32 roundings of Q, S and the result, N x N complex64 each -- 32 N^2 bytes either way);
//   * the twiddle tables exp(-2 pi i j / N) of every power of two 8 <= N <= kNoAllocMaxN (FP64 and FP32), written once
//     per device when the array is set up;
//   * the per-k phase tables e^{-2i k2 x_j}, e^{-2i k1 y_j} (FP64 and FP32), k itself, the Taylor data (d_n, c_n,
//     R(0)) and the per-tile partial sums of the moment reduction.
// Nothing in it has to start at zero: every call writes each part it reads before reading it.  All calls on one GPU
// share that GPU's copy (it keeps the last call's contents), so calls that overlap on one GPU race: serialise them on
// one stream.
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
constexpr size_t kOffTw64 = align256(kOffBig + 32 * kNMax);          // FP64 twiddles, every N
constexpr size_t kOffTw32 = align256(kOffTw64 + kTwEntries * sizeof(c64));
constexpr size_t kOffPhase = align256(kOffTw32 + kTwEntries * sizeof(c32));  // ex, ey (FP64), ex32, ey32 (FP32)
constexpr size_t kOffK = align256(kOffPhase + (size_t)kNoAllocMaxN * 2 * (sizeof(c64) + sizeof(c32)));
constexpr size_t kOffMom = align256(kOffK + sizeof(c64));            // coefG, dmom (FP64), dmom32
constexpr size_t kOffPartMom = align256(kOffMom + (size_t)kNMom * (2 * sizeof(c64) + sizeof(c32)));
// moment partials: 2 kNMom values per tile, at most N tiles per entry (one line per tile)
constexpr size_t kOffPartVec = align256(kOffPartMom + 2 * (size_t)kNMom * kNoAllocMaxN * sizeof(double));
constexpr size_t kScratchBytes = align256(kOffPartVec + (size_t)kNoAllocMaxN * sizeof(double));
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_na_mutex;
static unsigned char* g_na_ptr[kMaxDevices];  // the device address of `scratch` on each device (null: not set up)
static c64 g_tw64[kTwEntries];                // host twiddle tables of every N (filled once)
static c32 g_tw32[kTwEntries];
static bool g_tw_ready = false;

// Set-up on device dev (with dev current, under g_na_mutex): the scratch array's device address, and its twiddle
// tables written once.
static int noalloc_setup(int dev, unsigned char** out) {
  if (g_na_ptr[dev]) {
    *out = g_na_ptr[dev];
    return DBAR_OK;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(DBAR_EDEVICE, std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(e));
  }
  if (!g_tw_ready) {
    for (int N = 8; N <= kNoAllocMaxN; N <<= 1) host_twiddles(N, g_tw64 + (N - 8), g_tw32 + (N - 8));
    g_tw_ready = true;
  }
  unsigned char* base = static_cast<unsigned char*>(p);
  if (hipMemcpy(base + kOffTw64, g_tw64, sizeof(g_tw64), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(base + kOffTw32, g_tw32, sizeof(g_tw32), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return fail(DBAR_EDEVICE, "upload of the twiddle tables into the scratch array failed");
  }
  g_na_ptr[dev] = base;
  *out = base;
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
  if ((rc = noalloc_setup(dev, &base))) return rc;
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
  P.tw64 = base + kOffTw64 + (size_t)(N - 8) * sizeof(c64);
  P.tw32 = base + kOffTw32 + (size_t)(N - 8) * sizeof(c32);
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
