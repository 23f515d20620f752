// Host-side launch interface of the D-bar kernels (no kernel code here).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "dbar_common.h"

namespace dbar {

// Which fused line-transform stage to run.  "rows" = lines along x / xi1 (contiguous), "cols" = along y / xi2.
enum class LineOp : int {
  RowsInvScaled = 0,  // out = IFFT_rows(phase * ci * in)                          (first pass of F^-1)
  ColsInvMoments = 1, // IFFT_cols(in), then FP64 moments sum z^n s, sum conj(z) s  -> part  (second pass, no store)
  RowsInvRegular = 2, // out = IFFT_rows(phase * ci * R),  R = (S - G)/xi, R(0) = (-i/2) dt   (S = in)
  ColsInvTailFwd = 3, // r = IFFT_cols(in); h = r + sum d_n omega_n; [hout = h]; u = q_k conj(h); out = FFT_cols(u)
  ColsInvTail = 4,    // r = IFFT_cols(in); hout = r + sum d_n omega_n                 (h only)
  RowsFwdEpilogue = 5,// X = FFT_rows(in); out = alpha S + beta cf phase X + gamma Y; optional |out|^2 -> part
  ColsFwdPotential = 6,// out = FFT_cols(Q e_k)                                      (first pass of F(q_k))
  ColsFwdPlain = 7,   // out = FFT_cols(in)
  ColsInvPlain = 8,   // out = IFFT_cols(in)
  // The operator on s = F^{-1} S (x-space form, three launches):
  RowsFwdMoments = 9, // moments sum z^n s, sum conj(z) s of the input (x-space) -> part; out = FFT_rows(in)
  ColsFwdRegularInv = 10, // S = cf phase FFT_cols(in); R = (S - G)/xi, R(0) = (-i/2) dt; out = IFFT_cols(phase ci R)
  RowsInvTailEpilogue = 11, // r = IFFT_rows(in); h = r + sum d_n omega_n; out = alpha S + beta q_k conj(h) + gamma Y;
                            // optional |out|^2 -> part and Gram-Schmidt products -> dot_part
};

struct LineArgs {
  int B = 1;                   // batch entries (grid.y)
  const int* act = nullptr;    // per-entry active flag (nullptr = all active)
  const void* in = nullptr;    size_t in_bs = 0;   // per-entry strides in complex elements
  void* out = nullptr;         size_t out_bs = 0;
  const void* S = nullptr;     size_t S_bs = 0;    // epilogue vector (alpha term)
  const void* Y = nullptr;     size_t Y_bs = 0;    // epilogue vector (gamma term)
  const void* Q = nullptr;     size_t Q_bs = 0;    // potential, same precision as the transform; stride 0 = shared
  const c64* ex = nullptr;     const c64* ey = nullptr;  // [b][N] tables e^{-2i k2 x_j}, e^{-2i k1 y_j}
  const c32* ex32 = nullptr;   const c32* ey32 = nullptr;  // the same rounded to FP32 (FP32 operator)
  size_t e_bs = 0;             // per-entry stride of ex / ey (N; 0 = one table shared by all entries)
  const int* shv = nullptr;    // per-entry grid offsets (m1, m2) of a = 2i conj(k): regularise about xi = a
  int tail_phase_out = 0;      // ColsInvTail with shv: return e_k F^{-1}(h/(xi - a)) instead of F^{-1}(h/(xi - a))
  int accumulate = 0;          // ColsInvTail: hout += result
  const c64* coefG = nullptr;  // [b][kNMom]: c_0..c_M, slot kMaxM+1 = R(0) = (-i/2) dt
  const c64* dmom = nullptr;   // [b][kNMom]: d_0..d_M (tail weights)
  const c32* dmom32 = nullptr; // the same rounded to FP32 (FP32 operator)
  void* hout = nullptr;        size_t hout_bs = 0;  // ColsInvTail(Fwd), RowsInvTail(Epilogue): h (optional on the latter)
  void* sout = nullptr;        size_t sout_bs = 0;  // ColsFwdRegularInv: S before the division (optional)
  void* out32 = nullptr;       size_t out32_bs = 0; // RowsInvTailEpilogue (FP64): the result rounded to FP32 (optional;
                                                    // out may then be null)
  double* part = nullptr;      // per-block partial sums [b][tile][nval]
  const void* tw = nullptr;    // twiddle table exp(-2 pi i j / N), j < N, in the transform's precision
  double L = 1.0, ci = 1.0, cf = 1.0;
  int M = 11;
  double alpha = 0.0, gamma = 0.0;
  int y_rhs = 0;               // RowsInvTailEpilogue: the gamma term is -i q_k, formed from the epilogue's own q_k
                               // (the x-space right-hand side; Y is not read)
  c64 beta{0.0, 0.0};
  int want_norm = 0;           // RowsFwdEpilogue, RowsInvTailEpilogue: accumulate |out|^2 partials
  int tile = 0;                // column stages: tile width variant (see tile_columns)
  // RowsFwdEpilogue, RowsInvTailEpilogue: Gram-Schmidt products Re<V_i, out> for i < dot_nv written as per-tile partials
  // dot_part[b][i][tile] (V_i of entry b at dotV + b * dotV_bs + i * N * N, the transform's precision); the last one,
  // V_{dot_nv - 1}, must be the epilogue's S (alpha != 0)
  const void* dotV = nullptr;  size_t dotV_bs = 0;
  int dot_nv = 0;
  double* dot_part = nullptr;
  int dot_self = 0;            // RowsInvTailEpilogue: |out|^2 as one more value, slot dot_nv (dot_nv + 1 per entry)
  // RowsInvTailEpilogue: per-entry Gram-Schmidt window inside a launch that covers more vectors.  Entries with
  // dot_full[b] == 0 take no products with the first dot_skip vectors (their partials are written as 0); entries with
  // dot_full[b] != 0 (orthogonalised against every vector) take all of them.  dot_full null: all entries take all.
  const int* dot_full = nullptr;
  int dot_skip = 0;
  // RowsFwdMoments: the pending Gram-Schmidt update of its input, in = in - sum_{i < upd_nv} upd_coef[b][i] V_i (V_i
  // at dotV as above), written back to upd_out (the input's own address), |in|^2 partials to upd_part[b][tile]
  const double* upd_coef = nullptr;  int upd_coef_bs = 0;
  int upd_nv = 0;
  double upd_sign = 1.0;       // -1: in += sum coef_i V_i
  int upd_v32 = 0;             // the V_i are FP32 (an FP64 launch updating with an FP32 basis)
  int upd_zero = 0;            // the input counts as zero (its loaded values are ignored)
  void* upd_out = nullptr;
  double* upd_part = nullptr;
};

// Number of blocks (tiles) per batch entry used by a line stage with the current tile choice; partial buffers are
// sized for the default (narrowest, most tiles) choice.
int line_tiles(int N, bool cols, bool fp64);
int line_tiles_variant(int N, bool cols, bool fp64, int variant);
int line_tiles_max(int N, bool cols, bool fp64);  // the most tiles over the variants (sizes partial buffers)
// Column-tile width choice per (N, precision): the number of valid variants (0: the default width; then up to two
// wider tiles, 2x and 4x, while the block has at most 1024 threads and its LDS fits; then half the default width),
// the current choice, and the columns of a variant.
constexpr int kMaxTileVariants = 4;
int tile_variants(int N, bool fp64);
int tile_variant(int N, bool fp64);
int tile_columns(int N, bool fp64, int variant);
void set_tile_variant(int N, bool fp64, int variant);
// Incremented whenever a tile choice changes (captured graphs hold kernels and tile counts of the old choice).
int tuning_epoch();

template <typename T, int N>
void launch_lines(LineOp op, const LineArgs& a, hipStream_t s);

template <typename T>
void launch_lines_any(int N, LineOp op, const LineArgs& a, hipStream_t s);

#define DBAR_FOR_EACH_N(X) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)
#define DBAR_EXTERN_N(NN)                                                              \
  extern template void launch_lines<double, NN>(LineOp, const LineArgs&, hipStream_t); \
  extern template void launch_lines<float, NN>(LineOp, const LineArgs&, hipStream_t);
DBAR_FOR_EACH_N(DBAR_EXTERN_N)
#undef DBAR_EXTERN_N

// ------------------------------------------------------------------------------------------------------------
// Vector (Krylov) kernels on the real 2n view of complex arrays; all accumulation in FP64.
// ------------------------------------------------------------------------------------------------------------
constexpr int kVecBlock = 256;
constexpr int kVecEPT = 4;                          // complex elements per thread per chunk
constexpr int kVecChunk = kVecBlock * kVecEPT;      // complex elements per block

struct VecArgs {
  int B = 1;
  const int* act = nullptr;
  size_t n = 0;                // complex elements per vector
  const void* V = nullptr;     size_t V_bs = 0;   // basis: vector i of entry b at V + b*V_bs + i*n
  int nv = 0;                  // number of basis vectors used
  void* w = nullptr;           size_t w_bs = 0;   // target vector
  const double* coef = nullptr; int coef_bs = 0;  // [b][i] coefficients
  double* part = nullptr;      // [b][value][block] partials
  int want_self = 0;           // dots: also |w|^2 as value nv; update: |w_new|^2 as value 0
};

template <typename T> void launch_dots(const VecArgs& a, hipStream_t s);          // part = <V_i, w>
template <typename T> void launch_update(const VecArgs& a, hipStream_t s);        // w -= sum coef_i V_i
template <typename TX, typename TV> void launch_axpy_multi(const VecArgs& a, hipStream_t s);  // w += sum coef_i V_i
template <typename TO, typename TI> void launch_convert(const void* in, size_t in_bs, void* out, size_t out_bs,
                                                       size_t n, int B, const int* act, double scale, hipStream_t s);
int vec_blocks(size_t n);

// Deterministic reduction of partial sums: out[b][v] = scale * sum_blk part[b][v][blk]
void launch_reduce(const double* part, int nval, int nblk, double* out, int B, const int* act, hipStream_t s);

// ------------------------------------------------------------------------------------------------------------
// Optional measurement: HIP events around every launch, grouped by stage, with the number of active batch entries
// of each launch logged on the device (so algorithmic bytes are exact without host synchronisation).
// ------------------------------------------------------------------------------------------------------------
enum Stage : int {
  kStageLines = 0,                 // + 2 * LineOp + (float ? 1 : 0)
  kStageDots = 32,                 // + (float ? 1 : 0)
  kStageUpdate = 34,
  kStageAxpy = 36,                 // f64 += f64 / f64 += f32 / f32 += f32: 36, 37, 38
  kStageReduce = 39,
  kStageConvert = 40,
  kStageMoments = 41,
  kStageControl = 42,
  kNumStages = 43,
};
const char* stage_name(int stage);
bool timer_on();
// bytes_per_entry counts for every active entry of the launch; bytes_once (arrays shared by all entries of the launch,
// such as one potential read at stride 0) counts once per launch with at least one active entry.
int timer_begin(int stage, double bytes_per_entry, int B, const int* act, hipStream_t s, double bytes_once);
void timer_end(int handle, hipStream_t s);

struct TimerScope {
  int h = -1;
  hipStream_t s;
  TimerScope(int stage, double bytes_per_entry, int B, const int* act, hipStream_t st, double bytes_once = 0.0)
      : s(st) {
    if (timer_on()) h = timer_begin(stage, bytes_per_entry, B, act, st, bytes_once);
  }
  ~TimerScope() {
    if (h >= 0) timer_end(h, s);
  }
};

}  // namespace dbar
