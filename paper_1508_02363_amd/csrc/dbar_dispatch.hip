// Run-time dispatch over the grid size N for the line-transform stages.
#include <algorithm>
#include <atomic>

#include "dbar_lines.h"

namespace dbar {

// ------------------------------------------------------------------------------------------------------------
// Column-tile width choices (set by the tuner; default 0 = the narrowest tile)
// ------------------------------------------------------------------------------------------------------------
static int size_index(int N) {
  int i = 0;
  for (int m = 8; m < N && i < 12; m <<= 1) ++i;
  return i;
}
static std::atomic<int> g_tile[2][12];  // [fp64][log2(N) - 3]
static std::atomic<int> g_epoch{0};

int tile_variants(int N, bool fp64) {
#define DBAR_VARIANTS(NN) \
  if (N == NN) return fp64 ? Tiling<double, NN>::variants() : Tiling<float, NN>::variants();
  DBAR_FOR_EACH_N(DBAR_VARIANTS)
#undef DBAR_VARIANTS
  return 1;
}

int tile_variant(int N, bool fp64) { return g_tile[fp64 ? 1 : 0][size_index(N)].load(); }

void set_tile_variant(int N, bool fp64, int variant) {
  if (variant < 0 || variant >= tile_variants(N, fp64)) variant = 0;
  if (g_tile[fp64 ? 1 : 0][size_index(N)].exchange(variant) != variant) ++g_epoch;
}

int tuning_epoch() { return g_epoch.load(); }

template <typename T, int N>
static int tile_cols(int variant) {
  using Tl = Tiling<T, N>;
  switch (variant) {
    case 1: return Tl::template cols_v<1>();
    case 2: return Tl::template cols_v<2>();
    case 3: return Tl::template cols_v<3>();
    default: return Tl::COLS;
  }
}

int line_tiles_variant(int N, bool cols, bool fp64, int variant) {
#define DBAR_TILES(NN)                                                                               \
  if (N == NN) {                                                                                     \
    if (fp64) return NN / (cols ? tile_cols<double, NN>(variant) : Tiling<double, NN>::ROWS);        \
    return NN / (cols ? tile_cols<float, NN>(variant) : Tiling<float, NN>::ROWS);                    \
  }
  DBAR_FOR_EACH_N(DBAR_TILES)
#undef DBAR_TILES
  return 0;
}

int line_tiles_max(int N, bool cols, bool fp64) {
  int t = 0;
  for (int v = 0; v < (cols ? tile_variants(N, fp64) : 1); ++v) t = std::max(t, line_tiles_variant(N, cols, fp64, v));
  return t;
}

int tile_columns(int N, bool fp64, int variant) { return N / line_tiles_variant(N, true, fp64, variant); }

int line_tiles(int N, bool cols, bool fp64) {
  return line_tiles_variant(N, cols, fp64, cols ? tile_variant(N, fp64) : 0);
}

// Algorithmic HBM bytes of one stage (each array read or written once): per batch entry, and once per launch for the
// potential when all entries share it (Q_bs = 0: one array read at stride 0 by every entry).
static double line_bytes_once(int N, LineOp op, const LineArgs& a, size_t es) {
  const bool reads_q = op == LineOp::ColsInvTailFwd || op == LineOp::RowsInvTailEpilogue ||
                       op == LineOp::ColsFwdPotential;
  return reads_q && a.Q_bs == 0 ? (double)N * N * es : 0.0;
}
static double line_bytes(int N, LineOp op, const LineArgs& a, size_t es) {
  const double P = (double)N * N * es;
  const double PQ = a.Q_bs == 0 ? 0.0 : P;  // the potential, when every entry reads its own
  switch (op) {
    case LineOp::RowsInvScaled: return 2 * P;
    case LineOp::ColsInvMoments: return P;
    case LineOp::RowsInvRegular: return 2 * P;
    case LineOp::ColsInvTailFwd: return 2 * P + PQ + (a.hout ? P : 0.0);
    case LineOp::ColsInvTail: return 2 * P;
    case LineOp::RowsFwdEpilogue:  // fused dots read V_i, i < dot_nv - 1, besides S (= V_{dot_nv - 1})
      return 2 * P + (a.alpha != 0.0 ? P : 0.0) + (a.gamma != 0.0 ? P : 0.0) +
             (a.dot_nv > 0 ? (a.dot_nv - (a.alpha != 0.0 ? 1 : 0)) * P : 0.0);
    case LineOp::ColsFwdPotential: return P + PQ;
    case LineOp::ColsFwdPlain: return 2 * P;
    case LineOp::ColsInvPlain: return 2 * P;
    case LineOp::RowsFwdMoments: return 2 * P + (a.upd_coef ? P + a.upd_nv * (a.upd_v32 ? P / 2 : P) : 0.0);
    case LineOp::ColsFwdRegularInv: return 2 * P + (a.sout ? P : 0.0);
    case LineOp::RowsInvTailEpilogue:  // in, Q (per entry unless shared), out, S, Y (unless formed from q_k), h, the
                                       // FP32 copy, earlier basis
      return P + PQ + (a.out ? P : 0.0) + (a.out32 ? P / 2 : 0.0) + (a.alpha != 0.0 ? P : 0.0) +
             (a.gamma != 0.0 && !a.y_rhs ? P : 0.0) + (a.hout ? P : 0.0) +
             (a.dot_nv > 0 ? (a.dot_nv - (a.alpha != 0.0 ? 1 : 0)) * P : 0.0);
  }
  return 0.0;
}

template <typename T>
void launch_lines_any(int N, LineOp op, const LineArgs& a_in, hipStream_t s) {
  TimerScope ts(kStageLines + 2 * static_cast<int>(op) + (sizeof(T) == 4 ? 1 : 0),
                line_bytes(N, op, a_in, sizeof(cx<T>)), a_in.B, a_in.act, s, line_bytes_once(N, op, a_in, sizeof(cx<T>)));
  LineArgs a = a_in;
  a.tile = tile_variant(N, sizeof(T) == 8);
  switch (N) {
#define DBAR_CASE(NN) \
  case NN:            \
    launch_lines<T, NN>(op, a, s); \
    break;
    DBAR_FOR_EACH_N(DBAR_CASE)
#undef DBAR_CASE
    default:
      break;
  }
}

template void launch_lines_any<double>(int, LineOp, const LineArgs&, hipStream_t);
template void launch_lines_any<float>(int, LineOp, const LineArgs&, hipStream_t);

}  // namespace dbar
