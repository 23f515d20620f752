// Run-time dispatch over the grid size N for the line-transform stages.
#include "dbar_lines.h"

namespace dbar {

int line_tiles(int N, bool cols, bool fp64) {
#define DBAR_TILES(NN)                                                                          \
  if (N == NN) {                                                                                \
    if (fp64) return NN / (cols ? Tiling<double, NN>::COLS : Tiling<double, NN>::ROWS);         \
    return NN / (cols ? Tiling<float, NN>::COLS : Tiling<float, NN>::ROWS);                     \
  }
  DBAR_FOR_EACH_N(DBAR_TILES)
#undef DBAR_TILES
  return 0;
}

// Algorithmic HBM bytes per batch entry of one stage (each array read or written once).
static double line_bytes(int N, LineOp op, const LineArgs& a, size_t es) {
  const double P = (double)N * N * es;
  switch (op) {
    case LineOp::RowsInvScaled: return 2 * P;
    case LineOp::ColsInvMoments: return P;
    case LineOp::RowsInvRegular: return 2 * P;
    case LineOp::ColsInvTailFwd: return 3 * P + (a.hout ? P : 0.0);
    case LineOp::ColsInvTail: return 2 * P;
    case LineOp::RowsFwdEpilogue: return 2 * P + (a.alpha != 0.0 ? P : 0.0) + (a.gamma != 0.0 ? P : 0.0);
    case LineOp::ColsFwdPotential: return 2 * P;
    case LineOp::ColsFwdPlain: return 2 * P;
    case LineOp::ColsInvPlain: return 2 * P;
  }
  return 0.0;
}

template <typename T>
void launch_lines_any(int N, LineOp op, const LineArgs& a, hipStream_t s) {
  TimerScope ts(kStageLines + 2 * static_cast<int>(op) + (sizeof(T) == 4 ? 1 : 0),
                line_bytes(N, op, a, sizeof(cx<T>)), a.B, a.act, s);
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
