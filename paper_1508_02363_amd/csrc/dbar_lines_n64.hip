// Line-transform kernels for N = 64 (one translation unit per grid size keeps builds parallel).
#include "dbar_lines.h"

namespace dbar {
DBAR_INSTANTIATE_N(64)
}  // namespace dbar
