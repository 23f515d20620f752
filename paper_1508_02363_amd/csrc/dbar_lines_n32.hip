// Line-transform kernels for N = 32 (one translation unit per grid size keeps builds parallel).
#include "dbar_lines.h"

namespace dbar {
DBAR_INSTANTIATE_N(32)
}  // namespace dbar
