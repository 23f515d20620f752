// Line-transform kernels for N = 2048 (one translation unit per grid size keeps builds parallel).
#include "dbar_lines.h"

namespace dbar {
DBAR_INSTANTIATE_N(2048)
}  // namespace dbar
