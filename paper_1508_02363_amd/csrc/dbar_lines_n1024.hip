// Line-transform kernels for N = 1024 (one translation unit per grid size keeps builds parallel).
#include "dbar_lines.h"

namespace dbar {
DBAR_INSTANTIATE_N(1024)
}  // namespace dbar
