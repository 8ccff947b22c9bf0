// Blocked red-black SOR pass kernels with FP64 storage
// (one translation unit per precision so they build in parallel).
#include "sor_kernels.h"

namespace sor {
SOR_BLOCKED_LAUNCHER(kF64, launch_blocked_f64)
}  // namespace sor
