// Blocked red-black SOR pass kernels with FP32 storage
// (one translation unit per precision so they build in parallel).
#include "sor_kernels.h"

namespace sor {
SOR_BLOCKED_LAUNCHER(kF32, launch_blocked_f32)
}  // namespace sor
