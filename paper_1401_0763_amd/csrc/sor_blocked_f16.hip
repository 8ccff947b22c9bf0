// Blocked red-black SOR pass kernels with binary16 storage
// (one translation unit per precision so they build in parallel).
#include "sor_kernels.h"

namespace sor {
SOR_BLOCKED_LAUNCHER(kF16, launch_blocked_f16)
}  // namespace sor
