// Blocked red-black SOR pass, FP32 storage, 2 iteration(s) per pass.
#include "sor_kernels.h"

namespace sor {
template hipError_t launch_blocked_PT<kF32, 2>(const GridView &, Ctl *,
                                              const Sched &, hipStream_t,
                                              const BlockShape &);
template int blocked_blocks_per_cu<kF32, 2>(bool);
}  // namespace sor
