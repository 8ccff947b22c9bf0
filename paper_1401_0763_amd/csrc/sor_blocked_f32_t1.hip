// Blocked red-black SOR pass, FP32 storage, 1 iteration(s) per pass.
#include "sor_kernels.h"

namespace sor {
template hipError_t launch_blocked_PT<kF32, 1>(const GridView &, Ctl *,
                                              const Sched &, hipStream_t,
                                              const BlockShape &);
template int blocked_blocks_per_cu<kF32, 1>(bool);
}  // namespace sor
