// Blocked red-black SOR pass, FP64 storage, 2 iteration(s) per pass.
#include "sor_kernels.h"

namespace sor {
template hipError_t launch_blocked_PT<kF64, 2>(const GridView &, Ctl *,
                                              const Sched &, hipStream_t,
                                              const BlockShape &);
template int blocked_blocks_per_cu<kF64, 2>(bool);
}  // namespace sor
