// Blocked Jacobi pass, FP64 storage, 8 iteration(s) per pass.
#include "sor_kernels.h"

namespace sor {
template hipError_t launch_blocked_PT<kF64, 8, 2>(const GridView &, Ctl *,
                                                 const Sched &, hipStream_t,
                                                 const BlockShape &);
template int blocked_blocks_per_cu<kF64, 8, 2>(bool);
}  // namespace sor
