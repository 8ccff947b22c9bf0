// Blocked red-black SOR pass, binary16 storage, 7 iteration(s) per pass.
#include "sor_kernels.h"

namespace sor {
template hipError_t launch_blocked_PT<kF16, 7>(const GridView &, Ctl *,
                                              const Sched &, hipStream_t,
                                              const BlockShape &);
template int blocked_blocks_per_cu<kF16, 7>(bool);
}  // namespace sor
