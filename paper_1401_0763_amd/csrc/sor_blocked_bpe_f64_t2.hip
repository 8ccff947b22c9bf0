// Blocked block-parallel red-black pass for blocks of even width, FP64
// storage, 2 iteration(s) per pass.
#include "sor_kernels.h"

namespace sor {
template hipError_t launch_blocked_PT<kF64, 2, 4>(const GridView &, Ctl *,
                                                 const Sched &, hipStream_t,
                                                 const BlockShape &);
template int blocked_blocks_per_cu<kF64, 2, 4>(bool);
}  // namespace sor
