// Blocked red-black SOR pass, FP32 storage, 7 iterations per pass, forming
// the maxima of iteration 6 alone / no maxima (one kernel each;
// iterations counted from 0 within the pass).
#include "sor_kernels.h"

namespace sor {
template hipError_t launch_blocked_PT<kF32, 7, 0, 6>(const GridView &, Ctl *,
                                                 const Sched &, hipStream_t,
                                                 const BlockShape &);
template hipError_t launch_blocked_PT<kF32, 7, 0, 7>(const GridView &, Ctl *,
                                                 const Sched &, hipStream_t,
                                                 const BlockShape &);
template int blocked_blocks_per_cu<kF32, 7, 0, 6>(bool);
}  // namespace sor
