// Blocked red-black SOR pass, FP64 storage, 6 iterations per pass, forming
// no maxima (one kernel each;
// iterations counted from 0 within the pass).
#include "sor_kernels.h"

namespace sor {
template hipError_t launch_blocked_PT<kF64, 6, 0, 6>(const GridView &, Ctl *,
                                                 const Sched &, hipStream_t,
                                                 const BlockShape &);
}  // namespace sor
