// Blocked red-black SOR pass, FP64 storage, 7 iterations per pass, forming
// the maxima of iteration 2 alone / the maxima of iteration 3 alone (one kernel each;
// iterations counted from 0 within the pass).
#include "sor_kernels.h"

namespace sor {
template hipError_t launch_blocked_PT<kF64, 7, 0, 2>(const GridView &, Ctl *,
                                                 const Sched &, hipStream_t,
                                                 const BlockShape &);
template hipError_t launch_blocked_PT<kF64, 7, 0, 3>(const GridView &, Ctl *,
                                                 const Sched &, hipStream_t,
                                                 const BlockShape &);
}  // namespace sor
