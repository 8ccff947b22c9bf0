// The Jacobi and four-colour orderings of the 2-D FP64 solve: launchers of
// the kernels in sor_variants.hip.  Grids use the 2-D padded layout (origin
// pointer at full-array cell (0, 0), `pitch` elements per row).
#pragma once
#include "sor_internal.h"

namespace sor {

// One Jacobi (over-relaxed for omega != 1) iteration from A into B; B's
// boundary ring must hold the boundary values.  Closes the pass.
hipError_t launch_jacobi_iteration(const double *A, double *B, const double *F,
                                   int64_t pitch, int n, double omega, Ctl *ctl,
                                   const Sched &sc, hipStream_t s);
// One four-colour iteration in place on A: colour 0, then colours 1 and 2
// (which never touch) in one launch, then colour 3, which closes the pass.
hipError_t launch_colour4_iteration(double *A, const double *F, int64_t pitch, int n,
                                    double omega, Ctl *ctl, const Sched &sc,
                                    hipStream_t s);

}  // namespace sor
