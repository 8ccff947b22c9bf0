// 3-D grids (7-point stencil on the unit cube): launchers of the set-up and
// iteration kernels in sor_3d.hip.
#pragma once
#include "sor_internal.h"

namespace sor {

constexpr int kMaxN3 = 1024;     // largest side accepted
// Elements per row of the padded (n+2)^3 array.
int64_t grid3_pitch(int n);
hipError_t launch_pack3d(const double *u, const double *bdy, const double *f, double *U,
                         double *F, int n, unsigned *bad, hipStream_t s);
hipError_t launch_unpack3d(const double *U, double *u, int n, hipStream_t s);
// One iteration: the red launch, then the black launch (which closes the
// pass for the device-side verdict).
hipError_t launch_sor3d_iteration(double *U, const double *F, int n, double omega,
                                  Ctl *ctl, const Sched &sc, hipStream_t s);

}  // namespace sor
