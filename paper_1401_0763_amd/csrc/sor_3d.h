// 3-D grids (7-point stencil on the unit cube): launchers of the set-up and
// iteration kernels in sor_3d.hip.
#pragma once
#include "sor_internal.h"

namespace sor {

constexpr int kMaxN3 = 1024;     // largest side accepted
// Elements per row of the padded (n+2)^3 array.
int64_t grid3_pitch(int n);
// Pack into U and (if not null) U2: interior from u, faces from bdy, the rest 0.
hipError_t launch_pack3d(const double *u, const double *bdy, const double *f, double *U,
                         double *U2, double *F, int n, unsigned *bad, hipStream_t s);
hipError_t launch_unpack3d(const double *U, double *u, int n, hipStream_t s);
// Streaming kernel tiling for T iterations per launch (ring 2T): core
// CX x CY x Zs cells, region RX = CX+4T by RY = CY+4T positions, ntx x nty x
// nzt tiles (one workgroup each).  cx, cy, zs = 0 pick automatically (the
// x-y shape with the least halo per core cell, then the z-range that fills
// whole rounds of `slots` resident workgroups with short walks); ok is false
// if the region exceeds a workgroup's positions.
struct Tiling3 {
  int CX, CY, Zs, RX, RY, ntx, nty, nzt, T;
  bool ok;
};
Tiling3 tiling3(int n, int T, int cx, int cy, int zs, int slots);
// Most region positions of a T-iteration workgroup.
int stream3d_positions(int T);
// Resident streaming workgroups per CU (0 if the query fails).
int stream3d_blocks_per_cu(int T, bool pois);
// T (1 or 2) iterations A -> B with tiling t (made for that T); boundary
// cells of B must hold the boundary values.  Closes one pass of T iterations.
hipError_t launch_sor3d_stream(const double *A, double *B, const double *F, int n,
                               double omega, const Tiling3 &t, int T, Ctl *ctl,
                               const Sched &sc, hipStream_t s);
// One iteration: the red launch, then the black launch (which closes the
// pass for the device-side verdict).
hipError_t launch_sor3d_iteration(double *U, const double *F, int n, double omega,
                                  Ctl *ctl, const Sched &sc, hipStream_t s);

}  // namespace sor
