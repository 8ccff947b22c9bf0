// Host-side internals of libsor shared by its host translation units: the
// context object, its device buffers, and error/validation helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/sor.h"
#include "sor_internal.h"

namespace sor {

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

enum BufRole {
  kGridA64, kGridB64, kF64Buf,     // plain FP64 solve; U64 of the mixed solve
  kGridA32, kGridB32, kF32Buf,     // plain FP32 solve; inner grids of mixed
  kLoRhs,                          // inner right-hand side of the mixed solve
  kPartials, kStats, kCtlBuf,
  kBatchArena, kBatchGrids, kBatchQueue, kBatchRing,   // batched solves
  kNumRoles
};

struct BatchState;   // defined in sor_batch_api.cpp

}  // namespace sor

struct sor_ctx {
  int device = 0;
  std::string err;
  int kernel = SOR_KERNEL_BLOCKED;
  sor_tiling tiling[3] = {{6, 0}, {6, 0}, {6, 0}};  // by precision; seg 0: by size
  bool depth_auto[3] = {true, true, true};             // depth chosen per solve until set
  sor::DevBuf bufs[sor::kNumRoles];
  sor::Ctl *host_ctl = nullptr;                        // pinned mirror
  double *host_stats = nullptr;                        // pinned [4]
  bool prof = false;                                   // time sweep launches
  std::vector<hipEvent_t> events;                      // start/stop pairs
  double prof_ms = 0.0;
  int64_t prof_launches = 0;
  sor::BatchState *batch = nullptr;                    // batched-solve state
  int cus = 0;                                         // compute units (lazy)
  int occ[3][sor::kTMax + 1][2] = {};                   // pass blocks per CU (lazy)
  // Blocked passes of the other orderings, by pass ordering (1 four-colour,
  // 2 Jacobi, 3 block-parallel; 0 unused); seg 0: by size.
  sor_tiling tiling_var[4] = {{0, 0}, {5, 0}, {8, 0}, {5, 0}};
  int occ_var[5][sor::kTMax + 1][2] = {};              // their pass blocks per CU (lazy;
                                                       // 4: block-parallel, even width)
  int tiling3d[4] = {0, 0, 0, 0};                      // 3-D T, cx, cy, zs; 0: auto
  int occ3[2][2] = {};                                 // 3-D stream blocks per CU (lazy)
  void *scratch = nullptr;                             // allocation-free solve's memory
};

namespace sor {

sor_status fail(sor_ctx *c, sor_status st, const char *fmt, ...);
sor_status ensure(sor_ctx *c, BufRole role, size_t bytes);
bool is_device_ptr(sor_ctx *c, const void *p);
sor_status check_common(sor_ctx *c, const void *u, const void *bdy,
                        const void *rhs, int32_t n, double omega);
int prec_index(int bits);
// Young's optimal omega 2/(1 + sin(pi/(n+1))) (sor_omega_opt).
double omega_opt(int n);
// Inner SOR iterations per correction of the mixed-precision solves when the
// caller passes none: n/2 rounded up to a multiple of the batched kernel's
// fixed depth kMixTMax (at least that depth), so that batched and served
// grids run in the fixed-depth kernel.  Measured on 4096^2 to 256^2 Poisson
// problems, about n/2 reaches a relative residual of 1e-8 in the least time
// (each correction then lowers the residual about 20-fold); 2n and n take
// longer.
inline int64_t mixed_inner_default(int n) {
  const int64_t half = n > 1 ? (int64_t)(n / 2) : 1;
  return (half + kMixTMax - 1) / kMixTMax * kMixTMax;
}
// Largest side of a mixed-precision solve with binary16 inner storage.  Above
// it the 11-bit significand cannot hold the smooth correction: the inner
// sweeps stop moving once the per-iteration change of a cell is below half an
// ulp of its value, and the rounding of a smooth field is itself smooth, so
// the correction is wrong in exactly the components SOR is slow to fix.
// Measured: the refinement reaches 1e-8 within 30 corrections up to n = 1024
// and stalls near a relative residual of 1e2-1e3 from n = 1536.
constexpr int kMaxN16 = 1024;
void batch_state_free(sor_ctx *c);
void mix_state_free(sor_ctx *c);
// Segment rows chosen from the grid side for one plain solve: as many tiles
// as the pass kernel has resident wavefront slots on the device (or a whole
// multiple of that when a single round would need segments above 768 rows),
// and at least twice the stage count (2T red-black, 3T four-colour, T
// Jacobi).
int auto_seg_rows(sor_ctx *c, int prec, int n, int T, bool pois, int ord = 0);
// Depth of a plain solve while the context's depth is automatic: 7 where the
// 7-deep pass kernel keeps two wavefronts per SIMD, else 6.
int auto_depth(sor_ctx *c, int prec, bool pois);
// Tiling of a plain solve of side n: the autotuned entry of its size class if
// there is one, else the context's tiling (depth from auto_depth while it is
// automatic) with seg_rows from auto_seg_rows when none was set.
sor_tiling tuned_tiling(sor_ctx *c, int prec, int n, bool pois);
// Tiling of one grid inside a batched launch (many grids share the chip, so
// a grid's own tile count does not need to fill it): the autotuned entry, else
// the context's tiling with 64 rows below n = 512 and 192 (FP64) or 96 rows
// above when none was set.
sor_tiling batch_tiling(sor_ctx *c, int prec, int n);
void clear_tuning(sor_ctx *c, int prec);
sor_status check_sched(sor_ctx *c, double tol, int64_t max_iters, int64_t K);
// One plain red-black solve (prec kF64 or kF32) on caller-provided working
// grids of layout L (origins A, B and, with a source, F) and two control
// blocks (ctl, ctl + 1): pack, sweep passes with device-side checks, unpack.
// Arguments must already be validated.  Allocates nothing while the
// context's profiling is off.
sor_status solve_plain_on(sor_ctx *c, int prec, const Layout &L, void *u, const void *bdy,
                          const void *rhs, void *A, void *B, void *F, Ctl *ctl, double omega,
                          const Sched &sc, hipStream_t s, sor_result *out, double *hist);
// Per-device set-up of the allocation-free entry point (sor_noalloc.hip),
// called by sor_ctx_create with the device current.
sor_status noalloc_init(sor_ctx *c);

}  // namespace sor

#define HIP_TRY(ctx, expr)                                                   \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      return ::sor::fail((ctx), SOR_EDEVICE, "%s: %s", #expr,                \
                         hipGetErrorString(e_));                             \
  } while (0)
