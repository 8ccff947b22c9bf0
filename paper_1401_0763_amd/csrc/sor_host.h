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
  sor_tiling tiling[3] = {{4, 192}, {4, 96}, {4, 96}};  // by precision
  sor::DevBuf bufs[sor::kNumRoles];
  sor::Ctl *host_ctl = nullptr;                        // pinned mirror
  double *host_stats = nullptr;                        // pinned [4]
  bool prof = false;                                   // time sweep launches
  std::vector<hipEvent_t> events;                      // start/stop pairs
  double prof_ms = 0.0;
  int64_t prof_launches = 0;
  sor::BatchState *batch = nullptr;                    // batched-solve state
};

namespace sor {

sor_status fail(sor_ctx *c, sor_status st, const char *fmt, ...);
sor_status ensure(sor_ctx *c, BufRole role, size_t bytes);
bool is_device_ptr(sor_ctx *c, const void *p);
sor_status check_common(sor_ctx *c, const void *u, const void *bdy,
                        const void *rhs, int32_t n, double omega);
int prec_index(int bits);
void batch_state_free(sor_ctx *c);
void mix_state_free(sor_ctx *c);
// Plain-solve tiling for a grid side: the autotuned entry of its size class,
// else the context's tiling for the precision.
sor_tiling tuned_tiling(sor_ctx *c, int prec, int n);
void clear_tuning(sor_ctx *c, int prec);

}  // namespace sor

#define HIP_TRY(ctx, expr)                                                   \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      return ::sor::fail((ctx), SOR_EDEVICE, "%s: %s", #expr,                \
                         hipGetErrorString(e_));                             \
  } while (0)
