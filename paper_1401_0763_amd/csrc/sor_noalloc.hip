// Allocation-free plain FP64 solve: sor_solve_f64 on working memory that is
// part of the library's code object instead of hipMalloc'd context buffers.
//
// `scratch` below is a device array of fixed size; each GPU holds its own
// copy (at its own address) from the moment the library's code is loaded on
// it until the process ends.  Host code never uses the array's name as a
// device address: sor_ctx_create resolves the address once per device with
// hipGetSymbolAddress (noalloc_init) and keeps it, and the solve hands that
// address to the kernels.  The solve carves two control blocks and the
// padded working grids A, B (and F with a source) out of it; packing writes
// every element of A, F and the non-interior part of B and the control
// blocks are reset, so nothing a previous call left behind is read.  Every
// call of one process on one GPU uses the same array, whatever its context
// or stream: two such calls in flight at the same time race.  (Each process
// has its own copy.)
#include <hip/hip_runtime.h>

#include <mutex>

#include "sor_host.h"

using namespace sor;

namespace {

// Working memory of the allocation-free solve (per GPU).
constexpr size_t kNoallocBytes = size_t(64) << 20;

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};           // scratch's address on each device
hipError_t g_err[kMaxDevices] = {};      // failure of its lookup, if any
bool g_done[kMaxDevices] = {};

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Bytes the solve needs for side n (FP64 grids A and B, F with a source, and
// the two control blocks).
size_t noalloc_need(int n, bool rhs) {
  const Layout L = make_layout(n, kF64);
  const size_t grid = round256((size_t)L.elems() * sizeof(double));
  return round256(2 * sizeof(Ctl)) + (rhs ? 3 : 2) * grid;
}

// Largest side whose working memory fits (the need grows with n).
int noalloc_max_n(bool rhs) {
  int lo = 1, hi = kMaxN;
  while (lo < hi) {
    const int mid = lo + (hi - lo + 1) / 2;
    if (noalloc_need(mid, rhs) <= kNoallocBytes) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace

namespace sor {

sor_status noalloc_init(sor_ctx *c) {
  const int d = c->device;
  if (d < 0 || d >= kMaxDevices) return SOR_OK;     // the solve reports it
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_done[d]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    g_ptr[d] = p;
    g_err[d] = e;
    g_done[d] = true;
  }
  c->scratch = g_ptr[d];
  return SOR_OK;
}

}  // namespace sor

extern "C" sor_status sor_solve_f64_noalloc(sor_ctx *c, double *u, const double *boundary,
                                            const double *rhs, int32_t n, double omega,
                                            double tol, int64_t max_iters,
                                            int64_t check_every, void *stream,
                                            sor_result *out, double *max_hist) {
  sor_status st = check_common(c, u, boundary, rhs, n, omega);
  if (st != SOR_OK) return st;
  if (!out) return fail(c, SOR_EINVAL, "out must not be NULL");
  if ((st = check_sched(c, tol, max_iters, check_every)) != SOR_OK) return st;
  if (!c->scratch) {
    hipError_t e = hipErrorInvalidDevice;
    if (c->device >= 0 && c->device < kMaxDevices) {
      std::lock_guard<std::mutex> lk(g_mu);
      e = g_err[c->device];
    }
    return fail(c, SOR_EDEVICE, "working memory of the allocation-free solve is not "
                "available on device %d: %s", c->device, hipGetErrorString(e));
  }
  const size_t need = noalloc_need(n, rhs != nullptr);
  if (need > kNoallocBytes)
    return fail(c, SOR_EINVAL, "n = %d needs %zu bytes of working memory; the "
                "allocation-free solve holds %zu (n <= %d without a source, "
                "n <= %d with one)", n, need, kNoallocBytes, noalloc_max_n(false),
                noalloc_max_n(true));
  const Layout L = make_layout(n, kF64);
  const size_t grid = round256((size_t)L.elems() * sizeof(double));
  unsigned char *base = (unsigned char *)c->scratch;
  Ctl *ctl = (Ctl *)base;
  unsigned char *g0 = base + round256(2 * sizeof(Ctl));
  double *A = (double *)g0 + L.origin_off();
  double *B = (double *)(g0 + grid) + L.origin_off();
  double *F = rhs ? (double *)(g0 + 2 * grid) + L.origin_off() : nullptr;
  // Profiling would create events on first use: off for this call.
  const bool prof = c->prof;
  c->prof = false;
  st = solve_plain_on(c, kF64, L, (void *)u, boundary, rhs, A, B, F, ctl, omega,
                      Sched{max_iters, check_every, tol}, (hipStream_t)stream, out, max_hist);
  c->prof = prof;
  return st;
}
