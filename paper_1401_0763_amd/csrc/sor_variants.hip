// The two alternatives to the red-black order that Mittal 2014 names, for the
// 2-D FP64 problem: Jacobi (Sec. 2.1: every cell from the previous
// iteration's values; omega != 1 gives the over-relaxed Jacobi iteration)
// and multi-colour SOR (Sec. 3.1) with four colours, colour(i, j) =
// 2 (i mod 2) + (j mod 2) on the full array, swept in the order 0, 1, 2, 3.
// Same Gauss-Seidel value ((N + S) + (W + E) [+ h*h*f]) * 0.25, its
// difference from the old value and the relaxation step each formed with one
// rounding, increment form of Eq. 1 and stopping rule (Algorithm 1) as the red-black path.
//
// Both kernels walk a strip of kVR rows with one thread per column pair
// (2t, 2t+1) of the full array, keeping the rows above, at and below the
// current one in registers; west and east neighbours outside the pair are
// loaded from memory.  Jacobi reads A and writes B (ping-pong).  The
// four-colour launches work in place: the cells one launch updates are
// pairwise non-adjacent, so every neighbour it reads is one no thread of the
// launch writes, and colours 1 and 2 (never adjacent, both bordering only 0
// and 3) share a launch, which gives the same result as sweeping 1 then 2.
#include "sor_kernels.h"
#include "sor_variants.h"

namespace sor {

constexpr int kVT = 256;    // threads per workgroup (column pairs)
constexpr int kVR = 32;     // rows per workgroup

struct VGrid {
  const double *A;     // input (Jacobi) or the grid itself (four-colour)
  double *B;           // output (Jacobi) or A again
  const double *F;     // h*h*f or nullptr
  int64_t pitch;
  int n;
  double omega;
};

__device__ __forceinline__ double2 ld_pair(const double *p) {
  return *reinterpret_cast<const double2 *>(p);
}

// Workgroup maximum and non-finite flag; then either merge into the pass
// slots (finish == 0) or report the pass (finish != 0, every workgroup of
// the launch reports once).
__device__ __forceinline__ void block_report(Ctl *ctl, const Sched &sc, double dmax, bool bad,
                                             int finish) {
  __shared__ double wmax[kVT / 64];
  __shared__ int wbad[kVT / 64];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const double wm = wave_max(dmax);
  const bool wb = __ballot(bad) != 0;
  if (lane == 0) {
    wmax[wave] = wm;
    wbad[wave] = wb;
  }
  __syncthreads();
  if (wave != 0) return;
  double mx[1] = {0.0};
  bool bb = false;
#pragma unroll
  for (int w = 0; w < kVT / 64; ++w) {
    mx[0] = fmax(mx[0], wmax[w]);
    bb = bb || wbad[w];
  }
  const unsigned block = blockIdx.x + gridDim.x * blockIdx.y;
  const int slot = (int)(block % kSlots);
  if (!finish) {
    if (lane == 0) {
      __hip_atomic_fetch_max(&ctl->slots[slot][0],
                             (unsigned long long)__double_as_longlong(mx[0]),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (bb)
        __hip_atomic_fetch_or(&ctl->nonfinite, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  report_pass<1>(ctl, sc, mx, 1, bb && lane == 0, slot, gridDim.x * gridDim.y);
}

__device__ __forceinline__ double relax(double self, double s, double omega) {
  return __builtin_fma(omega, __builtin_fma(0.25, s, -self), self);
}

template <bool POIS>
__global__ __launch_bounds__(kVT) void jacobi_kernel(VGrid g, Ctl *ctl, Sched sc) {
  if (ctl_stopped(ctl)) return;
  const int n = g.n;
  const int64_t P = g.pitch;
  const int t = blockIdx.x * kVT + threadIdx.x;
  const int j = 2 * t;
  const int r0 = 1 + blockIdx.y * kVR, r1 = min(r0 + kVR, n + 1);
  double dmax = 0.0;
  bool bad = false;
  if (t <= n / 2) {
    const bool up0 = j >= 1 && j <= n, up1 = j + 1 <= n;
    const double *a = g.A + j;
    double2 nr = ld_pair(a + (int64_t)(r0 - 1) * P), mr = ld_pair(a + (int64_t)r0 * P);
    for (int i = r0; i < r1; ++i) {
      const int64_t o = (int64_t)i * P;
      const double2 sr = ld_pair(a + o + P);
      const double w = a[o - 1], e = a[o + 2];
      double2 out = mr;
      if (up0) {
        double s = (nr.x + sr.x) + (w + mr.y);
        if (POIS) s = s + g.F[o + j];
        out.x = relax(mr.x, s, g.omega);
        dmax = fmax(dmax, fabs(out.x - mr.x));
        bad = bad || !__builtin_isfinite(out.x);
      }
      if (up1) {
        double s = (nr.y + sr.y) + (mr.x + e);
        if (POIS) s = s + g.F[o + j + 1];
        out.y = relax(mr.y, s, g.omega);
        dmax = fmax(dmax, fabs(out.y - mr.y));
        bad = bad || !__builtin_isfinite(out.y);
      }
      *reinterpret_cast<double2 *>(g.B + o + j) = out;
      nr = mr;
      mr = sr;
    }
  }
  block_report(ctl, sc, dmax, bad, 1);
}

// Cells of the colours in `mask` (bit c = colour c) are updated in place.
template <bool POIS>
__global__ __launch_bounds__(kVT) void colour4_kernel(VGrid g, Ctl *ctl, Sched sc,
                                                      unsigned mask, int finish) {
  if (ctl_stopped(ctl)) return;
  const int n = g.n;
  const int64_t P = g.pitch;
  const int t = blockIdx.x * kVT + threadIdx.x;
  const int j = 2 * t;
  const int r0 = 1 + blockIdx.y * kVR, r1 = min(r0 + kVR, n + 1);
  double dmax = 0.0;
  bool bad = false;
  if (t <= n / 2) {
    const bool in0 = j >= 1 && j <= n, in1 = j + 1 <= n;
    double *a = g.B + j;
    double2 nr = ld_pair(a + (int64_t)(r0 - 1) * P), mr = ld_pair(a + (int64_t)r0 * P);
    for (int i = r0; i < r1; ++i) {
      const int64_t o = (int64_t)i * P;
      const double2 sr = ld_pair(a + o + P);
      const int c0 = 2 * (i & 1);                   // colour of column j (even)
      const bool up0 = in0 && (mask >> c0 & 1u), up1 = in1 && (mask >> (c0 + 1) & 1u);
      if (up0) {
        double s = (nr.x + sr.x) + (a[o - 1] + mr.y);
        if (POIS) s = s + g.F[o + j];
        const double nu = relax(mr.x, s, g.omega);
        dmax = fmax(dmax, fabs(nu - mr.x));
        bad = bad || !__builtin_isfinite(nu);
        mr.x = nu;
        a[o] = nu;
      }
      if (up1) {
        double s = (nr.y + sr.y) + (mr.x + a[o + 2]);
        if (POIS) s = s + g.F[o + j + 1];
        const double nu = relax(mr.y, s, g.omega);
        dmax = fmax(dmax, fabs(nu - mr.y));
        bad = bad || !__builtin_isfinite(nu);
        mr.y = nu;
        a[o + 1] = nu;
      }
      nr = mr;
      mr = sr;
    }
  }
  block_report(ctl, sc, dmax, bad, finish);
}

namespace {
dim3 variant_grid(int n) {
  return dim3((unsigned)((n / 2 + 1 + kVT - 1) / kVT), (unsigned)((n + kVR - 1) / kVR));
}
}  // namespace

hipError_t launch_jacobi_iteration(const double *A, double *B, const double *F,
                                   int64_t pitch, int n, double omega, Ctl *ctl,
                                   const Sched &sc, hipStream_t s) {
  const VGrid g{A, B, F, pitch, n, omega};
  if (F)
    hipLaunchKernelGGL(jacobi_kernel<true>, variant_grid(n), dim3(kVT), 0, s, g, ctl, sc);
  else
    hipLaunchKernelGGL(jacobi_kernel<false>, variant_grid(n), dim3(kVT), 0, s, g, ctl, sc);
  return hipGetLastError();
}

hipError_t launch_colour4_iteration(double *A, const double *F, int64_t pitch, int n,
                                    double omega, Ctl *ctl, const Sched &sc,
                                    hipStream_t s) {
  const VGrid g{A, A, F, pitch, n, omega};
  const unsigned masks[3] = {0x1u, 0x6u, 0x8u};
  for (int k = 0; k < 3; ++k) {
    if (F)
      hipLaunchKernelGGL(colour4_kernel<true>, variant_grid(n), dim3(kVT), 0, s, g, ctl, sc,
                         masks[k], k == 2 ? 1 : 0);
    else
      hipLaunchKernelGGL(colour4_kernel<false>, variant_grid(n), dim3(kVT), 0, s, g, ctl, sc,
                         masks[k], k == 2 ? 1 : 0);
  }
  return hipGetLastError();
}

}  // namespace sor
