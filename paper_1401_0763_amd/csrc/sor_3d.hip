// 3-D red-black SOR on the 7-point stencil of the unit cube: the extension of
// Mittal 2014's method that its Sec. 5 names as future work.  Same update
// (Sec. 2.1 Eq. 1 in increment form), colouring (Sec. 3.1 with one more
// axis: red = z + y + x even, red first) and stopping rule (Algorithm 1) as
// the 2-D path; the Gauss-Seidel value is ((W + E) + (N + S)) + (D + U)
// (+ h*h*f) times fl(1/6).
//
// One launch per colour, one thread per cell of that colour, in place; each
// thread walks kZ3 planes.  A block reduces its cells' largest change in LDS
// and merges it into the pass slots; the black launch's last block evaluates
// the check (report_pass), so a solve runs with the same device-side verdict
// and early exit as the 2-D passes.
#include "sor_kernels.h"
#include "sor_3d.h"

namespace sor {

constexpr int kX3 = 64;      // threads along x (cells of one colour)
constexpr int kY3 = 4;       // rows per block
constexpr int kZ3 = 4;       // planes per thread

// Device grid of side n: V[z][y][x] at base[(z * (n+2) + y) * px + x].
struct Grid3 {
  double *U;
  const double *F;     // h*h*f, same layout, or nullptr
  int64_t px;          // elements per row
  int n;
  double omega;
};

template <bool POIS>
__global__ __launch_bounds__(kX3 * kY3) void sor3d_colour_kernel(Grid3 g, Ctl *ctl,
                                                                 Sched sc, int colour,
                                                                 int finish) {
  if (ctl && ctl_stopped(ctl)) return;
  const int n = g.n;
  const int64_t px = g.px, plane = px * (int64_t)(n + 2);
  const int y = blockIdx.y * kY3 + (int)(threadIdx.x / kX3) + 1;
  const int t = blockIdx.x * kX3 + (int)(threadIdx.x % kX3);
  const double SIXTH = 1.0 / 6.0;
  double dmax = 0.0;
  bool bad = false;
  if (y <= n) {
#pragma unroll
    for (int dz = 0; dz < kZ3; ++dz) {
      const int z = blockIdx.z * kZ3 + dz + 1;
      const int x = 1 + ((z + y + 1 + colour) & 1) + 2 * t;   // first x of the colour
      if (z > n || x > n) continue;
      const int64_t c = (int64_t)z * plane + (int64_t)y * px + x;
      const double self = g.U[c];
      double s = ((g.U[c - 1] + g.U[c + 1]) + (g.U[c - px] + g.U[c + px])) +
                 (g.U[c - plane] + g.U[c + plane]);
      if (POIS) s = s + g.F[c];
      const double gs = SIXTH * s;
      const double nu = self + g.omega * (gs - self);
      dmax = fmax(dmax, fabs(nu - self));
      bad = bad || !__builtin_isfinite(nu);
      g.U[c] = nu;
    }
  }
  if (!ctl) return;
  // Block maximum (LDS), then one report per block from its first wave.
  __shared__ double wmax[kX3 * kY3 / 64];
  __shared__ int wbad[kX3 * kY3 / 64];
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
  for (int k = 0; k < kX3 * kY3 / 64; ++k) {
    mx[0] = fmax(mx[0], wmax[k]);
    bb = bb || wbad[k];
  }
  const unsigned block = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const int slot = (int)(block % kSlots);
  if (!finish) {
    if (lane == 0) {
      __hip_atomic_fetch_max(&ctl->slots[slot][0],
                             (unsigned long long)__double_as_longlong(mx[0]),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (bb)
        __hip_atomic_fetch_or(&ctl->nonfinite, 1u, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  report_pass<1>(ctl, sc, mx, 1, bb && lane == 0, slot,
                 gridDim.x * gridDim.y * gridDim.z);
}

// Pack u (n^3), the six faces (6 n^2) and h*h*f into the padded grid; every
// element of the allocation is written (edges, corners and padding are 0).
// Block (x-chunk, y, z) over the full (n+2)^2 x px allocation.
__global__ void pack3d_kernel(const double *u, const double *bdy, const double *f,
                              double *U, double *F, int64_t px, int n, double h2,
                              unsigned *bad) {
  const int64_t xa = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (xa >= px) return;
  const int x = (int)xa, y = blockIdx.y, z = blockIdx.z;
  const size_t nn = (size_t)n * n;
  const bool ix = x >= 1 && x <= n, iy = y >= 1 && y <= n, iz = z >= 1 && z <= n;
  double v = 0.0, fv = 0.0;
  if (ix && iy && iz) {
    const size_t k = ((size_t)(z - 1) * n + (y - 1)) * n + (x - 1);
    v = u[k];
    if (f) fv = h2 * f[k];
  } else if (iy && iz && (x == 0 || x == n + 1)) {
    v = bdy[(x == 0 ? 0 : 1) * nn + (size_t)(z - 1) * n + (y - 1)];
  } else if (ix && iz && (y == 0 || y == n + 1)) {
    v = bdy[(y == 0 ? 2 : 3) * nn + (size_t)(z - 1) * n + (x - 1)];
  } else if (ix && iy && (z == 0 || z == n + 1)) {
    v = bdy[(z == 0 ? 4 : 5) * nn + (size_t)(y - 1) * n + (x - 1)];
  }
  const int64_t c = ((int64_t)z * (n + 2) + y) * px + x;
  U[c] = v;
  if (F) F[c] = fv;
  if (bad && (!__builtin_isfinite(v) || !__builtin_isfinite(fv))) *bad = 1u;
}

__global__ void unpack3d_kernel(const double *U, double *u, int64_t px, int n) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const int y = blockIdx.y + 1, z = blockIdx.z + 1;
  if (x > n) return;
  u[((size_t)(z - 1) * n + (y - 1)) * n + (x - 1)] = U[((int64_t)z * (n + 2) + y) * px + x];
}

int64_t grid3_pitch(int n) { return ((int64_t)n + 2 + 31) / 32 * 32; }

hipError_t launch_pack3d(const double *u, const double *bdy, const double *f, double *U,
                         double *F, int n, unsigned *bad, hipStream_t s) {
  const int64_t px = grid3_pitch(n);
  const double h = 1.0 / (double)(n + 1);
  const dim3 grid((unsigned)((px + 255) / 256), (unsigned)(n + 2), (unsigned)(n + 2));
  hipLaunchKernelGGL(pack3d_kernel, grid, dim3(256), 0, s, u, bdy, f, U, F, px, n, h * h, bad);
  return hipGetLastError();
}

hipError_t launch_unpack3d(const double *U, double *u, int n, hipStream_t s) {
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)n, (unsigned)n);
  hipLaunchKernelGGL(unpack3d_kernel, grid, dim3(256), 0, s, U, u, grid3_pitch(n), n);
  return hipGetLastError();
}

// One iteration: the red launch, then the black launch that closes the pass.
hipError_t launch_sor3d_iteration(double *U, const double *F, int n, double omega,
                                  Ctl *ctl, const Sched &sc, hipStream_t s) {
  const Grid3 g{U, F, grid3_pitch(n), n, omega};
  const int half = (n + 1) / 2;                      // most cells of one colour per row
  const dim3 grid((unsigned)((half + kX3 - 1) / kX3), (unsigned)((n + kY3 - 1) / kY3),
                  (unsigned)((n + kZ3 - 1) / kZ3));
  for (int colour = 0; colour < 2; ++colour) {
    if (F)
      hipLaunchKernelGGL(sor3d_colour_kernel<true>, grid, dim3(kX3 * kY3), 0, s, g, ctl, sc,
                         colour, colour);
    else
      hipLaunchKernelGGL(sor3d_colour_kernel<false>, grid, dim3(kX3 * kY3), 0, s, g, ctl, sc,
                         colour, colour);
  }
  return hipGetLastError();
}

}  // namespace sor
