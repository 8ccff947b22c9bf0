// 3-D red-black SOR on the 7-point stencil of the unit cube: the extension of
// Mittal 2014's method that its Sec. 5 names as future work.  Same update
// (Sec. 2.1 Eq. 1 in increment form), colouring (Sec. 3.1 with one more
// axis: red = z + y + x even, red first) and stopping rule (Algorithm 1) as
// the 2-D path; the Gauss-Seidel value is ((W + E) + (N + S)) + (D + U)
// (+ h*h*f) times fl(1/6).
//
// Two kernels.  The streaming kernel (default) applies one whole iteration
// per launch from grid A into grid B: a workgroup owns a tile (an x-y patch
// and a range of z-planes) and walks it plane by plane, red half-sweep on
// plane z and black half-sweep on plane z-1 in the same step, with the
// planes in flight in registers and the current two in LDS.  The colour
// kernel (one launch per half-sweep, in place, one thread per cell) is the
// readable reference.  Both close each iteration with the device-side verdict
// (report_pass), so a solve runs with the same early exit as the 2-D passes.
#include <algorithm>

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

// ---------------------------------------------------------------------------
// Streaming kernel.  Tile = core [x0, x0+CX) x [y0, y0+CY) x [z0, z1) of
// interior cells; region = core plus a ring of 2 cells in x and y (RX = CX+4,
// RY = CY+4 positions), held as RX*RY positions, kK3 per thread (position
// p = thread + kT3*k, row-major in the region).  Step s handles plane
// zr = z0-1+s:
//   1. write plane zr (values of the previous iteration) to LDS, barrier;
//   2. red half-sweep of plane zr on the region minus its outer ring (the
//      black cells it reads, in the plane from LDS and above and below from
//      registers, are all still old);
//   3. black half-sweep of plane zr-1 on the core (its red neighbours: plane
//      zr-1 in LDS from step s-1, planes zr-2 and zr in registers, all new),
//      then store the core of plane zr-1 (both colours) to B.
// Steps run from zr = z0-1 to zr = z1, so red values of planes z0-1 and z1
// and of the ring are computed redundantly (also by the tiles that own them,
// from the same old values, so identically) and never stored.  Three LDS
// plane buffers (plane z in buffer z mod 3) need one barrier per step: the
// red sweep writes red cells of buffer zr while other threads read its black
// cells; the black sweep reads buffer zr-1 written before this step's
// barrier; buffer zr was last read by the black sweep of step s-2.
// Positions outside the grid load a clamped (in-bounds) address and are
// never updated nor read by an update.
// ---------------------------------------------------------------------------
constexpr int kT3 = 256;            // threads per workgroup
constexpr int kK3 = 8;              // positions per thread per plane
constexpr int kP3 = kT3 * kK3;      // most positions in a region
constexpr int kD3 = 2;              // planes loaded ahead of the one first needed
constexpr int kW3 = kD3 + 4;        // planes in registers: zr-2 .. zr+1, plus kD3 in flight

struct Geo3 {
  const double *A;      // iteration input
  double *B;            // iteration output
  const double *F;      // h*h*f or nullptr
  int64_t px, plane;    // elements per row, per plane
  int n, RX, RY, CX, CY, Zs, ntx, nty;
  double omega;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

template <bool POIS>
__global__ __launch_bounds__(kT3) void sor3d_stream_kernel(Geo3 g, Ctl *ctl, Sched sc) {
  if (ctl_stopped(ctl)) return;
  __shared__ double L[3][kP3];
  __shared__ double wmax[kT3 / 64];
  __shared__ int wbad[kT3 / 64];
  const int tid = threadIdx.x, n = g.n, RX = g.RX;
  int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int tx = tile % g.ntx;
  tile /= g.ntx;
  const int ty = tile % g.nty, tz = tile / g.nty;
  const int x0 = 1 + tx * g.CX, y0 = 1 + ty * g.CY, z0 = 1 + tz * g.Zs;
  const int z1 = min(z0 + g.Zs, n + 1);
  const int nsteps = z1 - z0 + 2;
  const int P = RX * g.RY;
  const double SIXTH = 1.0 / 6.0;
  const double omega = g.omega;

  // Per-position set-up: in-plane offset (clamped) and masks.
  int off[kK3];
  unsigned valid = 0, ring = 0, core = 0, par = 0;
#pragma unroll
  for (int k = 0; k < kK3; ++k) {
    const int p = tid + kT3 * k;
    off[k] = 0;
    if (p < P) {
      const int ry = p / RX, rx = p - ry * RX;
      const int x = x0 - 2 + rx, y = y0 - 2 + ry;
      const bool inter = x >= 1 && x <= n && y >= 1 && y <= n;
      off[k] = (int)(clampi(y, 0, n + 1) * g.px + clampi(x, 0, n + 1));
      valid |= 1u << k;
      if (inter && rx >= 1 && rx <= RX - 2 && ry >= 1 && ry <= g.RY - 2) ring |= 1u << k;
      if (inter && rx >= 2 && rx <= RX - 3 && ry >= 2 && ry <= g.RY - 3) core |= 1u << k;
      if ((x + y) & 1) par |= 1u << k;
    }
  }

  double v[kW3][kK3];
  double f[kW3][kK3];
  auto load_u = [&](double (&dst)[kK3], int z) {
    const double *b = g.A + (int64_t)clampi(z, 0, n + 1) * g.plane;
#pragma unroll
    for (int k = 0; k < kK3; ++k) dst[k] = (valid >> k & 1u) ? b[off[k]] : 0.0;
  };
  auto load_f = [&](double (&dst)[kK3], int z) {
    const double *b = g.F + (int64_t)clampi(z, 0, n + 1) * g.plane;
#pragma unroll
    for (int k = 0; k < kK3; ++k) dst[k] = (valid >> k & 1u) ? b[off[k]] : 0.0;
  };

  // Plane zr + j of step s lives in register slot (s + 1 + j) mod kW3.
  // Before step 0 (zr = z0-1): planes z0-2 .. z0+kD3 of u, z0-1 .. z0+kD3-1 of f.
#pragma unroll
  for (int j = -1; j <= kD3 + 1; ++j) load_u(v[(1 + j) % kW3], z0 - 1 + j);
  if (POIS) {
#pragma unroll
    for (int j = 0; j <= kD3; ++j) load_f(f[(1 + j) % kW3], z0 - 1 + j);
  }

  double dmax = 0.0;
  bool bad = false;
  for (int sb = 0; sb < nsteps; sb += kW3) {
#pragma unroll
    for (int i = 0; i < kW3; ++i) {
      const int s = sb + i;
      if (s >= nsteps) break;
      const int zr = z0 - 1 + s;
      const int c0 = (i + 1) % kW3;               // plane zr
      const int cm1 = (i + kW3) % kW3;            // zr - 1
      const int cm2 = (i + kW3 - 1) % kW3;        // zr - 2
      const int cp1 = (i + 2) % kW3;              // zr + 1
      double *Lr = L[zr % 3];
      const double *Lb = L[(zr + 2) % 3];          // plane zr - 1
#pragma unroll
      for (int k = 0; k < kK3; ++k)
        if (valid >> k & 1u) Lr[tid + kT3 * k] = v[c0][k];
      __syncthreads();
      if (zr >= 1 && zr <= n) {
#pragma unroll
        for (int k = 0; k < kK3; ++k) {
          if ((ring >> k & 1u) && (((par >> k) + (unsigned)zr) & 1u) == 0u) {
            const int p = tid + kT3 * k;
            const double self = v[c0][k];
            double sum = ((Lr[p - 1] + Lr[p + 1]) + (Lr[p - RX] + Lr[p + RX])) +
                         (v[cm1][k] + v[cp1][k]);
            if (POIS) sum = sum + f[c0][k];
            const double gs = SIXTH * sum;
            const double nu = self + omega * (gs - self);
            v[c0][k] = nu;
            Lr[p] = nu;
            if (core >> k & 1u) {
              dmax = fmax(dmax, fabs(nu - self));
              bad = bad || !__builtin_isfinite(nu);
            }
          }
        }
      }
      const int zb = zr - 1;
      if (zb >= z0) {
#pragma unroll
        for (int k = 0; k < kK3; ++k) {
          if ((core >> k & 1u) && (((par >> k) + (unsigned)zb) & 1u) == 1u) {
            const int p = tid + kT3 * k;
            const double self = v[cm1][k];
            double sum = ((Lb[p - 1] + Lb[p + 1]) + (Lb[p - RX] + Lb[p + RX])) +
                         (v[cm2][k] + v[c0][k]);
            if (POIS) sum = sum + f[cm1][k];
            const double gs = SIXTH * sum;
            const double nu = self + omega * (gs - self);
            v[cm1][k] = nu;
            dmax = fmax(dmax, fabs(nu - self));
            bad = bad || !__builtin_isfinite(nu);
          }
        }
        double *out = g.B + (int64_t)zb * g.plane;
#pragma unroll
        for (int k = 0; k < kK3; ++k)
          if (core >> k & 1u) out[off[k]] = v[cm1][k];
      }
      // Plane zr-2 of u is dead: its slot takes plane zr+kD3+2.  f's planes
      // zr-1 .. zr+kD3 stay live; f plane zr+kD3+1 takes the free slot.
      if (zr + kD3 + 2 <= z1 + 1) load_u(v[cm2], zr + kD3 + 2);
      if (POIS && zr + kD3 + 1 <= z1) load_f(f[(i + kD3 + 2) % kW3], zr + kD3 + 1);
    }
  }

  // Workgroup maximum, one report per workgroup from its first wave.
  const int wave = tid / 64, lane = tid % 64;
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
  for (int w = 0; w < kT3 / 64; ++w) {
    mx[0] = fmax(mx[0], wmax[w]);
    bb = bb || wbad[w];
  }
  report_pass<1>(ctl, sc, mx, 1, bb && lane == 0, (int)(blockIdx.x % kSlots), gridDim.x);
}

// Pack u (n^3), the six faces (6 n^2) and h*h*f into the padded grid; every
// element of the allocation is written (edges, corners and padding are 0).
// Block (x-chunk, y, z) over the full (n+2)^2 x px allocation.
__global__ void pack3d_kernel(const double *u, const double *bdy, const double *f,
                              double *U, double *U2, double *F, int64_t px, int n,
                              double h2, unsigned *bad) {
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
  if (U2) U2[c] = v;
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
                         double *U2, double *F, int n, unsigned *bad, hipStream_t s) {
  const int64_t px = grid3_pitch(n);
  const double h = 1.0 / (double)(n + 1);
  const dim3 grid((unsigned)((px + 255) / 256), (unsigned)(n + 2), (unsigned)(n + 2));
  hipLaunchKernelGGL(pack3d_kernel, grid, dim3(256), 0, s, u, bdy, f, U, U2, F, px, n, h * h,
                     bad);
  return hipGetLastError();
}

hipError_t launch_unpack3d(const double *U, double *u, int n, hipStream_t s) {
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)n, (unsigned)n);
  hipLaunchKernelGGL(unpack3d_kernel, grid, dim3(256), 0, s, U, u, grid3_pitch(n), n);
  return hipGetLastError();
}

// Automatic choice: among equal x-strips (core cx, region at least 32 wide
// for coalesced rows, or the whole side) and the tallest equal y-bands that
// fit, the x-y shape with the fewest region positions per core cell; then the
// z-range length (at least 4 planes) minimising (rounds of resident
// workgroups) x (planes a tile walks, Zs + 4, plus about 2 planes of
// start-up), so that the tiles fill whole rounds without long walks.
Tiling3 tiling3(int n, int cx, int cy, int zs, int slots) {
  Tiling3 t{};
  auto shape = [&](int ntx) {
    Tiling3 r{};
    r.ntx = ntx;
    r.CX = (n + ntx - 1) / ntx;
    r.RX = r.CX + 4;
    int cyw = cy > 0 ? cy : std::min(kP3 / r.RX, n + 4) - 4;
    cyw = std::max(1, std::min(cyw, n));
    r.nty = (n + cyw - 1) / cyw;
    r.CY = (n + r.nty - 1) / r.nty;
    r.RY = r.CY + 4;
    return r;
  };
  if (cx > 0) {
    t = shape((n + cx - 1) / cx);
  } else {
    double best = 1e30;
    for (int ntx = 1; ntx <= n; ++ntx) {
      const Tiling3 r = shape(ntx);
      if (r.RX * 5 > kP3) continue;
      if (r.RX < 32 && ntx > 1) break;                 // narrower strips only shrink
      if (r.RX * r.RY > kP3) continue;
      const double cost = (double)r.RX * r.RY / ((double)r.CX * r.CY);
      if (cost < best - 1e-9) {
        best = cost;
        t = r;
      }
      if (r.CX == 1) break;
    }
    if (best == 1e30) t = shape((n + 123) / 124);
  }
  const int nxy = t.ntx * t.nty;
  int zsw = zs;
  if (zsw <= 0) {
    double best = 1e30;
    for (int nzt = 1; nzt <= n; ++nzt) {
      const int Zs = (n + nzt - 1) / nzt;
      if (nzt > 1 && (n + Zs - 1) / Zs != nzt) continue;   // same Zs as a smaller count
      if (Zs < std::min(n, 4)) continue;                   // walks of 1-3 planes load 5-7
      const long long tiles = (long long)nxy * nzt;
      const long long rounds = (tiles + std::max(slots, 1) - 1) / std::max(slots, 1);
      const double cost = (double)rounds * (Zs + 6);
      if (cost < best - 1e-9) {
        best = cost;
        zsw = Zs;
      }
    }
  }
  zsw = std::max(1, std::min(zsw, n));
  t.nzt = (n + zsw - 1) / zsw;
  t.Zs = (n + t.nzt - 1) / t.nzt;
  t.ok = t.RX * t.RY <= kP3;
  return t;
}

int stream3d_blocks_per_cu(bool pois) {
  int b = 0;
  hipError_t e = pois ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &b, sor3d_stream_kernel<true>, kT3, 0)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &b, sor3d_stream_kernel<false>, kT3, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return b;
}

hipError_t launch_sor3d_stream(const double *A, double *B, const double *F, int n,
                               double omega, const Tiling3 &t, Ctl *ctl, const Sched &sc,
                               hipStream_t s) {
  const int64_t px = grid3_pitch(n);
  const Geo3 g{A, B, F, px, px * (int64_t)(n + 2), n, t.RX, t.RY, t.CX, t.CY, t.Zs,
               t.ntx, t.nty, omega};
  const unsigned blocks = (unsigned)(t.ntx * t.nty * t.nzt);
  if (F)
    hipLaunchKernelGGL(sor3d_stream_kernel<true>, dim3(blocks), dim3(kT3), 0, s, g, ctl, sc);
  else
    hipLaunchKernelGGL(sor3d_stream_kernel<false>, dim3(blocks), dim3(kT3), 0, s, g, ctl, sc);
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
