// 3-D red-black SOR on the 7-point stencil of the unit cube: the extension of
// Mittal 2014's method that its Sec. 5 names as future work.  Same update
// (Sec. 2.1 Eq. 1 in increment form), colouring (Sec. 3.1 with one more
// axis: red = z + y + x even, red first) and stopping rule (Algorithm 1) as
// the 2-D path; the Gauss-Seidel value is ((W + E) + (N + S)) + (D + U)
// (+ h*h*f) times fl(1/6), and the relaxation step u + w (g - u) is one fused
// multiply-add.
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
      const double nu = __builtin_fma(g.omega, gs - self, self);
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
// Streaming kernel, T iterations (S = 2T half-sweeps) per launch.  Tile =
// core [x0, x0+CX) x [y0, y0+CY) x [z0, z1) of interior cells; region = core
// plus a ring of S cells in x and y (RX = CX+2S by RY = CY+2S positions),
// held as RX*RY positions in row-major order, kK3 per thread.  One
// iteration per launch: thread t holds positions t + 256k (contiguous loads
// and LDS accesses) and masks each half-sweep to its colour.  Two per launch
// (twice the half-sweeps per loaded plane): RX is made odd (one more loaded
// column when CX+2S is even), so the colour parity of position p is that of
// p plus a tile constant; waves 0-1 hold the positions of one parity and
// waves 2-3 the other (p = 2(t + 128k) + parity offset), and each half-sweep
// runs on the two waves whose cells have its colour while the other two skip
// it.  The tile walks planes upwards: step s loads plane
// zr = z0-(S-1)+s into the pipeline and applies the S half-sweeps as stages,
// stage k (colour k mod 2, i.e. iteration k/2's red or black phase) to plane
// zr-k, in the order k = 0 .. S-1:
//   - stage k at plane q needs the other colour of q at stage k-1 (done at
//     step s-1), of q+1 (stage k-1 earlier in this step) and of q-1 (stage
//     k-1 two steps ago; stage k+1 reaches q-1 only after stage k in this
//     step), so every update sees exactly the two-phase iteration's values;
//   - the dependency cone shrinks by one cell per stage, so stage k updates
//     positions at distance >= k+1 from the region's edge and planes
//     z0-(S-1-k) .. z1-1+(S-1-k); after the last stage the core of plane
//     zr-(S-1) is final and stored to B.  Every value computed outside the
//     core equals the one the tile owning that cell computes (same inputs),
//     so all updates may enter the maxima.
// In-plane neighbours come from LDS: plane q lives in buffer (step at which
// stage 0 took it) mod (S+1); each stage reads one colour of its plane's
// buffer (written by the previous stage a step earlier) and writes the other.
// One barrier per step suffices: the buffer written before it (the new
// plane) was last read two steps earlier, and within a step the stages touch
// different buffers, each reading one colour and writing the other.  Planes
// zr-S .. zr+1 and kD3 more (loads in flight) live in registers.  Positions
// outside the grid load a clamped (in-bounds) address and are never updated
// nor read by an update.
// ---------------------------------------------------------------------------
constexpr int kT3 = 256;            // threads per workgroup
constexpr int kK3 = 8;              // positions per thread per plane
// Planes loaded ahead of the one first needed.  A step takes microseconds, so
// the next plane's load has a step to arrive; loading more ahead only holds
// registers (0 ran as fast as 2 on Laplace problems and 1-7 % faster with a
// source, whose planes then leave more room).
constexpr int kD3 = 0;

template <int T>
struct Stream3 {
  static constexpr int S = 2 * T;                  // stages (half-sweeps)
  static constexpr int B = S + 1;                  // LDS plane buffers
  static constexpr int W = S + kD3 + 2;            // register planes
  // Most positions in a region: three buffers of 2048 (48 KB, 3 workgroups
  // per CU) for one iteration; five of 2032 (79 KB, 2 per CU) for two.
  static constexpr int P = T == 1 ? kT3 * kK3 : 2032;
};

int stream3d_positions(int T) { return T == 1 ? Stream3<1>::P : Stream3<2>::P; }

struct Geo3 {
  const double *A;      // input of the launch
  double *B;            // output of the launch
  const double *F;      // h*h*f or nullptr
  int64_t px, plane;    // elements per row, per plane
  int n, RX, RY, CX, CY, Zs, ntx, nty;
  double omega;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

template <int T, bool POIS>
__global__ __launch_bounds__(kT3) void sor3d_stream_kernel(Geo3 g, Ctl *ctl, Sched sc) {
  constexpr int S = Stream3<T>::S, B = Stream3<T>::B, W = Stream3<T>::W;
  constexpr int PL = Stream3<T>::P;
  if (ctl_stopped(ctl)) return;
  // With T = 2 each plane buffer has one more slot, a sink for the writes of
  // positions outside the region (so the half-sweeps need no per-position
  // branch, see below).
  constexpr int PLS = T == 2 ? PL + 1 : PL;
  __shared__ double L[B * PLS];
  __shared__ double wmax[kT3 / 64][T];
  __shared__ int wbad[kT3 / 64];
  const int tid = threadIdx.x, n = g.n, RX = g.RX, RY = g.RY;
  int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int tx = tile % g.ntx;
  tile /= g.ntx;
  const int ty = tile % g.nty, tz = tile / g.nty;
  const int x0 = 1 + tx * g.CX, y0 = 1 + ty * g.CY, z0 = 1 + tz * g.Zs;
  const int z1 = min(z0 + g.Zs, n + 1);
  const int zbeg = z0 - (S - 1);                 // stage 0's first plane
  // Position of this thread's k-th cell; with CLS, the parity class of its
  // cells, (x + y) mod 2, is wave-uniform.
  constexpr bool CLS = T == 2;
  const int cls = tid >> 7, tc = tid & 127;
  const int poff = (cls + x0 + y0) & 1;          // p = 2j + poff has (x + y) % 2 == cls
  auto pos = [&](int k) { return CLS ? 2 * (tc + (kT3 / 2) * k) + poff : tid + kT3 * k; };
  const int nsteps = (z1 - z0) + 2 * S - 2;
  const int zlast = z1 + S - 1;                  // highest plane read
  const int P = RX * RY;
  const double SIXTH = 1.0 / 6.0;
  const double omega = g.omega;

  // Per-position set-up: in-plane offset (clamped) and masks.
  int off[kK3];
  unsigned valid = 0, core = 0, par = 0, act[S];
#pragma unroll
  for (int k = 0; k < S; ++k) act[k] = 0;
#pragma unroll
  for (int k = 0; k < kK3; ++k) {
    const int p = pos(k);
    off[k] = 0;
    if (p < P) {
      const int ry = p / RX, rx = p - ry * RX;
      const int x = x0 - S + rx, y = y0 - S + ry;
      const bool inter = x >= 1 && x <= n && y >= 1 && y <= n;
      const int dist = min(min(rx, RX - 1 - rx), min(ry, RY - 1 - ry));
      off[k] = (int)(clampi(y, 0, n + 1) * g.px + clampi(x, 0, n + 1));
      valid |= 1u << k;
#pragma unroll
      for (int st = 0; st < S; ++st)
        if (inter && dist >= st + 1) act[st] |= 1u << k;
      if (inter && dist >= S) core |= 1u << k;
      if ((x + y) & 1) par |= 1u << k;
    }
  }

  // T = 2, branch-free half-sweeps: every position of the thread computes an
  // update; one at distance 0 from the region edge or outside the region
  // reads its neighbours around an interior position instead (nb), positions
  // outside the region write to the sink slot PL (wr), and a position that is
  // not active in the stage keeps its value (a select, not a branch).
  int nb[CLS ? kK3 : 1], wr[CLS ? kK3 : 1];
  if constexpr (CLS) {
#pragma unroll
    for (int k = 0; k < kK3; ++k) {
      nb[k] = (act[0] >> k & 1u) ? pos(k) : RX + 1;
      wr[k] = (valid >> k & 1u) ? pos(k) : PL;
    }
  }

  double v[W][kK3];
  double f[POIS ? W : 1][kK3];
  // Every position loads (positions outside the region read the plane's
  // first cell, off = 0, and their values are never used) and stores go
  // through a buffer resource whose dropped offset discards them: no memory
  // instruction sits under a per-position branch, so the compiler can count
  // the loads in flight across steps instead of draining them at each join.
  auto load_u = [&](double (&dst)[kK3], int z) {
    const double *b = g.A + (int64_t)clampi(z, 0, n + 1) * g.plane;
#pragma unroll
    for (int k = 0; k < kK3; ++k) dst[k] = b[off[k]];
  };
  auto load_f = [&](double (&dst)[kK3], int z) {
    const double *b = g.F + (int64_t)clampi(z, 0, n + 1) * g.plane;
#pragma unroll
    for (int k = 0; k < kK3; ++k) dst[k] = b[off[k]];
  };
  const unsigned plane_bytes = (unsigned)(g.plane * (int64_t)sizeof(double));   // < 2^31

  // Plane zbeg + j lives in register slot (1 + j) mod W, i.e. plane zr + j
  // of step s in slot (s + 1 + j) mod W.  Before step 0: u planes
  // j = -1 .. kD3+1, f planes j = 0 .. kD3.
#pragma unroll
  for (int j = -1; j <= kD3 + 1; ++j) load_u(v[(1 + j) % W], zbeg + j);
  if constexpr (POIS) {
#pragma unroll
    for (int j = 0; j <= kD3; ++j) load_f(f[(1 + j) % W], zbeg + j);
  }

  double m[T];
#pragma unroll
  for (int t = 0; t < T; ++t) m[t] = 0.0;
  bool bad = false;
  for (int sb = 0; sb < nsteps; sb += W) {
    static_for<0, W>([&](auto I) __attribute__((always_inline)) {
      constexpr int i = decltype(I)::value;
      // Steps past the walk (the last chunk's tail) keep the plane traffic and
      // the barrier but update nothing and store nothing, so every step
      // issues the same memory instructions.
      const int s = sb + i;
      const bool live = s < nsteps;
      const int zr = zbeg + s;
      {
        double *Lz = L + (s % B) * PLS;
        const int c0 = (i + 1) % W;
#pragma unroll
        for (int k = 0; k < kK3; ++k)
          if (valid >> k & 1u) Lz[pos(k)] = v[c0][k];
      }
      __syncthreads();
      static_for<0, S>([&](auto K) __attribute__((always_inline)) {
        constexpr int st = decltype(K)::value;
        const int q = zr - st;                       // this stage's plane
        if (live && s >= 2 * st && q >= 1 && q <= n &&
            (!CLS || ((cls + q) & 1) == (st & 1))) {
          constexpr int cs = ((i + 1 - st) % W + W) % W;     // plane q
          constexpr int cd = ((i - st) % W + W) % W;         // q - 1
          constexpr int cu = ((i + 2 - st) % W + W) % W;     // q + 1
          double *Lq = L + ((s - st) % B) * PLS;
          if constexpr (CLS) {
            // The LDS reads of a group of positions (all eight: a group of
            // four ran 1-2 % slower) go first, so they are in flight together
            // (the cells a half-sweep writes are never the ones it reads, but
            // the compiler cannot know that).
            constexpr int G = 8;
            static_assert(kK3 % G == 0, "whole groups");
#pragma unroll
            for (int g0 = 0; g0 < kK3; g0 += G) {
              double ls[G];
#pragma unroll
              for (int j = 0; j < G; ++j) {
                const int p = nb[g0 + j];
                ls[j] = (Lq[p - 1] + Lq[p + 1]) + (Lq[p - RX] + Lq[p + RX]);
              }
#pragma unroll
              for (int j = 0; j < G; ++j) {
                const int k = g0 + j;
                const double self = v[cs][k];
                double sum = ls[j] + (v[cd][k] + v[cu][k]);
                if constexpr (POIS) sum = sum + f[cs][k];
                const double gs = SIXTH * sum;
                const double up = __builtin_fma(omega, gs - self, self);
                const double nu = (act[st] >> k & 1u) ? up : self;
                v[cs][k] = nu;
                if constexpr (st + 1 < S) Lq[wr[k]] = nu;
                m[st >> 1] = fmax(m[st >> 1], fabs(nu - self));
                bad = bad || !__builtin_isfinite(nu);
              }
            }
          } else {
#pragma unroll
          for (int k = 0; k < kK3; ++k) {
            if ((act[st] >> k & 1u) &&
                (CLS || (((par >> k) + (unsigned)q) & 1u) == (unsigned)(st & 1))) {
              const int p = pos(k);
              const double self = v[cs][k];
              double sum = ((Lq[p - 1] + Lq[p + 1]) + (Lq[p - RX] + Lq[p + RX])) +
                           (v[cd][k] + v[cu][k]);
              if constexpr (POIS) sum = sum + f[cs][k];
              const double gs = SIXTH * sum;
              const double nu = __builtin_fma(omega, gs - self, self);
              v[cs][k] = nu;
              if constexpr (st + 1 < S) Lq[p] = nu;
              m[st >> 1] = fmax(m[st >> 1], fabs(nu - self));
              bad = bad || !__builtin_isfinite(nu);
            }
          }
          }
        }
      });
      // Plane zr-(S-1) has had every stage: store its core (the stores of
      // the first 2S-2 steps, whose plane is not final yet, are dropped).
      {
        constexpr int cf = ((i + 2 - S) % W + W) % W;
        const unsigned drop = (live && s >= 2 * S - 2) ? 0u : kDrop;
        const auto out = make_rsrc(g.B + (int64_t)clampi(zr - (S - 1), 0, n + 1) * g.plane,
                                   plane_bytes);
#pragma unroll
        for (int k = 0; k < kK3; ++k) {
          using v2 = unsigned __attribute__((ext_vector_type(2)));
          const unsigned so = (core >> k & 1u) ? (unsigned)off[k] * 8u : kDrop;
          __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2, v[cf][k]), out,
                                                (int)(so | drop), 0, 0);
        }
      }
      // u plane zr-S is dead: its slot takes plane zr+kD3+2.  f planes
      // zr-(S-2) .. zr+kD3 stay live; f plane zr+kD3+1 takes a free slot.
      // Loads past the last plane read a clamped plane and are never used.
      load_u(v[(i + kD3 + 3) % W], min(zr + kD3 + 2, zlast));
      if constexpr (POIS) load_f(f[(i + kD3 + 2) % W], min(zr + kD3 + 1, zlast - 1));
    });
  }

  // Workgroup maxima, one report per workgroup from its first wave.
  const int wave = tid / 64, lane = tid % 64;
  const bool wb = __ballot(bad) != 0;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const double wm = wave_max(m[t]);
    if (lane == 0) wmax[wave][t] = wm;
  }
  if (lane == 0) wbad[wave] = wb;
  __syncthreads();
  if (wave != 0) return;
  double mx[T];
  bool bb = false;
#pragma unroll
  for (int t = 0; t < T; ++t) mx[t] = 0.0;
#pragma unroll
  for (int w = 0; w < kT3 / 64; ++w) {
#pragma unroll
    for (int t = 0; t < T; ++t) mx[t] = fmax(mx[t], wmax[w][t]);
    bb = bb || wbad[w];
  }
  report_pass<T>(ctl, sc, mx, T, bb && lane == 0, (int)(blockIdx.x % kSlots), gridDim.x);
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
// workgroups) x (planes a tile walks, Zs + 2S, plus about 2 planes of
// start-up), so that the tiles fill whole rounds without long walks.
Tiling3 tiling3(int n, int T, int cx, int cy, int zs, int slots) {
  Tiling3 t{};
  const int ring = 2 * T, PL = stream3d_positions(T);
  auto shape = [&](int ntx) {
    Tiling3 r{};
    r.ntx = ntx;
    r.CX = (n + ntx - 1) / ntx;
    r.RX = r.CX + 2 * ring + ((T == 2 && !(r.CX & 1)) ? 1 : 0);   // odd for T = 2
    int cyw = cy > 0 ? cy : std::min(PL / r.RX, n + 2 * ring) - 2 * ring;
    cyw = std::max(1, std::min(cyw, n));
    r.nty = (n + cyw - 1) / cyw;
    r.CY = (n + r.nty - 1) / r.nty;
    r.RY = r.CY + 2 * ring;
    return r;
  };
  if (cx > 0) {
    t = shape((n + cx - 1) / cx);
  } else {
    double best = 1e30;
    for (int ntx = 1; ntx <= n; ++ntx) {
      const Tiling3 r = shape(ntx);
      if (r.RX * (1 + 2 * ring) > PL) continue;
      if (r.RX < 32 && ntx > 1) break;                 // narrower strips only shrink
      if (r.RX * r.RY > PL) continue;
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
      if (Zs < std::min(n, 4)) continue;                   // walks of 1-3 planes load many
      const long long tiles = (long long)nxy * nzt;
      const long long rounds = (tiles + std::max(slots, 1) - 1) / std::max(slots, 1);
      const double cost = (double)rounds * (Zs + 2 * ring + 2);
      if (cost < best - 1e-9) {
        best = cost;
        zsw = Zs;
      }
    }
  }
  zsw = std::max(1, std::min(zsw, n));
  t.nzt = (n + zsw - 1) / zsw;
  t.Zs = (n + t.nzt - 1) / t.nzt;
  t.T = T;
  t.ok = t.RX * t.RY <= PL;
  return t;
}

int stream3d_blocks_per_cu(int T, bool pois) {
  int b = 0;
  hipError_t e;
  if (T == 1)
    e = pois ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, sor3d_stream_kernel<1, true>, kT3, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, sor3d_stream_kernel<1, false>, kT3, 0);
  else
    e = pois ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, sor3d_stream_kernel<2, true>, kT3, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, sor3d_stream_kernel<2, false>, kT3, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return b;
}

hipError_t launch_sor3d_stream(const double *A, double *B, const double *F, int n,
                               double omega, const Tiling3 &t, int T, Ctl *ctl,
                               const Sched &sc, hipStream_t s) {
  if (T != 1 && T != 2) return hipErrorInvalidValue;
  const int64_t px = grid3_pitch(n);
  const Geo3 g{A, B, F, px, px * (int64_t)(n + 2), n, t.RX, t.RY, t.CX, t.CY, t.Zs,
               t.ntx, t.nty, omega};
  const unsigned blocks = (unsigned)(t.ntx * t.nty * t.nzt);
  const dim3 grid(blocks), block(kT3);
  if (T == 1) {
    if (F) hipLaunchKernelGGL((sor3d_stream_kernel<1, true>), grid, block, 0, s, g, ctl, sc);
    else hipLaunchKernelGGL((sor3d_stream_kernel<1, false>), grid, block, 0, s, g, ctl, sc);
  } else {
    if (F) hipLaunchKernelGGL((sor3d_stream_kernel<2, true>), grid, block, 0, s, g, ctl, sc);
    else hipLaunchKernelGGL((sor3d_stream_kernel<2, false>), grid, block, 0, s, g, ctl, sc);
  }
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
