// Device code of libsor: red-black SOR sweeps for gfx950 (MI355X).
//
// Method (Mittal 2014): Sec. 2.1 Eq. 1 (SOR update), Sec. 3.1 with Fig. 1-2
// (red-black colouring, red phase then black phase, stride-2 visiting without
// a branch per cell), Algorithm 1 (iteration loop, check every K iterations,
// strict stopping rule on the largest change of one iteration).
//
// Every update is evaluated exactly as
//   s = (N + S) + (W + E); [s = s + F]; u' = fma(w, fma(0.25, s, -u), u)
// with -ffp-contract=off, so an FP64 sweep reproduces the CPU definition bit
// for bit whatever the tiling.
#include "sor_kernels.h"

#include <float.h>

namespace sor {

// ---------------------------------------------------------------------------
// Simple kernel: one launch per colour, one thread per cell of that colour,
// in place.  Row i's cells of colour c are j = j0 + 2t with j0 the first
// column >= 1 where (i + j) % 2 == c (Fig. 2's stride-2 loop, no branch per
// cell).  The black launch also closes the iteration (finisher).
// ---------------------------------------------------------------------------
template <int P, bool POIS>
__global__ __launch_bounds__(256) void simple_colour_kernel(GridView g, Ctl *ctl,
                                                            Sched sc, int colour,
                                                            int finish) {
  if (ctl && ctl_stopped(ctl)) return;
  using st = typename PT<P>::st;
  using ct = typename PT<P>::ct;
  const int i = blockIdx.y + 1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = 1 + ((i + 1 + colour) & 1) + 2 * t;
  ct d = (ct)0;
  bool bad = false;
  if (j <= g.n) {
    st *U = (st *)g.in;
    const st *F = (const st *)g.F;
    const int64_t p = g.pitch;
    const int64_t c = (int64_t)i * p + j;
    const ct self = (ct)U[c];
    ct s = ((ct)U[c - p] + (ct)U[c + p]) + ((ct)U[c - 1] + (ct)U[c + 1]);
    if (POIS) s = s + (ct)F[c];
    const ct dg = vfma((ct)0.25, s, -self);
    ct nu;
    if constexpr (P == kF16) nu = (ct)(st)(self + (ct)g.omega * dg);   // see blocked_tile
    else nu = vfma((ct)g.omega, dg, self);
    d = vabs(nu - self);
    bad = !__builtin_isfinite(nu);
    U[c] = (st)nu;
  }
  if (!ctl) return;
  double mx[1] = {wave_max((double)d)};
  const int slot = (blockIdx.x + blockIdx.y * gridDim.x) % kSlots;
  if (!finish) {
    const bool anybad = __ballot(bad) != 0;
    if ((threadIdx.x & 63) == 0) {
      __hip_atomic_fetch_max(&ctl->slots[slot][0],
                             (unsigned long long)__double_as_longlong(mx[0]),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (anybad)
        __hip_atomic_fetch_or(&ctl->nonfinite, 1u, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  report_pass<1>(ctl, sc, mx, 1, bad, slot,
                 gridDim.x * gridDim.y * (blockDim.x / 64));
}

// ---------------------------------------------------------------------------
// Grid set-up kernels.
// ---------------------------------------------------------------------------
__global__ void ctl_reset_kernel(Ctl *ctl) {
  const int t = threadIdx.x;
  unsigned long long *s = &ctl->slots[0][0];
  for (int k = t; k < kSlots * kTMax; k += blockDim.x) s[k] = 0ull;
  for (int k = t; k < kHistCap; k += blockDim.x) ctl->hist[k] = 0.0;
  if (t == 0) {
    ctl->counter = 0;
    ctl->nonfinite = ctl->input_nonfinite;   // inputs packed for this solve
    ctl->input_nonfinite = 0;
    ctl->stop = 0;
    ctl->stop_tentative = 0;
    ctl->it_base = 0;
    ctl->stop_iter = 0;
    ctl->stop_max = 0.0;
    ctl->last_iter = 0;
    ctl->last_max = __longlong_as_double(0x7ff8000000000000LL);
    ctl->passes_done = 0;
  }
}

// The set-up kernels below cover a grid's whole allocation: rows -kMY ..
// n+1+kMY and every column of the pitch, relative to the origin.  Cells off
// the (n+2) x (n+2) grid are set to 0, so the tiles' halo loads (which reach
// into this padding) only ever see finite values, whatever the memory held
// before.  Launch: one block row per allocated row, x over the pitch.

// Embed u (n*n) and the boundary edges (north, south, west, east) into the
// working grid A; the boundary ring and the padding also go to B (the
// ping-pong partner).
template <typename st>
__global__ void pack_kernel(const st *u, const st *bdy, st *A, st *B,
                            int64_t pitch, int n, unsigned *bad) {
  const int64_t ca = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ca >= pitch) return;
  const int c = (int)ca - kMX;
  const int r = (int)blockIdx.y - kMY;
  const bool in_r = r >= 1 && r <= n, in_c = c >= 1 && c <= n;
  st val = (st)0;
  if (in_r && in_c) val = u[(int64_t)(r - 1) * n + (c - 1)];
  else if (r == 0 && in_c) val = bdy[c - 1];
  else if (r == n + 1 && in_c) val = bdy[n + c - 1];
  else if (c == 0 && in_r) val = bdy[2 * n + r - 1];
  else if (c == n + 1 && in_r) val = bdy[3 * n + r - 1];
  const int64_t o = (int64_t)r * pitch + c;
  A[o] = val;
  if (B && !(in_r && in_c)) B[o] = val;
  if (bad && !__builtin_isfinite(val)) *bad = 1u;
}

// F = h*h*f on the interior, 0 elsewhere; the product is formed in double
// and rounded once to the storage type.
template <typename st>
__global__ void pack_rhs_kernel(const st *f, st *F, int64_t pitch, int n,
                                double h2, unsigned *bad) {
  const int64_t ca = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ca >= pitch) return;
  const int c = (int)ca - kMX;
  const int r = (int)blockIdx.y - kMY;
  st val = (st)0;
  if (r >= 1 && r <= n && c >= 1 && c <= n)
    val = (st)(h2 * (double)f[(int64_t)(r - 1) * n + (c - 1)]);
  F[(int64_t)r * pitch + c] = val;
  if (bad && !__builtin_isfinite(val)) *bad = 1u;
}

template <typename st>
__global__ void unpack_kernel(const st *A, st *u, int64_t pitch, int n) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y + 1;
  if (c >= n) return;
  u[(int64_t)(r - 1) * n + c] = A[(int64_t)r * pitch + c + 1];
}

template <typename st>
__global__ void fill_zero_kernel(st *A, int64_t pitch, int n) {
  const int64_t ca = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ca >= pitch) return;
  const int r = (int)blockIdx.y - kMY;
  A[(int64_t)r * pitch + (ca - kMX)] = (st)0;
}

// ---------------------------------------------------------------------------
// FP64 residual r = (F + ((N + S) + (W + E))) - 4u with the squared norms of r
// and of b = F + (boundary neighbours), and max |r|; per-block partials in a
// fixed tree order, then a one-block reduction in a fixed order.
// ---------------------------------------------------------------------------
constexpr int kResBlock = 256;

__device__ __forceinline__ void block_reduce3(double &a, double &b, double &c) {
  __shared__ double sh[3][kResBlock / 64];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
    c = fmax(c, __shfl_xor(c, o, 64));
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) { sh[0][w] = a; sh[1][w] = b; sh[2][w] = c; }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = sh[0][0]; b = sh[1][0]; c = sh[2][0];
    for (int k = 1; k < kResBlock / 64; ++k) {
      a += sh[0][k]; b += sh[1][k]; c = fmax(c, sh[2][k]);
    }
  }
}

__global__ __launch_bounds__(kResBlock) void residual_kernel(
    const double *U, const double *F, int64_t pitch, int n, double *r,
    double *partials, void *lo, int prec_lo, int64_t lo_pitch, int scale_exp) {
  const int i = blockIdx.y + 1;
  const int j = blockIdx.x * kResBlock + threadIdx.x + 1;
  double r2 = 0.0, b2 = 0.0, mr = 0.0;
  if (j <= n) {
    const int64_t c = (int64_t)i * pitch + j;
    const double s = (U[c - pitch] + U[c + pitch]) + (U[c - 1] + U[c + 1]);
    const double t = F ? F[c] + s : s;
    const double rr = t - 4.0 * U[c];
    const double nb = (i == 1) ? U[c - pitch] : 0.0;
    const double sb = (i == n) ? U[c + pitch] : 0.0;
    const double wb = (j == 1) ? U[c - 1] : 0.0;
    const double eb = (j == n) ? U[c + 1] : 0.0;
    const double bs = (nb + sb) + (wb + eb);
    const double bb = F ? F[c] + bs : bs;
    if (r) r[(int64_t)(i - 1) * n + (j - 1)] = rr;
    if (lo) {
      const float v = (float)ldexp(rr, scale_exp);
      const int64_t lc = (int64_t)i * lo_pitch + j;
      if (prec_lo == kF32) ((float *)lo)[lc] = v;
      else ((_Float16 *)lo)[lc] = (_Float16)v;
    }
    r2 = rr * rr;
    b2 = bb * bb;
    mr = fabs(rr);
  }
  block_reduce3(r2, b2, mr);
  if (threadIdx.x == 0) {
    const int64_t blk = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    partials[3 * blk + 0] = r2;
    partials[3 * blk + 1] = b2;
    partials[3 * blk + 2] = mr;
  }
}

__global__ __launch_bounds__(kResBlock) void residual_finalize_kernel(
    const double *partials, int64_t nblk, double *stats) {
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t k = threadIdx.x; k < nblk; k += kResBlock) {
    a += partials[3 * k + 0];
    b += partials[3 * k + 1];
    c = fmax(c, partials[3 * k + 2]);
  }
  block_reduce3(a, b, c);
  if (threadIdx.x == 0) { stats[0] = a; stats[1] = b; stats[2] = c; }
}

// U += (double)E * 2^-p on the interior; max |correction| into *maxbits.
// A block covers 256 columns of every gridDim.y-th row and adds its maximum
// with one atomic: the maxima of all blocks meet at one address, where
// same-address atomics complete one after another (about 11 ns each), so
// one atomic per wavefront of a one-row block (2^18 at 4096^2) took 3 ms
// against well under 0.1 ms for the grid traffic.
constexpr int kAccRowBlocks = 64;

__global__ __launch_bounds__(256) void accumulate_kernel(
    double *U, int64_t pitch, const void *E, int prec_lo, int64_t lo_pitch,
    int n, int scale_exp, unsigned long long *maxbits) {
  __shared__ double sh[256 / 64];
  const int j = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const double inv = ldexp(1.0, -scale_exp);
  double d = 0.0;
  if (j <= n) {
#pragma unroll 4
    for (int i = blockIdx.y + 1; i <= n; i += gridDim.y) {
      const int64_t lc = (int64_t)i * lo_pitch + j;
      const double e = prec_lo == kF32 ? (double)((const float *)E)[lc]
                                       : (double)(float)((const _Float16 *)E)[lc];
      const double corr = e * inv;
      const int64_t c = (int64_t)i * pitch + j;
      U[c] = U[c] + corr;
      d = fmax(d, fabs(corr));
    }
  }
  d = wave_max(d);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = d;
  __syncthreads();
  if (maxbits && threadIdx.x == 0) {
    for (int w = 1; w < 256 / 64; ++w) d = fmax(d, sh[w]);
    __hip_atomic_fetch_max(maxbits, (unsigned long long)__double_as_longlong(d),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
BlockGeom block_geom(int prec, int T, int ord) {
  BlockGeom g;
  g.V = prec_cells(prec);
  g.S = order_stages(ord, T);
  g.H = order_row_halo(ord, T);
  g.A = ((g.S + g.V - 1) / g.V) * g.V;
  g.CW = kLanes * g.V - 2 * g.A;
  g.W = order_window_rows(ord, T);
  return g;
}

Layout make_layout(int n, int prec) {
  Layout L;
  L.n = n;
  const int esz = prec_bytes(prec);
  const int64_t need = kMX + (int64_t)n + kLanes * prec_cells(prec) + 1;
  const int64_t q = 256 / esz;                 // 256-byte row alignment
  L.pitch = (need + q - 1) / q * q;
  L.rows = (int64_t)n + 2 + 2 * kMY;
  return L;
}

hipError_t launch_ctl_reset(Ctl *ctl, hipStream_t s) {
  hipLaunchKernelGGL(ctl_reset_kernel, dim3(1), dim3(256), 0, s, ctl);
  return hipGetLastError();
}

// One block row per allocated row (n + 2 + 2*kMY), x over the pitch.
static dim3 alloc_grid(int64_t pitch, int n) {
  return dim3((unsigned)((pitch + 255) / 256), (unsigned)(n + 2 + 2 * kMY));
}

hipError_t launch_pack(int prec, const void *u, const void *bdy, void *A,
                       void *B, int64_t pitch, int n, unsigned *bad, hipStream_t s) {
  switch (prec) {
    case kF64: hipLaunchKernelGGL(pack_kernel<double>, alloc_grid(pitch, n), dim3(256), 0, s,
                                  (const double *)u, (const double *)bdy, (double *)A,
                                  (double *)B, pitch, n, bad); break;
    case kF32: hipLaunchKernelGGL(pack_kernel<float>, alloc_grid(pitch, n), dim3(256), 0, s,
                                  (const float *)u, (const float *)bdy, (float *)A,
                                  (float *)B, pitch, n, bad); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pack_rhs(int prec, const void *f, void *F, int64_t pitch, int n,
                           unsigned *bad, hipStream_t s) {
  const double h = 1.0 / (double)(n + 1);
  const double h2 = h * h;
  switch (prec) {
    case kF64: hipLaunchKernelGGL(pack_rhs_kernel<double>, alloc_grid(pitch, n), dim3(256), 0, s,
                                  (const double *)f, (double *)F, pitch, n, h2, bad); break;
    case kF32: hipLaunchKernelGGL(pack_rhs_kernel<float>, alloc_grid(pitch, n), dim3(256), 0, s,
                                  (const float *)f, (float *)F, pitch, n, h2, bad); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_unpack(int prec, const void *A, void *u, int64_t pitch, int n,
                         hipStream_t s) {
  const dim3 grid((n + 255) / 256, n);
  switch (prec) {
    case kF64: hipLaunchKernelGGL(unpack_kernel<double>, grid, dim3(256), 0, s,
                                  (const double *)A, (double *)u, pitch, n); break;
    case kF32: hipLaunchKernelGGL(unpack_kernel<float>, grid, dim3(256), 0, s,
                                  (const float *)A, (float *)u, pitch, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill_zero(int prec, void *A, int64_t pitch, int n, hipStream_t s) {
  switch (prec) {
    case kF64: hipLaunchKernelGGL(fill_zero_kernel<double>, alloc_grid(pitch, n), dim3(256), 0, s,
                                  (double *)A, pitch, n); break;
    case kF32: hipLaunchKernelGGL(fill_zero_kernel<float>, alloc_grid(pitch, n), dim3(256), 0, s,
                                  (float *)A, pitch, n); break;
    case kF16: hipLaunchKernelGGL(fill_zero_kernel<_Float16>, alloc_grid(pitch, n), dim3(256), 0, s,
                                  (_Float16 *)A, pitch, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The blocked passes are instantiated in the sor_blocked_*_t*.hip units.
#define SOR_EXTERN_BLOCKED(P, T)                                               \
  extern template hipError_t launch_blocked_PT<P, T>(                          \
      const GridView &, Ctl *, const Sched &, hipStream_t, const BlockShape &); \
  extern template int blocked_blocks_per_cu<P, T>(bool);
#define SOR_EXTERN_BLOCKED_ALL(P)                                              \
  SOR_EXTERN_BLOCKED(P, 1) SOR_EXTERN_BLOCKED(P, 2) SOR_EXTERN_BLOCKED(P, 3)   \
  SOR_EXTERN_BLOCKED(P, 4) SOR_EXTERN_BLOCKED(P, 5) SOR_EXTERN_BLOCKED(P, 6)   \
  SOR_EXTERN_BLOCKED(P, 7) SOR_EXTERN_BLOCKED(P, 8)
SOR_EXTERN_BLOCKED_ALL(kF64)
SOR_EXTERN_BLOCKED_ALL(kF32)
SOR_EXTERN_BLOCKED_ALL(kF16)
// Red-black passes that form the maxima of one iteration (MX = 0..T-1) or
// of none (MX = T), in the sor_blocked_*_t*_mx*.hip units: FP64 and FP32 at
// depths 6 and 7 (the automatic depths), and for binary16 inner sweeps,
// which check only at their last iteration, the variant without maxima.
#define SOR_EXTERN_MX(P, T, MX)                                                \
  extern template hipError_t launch_blocked_PT<P, T, 0, MX>(                   \
      const GridView &, Ctl *, const Sched &, hipStream_t, const BlockShape &);
#define SOR_EXTERN_MX6(P)                                                      \
  SOR_EXTERN_MX(P, 6, 0) SOR_EXTERN_MX(P, 6, 1) SOR_EXTERN_MX(P, 6, 2)         \
  SOR_EXTERN_MX(P, 6, 3) SOR_EXTERN_MX(P, 6, 4) SOR_EXTERN_MX(P, 6, 5)         \
  SOR_EXTERN_MX(P, 6, 6)
#define SOR_EXTERN_MX7(P)                                                      \
  SOR_EXTERN_MX(P, 7, 0) SOR_EXTERN_MX(P, 7, 1) SOR_EXTERN_MX(P, 7, 2)         \
  SOR_EXTERN_MX(P, 7, 3) SOR_EXTERN_MX(P, 7, 4) SOR_EXTERN_MX(P, 7, 5)         \
  SOR_EXTERN_MX(P, 7, 6) SOR_EXTERN_MX(P, 7, 7)
SOR_EXTERN_MX6(kF64) SOR_EXTERN_MX7(kF64)
SOR_EXTERN_MX6(kF32) SOR_EXTERN_MX7(kF32)
SOR_EXTERN_MX(kF16, 6, 6) SOR_EXTERN_MX(kF16, 7, 7)
extern template int blocked_blocks_per_cu<kF64, 6, 0, 5>(bool);
extern template int blocked_blocks_per_cu<kF64, 7, 0, 6>(bool);
extern template int blocked_blocks_per_cu<kF32, 6, 0, 5>(bool);
extern template int blocked_blocks_per_cu<kF32, 7, 0, 6>(bool);
extern template int blocked_blocks_per_cu<kF16, 6, 0, 6>(bool);
extern template int blocked_blocks_per_cu<kF16, 7, 0, 7>(bool);

// Which maxima variants a (precision, depth) has: 2 one per iteration and
// none, 1 none only, 0 only the pass forming every maximum.
constexpr int rb_mx_variants(int P, int T) {
  return (T == 6 || T == 7) ? (P == kF16 ? 1 : 2) : 0;
}

// The red-black pass of depth T forming the maxima that mx selects (-1
// every iteration, 0..T-1 that one, T none), or, where that variant is
// not built, every maximum (a superset: the stopping rule reads the same
// values).
template <int P, int T, int M = 0>
static hipError_t launch_rb(int mx, const GridView &v, Ctl *ctl, const Sched &sc,
                            hipStream_t s) {
  if constexpr (rb_mx_variants(P, T) == 2 && M < T) {
    if (mx == M) return launch_blocked_PT<P, T, 0, M>(v, ctl, sc, s);
    return launch_rb<P, T, M + 1>(mx, v, ctl, sc, s);
  } else {
    if constexpr (rb_mx_variants(P, T) >= 1)
      if (mx == T) return launch_blocked_PT<P, T, 0, T>(v, ctl, sc, s);
    return launch_blocked_PT<P, T>(v, ctl, sc, s);
  }
}
#define SOR_EXTERN_BLOCKED_ORD(T, ORD)                                         \
  extern template hipError_t launch_blocked_PT<kF64, T, ORD>(                  \
      const GridView &, Ctl *, const Sched &, hipStream_t, const BlockShape &); \
  extern template int blocked_blocks_per_cu<kF64, T, ORD>(bool);
SOR_EXTERN_BLOCKED_ORD(1, 1) SOR_EXTERN_BLOCKED_ORD(2, 1)
SOR_EXTERN_BLOCKED_ORD(3, 1) SOR_EXTERN_BLOCKED_ORD(4, 1) SOR_EXTERN_BLOCKED_ORD(5, 1)
SOR_EXTERN_BLOCKED_ORD(1, 2) SOR_EXTERN_BLOCKED_ORD(2, 2)
SOR_EXTERN_BLOCKED_ORD(3, 2) SOR_EXTERN_BLOCKED_ORD(4, 2)
SOR_EXTERN_BLOCKED_ORD(5, 2) SOR_EXTERN_BLOCKED_ORD(6, 2)
SOR_EXTERN_BLOCKED_ORD(7, 2) SOR_EXTERN_BLOCKED_ORD(8, 2)
SOR_EXTERN_BLOCKED_ORD(1, 3) SOR_EXTERN_BLOCKED_ORD(2, 3)
SOR_EXTERN_BLOCKED_ORD(3, 3) SOR_EXTERN_BLOCKED_ORD(4, 3)
SOR_EXTERN_BLOCKED_ORD(5, 3) SOR_EXTERN_BLOCKED_ORD(6, 3)
SOR_EXTERN_BLOCKED_ORD(7, 3) SOR_EXTERN_BLOCKED_ORD(8, 3)
SOR_EXTERN_BLOCKED_ORD(1, 4) SOR_EXTERN_BLOCKED_ORD(2, 4)
SOR_EXTERN_BLOCKED_ORD(3, 4) SOR_EXTERN_BLOCKED_ORD(4, 4)
SOR_EXTERN_BLOCKED_ORD(5, 4) SOR_EXTERN_BLOCKED_ORD(6, 4)
SOR_EXTERN_BLOCKED_ORD(7, 4) SOR_EXTERN_BLOCKED_ORD(8, 4)

// Passes of the other orderings (FP64 only).
template <int ORD>
static hipError_t launch_blocked_ord(int T, const GridView &v, Ctl *ctl, const Sched &sc,
                                     hipStream_t s, const BlockShape &bs) {
  switch (T) {
    case 1: return launch_blocked_PT<kF64, 1, ORD>(v, ctl, sc, s, bs);
    case 2: return launch_blocked_PT<kF64, 2, ORD>(v, ctl, sc, s, bs);
    case 3: return launch_blocked_PT<kF64, 3, ORD>(v, ctl, sc, s, bs);
    case 4: return launch_blocked_PT<kF64, 4, ORD>(v, ctl, sc, s, bs);
  }
  if constexpr (ORD == 1) {
    if (T == 5) return launch_blocked_PT<kF64, 5, ORD>(v, ctl, sc, s, bs);
  }
  if constexpr (ORD >= 2) {
    switch (T) {
      case 5: return launch_blocked_PT<kF64, 5, ORD>(v, ctl, sc, s, bs);
      case 6: return launch_blocked_PT<kF64, 6, ORD>(v, ctl, sc, s, bs);
      case 7: return launch_blocked_PT<kF64, 7, ORD>(v, ctl, sc, s, bs);
      case 8: return launch_blocked_PT<kF64, 8, ORD>(v, ctl, sc, s, bs);
    }
  }
  return hipErrorInvalidValue;
}

template <int ORD>
static int blocked_blocks_per_cu_ord(int T, bool pois) {
  switch (T) {
    case 1: return blocked_blocks_per_cu<kF64, 1, ORD>(pois);
    case 2: return blocked_blocks_per_cu<kF64, 2, ORD>(pois);
    case 3: return blocked_blocks_per_cu<kF64, 3, ORD>(pois);
    case 4: return blocked_blocks_per_cu<kF64, 4, ORD>(pois);
  }
  if constexpr (ORD == 1) {
    if (T == 5) return blocked_blocks_per_cu<kF64, 5, ORD>(pois);
  }
  if constexpr (ORD >= 2) {
    switch (T) {
      case 5: return blocked_blocks_per_cu<kF64, 5, ORD>(pois);
      case 6: return blocked_blocks_per_cu<kF64, 6, ORD>(pois);
      case 7: return blocked_blocks_per_cu<kF64, 7, ORD>(pois);
      case 8: return blocked_blocks_per_cu<kF64, 8, ORD>(pois);
    }
  }
  return 0;
}

template <int P>
static hipError_t launch_blocked_P(int T, const GridView &v, Ctl *ctl,
                                   const Sched &sc, hipStream_t s, int mx) {
  switch (T) {
    case 1: return launch_blocked_PT<P, 1>(v, ctl, sc, s);
    case 2: return launch_blocked_PT<P, 2>(v, ctl, sc, s);
    case 3: return launch_blocked_PT<P, 3>(v, ctl, sc, s);
    case 4: return launch_blocked_PT<P, 4>(v, ctl, sc, s);
    case 5: return launch_blocked_PT<P, 5>(v, ctl, sc, s);
    case 6: return launch_rb<P, 6>(mx, v, ctl, sc, s);
    case 7: return launch_rb<P, 7>(mx, v, ctl, sc, s);
    case 8: return launch_blocked_PT<P, 8>(v, ctl, sc, s);
  }
  return hipErrorInvalidValue;
}

// Occupancy of the pass a solve mostly runs: with a maxima variant, the one
// forming the maxima of its last iteration (a solve checking every T or
// more iterations has at most one check per pass), or, with binary16
// storage, the one forming none (inner sweeps check only at their end).
template <int P, int T>
static int blocked_blocks_per_cu_rb(bool pois) {
  if constexpr (rb_mx_variants(P, T) == 2) return blocked_blocks_per_cu<P, T, 0, T - 1>(pois);
  else if constexpr (rb_mx_variants(P, T) == 1) return blocked_blocks_per_cu<P, T, 0, T>(pois);
  else return blocked_blocks_per_cu<P, T>(pois);
}

template <int P>
static int blocked_blocks_per_cu_P(int T, bool pois) {
  switch (T) {
    case 1: return blocked_blocks_per_cu<P, 1>(pois);
    case 2: return blocked_blocks_per_cu<P, 2>(pois);
    case 3: return blocked_blocks_per_cu<P, 3>(pois);
    case 4: return blocked_blocks_per_cu<P, 4>(pois);
    case 5: return blocked_blocks_per_cu<P, 5>(pois);
    case 6: return blocked_blocks_per_cu_rb<P, 6>(pois);
    case 7: return blocked_blocks_per_cu_rb<P, 7>(pois);
    case 8: return blocked_blocks_per_cu<P, 8>(pois);
  }
  return 0;
}

int blocked_blocks_per_cu(int prec, int T, bool pois, int ord) {
  if (ord) {
    if (prec != kF64) return 0;
    switch (ord) {
      case 1: return blocked_blocks_per_cu_ord<1>(T, pois);
      case 2: return blocked_blocks_per_cu_ord<2>(T, pois);
      case 3: return blocked_blocks_per_cu_ord<3>(T, pois);
      case 4: return blocked_blocks_per_cu_ord<4>(T, pois);
    }
    return 0;
  }
  switch (prec) {
    case kF64: return blocked_blocks_per_cu_P<kF64>(T, pois);
    case kF32: return blocked_blocks_per_cu_P<kF32>(T, pois);
    case kF16: return blocked_blocks_per_cu_P<kF16>(T, pois);
  }
  return 0;
}

bool blocked_T_supported(int T) {
  return T >= 1 && T <= kTMax;
}

bool blocked_ord_T_supported(int ord, int T) {
  return T >= 1 && T <= (ord == 1 ? kTMaxC4 : kTMax);
}

hipError_t launch_blocked_pass(int prec, int T, const GridView &v, Ctl *ctl,
                               const Sched &sc, hipStream_t s, int ord,
                               const BlockShape &bs, int mx) {
  if (ord) {
    if (prec != kF64) return hipErrorInvalidValue;
    switch (ord) {
      case 1: return launch_blocked_ord<1>(T, v, ctl, sc, s, bs);
      case 2: return launch_blocked_ord<2>(T, v, ctl, sc, s, bs);
      case 3: return launch_blocked_ord<3>(T, v, ctl, sc, s, bs);
      case 4: return launch_blocked_ord<4>(T, v, ctl, sc, s, bs);
    }
    return hipErrorInvalidValue;
  }
  switch (prec) {
    case kF64: return launch_blocked_P<kF64>(T, v, ctl, sc, s, mx);
    case kF32: return launch_blocked_P<kF32>(T, v, ctl, sc, s, mx);
    case kF16: return launch_blocked_P<kF16>(T, v, ctl, sc, s, mx);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_simple_iteration(int prec, const GridView &v, Ctl *ctl,
                                   const Sched &sc, hipStream_t s) {
  const int per_row = (v.n + 1) / 2;   // most cells of one colour in a row
  const dim3 grid((per_row + 255) / 256, v.n);
  for (int colour = 0; colour < 2; ++colour) {
    const int fin = colour == 1;
    switch (prec) {
      case kF64:
        if (v.F) hipLaunchKernelGGL((simple_colour_kernel<kF64, true>), grid, dim3(256), 0, s, v, ctl, sc, colour, fin);
        else hipLaunchKernelGGL((simple_colour_kernel<kF64, false>), grid, dim3(256), 0, s, v, ctl, sc, colour, fin);
        break;
      case kF32:
        if (v.F) hipLaunchKernelGGL((simple_colour_kernel<kF32, true>), grid, dim3(256), 0, s, v, ctl, sc, colour, fin);
        else hipLaunchKernelGGL((simple_colour_kernel<kF32, false>), grid, dim3(256), 0, s, v, ctl, sc, colour, fin);
        break;
      case kF16:
        if (v.F) hipLaunchKernelGGL((simple_colour_kernel<kF16, true>), grid, dim3(256), 0, s, v, ctl, sc, colour, fin);
        else hipLaunchKernelGGL((simple_colour_kernel<kF16, false>), grid, dim3(256), 0, s, v, ctl, sc, colour, fin);
        break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

int64_t residual_partials(int n) {
  return (int64_t)((n + kResBlock - 1) / kResBlock) * n;
}

hipError_t launch_residual(const double *U, const double *F, int64_t pitch, int n,
                           double *r, double *partials, double *stats, void *lo,
                           int prec_lo, int64_t lo_pitch, int scale_exp,
                           hipStream_t s) {
  const dim3 grid((n + kResBlock - 1) / kResBlock, n);
  hipLaunchKernelGGL(residual_kernel, grid, dim3(kResBlock), 0, s, U, F, pitch, n, r,
                     partials, lo, prec_lo, lo_pitch, scale_exp);
  hipLaunchKernelGGL(residual_finalize_kernel, dim3(1), dim3(kResBlock), 0, s,
                     (const double *)partials, residual_partials(n), stats);
  return hipGetLastError();
}

hipError_t launch_accumulate(double *U, int64_t pitch, const void *E, int prec_lo,
                             int64_t lo_pitch, int n, int scale_exp,
                             unsigned long long *maxbits, hipStream_t s) {
  const dim3 grid((n + 255) / 256, n < kAccRowBlocks ? n : kAccRowBlocks);
  hipLaunchKernelGGL(accumulate_kernel, grid, dim3(256), 0, s, U, pitch, E, prec_lo,
                     lo_pitch, n, scale_exp, maxbits);
  return hipGetLastError();
}

}  // namespace sor
