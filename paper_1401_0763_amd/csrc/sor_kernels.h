// Device-side building blocks of libsor shared by its translation units:
// precision traits, cross-lane moves, the per-pass stopping-rule evaluation
// and the temporally blocked sweep of one tile.
//
// Method (Mittal 2014): Sec. 2.1 Eq. 1 (SOR update), Sec. 3.1 with Fig. 1-2
// (red-black colouring, red phase then black phase), Algorithm 1 (iteration
// loop, check every K iterations, strict stopping rule on the largest change
// of one iteration).
#pragma once

#include "sor_internal.h"

namespace sor {

// ---------------------------------------------------------------------------
// Precision traits: storage type, arithmetic type, cells per lane.
// ---------------------------------------------------------------------------
template <int P> struct PT;
template <> struct PT<kF64> { using st = double;   using ct = double; static constexpr int V = 2; };
template <> struct PT<kF32> { using st = float;    using ct = float;  static constexpr int V = 4; };
template <> struct PT<kF16> { using st = _Float16; using ct = float;  static constexpr int V = 4; };

template <int P>
struct alignas(sizeof(typename PT<P>::st) * PT<P>::V) Vec {
  typename PT<P>::st v[PT<P>::V];
};

// ---------------------------------------------------------------------------
// Cross-lane moves.  DPP wave_shr:1 hands every lane the value of the lane
// below it (lane i receives lane i-1); wave_shl:1 the lane above.  Lanes at
// the wave edge receive 0 (bound_ctrl); they only ever feed halo cells.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int dpp_from_left_i(int x) {
  return __builtin_amdgcn_mov_dpp(x, 0x138, 0xf, 0xf, true);
}
__device__ __forceinline__ int dpp_from_right_i(int x) {
  return __builtin_amdgcn_mov_dpp(x, 0x130, 0xf, 0xf, true);
}
__device__ __forceinline__ float from_left(float x) {
  return __int_as_float(dpp_from_left_i(__float_as_int(x)));
}
__device__ __forceinline__ float from_right(float x) {
  return __int_as_float(dpp_from_right_i(__float_as_int(x)));
}
__device__ __forceinline__ double from_left(double x) {
  return __hiloint2double(dpp_from_left_i(__double2hiint(x)),
                          dpp_from_left_i(__double2loint(x)));
}
__device__ __forceinline__ double from_right(double x) {
  return __hiloint2double(dpp_from_right_i(__double2hiint(x)),
                          dpp_from_right_i(__double2loint(x)));
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

__device__ __forceinline__ float vabs(float x) { return fabsf(x); }
__device__ __forceinline__ double vabs(double x) { return fabs(x); }
__device__ __forceinline__ float vmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return fmax(a, b); }

// Spread consecutive tiles over the 8 XCDs in contiguous runs: workgroups are
// dispatched round-robin over XCDs, so block b runs on XCD b % 8; mapping it
// to tile xcd * per + ... keeps vertically and horizontally adjacent tiles
// (which share halo rows) in the same XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int xcd = b & 7, k = b >> 3;
  const int per = nb >> 3, rem = nb & 7;
  return xcd * per + (xcd < rem ? xcd : rem) + k;
}

// ---------------------------------------------------------------------------
// Control block helpers (agent-scope atomics: the 8 XCDs' L2s are not
// coherent for plain stores, agent-scope atomics are).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int ctl_stopped(const Ctl *ctl) {
  return __hip_atomic_load(&ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish this wave's per-iteration maxima (already wave-reduced, in lane 0)
// and, if it is the last wave of the pass, evaluate the stopping rule for the
// pass's iterations (Algorithm 1), record each iteration's change, and reset
// the slots for the next pass.
template <int T>
__device__ __forceinline__ void report_pass(Ctl *ctl, const Sched &sc,
                                            const double (&mx)[T], int t_run,
                                            bool bad, int slot,
                                            unsigned waves_total) {
  const int lane = threadIdx.x & 63;
  const bool anybad = __ballot(bad) != 0;
  unsigned prev = 0;
  if (lane == 0) {
#pragma unroll
    for (int t = 0; t < T; ++t)
      __hip_atomic_fetch_max(&ctl->slots[slot][t],
                             (unsigned long long)__double_as_longlong(mx[t]),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (anybad)
      __hip_atomic_fetch_or(&ctl->nonfinite, 1u, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT);
    prev = __hip_atomic_fetch_add(&ctl->counter, 1u, __ATOMIC_ACQ_REL,
                                  __HIP_MEMORY_SCOPE_AGENT);
  }
  prev = __shfl(prev, 0, 64);
  if (prev != waves_total - 1) return;

  // Last wave of the pass: gather the slots (lane s reads slot s).
  double it_max[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    unsigned long long b = __hip_atomic_load(&ctl->slots[lane][t], __ATOMIC_ACQUIRE,
                                             __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ctl->slots[lane][t], 0ull, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    it_max[t] = wave_max(__longlong_as_double((long long)b));
  }
  if (lane == 0) {
    const long long it0 = __hip_atomic_load(&ctl->it_base, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
    const unsigned nonf = __hip_atomic_load(&ctl->nonfinite, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
    int stop = ctl->stop;
    for (int t = 0; t < t_run; ++t) {
      const long long it = it0 + t + 1;
      ctl->hist[(it - 1) % kHistCap] = it_max[t];
      if (stop == 0 && (it % sc.check_every == 0 || it == sc.max_iters)) {
        ctl->last_iter = it;
        ctl->last_max = it_max[t];
        if (it_max[t] < sc.tol) {
          stop = 1;
          ctl->stop_iter = it;
          ctl->stop_max = it_max[t];
        }
      }
    }
    if (nonf) {
      stop = 2;
      ctl->stop_iter = it0 + t_run;
      ctl->stop_max = it_max[t_run - 1];
    }
    ctl->it_base = it0 + t_run;
    ctl->passes_done += 1;
    __hip_atomic_store(&ctl->stop, stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ctl->counter, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// Temporally blocked streaming sweep of one tile by one wavefront.
//
// The tile is a column strip of 64*V cells (V per lane, so one 16-byte access
// per lane per row; 8 bytes for binary16 storage) and a row segment of
// seg_rows output rows.  The wave walks down the rows; at step r it applies
// S = 2T half-sweeps as a pipeline: stage k (k = 0..S-1) updates row r-k with
// colour k&1 (red first, Sec. 3.1), i.e. stage k is iteration k/2's red or
// black phase.  Stage k at row q reads row q+1 after stage k-1 updated it in
// this same step, row q-1 after stage k-1 updated it one step earlier, and
// row q's own other-colour cells at level k-1, so every update sees exactly
// the values the two-phase iteration of Algorithm 1 gives it.  Rows live in a
// rotating register window; horizontal neighbours in the adjacent lane arrive
// by DPP.
//
// Values near the strip and segment edges depend on cells outside the tile
// and are wrong after enough stages (the dependency cone grows one cell per
// half-sweep), so the tile loads a halo of A >= S columns and S rows on each
// side and stores only its core (CW columns x seg_rows rows).  Input and
// output are separate grids (ping-pong), so halos are read at the pass's
// starting level whatever order tiles run in.
//
// Only the first 2*t_run stages are applied (t_run <= T iterations); the
// rest leave the rows untouched, which lets one kernel finish a solve whose
// iteration budget is not a multiple of T.
//
// Boundary and out-of-grid cells are never changed: their update is computed
// and discarded by a select, so the unrolled body has no branches.
//
// m[t] receives the largest |u' - u| of iteration t over the tile's core
// cells (0 in halo lanes); bad is set if a stored interior value is not
// finite.
// ---------------------------------------------------------------------------
template <int P, int T, bool POIS>
__device__ __forceinline__ void blocked_tile(const GridView &g, int tile,
                                             int t_run,
                                             typename PT<P>::ct (&m)[T],
                                             bool &bad) {
  using st = typename PT<P>::st;
  using ct = typename PT<P>::ct;
  constexpr int V = PT<P>::V;
  constexpr int S = 2 * T;
  constexpr int A = ((S + V - 1) / V) * V;
  constexpr int WV = kLanes * V;
  constexpr int CW = WV - 2 * A;
  constexpr int D = 2;                           // rows prefetched ahead
  constexpr int W = ((S + D + 2) + 1) & ~1;      // window rows (even)

  const int lane = threadIdx.x & 63;
  const int n = g.n;
  const int strip = tile % g.nstrips;
  const int seg = tile / g.nstrips;
  const int col0 = strip * CW - A + lane * V;    // even: parity below is static
  const int a = seg * g.seg_rows - S;            // first loaded row (even)
  const int core0 = seg * g.seg_rows;
  const int core1 = min(core0 + g.seg_rows, n + 1);
  const int b = core1 + S;                       // one past the last loaded row
  const int rlo = max(core0, 1);
  const int rhi = min(core1, n + 1);
  const int s_run = 2 * t_run;
  const bool lane_core = (lane * V >= A) && (lane * V < WV - A);
  const bool lane_store = lane_core && (col0 <= n) && (col0 + V - 1 >= 1);
  bool ok[V];
#pragma unroll
  for (int v = 0; v < V; ++v) ok[v] = (col0 + v >= 1) && (col0 + v <= n);
  const ct om = (ct)g.omega;
  const int64_t pitch = g.pitch;
  const st *in = (const st *)g.in + col0;
  st *out = (st *)g.out + col0;
  const st *F = nullptr;
  if constexpr (POIS) F = (const st *)g.F + col0;

  ct w[W][V];
  ct fw[POIS ? W : 1][V];
#pragma unroll
  for (int s = 0; s < W; ++s)
#pragma unroll
    for (int v = 0; v < V; ++v) {
      w[s][v] = (ct)0;
      if constexpr (POIS) fw[s][v] = (ct)0;
    }
#pragma unroll
  for (int t = 0; t < T; ++t) m[t] = (ct)0;

  // Prologue: rows a .. a+D+1 into slots 0 .. D+1 (b - a >= 2S + 1 > D + 2).
#pragma unroll
  for (int s = 0; s < D + 2; ++s) {
    const Vec<P> x = *(const Vec<P> *)(in + (int64_t)(a + s) * pitch);
#pragma unroll
    for (int v = 0; v < V; ++v) w[s][v] = (ct)x.v[v];
    if constexpr (POIS) {
      const Vec<P> y = *(const Vec<P> *)(F + (int64_t)(a + s) * pitch);
#pragma unroll
      for (int v = 0; v < V; ++v) fw[s][v] = (ct)y.v[v];
    }
  }

  const int nsteps = b - a - 2;                  // steps r = a+1 .. b-2
  for (int base = 0; base < nsteps; base += W) {
#pragma unroll
    for (int i = 0; i < W; ++i) {
      const int step = base + i;
      if (step < nsteps) {
        const int r = a + 1 + step;
        // Prefetch row r+D+1 into its slot ((row - a) mod W).
        const int rp = r + D + 1;
        if (rp < b) {
          const int sp = (i + D + 2) % W;
          const Vec<P> x = *(const Vec<P> *)(in + (int64_t)rp * pitch);
#pragma unroll
          for (int v = 0; v < V; ++v) w[sp][v] = (ct)x.v[v];
          if constexpr (POIS) {
            const Vec<P> y = *(const Vec<P> *)(F + (int64_t)rp * pitch);
#pragma unroll
            for (int v = 0; v < V; ++v) fw[sp][v] = (ct)y.v[v];
          }
        }
        // Stages: k-th half-sweep on row r-k.
#pragma unroll
        for (int k = 0; k < S; ++k) {
          const int q = r - k;
          const bool row_upd = (q >= 1) && (q <= n) && (k < s_run);   // uniform
          const bool row_cnt = (q >= rlo) && (q < rhi);                // uniform
          const int sq = ((i + 1 - k) % W + W) % W;
          const int su = (sq + W - 1) % W;
          const int sd = (sq + 1) % W;
          // Cells of colour k&1 in this lane: (q + col0 + v + k) even, and
          // q + k has the parity of 1 + i because a, base and W are even.
          const int v0 = (1 + i) & 1;
#pragma unroll
          for (int v = v0; v < V; v += 2) {
            const ct self = w[sq][v];
            const ct left = (v == 0) ? from_left(w[sq][V - 1]) : w[sq][(v + V - 1) % V];
            const ct right = (v == V - 1) ? from_right(w[sq][0]) : w[sq][(v + 1) % V];
            ct s = (w[su][v] + w[sd][v]) + (left + right);
            if constexpr (POIS) s = s + fw[sq][v];
            const ct gs = (ct)0.25 * s;
            ct nu = self + om * (gs - self);
            if constexpr (P == kF16) nu = (ct)(st)nu;
            nu = (row_upd && ok[v]) ? nu : self;
            const ct d = vabs(nu - self);
            w[sq][v] = nu;
            m[k >> 1] = vmax(m[k >> 1], row_cnt ? d : (ct)0);
          }
        }
        // Row r-S+1 has now had all S half-sweeps: store it if it is core.
        const int qo = r - S + 1;
        if (qo >= rlo && qo < rhi) {
          const int so = ((i + 2 - S) % W + W) % W;
          if (lane_store) {
            Vec<P> x;
#pragma unroll
            for (int v = 0; v < V; ++v) {
              x.v[v] = (st)w[so][v];
              if (ok[v] && !__builtin_isfinite(w[so][v])) bad = true;
            }
            *(Vec<P> *)(out + (int64_t)qo * pitch) = x;
          }
        }
      }
    }
  }
  if (!lane_core) {
#pragma unroll
    for (int t = 0; t < T; ++t) m[t] = (ct)0;
  }
}

// One blocked pass over a whole grid: one wavefront per tile, t_run <= T
// iterations from g.in into g.out.  With a control block, the pass first
// exits if an earlier pass met the stopping rule, then reports its maxima.
template <int P, int T, bool POIS>
__global__ __launch_bounds__(64) void blocked_pass_kernel(GridView g, Ctl *ctl,
                                                          Sched sc, int t_run) {
  if (ctl && ctl_stopped(ctl)) return;
  using ct = typename PT<P>::ct;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  ct m[T];
  bool bad = false;
  blocked_tile<P, T, POIS>(g, tile, t_run, m, bad);
  if (!ctl) return;
  double mx[T];
#pragma unroll
  for (int t = 0; t < T; ++t) mx[t] = wave_max((double)m[t]);
  report_pass<T>(ctl, sc, mx, t_run, bad, blockIdx.x % kSlots, gridDim.x);
}

// Host-side dispatch of blocked passes for one precision (defined in the
// per-precision translation units).
#define SOR_BLOCKED_LAUNCHER(P, NAME)                                          \
  template <int T>                                                             \
  static void NAME##_T(const GridView &v, Ctl *ctl, const Sched &sc,           \
                       int t_run, hipStream_t s) {                             \
    const dim3 grid((unsigned)v.nstrips * (unsigned)v.nseg);                   \
    if (v.F)                                                                   \
      hipLaunchKernelGGL((blocked_pass_kernel<P, T, true>), grid, dim3(64), 0, \
                         s, v, ctl, sc, t_run);                                \
    else                                                                       \
      hipLaunchKernelGGL((blocked_pass_kernel<P, T, false>), grid, dim3(64),   \
                         0, s, v, ctl, sc, t_run);                             \
  }                                                                            \
  hipError_t NAME(int T, const GridView &v, Ctl *ctl, const Sched &sc,         \
                  int t_run, hipStream_t s) {                                  \
    switch (T) {                                                               \
      case 1: NAME##_T<1>(v, ctl, sc, t_run, s); break;                        \
      case 2: NAME##_T<2>(v, ctl, sc, t_run, s); break;                        \
      case 3: NAME##_T<3>(v, ctl, sc, t_run, s); break;                        \
      case 4: NAME##_T<4>(v, ctl, sc, t_run, s); break;                        \
      case 6: NAME##_T<6>(v, ctl, sc, t_run, s); break;                        \
      case 8: NAME##_T<8>(v, ctl, sc, t_run, s); break;                        \
      default: return hipErrorInvalidValue;                                    \
    }                                                                          \
    return hipGetLastError();                                                  \
  }

}  // namespace sor
