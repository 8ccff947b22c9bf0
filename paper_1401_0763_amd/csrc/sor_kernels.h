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

#include <type_traits>

// Rows a wavefront loads ahead of the row it is updating.
#ifndef SOR_PREFETCH
#define SOR_PREFETCH 4
#endif
// Register-window periods unrolled per loop iteration of the row walk.
#ifndef SOR_UNROLL
#define SOR_UNROLL 1
#endif

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

// Compile-time loop: calls f(std::integral_constant<int, I>) for I = B..E-1.
// Used where an index selects a register (window slot, stage), so the index
// must be a constant however large the unrolled body grows.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

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
// Raw buffer access.  A buffer resource (base, byte extent) lives in SGPRs;
// each access adds a per-lane VGPR offset and a wave-uniform SGPR offset.  A
// store whose per-lane offset has bit 31 set lies beyond the resource's
// extent (which is kept below 2^31) and is dropped by the hardware, which
// gives predicated stores without a branch.
// ---------------------------------------------------------------------------
constexpr unsigned kDrop = 0x80000000u;
constexpr unsigned kRsrcWord3 = 0x00020000u;   // gfx9 raw buffer, 32-bit format

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base,
                                                             unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes,
                                           (int)kRsrcWord3);
}

template <int P>
__device__ __forceinline__ Vec<P> buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff,
                                           unsigned soff) {
  if constexpr (sizeof(Vec<P>) == 16) {
    return __builtin_bit_cast(Vec<P>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
  } else {
    return __builtin_bit_cast(Vec<P>, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
  }
}

template <int P>
__device__ __forceinline__ void buf_store(const Vec<P> &x, __amdgpu_buffer_rsrc_t r,
                                          unsigned voff, unsigned soff) {
  if constexpr (sizeof(Vec<P>) == 16) {
    using v4 = unsigned __attribute__((ext_vector_type(4)));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4, x), r, (int)voff, (int)soff, 0);
  } else {
    using v2 = unsigned __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2, x), r, (int)voff, (int)soff, 0);
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
// The step loop runs in chunks of W steps with no branch inside a chunk, so
// the compiler can overlap the stages of neighbouring steps: loads read a
// clamped row (always inside the tile's rows), stores of rows outside the
// core are dropped by an out-of-range offset, and the per-iteration maxima
// weight each change by 1 (core row) or 0 (halo row).  MASK tiles touch the
// boundary ring or lie partly outside the grid; their boundary and
// out-of-grid cells keep their value through a select.  Other tiles hold
// interior cells only and need no mask.
//
// m[t] receives the largest |u' - u| of iteration t over the tile's core
// cells (0 in halo lanes); bad is set if a stored interior value is not
// finite.
// ---------------------------------------------------------------------------
template <int P, int T, bool POIS, bool MASK>
__device__ __forceinline__ void blocked_tile(const GridView &g, int tile,
                                             typename PT<P>::ct (&m)[T],
                                             bool &bad) {
  using st = typename PT<P>::st;
  using ct = typename PT<P>::ct;
  constexpr int V = PT<P>::V;
  constexpr int S = 2 * T;
  constexpr int A = ((S + V - 1) / V) * V;
  constexpr int WV = kLanes * V;
  constexpr int CW = WV - 2 * A;
  constexpr int D = SOR_PREFETCH;                // rows prefetched ahead
  constexpr int W = ((S + D + 2) + 1) & ~1;      // window rows (even)
  constexpr int ESZ = (int)sizeof(st);

  const int lane = threadIdx.x & 63;
  const int n = g.n;
  const int strip = tile % g.nstrips;
  const int seg = tile / g.nstrips;
  const int j0 = strip * CW - A;                 // first column of the strip
  const int col0 = j0 + lane * V;                // even: parity below is static
  const int a = seg * g.seg_rows - S;            // first loaded row (even)
  const int core0 = seg * g.seg_rows;
  const int core1 = min(core0 + g.seg_rows, n + 1);
  const int b = core1 + S;                       // one past the last loaded row
  const int rlo = max(core0, 1);
  const int rhi = min(core1, n + 1);
  const bool lane_core = (lane * V >= A) && (lane * V < WV - A);
  const bool lane_store = lane_core && (col0 <= n) && (col0 + V - 1 >= 1);
  bool ok[V];
#pragma unroll
  for (int v = 0; v < V; ++v) ok[v] = (col0 + v >= 1) && (col0 + v <= n);
  const ct om = (ct)g.omega;
  const unsigned rowbytes = (unsigned)(g.pitch * ESZ);
  const unsigned extent = (unsigned)(b - a) * rowbytes;     // < 2^31
  const int64_t tile_off = (int64_t)a * g.pitch + j0;
  const auto rin = make_rsrc((const st *)g.in + tile_off, extent);
  const auto rout = make_rsrc((st *)g.out + tile_off, extent);
  __amdgpu_buffer_rsrc_t rf;
  if constexpr (POIS) rf = make_rsrc((const st *)g.F + tile_off, extent);
  const unsigned lane_off = (unsigned)(lane * V * ESZ);
  const unsigned st_off = lane_store ? lane_off : kDrop;

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
    const Vec<P> x = buf_load<P>(rin, lane_off, (unsigned)s * rowbytes);
#pragma unroll
    for (int v = 0; v < V; ++v) w[s][v] = (ct)x.v[v];
    if constexpr (POIS) {
      const Vec<P> y = buf_load<P>(rf, lane_off, (unsigned)s * rowbytes);
#pragma unroll
      for (int v = 0; v < V; ++v) fw[s][v] = (ct)y.v[v];
    }
  }

  const int nsteps = b - a - 2;                  // steps r = a+1 .. b-2
  constexpr int CH = W * SOR_UNROLL;             // steps per loop iteration
  for (int base = 0; base < nsteps; base += CH) {
    static_for<0, CH>([&](auto I) __attribute__((always_inline)) {
      constexpr int i = decltype(I)::value;
      const int r = a + 1 + base + i;
      // Prefetch row r+D+1 (clamped to the tile) into its slot ((row-a) mod W).
      {
        constexpr int sp = (i + D + 2) % W;
        const int rp = min(r + D + 1, b - 1);
        const unsigned soff = (unsigned)(rp - a) * rowbytes;
        const Vec<P> x = buf_load<P>(rin, lane_off, soff);
#pragma unroll
        for (int v = 0; v < V; ++v) w[sp][v] = (ct)x.v[v];
        if constexpr (POIS) {
          const Vec<P> y = buf_load<P>(rf, lane_off, soff);
#pragma unroll
          for (int v = 0; v < V; ++v) fw[sp][v] = (ct)y.v[v];
        }
      }
      // Stages: k-th half-sweep on row r-k.
      static_for<0, S>([&](auto K) __attribute__((always_inline)) {
        constexpr int k = decltype(K)::value;
        constexpr int sq = ((i + 1 - k) % W + W) % W;
        constexpr int su = (sq + W - 1) % W;
        constexpr int sd = (sq + 1) % W;
        // Cells of colour k&1 in this lane: (q + col0 + v + k) even, and
        // q + k has the parity of 1 + i because a, base and W are even.
        constexpr int v0 = (1 + i) & 1;
        const int q = r - k;
        const ct cnt = (q >= rlo && q < rhi) ? (ct)1 : (ct)0;        // uniform
        const bool row_upd = (q >= 1) && (q <= n);                   // uniform
        static_for<0, V / 2>([&](auto J) __attribute__((always_inline)) {
          constexpr int v = v0 + 2 * decltype(J)::value;
          const ct self = w[sq][v];
          ct left, right;
          if constexpr (v == 0) left = from_left(w[sq][V - 1]);
          else left = w[sq][v - 1];
          if constexpr (v == V - 1) right = from_right(w[sq][0]);
          else right = w[sq][v + 1];
          ct s = (w[su][v] + w[sd][v]) + (left + right);
          if constexpr (POIS) s = s + fw[sq][v];
          const ct gs = (ct)0.25 * s;
          ct nu = self + om * (gs - self);
          if constexpr (P == kF16) nu = (ct)(st)nu;
          if constexpr (MASK) nu = (row_upd && ok[v]) ? nu : self;
          const ct d = vabs(nu - self);
          w[sq][v] = nu;
          m[k >> 1] = vmax(m[k >> 1], d * cnt);
        });
      });
      // Row r-S+1 has now had all S half-sweeps: store it if it is core.
      {
        constexpr int so = ((i + 2 - S) % W + W) % W;
        const int qo = r - S + 1;
        const bool row_ok = (qo >= rlo) && (qo < rhi);
        Vec<P> x;
        bool nf = false;
#pragma unroll
        for (int v = 0; v < V; ++v) {
          x.v[v] = (st)w[so][v];
          nf = nf | (ok[v] && !__builtin_isfinite(w[so][v]));
        }
        bad = bad | (nf && row_ok && lane_store);
        buf_store<P>(x, rout, st_off | (row_ok ? 0u : kDrop),
                     row_ok ? (unsigned)(qo - a) * rowbytes : 0u);
      }
    });
  }
  if (!lane_core) {
#pragma unroll
    for (int t = 0; t < T; ++t) m[t] = (ct)0;
  }
}

// One blocked pass over a whole grid: one wavefront per tile, T iterations
// from g.in into g.out.  With a control block, the pass first exits if an
// earlier pass met the stopping rule, then reports its maxima.
template <int P, int T, bool POIS>
__global__ __launch_bounds__(64) void blocked_pass_kernel(GridView g, Ctl *ctl,
                                                          Sched sc) {
  if (ctl && ctl_stopped(ctl)) return;
  using ct = typename PT<P>::ct;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  constexpr int V = PT<P>::V;
  constexpr int S = 2 * T;
  constexpr int A = ((S + V - 1) / V) * V;
  constexpr int CW = kLanes * V - 2 * A;
  // A tile needs masking if its loaded rows or columns reach the boundary
  // ring or beyond (rows a..b-1, columns j0..j0+64V-1).
  const int strip = tile % g.nstrips, seg = tile / g.nstrips;
  const int j0 = strip * CW - A;
  const int a = seg * g.seg_rows - S;
  const int b = min(a + S + g.seg_rows, g.n + 1) + S;
  const bool mask = (j0 < 1) || (j0 + kLanes * V - 1 > g.n) || (a < 1) || (b - 1 > g.n);
  ct m[T];
  bool bad = false;
  if (mask)
    blocked_tile<P, T, POIS, true>(g, tile, m, bad);
  else
    blocked_tile<P, T, POIS, false>(g, tile, m, bad);
  if (!ctl) return;
  double mx[T];
#pragma unroll
  for (int t = 0; t < T; ++t) mx[t] = wave_max((double)m[t]);
  report_pass<T>(ctl, sc, mx, T, bad, blockIdx.x % kSlots, gridDim.x);
}

// ---------------------------------------------------------------------------
// Work queue of the persistent batched kernels (see BQueue / BItem).
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long ld_acq(const unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish items (grid g, 0..ntiles-1) (whole wave).
__device__ inline void bq_publish(BQueue *q, BItem *ring, int g, int ntiles) {
  const int lane = threadIdx.x & 63;
  unsigned long long base = 0;
  if (lane == 0)
    base = __hip_atomic_fetch_add(&q->tail, (unsigned long long)ntiles,
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  base = __shfl(base, 0, 64);
  const unsigned long long gen = q->gen, mask = q->mask;
  for (int i = lane; i < ntiles; i += 64) {
    const unsigned long long idx = base + (unsigned long long)i;
    BItem *it = &ring[idx & mask];
    __hip_atomic_store(&it->payload, ((unsigned long long)g << 32) | (unsigned)i,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&it->tag, bq_tag(gen, idx), __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Take the next item.  Returns false when no grid has work left (or a wait
// exceeded the deadline, which raises q->error).  Every lane waits.
__device__ inline bool bq_take(BQueue *q, BItem *ring, int &g, int &tile) {
  const int lane = threadIdx.x & 63;
  unsigned long long idx = 0;
  if (lane == 0)
    idx = __hip_atomic_fetch_add(&q->head, 1ull, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
  idx = __shfl(idx, 0, 64);
  BItem *it = &ring[idx & q->mask];
  const unsigned long long want = bq_tag(q->gen, idx);
  const long long t0 = wall_clock64();
  for (;;) {
    if (ld_acq(&it->tag) == want) break;
    if (__hip_atomic_load(&q->remaining, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) <= 0)
      return false;
    if (__hip_atomic_load(&q->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return false;
    if (wall_clock64() - t0 > q->deadline_ticks) {
      if (lane == 0)
        __hip_atomic_fetch_or(&q->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(8);
  }
  const unsigned long long p = __hip_atomic_load(&it->payload, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
  g = (int)(p >> 32);
  tile = (int)(p & 0xffffffffu);
  return true;
}

// Host-side launch of the blocked pass for one (precision, T); each pair is
// instantiated in its own translation unit so the unrolled bodies compile in
// parallel.
template <int P, int T>
hipError_t launch_blocked_PT(const GridView &v, Ctl *ctl, const Sched &sc,
                             hipStream_t s) {
  const dim3 grid((unsigned)v.nstrips * (unsigned)v.nseg);
  if (v.F)
    hipLaunchKernelGGL((blocked_pass_kernel<P, T, true>), grid, dim3(64), 0, s,
                       v, ctl, sc);
  else
    hipLaunchKernelGGL((blocked_pass_kernel<P, T, false>), grid, dim3(64), 0, s,
                       v, ctl, sc);
  return hipGetLastError();
}

}  // namespace sor
