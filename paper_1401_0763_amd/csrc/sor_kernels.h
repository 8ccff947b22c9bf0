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

#include <limits>
#include <type_traits>

// Rows a wavefront loads ahead of the row it is updating.
#ifndef SOR_PREFETCH
#define SOR_PREFETCH 4
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


// The value of x in the adjacent lane (DPP wave shift by one lane: CTRL
// kDppWaveShr1 reads lane i-1, kDppWaveShl1 lane i+1; the lane at the end
// of the wave reads 0).  A 64-bit value moves as two 32-bit halves.  The
// compiler keeps the wait state a DPP read needs after a vector write.
constexpr int kDppWaveShr1 = 0x138;
constexpr int kDppWaveShl1 = 0x130;
template <int CTRL>
__device__ __forceinline__ float lane_shift(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

__device__ __forceinline__ float vabs(float x) { return fabsf(x); }
__device__ __forceinline__ double vabs(double x) { return fabs(x); }
__device__ __forceinline__ float vmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ float vfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double vfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ double vmax(double a, double b) { return fmax(a, b); }
// High 32 bits of a double's bit pattern, all 32 of a float's.
__device__ __forceinline__ unsigned high_bits(double x) { return (unsigned)__double2hiint(x); }
__device__ __forceinline__ unsigned high_bits(float x) { return __float_as_uint(x); }

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
// the slots for the next pass.  last_formed is false for a pass that formed
// no maximum for its last iteration: a non-finite grid then reports NaN as
// its change.
template <int T>
__device__ __forceinline__ void report_pass(Ctl *ctl, const Sched &sc,
                                            const double (&mx)[T], int t_run,
                                            bool bad, int slot,
                                            unsigned waves_total,
                                            bool last_formed = true) {
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
    // The finishing wave reads only the slots and the flag, which are
    // device-scope atomics: waiting for them to complete orders them before
    // the counter.  An agent-scope release here would write back this XCD's
    // whole L2 once per wave; the grid itself is published at the kernel's
    // end.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    prev = __hip_atomic_fetch_add(&ctl->counter, 1u, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  }
  prev = __shfl(prev, 0, 64);
  if (prev != waves_total - 1) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

  // Last wave of the pass: gather the slots (lane s reads slot s).
  double it_max[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    // Relaxed: the fence above already acquired (an acquire load would
    // invalidate the XCD's L2 once per slot).
    unsigned long long b = __hip_atomic_load(&ctl->slots[lane][t], __ATOMIC_RELAXED,
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
      if (stop == 1 && ctl->stop_iter < it0 + t_run) {
        // The rule was met at an iteration inside the pass, and some cell is
        // non-finite by the pass's end: whether it already was at the
        // stopping iteration is decided by the truncated re-run.
        ctl->stop_tentative = 1;
      } else {
        stop = 2;
        ctl->stop_iter = it0 + t_run;
        ctl->stop_max = last_formed ? it_max[t_run - 1] : __builtin_nan("");
      }
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

// Cache policy of the sweep's grid accesses.  kCohDefault: cached in the
// XCD's L2 (visibility to other XCDs comes with the kernel's end).  kCohAgent:
// device-scope loads and stores (the form of relaxed agent-scope atomic
// accesses), for kernels whose wavefronts read, in the same launch, cells
// that wavefronts on other XCDs wrote.
constexpr int kCohDefault = 0;
constexpr int kCohAgent = 16;      // SC1

template <int P, int AUX = kCohDefault>
__device__ __forceinline__ Vec<P> buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff,
                                           unsigned soff) {
  if constexpr (sizeof(Vec<P>) == 16) {
    return __builtin_bit_cast(Vec<P>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, AUX));
  } else {
    return __builtin_bit_cast(Vec<P>, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, AUX));
  }
}

// The store's SGPR offset field is the constant 0 and the row offset goes
// into the per-lane offset (the sum stays below 2^32, and a lane whose
// offset carries kDrop stays beyond the extent).  A store of more than 8
// bytes reads its data registers after it issues, so a vector instruction
// that overwrites them at once needs a wait state between the two; the
// compiler inserts it only when the SGPR offset is not a register.  With a
// register there, the register allocator reused a dead data register for
// the next instruction's result right behind the store, and at 4096^2
// some stored cells got a wrong low word, in different cells from run to
// run.
template <int P, int AUX = kCohDefault>
__device__ __forceinline__ void buf_store(const Vec<P> &x, __amdgpu_buffer_rsrc_t r,
                                          unsigned voff, unsigned soff) {
  const int off = (int)(voff + soff);
  if constexpr (sizeof(Vec<P>) == 16) {
    using v4 = unsigned __attribute__((ext_vector_type(4)));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4, x), r, off, 0, AUX);
  } else {
    using v2 = unsigned __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2, x), r, off, 0, AUX);
  }
}

// Stage pipelines of the blocked tile by ordering: red-black (0) and
// block-parallel red-black (3; 4 for blocks of even width) apply 2
// half-sweeps per iteration; the four-colour ordering (1) 3 (colour 0,
// colours 1 and 2, colour 3); Jacobi (2) one sweep of every cell from the
// previous iterate.  The row halo is the stage count rounded up to even, so
// a tile's first loaded row keeps the parity of its first core row.  The
// register window holds the stage rows, their neighbours and the
// SOR_PREFETCH rows loaded ahead, rounded up to even; the row walk runs in
// chunks of that many steps.
__host__ __device__ constexpr int order_stages(int ord, int T) {
  return (ord == 0 || ord >= 3 ? 2 : ord == 1 ? 3 : 1) * T;
}
__host__ __device__ constexpr int order_row_halo(int ord, int T) {
  return (order_stages(ord, T) + 1) / 2 * 2;
}
__host__ __device__ constexpr int order_window_rows(int ord, int T) {
  return ((order_stages(ord, T) + SOR_PREFETCH + 2) + 1) / 2 * 2;
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
// rotating register window.
//
// All stages of one step update cells of the same parity v0 within a lane,
// and the one neighbour that lies in the adjacent lane (left of cell 0 when
// v0 = 0, right of cell V-1 when v0 = 1) is a cell that stage k-1 updated one
// step earlier and that no stage has written since (stage 0: a cell of the
// newly loaded row).  Each stage reads it straight from the adjacent lane's
// window register with a DPP wave shift (lane_shift), a vector move that
// needs no LDS; the block-parallel stages read an old value the same way
// from the adjacent lane's ob1.  (An earlier form sent every edge value
// through the LDS crossbar as it was made, 2 permutes per stage, which
// bounded the pass.)
//
// Values near the strip and segment edges depend on cells outside the tile
// and are wrong after enough stages (the dependency cone grows one cell per
// half-sweep), so the tile loads a halo of A >= S columns and H >= S rows on
// each side and stores only its core (CW columns x seg_rows rows).  Input and
// output are separate grids (ping-pong), so halos are read at the pass's
// starting level whatever order tiles run in.
//
// The other orderings (ORD, FP64 only) run the same walk, window, halo and
// stores with their own stage lists; they are described where they branch
// off below.  The block-parallel ordering (3) is the red-black pipeline in
// which a black cell takes a red neighbour that lies in another block (of
// bs.rows x bs.cols interior cells) at its value before this
// iteration's red half-sweep: each red stage keeps the values it overwrites
// for the two steps in which the next stage can still need them, and sends
// the old edge value across lanes beside the new one.  The dependency cone
// is the red-black one (a black cell's update reaches two cells back into
// the previous iterate), so the halo is unchanged.  With blocks of even
// width (ordering 4) every column edge falls between the two cells of one
// lane (blocks start at odd columns, lanes at even ones), so no old value
// crosses lanes and one flag per lane says whether its pair is split.
//
// One branch-free body serves every tile.  Boundary and out-of-grid cells
// must keep their value; they get a relaxation factor of 0 instead of omega
// (u + 0*(g - u) = u for finite g): per lane for columns, and per window slot
// for rows, where each slot also carries the weight (1 for core rows, 0 for
// halo rows) of its changes in the maxima.  Loads read a clamped row (always
// inside the tile's rows) and stores of non-core rows are dropped through an
// out-of-range offset.
//
// m[t] receives the largest |u' - u| of iteration t over the tile's core
// cells (0 in halo lanes).  MX (red-black only) names the iterations whose
// maxima are formed: -1 all of them, 0..T-1 that one alone, T none; the
// stopping rule reads only the maxima of check iterations, and a pass
// holds at most one of them when the check interval is at least T, so the
// change, its weight and the running maximum (three of the update's eight
// vector instructions) are left out of the other iterations.  m[t] of an
// iteration left out stays 0.
//
// bad is set when an interior core cell is not finite at the end of the
// pass.  Non-finite values are absorbing for interior cells (an infinite
// cell's next update is inf - inf or NaN, and a NaN stays NaN), so a cell
// that turns non-finite at any iteration of the pass is non-finite when its
// row is stored.  The maxima are no test for it: the max drops NaN (made
// from finite operands as +inf + -inf), and a change can overflow between
// two finite values, which Algorithm 1 counts as an ordinary large change.
// Non-finite inputs are caught when they are packed.
//
// DYN (red-black only): the tile has the geometry of depth T but applies only
// the first s_run (even, 2..2T) half-sweeps, i.e. s_run/2 iterations; the
// others are skipped by a wave-uniform branch, and m[t] stays 0 for the
// iterations not applied.  The halo sized for T covers any smaller depth, so
// the core cells get exactly the s_run/2-iteration result.
// ---------------------------------------------------------------------------
template <int P, int T, bool POIS, int COH = kCohDefault, int ORD = 0, bool DYN = false,
          int MX = -1>
__device__ __forceinline__ void blocked_tile(const GridView &g, int tile,
                                             typename PT<P>::ct (&m)[T],
                                             bool &bad, int s_run = 2 * T,
                                             const BlockShape bs = BlockShape{}) {
  using st = typename PT<P>::st;
  using ct = typename PT<P>::ct;
  constexpr int V = PT<P>::V;
  static_assert(ORD == 0 || P == kF64, "other orderings are instantiated for FP64");
  static_assert(!DYN || ORD == 0, "a run-time depth is implemented for red-black passes");
  static_assert(ORD < 3 || PT<P>::V == 2, "block-parallel passes hold one red cell per lane");
  static_assert(MX == -1 || (ORD == 0 && !DYN && MX >= 0 && MX <= T),
                "maxima of selected iterations are implemented for fixed-depth red-black passes");
  constexpr int S = order_stages(ORD, T);        // stages (half-sweeps or colour sweeps)
  constexpr int H = order_row_halo(ORD, T);      // halo rows (even)
  constexpr int A = ((S + V - 1) / V) * V;
  constexpr int WV = kLanes * V;
  constexpr int CW = WV - 2 * A;
  constexpr int D = SOR_PREFETCH;                // rows prefetched ahead
  constexpr int W = order_window_rows(ORD, T);   // window rows (even)
  constexpr int ESZ = (int)sizeof(st);

  const int lane = threadIdx.x & 63;
  const int n = g.n;
  const int strip = tile % g.nstrips;
  const int seg = tile / g.nstrips;
  const int j0 = strip * CW - A;                 // first column of the strip
  const int col0 = j0 + lane * V;                // even: parity below is static
  const int a = seg * g.seg_rows - H;            // first loaded row (even)
  const int core0 = seg * g.seg_rows;
  const int core1 = min(core0 + g.seg_rows, n + 1);
  const int b = core1 + H;                       // one past the last loaded row
  const int rlo = max(core0, 1);
  const int rhi = min(core1, n + 1);
  const bool lane_core = (lane * V >= A) && (lane * V < WV - A);
  const bool lane_store = lane_core && (col0 <= n) && (col0 + V - 1 >= 1);
  ct omc[V];                                     // omega, or 0 off the interior
#pragma unroll
  for (int v = 0; v < V; ++v)
    omc[v] = (col0 + v >= 1 && col0 + v <= n) ? (ct)g.omega : (ct)0;
  const unsigned rowbytes = (unsigned)(g.pitch * ESZ);
  const unsigned extent = (unsigned)(b - a) * rowbytes;     // < 2^31
  const int64_t tile_off = (int64_t)a * g.pitch + j0;
  const auto rin = make_rsrc((const st *)g.in + tile_off, extent);
  const auto rout = make_rsrc((st *)g.out + tile_off, extent);
  // A null source reads as zeros (a resource of no records returns 0 for
  // every load).  Adding +0 changes the neighbour sum only when it is -0, and
  // then the update still gives the same value and change (0.25 * s - u is
  // -u, or a zero whose sign the relaxation step loses), so a Laplace grid
  // gets the same bits through this path as through the one without a source.
  __amdgpu_buffer_rsrc_t rf;
  if constexpr (POIS)
    rf = g.F ? make_rsrc((const st *)g.F + tile_off, extent) : make_rsrc(g.in, 0u);
  const unsigned lane_off = (unsigned)(lane * V * ESZ);
  const unsigned st_off = lane_store ? lane_off : kDrop;
  // Non-finite test of the stored interior cells: the largest high word (sign
  // cleared) of their bit patterns is at least that of infinity exactly when
  // one of them is an infinity or a NaN; integer operations, two per cell.
  unsigned fmask[V];                             // 0x7fffffff on interior cells
#pragma unroll
  for (int v = 0; v < V; ++v) fmask[v] = (lane_store && omc[v] != (ct)0) ? 0x7fffffffu : 0u;
  unsigned fhi = 0;
  // Block-parallel: per cell of this lane, whether its west (bx_w) or east
  // (bx_e) neighbour lies in another block; per window slot (bit), whether
  // the row's north (rx_n) or south (rx_s) neighbour does.  Cells and rows
  // off the interior never change, so their flags do not matter.
  constexpr bool BP = ORD == 3 || ORD == 4;
  constexpr bool BPE = ORD == 4;                 // even block width
  bool bx_w[V], bx_e[V];
  bool bx_in = false;                            // BPE: a block edge splits this lane's pair
  unsigned hx_in = 0u, hx_w[V] = {}, hx_e[V] = {};   // the same flags as all-ones masks
  unsigned rx_n = 0, rx_s = 0;
  int rib = 0;                                   // (row - 1) mod blk_rows of the next load
  if constexpr (BP) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int c = col0 + v;
      bx_w[v] = c >= 2 && c <= n && (c - 1) % bs.cols == 0;
      bx_e[v] = c >= 1 && c < n && c % bs.cols == 0;
    }
    bx_in = bx_e[0];
    hx_in = bx_in ? 0xffffffffu : 0u;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      hx_w[v] = bx_w[v] ? 0xffffffffu : 0u;
      hx_e[v] = bx_e[v] ? 0xffffffffu : 0u;
    }
    rib = ((a - 1) % bs.rows + bs.rows) % bs.rows;
  }

  ct w[W][V];                                    // row window
  ct fw[POIS ? W : 1][V];                        // h*h*f of the window rows
  ct wc[W];                                      // slot weight in the maxima
  ct wr[W];                                      // 1 for interior rows, else 0
#pragma unroll
  for (int s = 0; s < W; ++s) {
    wc[s] = (ct)0;
    wr[s] = (ct)0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      w[s][v] = (ct)0;
      if constexpr (POIS) fw[s][v] = (ct)0;
    }
  }
#pragma unroll
  for (int t = 0; t < T; ++t) m[t] = (ct)0;

  // Row rn (clamped to the tile) into window slot SP, with its attributes.
  auto load_row = [&](int rn, auto SP) __attribute__((always_inline)) {
    constexpr int sp = decltype(SP)::value;
    if constexpr (MX < 0 || P != kF64) wc[sp] = (rn >= rlo && rn < rhi) ? (ct)1 : (ct)0;
    wr[sp] = (rn >= 1 && rn <= n) ? (ct)1 : (ct)0;
    if constexpr (BP) {
      const unsigned bit = 1u << sp;
      rx_n = (rn >= 2 && rn <= n && rib == 0) ? (rx_n | bit) : (rx_n & ~bit);
      rx_s = (rn >= 1 && rn < n && rib == bs.rows - 1) ? (rx_s | bit) : (rx_s & ~bit);
      rib = rib + 1 == bs.rows ? 0 : rib + 1;
    }
    const unsigned soff = (unsigned)(min(rn, b - 1) - a) * rowbytes;
    const Vec<P> x = buf_load<P, COH>(rin, lane_off, soff);
#pragma unroll
    for (int v = 0; v < V; ++v) w[sp][v] = (ct)x.v[v];
    if constexpr (POIS) {
      const Vec<P> y = buf_load<P, COH>(rf, lane_off, soff);
#pragma unroll
      for (int v = 0; v < V; ++v) fw[sp][v] = (ct)y.v[v];
    }
  };
  // Prologue: rows a .. a+D+1 into slots 0 .. D+1 (b - a >= 2S + 1 > D + 2).
  static_for<0, D + 2>([&](auto SP) __attribute__((always_inline)) {
    load_row(a + decltype(SP)::value, SP);
  });

  // Block-parallel: the red values that red stage t overwrote this step
  // (ob0), one step earlier (ob1) and two steps earlier (ob2); an old value
  // in the adjacent lane is that lane's ob1.
  constexpr int TB = BP ? T : 1;
  ct ob0[TB], ob1[TB], ob2[TB];
#pragma unroll
  for (int t = 0; t < TB; ++t) {
    ob0[t] = ob1[t] = ob2[t] = (ct)0;
  }
  // Jacobi: every stage needs the row above its row at its own input level
  // (pv), which the stage itself overwrote one step earlier.
  constexpr int SJ = ORD == 2 ? S : 1;
  ct pv[SJ][V];
#pragma unroll
  for (int k = 0; k < SJ; ++k) {
#pragma unroll
    for (int v = 0; v < V; ++v) pv[k][v] = (ct)0;
  }
  if constexpr (ORD == 2) {
#pragma unroll
    for (int v = 0; v < V; ++v) pv[0][v] = w[0][v];
  }

  // Wait here for the prologue's loads.  The loop head joins
  // this path with the loop's back edge; without the wait the compiler takes
  // the prologue's most recent load as pending there and drains the memory
  // queue at the head of every chunk instead of once per tile.
  __builtin_amdgcn_s_waitcnt(0x0070);   // vmcnt(0) lgkmcnt(0)
  // Steps r = a+1 .. b-2 in chunks of W, so window slots are static.
  const int nsteps = b - a - 2;
  for (int base = 0; base < nsteps; base += W) {
    static_for<0, W>([&](auto I) __attribute__((always_inline)) {
      constexpr int i = decltype(I)::value;
      const int r = a + 1 + base + i;
      load_row(r + D + 1, std::integral_constant<int, (i + D + 2) % W>{});
      // Cells of colour k&1 in this lane at stage k: (q + col0 + v + k) even,
      // and q + k = r has the parity of 1 + i because a, base and W are even.
      constexpr int v0 = (1 + i) & 1;
      if constexpr (ORD == 0 || BP) {
      if constexpr (BP) {
#pragma unroll
        for (int t = 0; t < T; ++t) {
          ob2[t] = ob1[t];
          ob1[t] = ob0[t];
        }
      }
      // Stage k (half-sweep k) on row r-k.
      static_for<0, S>([&](auto K) __attribute__((always_inline)) {
        constexpr int k = decltype(K)::value;
        constexpr int sq = ((i + 1 - k) % W + W) % W;
        constexpr int su = (sq + W - 1) % W;
        constexpr int sd = (sq + 1) % W;
        if (!DYN || k == 0 || k < s_run) {
        static_for<0, V / 2>([&](auto JV) __attribute__((always_inline)) {
          constexpr int v = v0 + 2 * decltype(JV)::value;
          const ct self = w[sq][v];
          // The neighbour in the adjacent lane is that lane's edge cell of
          // the same row, which stage k-1 updated one step earlier and no
          // stage has written since; a DPP wave shift reads it from there
          // at the point of use.
          ct left = v == 0 ? lane_shift<kDppWaveShr1>(w[sq][V - 1]) : w[sq][v == 0 ? 0 : v - 1];
          ct right = v == V - 1 ? lane_shift<kDppWaveShl1>(w[sq][0])
                                : w[sq][v == V - 1 ? 0 : v + 1];
          ct up = w[su][v], down = w[sd][v];
          if constexpr (BP && (k & 1)) {
            // Black half-sweep of iteration k/2: a red neighbour in another
            // block at its value before this iteration's red half-sweep (row
            // above: kept two steps ago, row below: this step, same row: one
            // step ago in this lane or sent from the adjacent one).
            constexpr int t = k >> 1;
            // The selects are bit-field inserts on the values' bit patterns
            // with 32-bit all-ones or zero masks (uniform for rows, per lane
            // for columns): selects on the conditions kept a 64-bit lane mask
            // per condition in SGPRs, and their spills cost more (the pass
            // runs 6-9 % faster this way).
            auto pick = [](ct a, ct b, unsigned mk) __attribute__((always_inline)) {
              const unsigned long long ab = __double_as_longlong(a), bb = __double_as_longlong(b);
              const unsigned long long m = ((unsigned long long)mk << 32) | mk;
              return __longlong_as_double((long long)((ab & m) | (bb & ~m)));
            };
            const unsigned mn = 0u - ((rx_n >> sq) & 1u), ms = 0u - ((rx_s >> sq) & 1u);
            up = pick(ob2[t], up, mn);
            down = pick(ob0[t], down, ms);
            if constexpr (BPE) {
              if constexpr (v == 0) right = pick(ob1[t], right, hx_in);
              else left = pick(ob1[t], left, hx_in);
            } else {
              left = pick(v == 0 ? lane_shift<kDppWaveShr1>(ob1[t]) : ob1[t], left, hx_w[v]);
              right = pick(v == V - 1 ? lane_shift<kDppWaveShl1>(ob1[t]) : ob1[t], right,
                           hx_e[v]);
            }
          }
          if constexpr (BP && !(k & 1)) {
            ob0[k >> 1] = self;
          }
          ct s = (up + down) + (left + right);
          if constexpr (POIS) s = s + fw[sq][v];
          const ct dg = vfma((ct)0.25, s, -self);      // Gauss-Seidel value - self
          // Eq. 1 with one rounding; with binary16 storage the step is rounded
          // to float (product, then sum) before the storage rounding, since a
          // fused multiply-add feeding that rounding becomes one mixed-
          // precision instruction that rounds once, straight to binary16.
          ct nu;
          if constexpr (P == kF16) nu = self + (omc[v] * wr[sq]) * dg;
          else nu = vfma(omc[v] * wr[sq], dg, self);
          if constexpr (P == kF16) nu = (ct)(st)nu;
          w[sq][v] = nu;
          if constexpr (MX < 0 || (k >> 1) == MX) {
            const ct d = vabs(nu - self);
            if constexpr (MX < 0 || P != kF64) {
              m[k >> 1] = vmax(m[k >> 1], d * wc[sq]);
            } else {
              // One maximum per FP64 pass: the row's weight is formed where
              // it is used (two stages per step) instead of kept per window
              // slot, which saves the slots' SGPRs (0.8 % of the 7-deep
              // pass).  Not for FP32: its 7-deep Poisson pass would then fit
              // two wavefronts per SIMD, and the tiles sized for two ran the
              // inner sweeps of the mixed solve at 1400 against 1580 GLUP/s.
              const int q = r - k;
              const ct wq = ((unsigned)(q - rlo) < (unsigned)(rhi - rlo)) ? (ct)1 : (ct)0;
              m[k >> 1] = vmax(m[k >> 1], d * wq);
            }
          }
        });
        }
        // No instruction moves across a stage.  A schedule that let
        // arithmetic cross this barrier once gave results that differed
        // from the oracle's after hundreds of iterations on a large grid;
        // the store-data wait state (buf_store) was missing then, and that
        // schedule was not tried again.
        __builtin_amdgcn_sched_barrier(0);
      });
      } else if constexpr (ORD == 1) {
      // Four-colour ordering: stage k is colour sweep k mod 3 of iteration
      // k/3 (colour 0 = even row and column, then colours 1 and 2 = the
      // black cells, then colour 3 = odd row and column).  Row q = r-k has
      // the static parity of 1+i-k; the cells a stage updates in this lane
      // have the static parity vpar(k, q) (none for colour 0 on odd rows and
      // colour 3 on even rows).  Stage k+1 takes the same row at the next
      // step, so the edge cell it needs from the adjacent lane is that lane's
      // cell as stage k left it; it is read from that lane's register (DPP
      // wave shift) at the point of use.
      auto vpar = [](int k, int pq) constexpr {
        const int c = k % 3;
        return c == 0 ? (pq == 0 ? 0 : -1) : c == 1 ? ((pq + 1) & 1) : (pq == 1 ? 1 : -1);
      };
      static_for<0, S>([&](auto K) __attribute__((always_inline)) {
        constexpr int k = decltype(K)::value;
        constexpr int sq = ((i + 1 - k) % W + W) % W;
        constexpr int su = (sq + W - 1) % W;
        constexpr int sd = (sq + 1) % W;
        constexpr int pq = ((1 + i - k) % 2 + 2) % 2;
        constexpr int vp = vpar(k, pq);
        if constexpr (vp >= 0) {
          static_for<0, V / 2>([&](auto JV) __attribute__((always_inline)) {
            constexpr int v = vp + 2 * decltype(JV)::value;
            const ct self = w[sq][v];
            const ct left = v == 0 ? lane_shift<kDppWaveShr1>(w[sq][V - 1])
                                   : w[sq][v == 0 ? 0 : v - 1];
            const ct right = v == V - 1 ? lane_shift<kDppWaveShl1>(w[sq][0])
                                        : w[sq][v == V - 1 ? 0 : v + 1];
            ct s = (w[su][v] + w[sd][v]) + (left + right);
            if constexpr (POIS) s = s + fw[sq][v];
            const ct dg = vfma((ct)0.25, s, -self);
            ct nu = vfma(omc[v] * wr[sq], dg, self);
            const ct d = vabs(nu - self);
            w[sq][v] = nu;
            m[k / 3] = vmax(m[k / 3], d * wc[sq]);
          });
        }
        __builtin_amdgcn_sched_barrier(0);
      });
      } else {
      // Jacobi: stage k is iteration k and updates every cell of row r-k
      // from level k of the rows above (pv[k]), at (its own, before any
      // write) and below (just updated by stage k-1), and of the cells in
      // the neighbouring lanes, which stage k-1 wrote one step earlier and
      // which are read from those lanes' registers (DPP wave shifts) before
      // this stage writes its own.
      static_for<0, S>([&](auto K) __attribute__((always_inline)) {
        constexpr int k = decltype(K)::value;
        constexpr int sq = ((i + 1 - k) % W + W) % W;
        constexpr int sd = (sq + 1) % W;
        ct nw[V];
        static_for<0, V>([&](auto VV) __attribute__((always_inline)) {
          constexpr int v = decltype(VV)::value;
          const ct self = w[sq][v];
          const ct left = v == 0 ? lane_shift<kDppWaveShr1>(w[sq][V - 1])
                                 : w[sq][v == 0 ? 0 : v - 1];
          const ct right = v == V - 1 ? lane_shift<kDppWaveShl1>(w[sq][0])
                                      : w[sq][v == V - 1 ? 0 : v + 1];
          ct s = (pv[k][v] + w[sd][v]) + (left + right);
          if constexpr (POIS) s = s + fw[sq][v];
          const ct dg = vfma((ct)0.25, s, -self);
          nw[v] = vfma(omc[v] * wr[sq], dg, self);
          m[k] = vmax(m[k], vabs(nw[v] - self) * wc[sq]);
        });
#pragma unroll
        for (int v = 0; v < V; ++v) {
          pv[k][v] = w[sq][v];
          w[sq][v] = nw[v];
        }
        __builtin_amdgcn_sched_barrier(0);
      });
      }
      // Row r-S+1 has had all S half-sweeps: store it if it is a core row.
      constexpr int so = ((i + 2 - S) % W + W) % W;
      const int qo = r - S + 1;
      const bool row_ok = (qo >= rlo) && (qo < rhi);
      Vec<P> x;
#pragma unroll
      for (int v = 0; v < V; ++v) x.v[v] = (st)w[so][v];
      buf_store<P, COH>(x, rout, st_off | (row_ok ? 0u : kDrop),
                   row_ok ? (unsigned)(qo - a) * rowbytes : 0u);
      const unsigned rmask = row_ok ? 0xffffffffu : 0u;
#pragma unroll
      for (int v = 0; v < V; ++v) fhi = max(fhi, high_bits(w[so][v]) & fmask[v] & rmask);
    });
  }
  bad = bad | (fhi >= high_bits(std::numeric_limits<ct>::infinity()));
#pragma unroll
  for (int t = 0; t < T; ++t)
    if (!lane_core) m[t] = (ct)0;
}

// One blocked pass over a whole grid: one wavefront per tile, T iterations
// from g.in into g.out.  With a control block, the pass first exits if an
// earlier pass met the stopping rule, then reports its maxima.
template <int P, int T, bool POIS, int ORD, int MX = -1>
__device__ __forceinline__ void blocked_pass_body(const GridView &g, Ctl *ctl,
                                                  const Sched &sc,
                                                  const BlockShape bs = BlockShape{}) {
  if (ctl && ctl_stopped(ctl)) return;
  using ct = typename PT<P>::ct;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  ct m[T];
  bool bad = false;
  blocked_tile<P, T, POIS, kCohDefault, ORD, false, MX>(g, tile, m, bad, 2 * T, bs);
  if (!ctl) return;
  double it_max[T];
#pragma unroll
  for (int t = 0; t < T; ++t)
    it_max[t] = (MX < 0 || t == MX) ? wave_max((double)m[t]) : 0.0;
  report_pass<T>(ctl, sc, it_max, T, bad, blockIdx.x % kSlots, gridDim.x,
                 MX < 0 || MX == T - 1);
}

// Red-black passes.  MX selects the iterations whose maxima are formed (-1
// all, 0..T-1 that one, T none); the host launches the variant that forms
// exactly those the stopping rule will read.
template <int P, int T, bool POIS, int MX = -1>
__global__ __launch_bounds__(64) void blocked_pass_kernel(GridView g, Ctl *ctl,
                                                          Sched sc) {
  blocked_pass_body<P, T, POIS, 0, MX>(g, ctl, sc);
}

// Four-colour passes.
template <int P, int T, bool POIS>
__global__ __launch_bounds__(64) void blocked_pass_c4_kernel(GridView g, Ctl *ctl,
                                                             Sched sc) {
  blocked_pass_body<P, T, POIS, 1>(g, ctl, sc);
}

// Jacobi passes.
template <int P, int T, bool POIS>
__global__ __launch_bounds__(64) void blocked_pass_jacobi_kernel(GridView g, Ctl *ctl,
                                                                 Sched sc) {
  blocked_pass_body<P, T, POIS, 2>(g, ctl, sc);
}

// Block-parallel passes (blocks of bs; of even width: the _even kernel).
template <int P, int T, bool POIS>
__global__ __launch_bounds__(64) void blocked_pass_bp_kernel(GridView g, Ctl *ctl,
                                                             Sched sc, BlockShape bs) {
  blocked_pass_body<P, T, POIS, 3>(g, ctl, sc, bs);
}
template <int P, int T, bool POIS>
__global__ __launch_bounds__(64) void blocked_pass_bp_even_kernel(GridView g, Ctl *ctl,
                                                                  Sched sc, BlockShape bs) {
  blocked_pass_body<P, T, POIS, 4>(g, ctl, sc, bs);
}

// Device-scope scalar loads and stores (relaxed agent-scope atomics, i.e.
// accesses that bypass a stale or dirty copy in one XCD's L2), for grid data
// that persistent kernels hand from one wavefront to another in one launch.
__device__ __forceinline__ double ld_agent(const double *p) {
  return __longlong_as_double(__hip_atomic_load(reinterpret_cast<const long long *>(p),
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_agent(double *p, double v) {
  __hip_atomic_store(reinterpret_cast<long long *>(p), __double_as_longlong(v),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_agent(const float *p) {
  return __int_as_float(__hip_atomic_load(reinterpret_cast<const int *>(p),
                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_agent(float *p, float v) {
  __hip_atomic_store(reinterpret_cast<int *>(p), __float_as_int(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ _Float16 ld_agent(const _Float16 *p) {
  return __builtin_bit_cast(_Float16, __hip_atomic_load(reinterpret_cast<const short *>(p),
                                                        __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_agent(_Float16 *p, _Float16 v) {
  __hip_atomic_store(reinterpret_cast<short *>(p), __builtin_bit_cast(short, v),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Count one finished work item whose device-scope stores must be visible to
// the wave that sees the count complete: wait for them, then a relaxed
// increment (an agent-scope release would also write back this XCD's L2).
__device__ __forceinline__ unsigned count_item_done(unsigned *counter) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  return __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Work queue of the persistent batched kernels (see BQueue / BItem).
// ---------------------------------------------------------------------------

// Publish items (grid g, 0..ntiles-1) (whole wave).
__device__ inline void bq_publish(BQueue *q, BItem *ring, int g, int ntiles) {
  const int lane = threadIdx.x & 63;
  unsigned long long base = 0;
  if (lane == 0)
    base = __hip_atomic_fetch_add(&q->tail, (unsigned long long)ntiles,
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  base = __shfl(base, 0, 64);
  const unsigned long long gen = q->gen, mask = q->mask;
  // Every payload, then one release fence, then every tag: a release store
  // per item would write back the XCD's L2 once per 64 items.
  for (int i = lane; i < ntiles; i += 64) {
    const unsigned long long idx = base + (unsigned long long)i;
    __hip_atomic_store(&ring[idx & mask].payload, ((unsigned long long)g << 32) | (unsigned)i,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  for (int i = lane; i < ntiles; i += 64) {
    const unsigned long long idx = base + (unsigned long long)i;
    __hip_atomic_store(&ring[idx & mask].tag, bq_tag(gen, idx), __ATOMIC_RELAXED,
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
  // Poll with relaxed loads and acquire once the item is there: an acquire
  // load at agent scope invalidates the XCD's L2 each time, which a waiting
  // wave would otherwise do on every poll, under the working waves' feet.
  // Waits back off from about 0.2 us to about 3 us between polls.
  int naps = 1;
  for (;;) {
    if (__hip_atomic_load(&it->tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == want) break;
    if (__hip_atomic_load(&q->remaining, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <= 0)
      return false;
    if (__hip_atomic_load(&q->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return false;
    if (wall_clock64() - t0 > q->deadline_ticks) {
      if (lane == 0)
        __hip_atomic_fetch_or(&q->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    for (int k = 0; k < naps; ++k) __builtin_amdgcn_s_sleep(8);
    naps = naps < 16 ? 2 * naps : 16;
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const unsigned long long p = __hip_atomic_load(&it->payload, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
  // The item is the same in every lane: keep it in scalar registers, so the
  // grid record and everything derived from it stay wave-uniform.
  g = __builtin_amdgcn_readfirstlane((int)(p >> 32));
  tile = __builtin_amdgcn_readfirstlane((int)(p & 0xffffffffu));
  return true;
}

// The pass kernel of an ordering (for the launchers below).
template <int P, int T, bool POIS, int ORD, int MX = -1> struct PassKernel {
  static constexpr auto k = blocked_pass_kernel<P, T, POIS, MX>;
};
template <int P, int T, bool POIS> struct PassKernel<P, T, POIS, 1> {
  static constexpr auto k = blocked_pass_c4_kernel<P, T, POIS>;
};
template <int P, int T, bool POIS> struct PassKernel<P, T, POIS, 2> {
  static constexpr auto k = blocked_pass_jacobi_kernel<P, T, POIS>;
};
template <int P, int T, bool POIS> struct PassKernel<P, T, POIS, 3> {
  static constexpr auto k = blocked_pass_bp_kernel<P, T, POIS>;
};
template <int P, int T, bool POIS> struct PassKernel<P, T, POIS, 4> {
  static constexpr auto k = blocked_pass_bp_even_kernel<P, T, POIS>;
};

// Host-side launch of the blocked pass for one (precision, T, ordering,
// maxima selection); each is instantiated in its own translation unit so
// the unrolled bodies compile in parallel.
template <int P, int T, int ORD = 0, int MX = -1>
hipError_t launch_blocked_PT(const GridView &v, Ctl *ctl, const Sched &sc,
                             hipStream_t s, const BlockShape &bs = BlockShape{}) {
  static_assert(MX == -1 || ORD == 0, "maxima selection is a red-black variant");
  const dim3 grid((unsigned)v.nstrips * (unsigned)v.nseg);
  if constexpr (ORD >= 3) {
    if (v.F)
      hipLaunchKernelGGL((PassKernel<P, T, true, ORD>::k), grid, dim3(64), 0, s, v, ctl, sc, bs);
    else
      hipLaunchKernelGGL((PassKernel<P, T, false, ORD>::k), grid, dim3(64), 0, s, v, ctl, sc, bs);
  } else {
    if (v.F)
      hipLaunchKernelGGL((PassKernel<P, T, true, ORD, MX>::k), grid, dim3(64), 0, s, v, ctl, sc);
    else
      hipLaunchKernelGGL((PassKernel<P, T, false, ORD, MX>::k), grid, dim3(64), 0, s, v, ctl, sc);
  }
  return hipGetLastError();
}

// Wavefronts of the pass kernel (one per workgroup) that one CU holds at once.
template <int P, int T, int ORD = 0, int MX = -1>
int blocked_blocks_per_cu(bool pois) {
  int nb = 0;
  const hipError_t e =
      pois ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                 &nb, reinterpret_cast<const void *>(PassKernel<P, T, true, ORD, MX>::k), 64, 0)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                 &nb, reinterpret_cast<const void *>(PassKernel<P, T, false, ORD, MX>::k), 64, 0);
  return e == hipSuccess ? nb : 0;
}

}  // namespace sor
