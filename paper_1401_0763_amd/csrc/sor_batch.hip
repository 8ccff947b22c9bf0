// Batched red-black SOR: many independent grids of different sizes, each
// with its own omega, tolerance and iteration limit, advanced by one
// persistent kernel (one wavefront per work item).
//
// Every grid follows Algorithm 1 of Mittal 2014 exactly as a single solve
// does (same blocked passes, same per-iteration maxima, same stopping rule
// and re-run of a truncated pass), so each grid's result is bit-identical to
// solving it alone, whatever else is in the batch.
#include "sor_kernels.h"

namespace sor {

// Depth of the next batched pass: the grid's depth, or what is left of a
// re-run or of the iteration limit.
__device__ __forceinline__ int batch_depth(long long left, int T) {
  return left < T ? (int)left : T;
}

// Grid g finished the pass whose tiles were queued: evaluate Algorithm 1's
// check for its iterations, then queue the next pass or retire the grid.
// Called by the whole wave that completed the pass's last tile.  Not inlined:
// merged into the kernel's loop it raises the kernel's register count enough
// to halve the resident wavefronts.
//
// The main kernel (TAIL false) runs only full passes of depth TM.  A grid
// whose next pass is shorter (a re-run up to an iteration inside the last
// pass, or the last iterations before max_iters) is parked: its pass goes to
// the tail queue (tq, tring), whose kernel runs after the main one and
// applies passes of any depth.
template <int P, int TM, bool TAIL>
__device__ __noinline__ void batch_grid_finish(BGrid *G, int g, BQueue *q, BItem *ring,
                                               BQueue *tq, BItem *tring) {
  const int lane = threadIdx.x & 63;
  const int T = G->pass_T;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  double it_max[kTMax];
#pragma unroll
  for (int t = 0; t < kTMax; ++t) {
    unsigned long long b = 0;
    if (lane < kBSlots && t < T) {
      b = __hip_atomic_load(&G->slots[lane][t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&G->slots[lane][t], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    it_max[t] = wave_max(__longlong_as_double((long long)b));
  }
  int next_T = 0;   // depth of the next pass, 0: retire the grid
  int nt = 0;       // its tiles
  if (lane == 0) {
    const unsigned nonf = __hip_atomic_load(&G->nonfinite, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    G->passes += 1;
    G->pass_budget -= 1;
    if (G->mode == 0) {
      const long long it0 = G->it_base;
      long long stop_at = 0;
      for (int t = 0; t < T; ++t) {
        const long long it = it0 + t + 1;
        if (stop_at == 0 && (it % G->check_every == 0 || it == G->max_iters)) {
          G->last_max = it_max[t];
          if (it_max[t] < G->tol) {
            stop_at = it;
            G->stop_iter = it;
            G->stop_max = it_max[t];
          }
        }
      }
      if (nonf) {
        G->status = 3;
        G->cur ^= 1;
        G->it_base = it0 + T;
        G->stop_iter = it0 + T;
      } else if (stop_at == it0 + T) {
        G->cur ^= 1;
        G->it_base = stop_at;
        G->status = 1;
      } else if (stop_at != 0) {
        // Met inside the pass: redo its first (stop_at - it0) iterations from
        // the pass input, which is still in place (grid `cur`).
        G->mode = 1;
        G->rerun_left = stop_at - it0;
        G->it_base = it0;
        next_T = batch_depth(G->rerun_left, G->T);
      } else {
        G->cur ^= 1;
        G->it_base = it0 + T;
        if (G->it_base >= G->max_iters) {
          G->status = 2;
          G->stop_iter = G->max_iters;
          G->stop_max = G->last_max;
        } else if (G->pass_budget <= 0) {
          G->status = 4;
        } else {
          next_T = batch_depth(G->max_iters - G->it_base, G->T);
        }
      }
    } else {
      G->cur ^= 1;
      G->it_base += T;
      G->rerun_left -= T;
      if (G->rerun_left <= 0) {
        G->status = 1;
        G->mode = 0;
      } else {
        next_T = batch_depth(G->rerun_left, G->T);
      }
    }
    if (next_T) {
      nt = blocked_ntiles(P, G->n, TM, G->seg_rows);
      G->pass_T = next_T;
      G->ntiles = nt;
    } else {
      G->t_done = wall_clock64();
    }
    __hip_atomic_store(&G->tiles_done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  next_T = __shfl(next_T, 0, 64);
  nt = __shfl(nt, 0, 64);
  const bool park = !TAIL && next_T != 0 && next_T < TM;
  if (park) {
    if (lane == 0) {
      __hip_atomic_fetch_add(&tq->remaining, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&q->remaining, -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    bq_publish(tq, tring, g, nt);
  } else if (next_T) {
    bq_publish(q, ring, g, nt);
  } else if (lane == 0) {
    __hip_atomic_fetch_add(&q->remaining, -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One tile of a pass of t_run (1..T) iterations (DYN; else exactly T), in
// the tile geometry of depth T (every pass of a grid has the same tiles).
template <int P, int T, bool POIS, bool DYN>
__device__ __forceinline__ void batch_tile(BGrid *G, int tile, int t_run,
                                           double (&mx)[kTMax], bool &bad) {
  using ct = typename PT<P>::ct;
  constexpr int V = PT<P>::V;
  constexpr int S = 2 * T;
  constexpr int A = ((S + V - 1) / V) * V;
  constexpr int CW = kLanes * V - 2 * A;
  GridView v;
  v.in = G->cur ? G->B : G->A;
  v.out = G->cur ? G->A : G->B;
  v.F = G->F;
  v.pitch = G->pitch;
  v.n = G->n;
  v.seg_rows = G->seg_rows;
  v.nstrips = (v.n + 1 + CW - 1) / CW;
  v.nseg = (v.n + 1 + v.seg_rows - 1) / v.seg_rows;
  v.omega = G->omega;
  ct m[T];
  // Tiles of this grid's next pass may run on other XCDs in this same launch.
  blocked_tile<P, T, POIS, kCohAgent, 0, DYN>(v, tile, m, bad, 2 * t_run);
#pragma unroll
  for (int t = 0; t < T; ++t) mx[t] = wave_max((double)m[t]);
}

// Persistent batched sweep: each wavefront takes items until no grid has work
// left.  Items of a grid's pass run in any order on any wavefront; the last
// one to finish closes the pass.  The main kernel has one tile body, of the
// fixed depth TM and with a source term (a grid without a source reads it as
// zero), which keeps the register count of a single pass kernel: a second
// body in the same kernel (another depth, or one without the source term),
// or a depth chosen at run time, costs it half its resident wavefronts.  The
// tail kernel (TAIL) applies the shorter passes of the parked grids with a
// run-time depth.
template <int P, int TM, bool POIS, bool TAIL>
__global__ __launch_bounds__(64) void batch_kernel(BGrid *grids, BQueue *q, BItem *ring,
                                                   BQueue *tq, BItem *tring) {
  const int lane = threadIdx.x & 63;
  if (lane == 0) {                          // launch start, for retire times
    long long zero = 0;
    __hip_atomic_compare_exchange_strong(&q->t0, &zero, (long long)wall_clock64(),
                                         __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
  }
  for (;;) {
    int g, tile;
    if (!bq_take(q, ring, g, tile)) return;
    BGrid *G = &grids[g];
    const int T = TAIL ? G->pass_T : TM;
    double mx[kTMax];
#pragma unroll
    for (int t = 0; t < kTMax; ++t) mx[t] = 0.0;
    bool bad = false;
    batch_tile<P, TM, POIS, TAIL>(G, tile, T, mx, bad);
    const bool anybad = __ballot(bad) != 0;
    unsigned prev = 0;
    if (lane == 0) {
      if (G->mode == 0) {
        const int slot = tile % kBSlots;
        for (int t = 0; t < T; ++t)
          __hip_atomic_fetch_max(&G->slots[slot][t],
                                 (unsigned long long)__double_as_longlong(mx[t]),
                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (anybad)
          __hip_atomic_fetch_or(&G->nonfinite, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      prev = count_item_done(&G->tiles_done);   // grid stores are device-scope
    }
    prev = __shfl(prev, 0, 64);
    if (prev == (unsigned)G->ntiles - 1) batch_grid_finish<P, TM, TAIL>(G, g, q, ring, tq, tring);
  }
}

// Pack every grid's caller arrays into its working grid A (and the ring into
// B), and F = h*h*f.  Block (x, y): allocated row x - kMY of grid y; the
// padding around the (n+2) x (n+2) grid is zeroed as well, since tile halos
// read it.
__global__ void batch_pack_kernel(BGrid *grids, int count) {
  BGrid &G = grids[blockIdx.y];
  const int n = G.n;
  const int r = (int)blockIdx.x - kMY;
  if (r > n + 1 + kMY) return;
  double *A = (double *)G.A, *B = (double *)G.B;
  double *F = (double *)G.F;
  const double h = 1.0 / (double)(n + 1);
  const double h2 = h * h;
  bool ok = true;
  for (int64_t ca = threadIdx.x; ca < G.pitch; ca += blockDim.x) {
    const int c = (int)ca - kMX;
    const bool in_r = r >= 1 && r <= n, in_c = c >= 1 && c <= n;
    double val = 0.0;
    if (in_r && in_c) val = G.user_u[(int64_t)(r - 1) * n + (c - 1)];
    else if (r == 0 && in_c) val = G.user_bdy[c - 1];
    else if (r == n + 1 && in_c) val = G.user_bdy[n + c - 1];
    else if (c == 0 && in_r) val = G.user_bdy[2 * n + r - 1];
    else if (c == n + 1 && in_r) val = G.user_bdy[3 * n + r - 1];
    const int64_t o = (int64_t)r * G.pitch + c;
    A[o] = val;
    if (!(in_r && in_c)) B[o] = val;
    ok = ok && __builtin_isfinite(val);
    if (F) {
      const double fv = (in_r && in_c) ? h2 * G.user_f[(int64_t)(r - 1) * n + (c - 1)] : 0.0;
      F[o] = fv;
      ok = ok && __builtin_isfinite(fv);
    }
  }
  if (!ok) G.nonfinite = 1u;      // sweeps detect only values turning non-finite
}

__global__ void batch_unpack_kernel(const BGrid *grids, int count) {
  const BGrid &G = grids[blockIdx.y];
  const int n = G.n;
  const int r = blockIdx.x + 1;
  if (r > n) return;
  const double *S = (const double *)(G.cur ? G.B : G.A);
  for (int c = threadIdx.x; c < n; c += blockDim.x)
    G.user_u[(int64_t)(r - 1) * n + c] = S[(int64_t)r * G.pitch + c + 1];
}

hipError_t launch_batch_pack(BGrid *grids, int count, int max_n, hipStream_t s) {
  hipLaunchKernelGGL(batch_pack_kernel, dim3(max_n + 2 + 2 * kMY, count), dim3(256), 0, s,
                     grids, count);
  return hipGetLastError();
}

hipError_t launch_batch_unpack(const BGrid *grids, int count, int max_n, hipStream_t s) {
  hipLaunchKernelGGL(batch_unpack_kernel, dim3(max_n, count), dim3(256), 0, s, grids, count);
  return hipGetLastError();
}

hipError_t launch_batch_f64(BGrid *grids, BQueue *q, BItem *ring, BQueue *tq, BItem *tring,
                            int waves, bool tail, hipStream_t s) {
  if (tail)
    hipLaunchKernelGGL((batch_kernel<kF64, kBatchT, true, true>), dim3(waves), dim3(64), 0, s,
                       grids, q, ring, tq, tring);
  else
    hipLaunchKernelGGL((batch_kernel<kF64, kBatchT, true, false>), dim3(waves), dim3(64), 0, s,
                       grids, q, ring, tq, tring);
  return hipGetLastError();
}

int batch_waves_per_cu_f64(bool tail) {
  int blocks = 0;
  const hipError_t e =
      tail ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                 &blocks, batch_kernel<kF64, kBatchT, true, true>, 64, 0)
           : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                 &blocks, batch_kernel<kF64, kBatchT, true, false>, 64, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 4;
  }
  // One persistent wavefront per SIMD at most (two ran the 512-grid batch
  // in 0.30 s against 0.237 s).
  return blocks > 0 ? (blocks < 4 ? blocks : 4) : 1;
}

}  // namespace sor
