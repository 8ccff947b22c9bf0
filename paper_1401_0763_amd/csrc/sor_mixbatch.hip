// Mixed-precision batched solves: FP64 defect correction (iterative
// refinement) around low-precision red-black SOR sweeps, for many grids in
// one persistent kernel.  Per grid the arithmetic is exactly that of
// sor_solve_mixed: r = b - A u in FP64, inner right-hand side fl(r * 2^p),
// a fixed number of red-black SOR iterations (Sec. 2.1 Eq. 1, Sec. 3.1) on
// the correction from zero, u += e * 2^-p.  Norm sums are formed per row
// block in a fixed order and then over row blocks in a fixed order, so a
// grid's result does not depend on the other grids of the batch.
#include "sor_kernels.h"

namespace sor {

__device__ __forceinline__ int mix_depth(long long left, int T) {
  return left < T ? (int)left : T;
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// FP64 residual r = (F + ((N + S) + (W + E))) - 4u and b = F + (boundary
// neighbours) at interior cell (i, j): the expressions of the residual kernel.
__device__ __forceinline__ void mix_resid_cell(const BMGrid &G, int i, int j,
                                               double &r, double &b) {
  const double *U = G.U;
  const int64_t p = G.pitch;
  const int64_t c = (int64_t)i * p + j;
  const double un = ld_agent(U + c - p), us = ld_agent(U + c + p);
  const double uw = ld_agent(U + c - 1), ue = ld_agent(U + c + 1);
  const double s = (un + us) + (uw + ue);
  const double t = G.F ? G.F[c] + s : s;
  r = t - 4.0 * ld_agent(U + c);
  const double nb = (i == 1) ? un : 0.0;
  const double sb = (i == G.n) ? us : 0.0;
  const double wb = (j == 1) ? uw : 0.0;
  const double eb = (j == G.n) ? ue : 0.0;
  const double bs = (nb + sb) + (wb + eb);
  b = G.F ? G.F[c] + bs : bs;
}

template <int PL>
__device__ __forceinline__ typename PT<PL>::st to_lo(double x) {
  const float v = (float)x;
  return (typename PT<PL>::st)v;
}

// One row block (rows 1 + t*kMixRows ...) of the RESID, CAST or ACCUM phase.
// Not inlined, like mix_finish: merged into the kernel's loop beside the tile
// body they raise its register count.
template <int PL>
__device__ __noinline__ void mix_rowblock(BMGrid *G, int t, int phase) {
  using st = typename PT<PL>::st;
  const int lane = threadIdx.x & 63;
  const int n = G->n;
  const int r0 = 1 + t * kMixRows;
  const int r1 = min(n, r0 + kMixRows - 1);
  const int pexp = G->scale_exp;
  const double inv = ldexp(1.0, -pexp);
  st *R = (st *)G->R;
  st *EA = (st *)G->EA;
  const st *E = (const st *)(G->cur ? G->EB : G->EA);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int i = r0; i <= r1; ++i) {
    for (int j = 1 + lane; j <= n; j += 64) {
      if (phase == kPhResid) {
        double r, b;
        mix_resid_cell(*G, i, j, r, b);
        a0 += r * r;
        a1 += b * b;
        a2 = fmax(a2, fabs(r));
      } else if (phase == kPhCast) {
        double r, b;
        mix_resid_cell(*G, i, j, r, b);
        const int64_t lc = (int64_t)i * G->lo_pitch + j;
        st_agent(R + lc, to_lo<PL>(ldexp(r, pexp)));
        st_agent(EA + lc, (st)0);
      } else {
        const int64_t lc = (int64_t)i * G->lo_pitch + j;
        const double corr = (double)(float)ld_agent(E + lc) * inv;
        const int64_t c = (int64_t)i * G->pitch + j;
        st_agent(G->U + c, ld_agent(G->U + c) + corr);
        a2 = fmax(a2, fabs(corr));
      }
    }
  }
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  a2 = wave_max(a2);
  if (lane == 0) {
    st_agent(G->partials + 3 * t + 0, a0);
    st_agent(G->partials + 3 * t + 1, a1);
    st_agent(G->partials + 3 * t + 2, a2);
  }
}

// One tile of a low-precision inner blocked pass of t_run (1..T) iterations
// (DYN; else exactly T) on the correction, in the tile geometry of depth T.
template <int PL, int T, bool DYN>
__device__ __forceinline__ bool mix_sweep_tile(BMGrid *G, int tile, int t_run) {
  using ct = typename PT<PL>::ct;
  constexpr int V = PT<PL>::V;
  constexpr int S = 2 * T;
  constexpr int A = ((S + V - 1) / V) * V;
  constexpr int CW = kLanes * V - 2 * A;
  GridView v;
  v.in = G->cur ? G->EB : G->EA;
  v.out = G->cur ? G->EA : G->EB;
  v.F = G->R;
  v.pitch = G->lo_pitch;
  v.n = G->n;
  v.seg_rows = G->seg_rows;
  v.nstrips = (v.n + 1 + CW - 1) / CW;
  v.nseg = (v.n + 1 + v.seg_rows - 1) / v.seg_rows;
  v.omega = G->omega;
  ct m[T];
  bool bad = false;
  // The next pass's tiles and the ACCUM phase may run on other XCDs in this
  // same launch.
  blocked_tile<PL, T, true, kCohAgent, 0, DYN>(v, tile, m, bad, 2 * t_run);
  return bad;
}

// Serial step after the last item of a phase (whole wave).
template <int PL>
__device__ __noinline__ void mix_finish(BMGrid *G, int g, BQueue *q, BItem *ring) {
  const int lane = threadIdx.x & 63;
  const int phase = G->phase;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (phase == kPhResid || phase == kPhAccum) {
    for (int k = lane; k < G->nrb; k += 64) {
      s0 += __hip_atomic_load(&G->partials[3 * k + 0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s1 += __hip_atomic_load(&G->partials[3 * k + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s2 = fmax(s2, __hip_atomic_load(&G->partials[3 * k + 2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    s2 = wave_max(s2);
  }
  int next = 0;        // 0: retire, 1: queue `nitems` items of the new phase
  int nitems = 0;
  if (lane == 0) {
    int done_status = 0;
    if (phase == kPhResid) {
      const double rel = s1 > 0.0 ? sqrt(s0) / sqrt(s1) : sqrt(s0);
      G->rel = rel;
      G->rinf = s2;
      if (!isfinite(rel)) done_status = 3;
      else if (rel <= G->rel_tol || s2 == 0.0) done_status = 1;
      else if (G->corr_tol > 0.0 && G->outer > 0 && G->last_corr < G->corr_tol) done_status = 1;
      else if (G->outer >= G->max_outer) done_status = 2;
      else {
        int e2;
        frexp(G->target / s2, &e2);
        G->scale_exp = e2 - 1;
        G->phase = kPhCast;
        nitems = G->nrb;
      }
    } else if (phase == kPhCast) {
      G->phase = kPhSweep;
      G->cur = 0;
      G->inner_left = G->inner_iters;
      G->pass_T = mix_depth(G->inner_left, G->T);
      nitems = blocked_ntiles(PL, G->n, kMixTMax, G->seg_rows);
    } else if (phase == kPhSweep) {
      G->passes += 1;
      G->cur ^= 1;
      G->inner_left -= G->pass_T;
      G->inner_total += G->pass_T;
      if (__hip_atomic_load(&G->nonfinite, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        done_status = 3;
      } else if (G->inner_left > 0) {
        G->pass_T = mix_depth(G->inner_left, G->T);
        nitems = blocked_ntiles(PL, G->n, kMixTMax, G->seg_rows);
      } else {
        G->phase = kPhAccum;
        nitems = G->nrb;
      }
    } else {
      G->last_corr = s2;
      G->outer += 1;
      G->phase = kPhResid;
      nitems = G->nrb;
    }
    if (done_status) {
      G->status = done_status;
    } else if (q->slice_ticks > 0 &&
               wall_clock64() - __hip_atomic_load(&q->t0, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT) > q->slice_ticks) {
      G->nitems = nitems;                // time slice over: status stays 0 and
                                         // the next launch queues these items
    } else {
      G->nitems = nitems;
      next = 1;
    }
    __hip_atomic_store(&G->items_done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  next = __shfl(next, 0, 64);
  nitems = __shfl(nitems, 0, 64);
  if (next) {
    bq_publish(q, ring, g, nitems);
  } else if (lane == 0) {
    __hip_atomic_fetch_add(&q->remaining, -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// DYN false: every inner pass has the full depth kMixTMax (each grid's inner
// iteration count is a multiple of it), one fixed tile body, two resident
// wavefronts per SIMD; DYN true: any inner count, passes of run-time depth,
// one resident wavefront per SIMD.
template <int PL, bool DYN>
__global__ __launch_bounds__(64) void mix_batch_kernel(BMGrid *grids, BQueue *q, BItem *ring) {
  const int lane = threadIdx.x & 63;
  if (lane == 0 && blockIdx.x == 0) {
    long long zero = 0;
    __hip_atomic_compare_exchange_strong(&q->t0, &zero, (long long)wall_clock64(),
                                         __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
  }
  for (;;) {
    int g, item;
    if (!bq_take(q, ring, g, item)) return;
    BMGrid *G = &grids[g];
    const int phase = G->phase;
    if (phase == kPhSweep) {
      const int T = DYN ? G->pass_T : kMixTMax;
      const bool bad = mix_sweep_tile<PL, kMixTMax, DYN>(G, item, T);
      if (__ballot(bad) != 0 && lane == 0)
        __hip_atomic_fetch_or(&G->nonfinite, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      mix_rowblock<PL>(G, item, phase);
    }
    unsigned prev = 0;
    if (lane == 0) prev = count_item_done(&G->items_done);   // grid data is device-scope
    prev = __shfl(prev, 0, 64);
    if (prev == (unsigned)G->nitems - 1) mix_finish<PL>(G, g, q, ring);
  }
}

// Pack the listed grids: U (and its ring), F = h*h*f, zero rings of EA, EB,
// R.  Block (x, y): allocated row x - kMY of listed grid y; the padding
// around each (n+2) x (n+2) grid is zeroed as well, since tile halos read it.
template <int PL>
__global__ void mix_pack_kernel(const BMGrid *grids, const int *slots, int count) {
  using st = typename PT<PL>::st;
  const BMGrid &G = grids[slots[blockIdx.y]];
  const int n = G.n;
  const int r = (int)blockIdx.x - kMY;
  if (r > n + 1 + kMY) return;
  const double h = 1.0 / (double)(n + 1);
  const double h2 = h * h;
  double *F = const_cast<double *>(G.F);
  const bool in_r = r >= 1 && r <= n;
  for (int64_t ca = threadIdx.x; ca < G.pitch; ca += blockDim.x) {
    const int c = (int)ca - kMX;
    const bool in_c = c >= 1 && c <= n;
    double val = 0.0;
    if (in_r && in_c) val = G.user_u[(int64_t)(r - 1) * n + (c - 1)];
    else if (r == 0 && in_c) val = G.user_bdy[c - 1];
    else if (r == n + 1 && in_c) val = G.user_bdy[n + c - 1];
    else if (c == 0 && in_r) val = G.user_bdy[2 * n + r - 1];
    else if (c == n + 1 && in_r) val = G.user_bdy[3 * n + r - 1];
    G.U[(int64_t)r * G.pitch + c] = val;
    if (F) F[(int64_t)r * G.pitch + c] = (in_r && in_c) ? h2 * G.user_f[(int64_t)(r - 1) * n + (c - 1)] : 0.0;
  }
  for (int64_t ca = threadIdx.x; ca < G.lo_pitch; ca += blockDim.x) {
    const int c = (int)ca - kMX;
    if (in_r && c >= 1 && c <= n) continue;
    const int64_t lc = (int64_t)r * G.lo_pitch + c;
    ((st *)G.EA)[lc] = (st)0;
    ((st *)G.EB)[lc] = (st)0;
    ((st *)G.R)[lc] = (st)0;
  }
}

__global__ void mix_unpack_kernel(const BMGrid *grids, const int *slots, int count) {
  const BMGrid &G = grids[slots[blockIdx.y]];
  const int n = G.n;
  const int r = blockIdx.x + 1;
  if (r > n) return;
  for (int c = threadIdx.x; c < n; c += blockDim.x)
    G.user_u[(int64_t)(r - 1) * n + c] = G.U[(int64_t)r * G.pitch + c + 1];
}

hipError_t launch_mix_pack(int prec_lo, const BMGrid *grids, const int *slots, int count,
                           int max_n, hipStream_t s) {
  if (prec_lo == kF32)
    hipLaunchKernelGGL(mix_pack_kernel<kF32>, dim3(max_n + 2 + 2 * kMY, count), dim3(256), 0, s, grids,
                       slots, count);
  else
    hipLaunchKernelGGL(mix_pack_kernel<kF16>, dim3(max_n + 2 + 2 * kMY, count), dim3(256), 0, s, grids,
                       slots, count);
  return hipGetLastError();
}

hipError_t launch_mix_unpack(const BMGrid *grids, const int *slots, int count, int max_n,
                             hipStream_t s) {
  hipLaunchKernelGGL(mix_unpack_kernel, dim3(max_n, count), dim3(256), 0, s, grids, slots,
                     count);
  return hipGetLastError();
}

hipError_t launch_mix_batch(int prec_lo, bool dyn, BMGrid *grids, BQueue *q, BItem *ring,
                            int waves, hipStream_t s) {
  if (prec_lo == kF32 && !dyn)
    hipLaunchKernelGGL((mix_batch_kernel<kF32, false>), dim3(waves), dim3(64), 0, s, grids, q, ring);
  else if (prec_lo == kF32)
    hipLaunchKernelGGL((mix_batch_kernel<kF32, true>), dim3(waves), dim3(64), 0, s, grids, q, ring);
  else if (!dyn)
    hipLaunchKernelGGL((mix_batch_kernel<kF16, false>), dim3(waves), dim3(64), 0, s, grids, q, ring);
  else
    hipLaunchKernelGGL((mix_batch_kernel<kF16, true>), dim3(waves), dim3(64), 0, s, grids, q, ring);
  return hipGetLastError();
}

int mix_waves_per_cu(int prec_lo, bool dyn) {
  int blocks = 0;
  hipError_t e;
  if (prec_lo == kF32 && !dyn)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, mix_batch_kernel<kF32, false>, 64, 0);
  else if (prec_lo == kF32)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, mix_batch_kernel<kF32, true>, 64, 0);
  else if (!dyn)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, mix_batch_kernel<kF16, false>, 64, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, mix_batch_kernel<kF16, true>, 64, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 4;
  }
  // One persistent wavefront per SIMD at most: with two (the FP32 kernel
  // fits two once its neighbour exchange moved to DPP) the 512-grid batch
  // took 0.231 s against 0.211 s, more waves waiting for items.
  return blocks > 0 ? (blocks < 4 ? blocks : 4) : 1;
}

}  // namespace sor
