// Host side of batched solves and of the tiling autotuner (C ABI in
// include/sor.h).
//
// A batch is laid out in one device arena (each grid's padded A and B grids
// and its h*h*f grid), described by an array of BGrid records, and advanced by
// one persistent kernel fed from a device ring buffer of (grid, tile) items.
// The upload / pack / persistent kernel / unpack / download sequence is
// captured once as a HIP graph and replayed while the batch shapes repeat
// (the graph reads the descriptors from pinned host staging buffers, so new
// caller pointers and parameters take effect on every replay).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <vector>

#include "sor_host.h"

namespace sor {

struct BatchState {
  hipStream_t stream = nullptr;          // internal stream (graph capture)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  BGrid *h_grids = nullptr;              // pinned staging
  size_t h_grids_cap = 0;
  BQueue *h_queue = nullptr;
  BItem *h_items = nullptr;
  size_t h_items_cap = 0;
  unsigned long long gen = 0;
  long long wall_khz = 0;
  hipGraphExec_t exec = nullptr;
  std::vector<long long> sig;            // shapes the graph was recorded for
  std::vector<double> done_ms;           // retire time of each grid of the last
                                         // batched FP64 solve (ms after launch start)
  // size class -> tiling, per precision: autotuner results for plain solves
  // (sor_autotune) and for grids inside batched launches (sor_autotune_batch)
  std::map<int, sor_tiling> tune[3];
  std::map<int, sor_tiling> tune_batch[3];
};

void batch_state_free(sor_ctx *c) {
  BatchState *b = c->batch;
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->h_grids) (void)hipHostFree(b->h_grids);
  if (b->h_queue) (void)hipHostFree(b->h_queue);
  if (b->h_items) (void)hipHostFree(b->h_items);
  delete b;
  c->batch = nullptr;
}

// Size class of a grid side: nearest half power of two (so 64, 90, 128, ...).
int size_class(int n) { return (int)std::lround(2.0 * std::log2((double)std::max(n, 1))); }

sor_tiling batch_tiling(sor_ctx *c, int prec, int n) {
  if (c->batch) {
    auto &m = c->batch->tune_batch[prec];
    auto it = m.find(size_class(n));
    if (it != m.end()) return it->second;
  }
  sor_tiling t = c->tiling[prec];
  if (prec == kF64) {
    // Depth-kBatchT tiles, one wavefront per SIMD: the batch autotuner's
    // choices on the 512-grid workload were 96-192 rows below n = 512 and
    // 384 from n = 512 on.
    if (t.seg_rows == 0) t.seg_rows = n < 512 ? 128 : 384;
    return t;
  }
  // Mixed inner sweeps: passes of the context's depth (6 unless set, the
  // persistent kernel's fixed depth), tiles as for FP64.
  if (t.seg_rows == 0) t.seg_rows = n < 512 ? 128 : 384;
  return t;
}

int auto_seg_rows(sor_ctx *c, int prec, int n, int T, bool pois, int ord) {
  if (c->cus <= 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) !=
            hipSuccess || cus <= 0)
      cus = 256;
    c->cus = cus;
  }
  int &occ = ord ? c->occ_var[ord][T][pois ? 1 : 0] : c->occ[prec][T][pois ? 1 : 0];
  if (occ <= 0) occ = std::max(1, blocked_blocks_per_cu(prec, T, pois, ord));
  const BlockGeom gm = block_geom(prec, T, ord);
  const long long strips = (n + 1 + gm.CW - 1) / gm.CW;
  // Resident wavefronts, counted at most two per SIMD: passes that fit three
  // measured faster with the taller tiles of the two-per-SIMD count.
  const long long slots = (long long)std::min(occ, 8) * c->cus;
  // At least 2S rows: on grids too small to fill the device, more and shorter
  // tiles measured faster than fewer tiles with relatively less halo.
  const int lo = 2 * gm.S, hi = 768;
  int seg = hi;
  for (int k = 1; k <= 64; ++k) {
    const long long segs = std::max(1LL, k * slots / strips);
    seg = (int)((n + 1 + segs - 1) / segs);
    if (seg <= hi) break;
  }
  seg = std::min(hi, std::max(lo, seg));
  // A tile walks seg + 2H - 2 steps in chunks of W: round seg up so that the
  // last chunk is full (fewer tiles, none of their steps wasted).
  const int over = (seg + 2 * gm.H - 2) % gm.W;
  if (over) seg += gm.W - over;
  return std::min(1024, seg + (seg & 1));
}

int auto_depth(sor_ctx *c, int prec, bool pois) {
  // FP64 and FP32: 7, which measured ahead of 6 (and 8) for Laplace and
  // Poisson problems alike.  Binary16 storage: 7 where its 7-deep pass keeps
  // two wavefronts on each of the CU's 4 SIMDs, else 6.
  if (prec != kF16) return 7;
  int &occ = c->occ[prec][7][pois ? 1 : 0];
  if (occ <= 0) occ = std::max(1, blocked_blocks_per_cu(prec, 7, pois));
  return occ >= 2 * 4 ? 7 : 6;
}

sor_tiling tuned_tiling(sor_ctx *c, int prec, int n, bool pois) {
  if (c->batch) {
    auto &m = c->batch->tune[prec];
    auto it = m.find(size_class(n));
    if (it != m.end()) return it->second;
  }
  sor_tiling t = c->tiling[prec];
  if (c->depth_auto[prec]) t.iters_per_pass = auto_depth(c, prec, pois);
  if (t.seg_rows == 0) t.seg_rows = auto_seg_rows(c, prec, n, t.iters_per_pass, pois);
  return t;
}

void clear_tuning(sor_ctx *c, int prec) {
  if (c->batch) {
    c->batch->tune[prec].clear();
    c->batch->tune_batch[prec].clear();
  }
}

namespace {

sor_status batch_state(sor_ctx *c, BatchState **out) {
  if (!c->batch) {
    BatchState *b = new (std::nothrow) BatchState;
    if (!b) return fail(c, SOR_ENOMEM, "out of host memory");
    c->batch = b;
    HIP_TRY(c, hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    HIP_TRY(c, hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
    HIP_TRY(c, hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    HIP_TRY(c, hipHostMalloc((void **)&b->h_queue, 2 * sizeof(BQueue), hipHostMallocDefault));
    int khz = 0;
    HIP_TRY(c, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device));
    b->wall_khz = khz > 0 ? khz : 100000;
  }
  *out = c->batch;
  return SOR_OK;
}

template <typename T>
sor_status host_grow(sor_ctx *c, T **p, size_t *cap, size_t need) {
  if (*cap >= need) return SOR_OK;
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  *cap = 0;
  size_t n = std::max(need, *cap * 2);
  HIP_TRY(c, hipHostMalloc((void **)p, n * sizeof(T), hipHostMallocDefault));
  *cap = n;
  return SOR_OK;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace
}  // namespace sor

using namespace sor;

extern "C" {

sor_status sor_batch_solve_f64(sor_ctx *c, const sor_grid_desc *grids, int32_t count,
                               void *stream, sor_result *results) {
  if (!c) return SOR_EINVAL;
  c->err.clear();
  if (!grids || !results || count < 1) return fail(c, SOR_EINVAL, "need grids, results and count >= 1");
  HIP_TRY(c, hipSetDevice(c->device));
  for (int g = 0; g < count; ++g) {
    const sor_grid_desc &d = grids[g];
    sor_status st = check_common(c, d.u, d.boundary, d.rhs, d.n, d.omega);
    if (st != SOR_OK) return fail(c, st, "grid %d: %s", g, c->err.c_str());
    if (!(d.tol >= 0.0) || d.max_iters < 1 || d.check_every < 1)
      return fail(c, SOR_EINVAL, "grid %d: tol, max_iters or check_every invalid", g);
  }
  BatchState *bs = nullptr;
  sor_status st = batch_state(c, &bs);
  if (st != SOR_OK) return st;

  // Arena layout, tilings and work estimates.  Every grid runs in one
  // persistent kernel of fixed depth kBatchT (queue 0), followed by a tail
  // kernel (queue 1) for the passes shorter than that depth.
  std::vector<Layout> lay(count);
  std::vector<size_t> offA(count), offB(count), offF(count);
  std::vector<int> seg(count);
  size_t arena = 0;
  long long items[2] = {0, 0}, max_items = 0;
  int ngrids[2] = {0, 0};
  int max_n = 0;
  for (int g = 0; g < count; ++g) {
    const int n = grids[g].n;
    lay[g] = make_layout(n, kF64);
    const size_t bytes = align_up((size_t)lay[g].elems() * sizeof(double), 256);
    offA[g] = arena; arena += bytes;
    offB[g] = arena; arena += bytes;
    if (grids[g].rhs) { offF[g] = arena; arena += bytes; }
    seg[g] = batch_tiling(c, kF64, n).seg_rows;
    const int nt = blocked_ntiles(kF64, n, kBatchT, seg[g]);
    const int q = grids[g].max_iters < kBatchT ? 1 : 0;      // first pass short: tail
    items[q] += nt;
    ngrids[q] += 1;
    max_items += nt;
    max_n = std::max(max_n, n);
  }
  const long long total_items = items[0] + items[1];
  // Ring capacity per queue: every grid has at most one pass queued, plus one
  // slot per waiting wavefront; doubled and rounded to a power of two.
  int cus = 0;
  HIP_TRY(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
  int waves[2];
  unsigned long long cap[2];
  for (int q = 0; q < 2; ++q) {
    waves[q] = std::max(1, cus) * batch_waves_per_cu_f64(q == 1);
    cap[q] = 1024;
    while (cap[q] < 2ull * (unsigned long long)(max_items + waves[q]) + 1024) cap[q] <<= 1;
  }

  if ((st = ensure(c, kBatchArena, arena)) ||
      (st = ensure(c, kBatchGrids, sizeof(BGrid) * (size_t)count)) ||
      (st = ensure(c, kBatchQueue, 2 * sizeof(BQueue))) ||
      (st = ensure(c, kBatchRing, sizeof(BItem) * (cap[0] + cap[1]))))
    return st;
  if ((st = host_grow(c, &bs->h_grids, &bs->h_grids_cap, (size_t)count)) ||
      (st = host_grow(c, &bs->h_items, &bs->h_items_cap, (size_t)std::max(1LL, total_items))))
    return st;

  char *base = (char *)c->bufs[kBatchArena].p;
  for (int g = 0; g < count; ++g) {
    const sor_grid_desc &d = grids[g];
    BGrid &G = bs->h_grids[g];
    std::memset(&G, 0, sizeof(BGrid));
    const size_t org = (size_t)lay[g].origin_off() * sizeof(double);
    G.A = base + offA[g] + org;
    G.B = base + offB[g] + org;
    G.F = d.rhs ? base + offF[g] + org : nullptr;
    G.user_u = d.u;
    G.user_bdy = d.boundary;
    G.user_f = d.rhs;
    G.pitch = lay[g].pitch;
    G.n = d.n;
    G.T = kBatchT;
    G.seg_rows = seg[g];
    G.omega = d.omega;
    G.tol = d.tol;
    G.max_iters = d.max_iters;
    G.check_every = d.check_every;
    G.pass_budget = LLONG_MAX;
    G.pass_T = (int)std::min<long long>(d.max_iters, kBatchT);
    G.ntiles = blocked_ntiles(kF64, d.n, kBatchT, G.seg_rows);
    G.last_max = NAN;
  }
  // Initial queues: pass 0 of every grid, largest expected work first (work
  // grows like n^3 at the optimal omega) so the longest chains start first.
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return grids[x].n > grids[y].n; });
  const unsigned long long gen = ++bs->gen & 0xffffffull;
  unsigned long long idx[2] = {0, 0};
  BItem *hit[2] = {bs->h_items, bs->h_items + items[0]};
  for (int g : order) {
    const BGrid &G = bs->h_grids[g];
    const int q = G.pass_T < G.T ? 1 : 0;
    for (int t = 0; t < G.ntiles; ++t, ++idx[q]) {
      hit[q][idx[q]].tag = bq_tag(gen, idx[q]);
      hit[q][idx[q]].payload = ((unsigned long long)g << 32) | (unsigned)t;
    }
  }
  for (int q = 0; q < 2; ++q) {
    BQueue &Q = bs->h_queue[q];
    std::memset(&Q, 0, sizeof(BQueue));
    Q.head = 0;
    Q.tail = idx[q];
    Q.gen = gen;
    Q.mask = cap[q] - 1;
    Q.remaining = ngrids[q];
    Q.error = 0;
    Q.deadline_ticks = bs->wall_khz * 1000ll * 20;   // 20 s without progress
  }

  BGrid *dG = (BGrid *)c->bufs[kBatchGrids].p;
  BQueue *dQ = (BQueue *)c->bufs[kBatchQueue].p;
  BItem *dR[2] = {(BItem *)c->bufs[kBatchRing].p, (BItem *)c->bufs[kBatchRing].p + cap[0]};
  const std::vector<long long> sig = {
      count, items[0], items[1], max_n, waves[0], waves[1], (long long)cap[0],
      (long long)cap[1], (long long)(uintptr_t)base, (long long)(uintptr_t)dG,
      (long long)(uintptr_t)dQ, (long long)(uintptr_t)dR[0],
      (long long)(uintptr_t)bs->h_grids, (long long)(uintptr_t)bs->h_queue,
      (long long)(uintptr_t)bs->h_items};
  bool record = !(bs->exec && bs->sig == sig);
  hipStream_t s = bs->stream;
  HIP_TRY(c, hipEventRecord(bs->ev_in, (hipStream_t)stream));
  HIP_TRY(c, hipStreamWaitEvent(s, bs->ev_in, 0));
  if (record) {
    if (bs->exec) { (void)hipGraphExecDestroy(bs->exec); bs->exec = nullptr; }
    hipGraph_t graph = nullptr;
    HIP_TRY(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    auto step = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    step(hipMemcpyAsync(dG, bs->h_grids, sizeof(BGrid) * count, hipMemcpyHostToDevice, s));
    step(hipMemcpyAsync(dQ, bs->h_queue, 2 * sizeof(BQueue), hipMemcpyHostToDevice, s));
    for (int q = 0; q < 2; ++q)
      if (items[q])
        step(hipMemcpyAsync(dR[q], hit[q], sizeof(BItem) * items[q], hipMemcpyHostToDevice, s));
    step(launch_batch_pack(dG, count, max_n, s));
    if (ngrids[0])
      step(launch_batch_f64(dG, dQ, dR[0], dQ + 1, dR[1], waves[0], false, s));
    step(launch_batch_f64(dG, dQ + 1, dR[1], dQ + 1, dR[1], waves[1], true, s));
    step(launch_batch_unpack(dG, count, max_n, s));
    step(hipMemcpyAsync(bs->h_grids, dG, sizeof(BGrid) * count, hipMemcpyDeviceToHost, s));
    step(hipMemcpyAsync(bs->h_queue, dQ, 2 * sizeof(BQueue), hipMemcpyDeviceToHost, s));
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(c, SOR_EDEVICE, "graph capture failed: %s",
                  hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(&bs->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      bs->exec = nullptr;
      return fail(c, SOR_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
    }
    bs->sig = sig;
  }
  HIP_TRY(c, hipGraphLaunch(bs->exec, s));
  HIP_TRY(c, hipEventRecord(bs->ev_out, s));
  HIP_TRY(c, hipStreamWaitEvent((hipStream_t)stream, bs->ev_out, 0));
  HIP_TRY(c, hipStreamSynchronize(s));

  for (int q = 0; q < 2; ++q)
    if (bs->h_queue[q].error) return fail(c, SOR_ETIMEOUT, "a queue wait exceeded its bound");
  sor_status overall = SOR_OK;
  bs->done_ms.assign(count, NAN);
  long long t0 = 0;                       // start of the first persistent launch
  for (int k = 0; k < 2; ++k)
    if (bs->h_queue[k].t0 > 0 && (t0 == 0 || bs->h_queue[k].t0 < t0)) t0 = bs->h_queue[k].t0;
  for (int g = 0; g < count; ++g) {
    const BGrid &G = bs->h_grids[g];
    if (G.t_done > 0 && t0 > 0)
      bs->done_ms[g] = (double)(G.t_done - t0) / (double)bs->wall_khz;
    sor_result &r = results[g];
    r = sor_result{};
    r.rel_residual = NAN;
    r.passes = G.passes;
    r.iterations = G.status == 2 ? G.max_iters : G.stop_iter;
    r.final_max_delta = G.stop_max;
    r.converged = G.status == 1;
    switch (G.status) {
      case 1: r.status = SOR_OK; break;
      case 2: r.status = SOR_NOT_CONVERGED; break;
      case 3: r.status = SOR_ENONFINITE; break;
      default: r.status = SOR_EDEVICE; break;
    }
    if (r.status == SOR_ENONFINITE) overall = SOR_ENONFINITE;
    else if (r.status == SOR_EDEVICE && overall >= 0) overall = SOR_EDEVICE;
    else if (r.status == SOR_NOT_CONVERGED && overall == SOR_OK) overall = SOR_NOT_CONVERGED;
  }
  if (overall == SOR_EDEVICE) return fail(c, SOR_EDEVICE, "a grid did not finish");
  return overall;
}

sor_status sor_batch_last_times(const sor_ctx *c, int32_t count, double *done_ms) {
  if (!c || !done_ms || count < 0) return SOR_EINVAL;
  const std::vector<double> *v = c->batch ? &c->batch->done_ms : nullptr;
  if (!v || (size_t)count != v->size()) return SOR_EINVAL;
  for (int g = 0; g < count; ++g) done_ms[g] = (*v)[g];
  return SOR_OK;
}

sor_status sor_autotune(sor_ctx *c, int32_t bits, int32_t n, sor_tiling *best) {
  if (!c) return SOR_EINVAL;
  c->err.clear();
  const int prec = prec_index(bits);
  if (prec != kF64 && prec != kF32) return fail(c, SOR_EINVAL, "bits must be 64 or 32");
  if (n < 1 || n > kMaxN) return fail(c, SOR_EINVAL, "n = %d outside 1..%d", n, kMaxN);
  HIP_TRY(c, hipSetDevice(c->device));
  BatchState *bs = nullptr;
  sor_status st = batch_state(c, &bs);
  if (st != SOR_OK) return st;
  const Layout L = make_layout(n, prec);
  const size_t bytes = (size_t)L.elems() * (size_t)prec_bytes(prec);
  const BufRole ra = prec == kF64 ? kGridA64 : kGridA32;
  const BufRole rb = prec == kF64 ? kGridB64 : kGridB32;
  if ((st = ensure(c, ra, bytes)) || (st = ensure(c, rb, bytes))) return st;
  char *A = (char *)c->bufs[ra].p + L.origin_off() * prec_bytes(prec);
  char *B = (char *)c->bufs[rb].p + L.origin_off() * prec_bytes(prec);
  hipStream_t s = bs->stream;
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  const Sched sc{1, 1, 0.0};
  sor_tiling bt = tuned_tiling(c, prec, n, false);
  double best_t = INFINITY;
  hipError_t e = hipSuccess;
  for (int T : {1, 2, 3, 4, 5, 6, 7, 8}) {
    for (int seg : {16, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768}) {
      if (seg > 2 * (n + 1) && seg != 16) continue;
      GridView v;
      v.in = A; v.out = B; v.F = nullptr; v.pitch = L.pitch; v.n = n;
      v.seg_rows = seg; v.omega = 1.5;
      const BlockGeom gm = block_geom(prec, T);
      v.nstrips = (n + 1 + gm.CW - 1) / gm.CW;
      v.nseg = (n + 1 + seg - 1) / seg;
      const int reps = 3;
      // Timed as a solve's passes run: forming the maxima of one iteration.
      const int mx = T - 1;
      if (e == hipSuccess) e = launch_blocked_pass(prec, T, v, nullptr, sc, s, 0, {}, mx);
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      for (int k = 0; k < reps && e == hipSuccess; ++k) {
        std::swap(v.in, *(const void **)&v.out);
        e = launch_blocked_pass(prec, T, v, nullptr, sc, s, 0, {}, mx);
      }
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) break;
      const double per_iter = ms / (reps * T);
      if (per_iter < best_t) {
        best_t = per_iter;
        bt.iters_per_pass = T;
        bt.seg_rows = seg;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(c, SOR_EDEVICE, "autotune: %s", hipGetErrorString(e));
  bs->tune[prec][size_class(n)] = bt;
  if (best) *best = bt;
  return SOR_OK;
}

sor_status sor_autotune_batch(sor_ctx *c, int32_t bits, int32_t n, sor_tiling *best) {
  if (!c) return SOR_EINVAL;
  c->err.clear();
  const int prec = prec_index(bits);
  if (prec < 0) return fail(c, SOR_EINVAL, "bits must be 64, 32 or 16");
  if (n < 8 || n > 8192) return fail(c, SOR_EINVAL, "n = %d outside 8..8192", n);
  HIP_TRY(c, hipSetDevice(c->device));
  BatchState *bs = nullptr;
  sor_status st = batch_state(c, &bs);
  if (st != SOR_OK) return st;
  // A batch of G identical grids, enough for about 16384 tiles at 4
  // iterations per pass and 64-row tiles (a queue as deep as in a large
  // mixed batch, where tile count matters less than halo per tile), capped
  // at 256 grids and 1 GiB.
  const BlockGeom g4 = block_geom(prec, 4);
  const long long tiles = (long long)((n + 1 + g4.CW - 1) / g4.CW) * ((n + 1 + 63) / 64);
  long long G = std::max(1LL, std::min(256LL, (16384 + tiles - 1) / tiles));
  G = std::max(1LL, std::min(G, (long long)((1ull << 30) / ((size_t)n * n * 8 * 3))));
  const size_t cells = (size_t)n * n;
  double *u = nullptr, *bdy = nullptr;
  if (hipMalloc(&u, sizeof(double) * cells * G) != hipSuccess ||
      hipMalloc(&bdy, sizeof(double) * 4 * n) != hipSuccess) {
    (void)hipGetLastError();
    if (u) (void)hipFree(u);
    return fail(c, SOR_ENOMEM, "autotune_batch: cannot allocate %lld grids of side %d", G, n);
  }
  std::vector<double> hb(4 * (size_t)n, 1.0);
  hipError_t he = hipMemcpy(bdy, hb.data(), sizeof(double) * 4 * n, hipMemcpyHostToDevice);
  const double omega = omega_opt(n);
  const int iters = 96;                                 // passes may end short
  std::vector<sor_grid_desc> gd((size_t)G);
  std::vector<sor_mixed_desc> md((size_t)G);
  for (long long g = 0; g < G; ++g) {
    gd[g] = sor_grid_desc{u + cells * g, bdy, nullptr, n, 0, omega, 0.0, iters, iters};
    md[g] = sor_mixed_desc{u + cells * g, bdy, nullptr, n, 0, omega, 0.0, 0.0, 1, iters};
  }
  std::vector<sor_result> res((size_t)G);
  auto &table = bs->tune_batch[prec];
  const int cls = size_class(n);
  const auto saved = table.find(cls) != table.end() ? table[cls] : sor_tiling{0, 0};
  sor_tiling bt{4, 64};
  double best_t = INFINITY;
  // Batched passes have a fixed depth (FP64) or run fastest at the
  // persistent kernel's fixed depth (mixed inner sweeps): only the tile
  // height is searched.
  const std::vector<int> depths{prec == kF64 ? kBatchT : kMixTMax};
  for (int T : depths) {
    for (int seg : {16, 32, 48, 64, 96, 128, 192, 256, 384}) {
      if (he != hipSuccess) break;
      if (seg > 2 * (n + 1) && seg != 16) continue;
      table[cls] = sor_tiling{T, seg};
      double tmin = INFINITY;
      for (int rep = 0; rep < 3; ++rep) {              // first run records the graph
        if (hipMemset(u, 0, sizeof(double) * cells * G) != hipSuccess) { he = hipErrorUnknown; break; }
        const auto t0 = std::chrono::steady_clock::now();
        const sor_status s2 =
            prec == kF64 ? sor_batch_solve_f64(c, gd.data(), (int32_t)G, nullptr, res.data())
                         : sor_batch_solve_mixed(c, md.data(), (int32_t)G, bits, nullptr, res.data());
        const auto t1 = std::chrono::steady_clock::now();
        if (s2 < 0) { he = hipErrorUnknown; break; }
        if (rep > 0) tmin = std::min(tmin, std::chrono::duration<double>(t1 - t0).count());
      }
      if (tmin < best_t) {
        best_t = tmin;
        bt = sor_tiling{T, seg};
      }
    }
  }
  (void)hipFree(u);
  (void)hipFree(bdy);
  if (he != hipSuccess) {
    if (saved.iters_per_pass) table[cls] = saved; else table.erase(cls);
    return fail(c, SOR_EDEVICE, "autotune_batch: %s", c->err.empty() ? "device error" : c->err.c_str());
  }
  table[cls] = bt;
  if (best) *best = bt;
  return SOR_OK;
}

}  // extern "C"
