// Host side of mixed-precision batched solves and of the serving loop.
//
// Both drive the mixed-precision persistent kernel (sor_mixbatch.hip) over a
// table of grid slots.  A slot holds one grid's whole state on the device: the
// FP64 iterate U and h*h*f, the low-precision inner iterate pair and
// right-hand side, per-row-block partial sums, and staging for the caller's
// arrays.  One launch advances every listed slot until it finishes or until
// the launch's time slice ends (the slot then resumes in the next launch at
// the phase it reached).
//
//   sor_batch_solve_mixed: all grids in one launch, no time limit, recorded as
//   a HIP graph and replayed while the batch shapes repeat.
//   sor_server_*: a background thread admits queued requests into free slots
//   when the memory budget allows, launches time-sliced epochs over all
//   resident requests, and retires finished ones (continuous batching).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <numeric>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sor_host.h"

namespace sor {


namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

constexpr int kServerMinSeg = 32;   // served grids use tiles of >= 32 rows

// Byte offsets of one slot's buffers inside its region.
struct SlotLayout {
  Layout L64, Llo;
  int nrb = 0;
  size_t U = 0, F = 0, EA = 0, EB = 0, R = 0, P = 0;   // device state
  size_t in_u = 0, in_b = 0, in_f = 0;                  // caller staging (server)
  size_t total = 0;
};

SlotLayout slot_layout(int n, int prec_lo, bool has_f, bool staging) {
  SlotLayout s;
  s.L64 = make_layout(n, kF64);
  s.Llo = make_layout(n, prec_lo);
  s.nrb = (n + kMixRows - 1) / kMixRows;
  const size_t b64 = align256((size_t)s.L64.elems() * 8);
  const size_t blo = align256((size_t)s.Llo.elems() * (size_t)prec_bytes(prec_lo));
  size_t o = 0;
  s.U = o; o += b64;
  if (has_f) { s.F = o; o += b64; }
  s.EA = o; o += blo;
  s.EB = o; o += blo;
  s.R = o; o += blo;
  s.P = o; o += align256((size_t)s.nrb * 3 * 8);
  if (staging) {
    s.in_u = o; o += align256((size_t)n * n * 8);
    s.in_b = o; o += align256((size_t)4 * n * 8);
    if (has_f) { s.in_f = o; o += align256((size_t)n * n * 8); }
  }
  s.total = o;
  return s;
}

// Fill a slot's descriptor (host copy) for a fresh grid at phase RESID.
void fill_slot(BMGrid &G, char *region, const SlotLayout &s, int prec_lo, int n,
               double *user_u, const double *user_bdy, const double *user_f,
               double omega, double rel_tol, double corr_tol, int64_t max_outer,
               int64_t inner_iters, const sor_tiling &t) {
  std::memset(&G, 0, sizeof(BMGrid));
  const int elo = prec_bytes(prec_lo);
  G.U = (double *)(region + s.U) + s.L64.origin_off();
  G.F = user_f ? (const double *)(region + s.F) + s.L64.origin_off() : nullptr;
  G.EA = region + s.EA + (size_t)s.Llo.origin_off() * elo;
  G.EB = region + s.EB + (size_t)s.Llo.origin_off() * elo;
  G.R = region + s.R + (size_t)s.Llo.origin_off() * elo;
  G.partials = (double *)(region + s.P);
  G.user_u = user_u;
  G.user_bdy = user_bdy;
  G.user_f = user_f;
  G.pitch = s.L64.pitch;
  G.lo_pitch = s.Llo.pitch;
  G.n = n;
  G.T = std::max(1, std::min(t.iters_per_pass, kMixTMax));
  G.seg_rows = t.seg_rows;
  G.nrb = s.nrb;
  G.omega = omega;
  G.rel_tol = rel_tol;
  G.corr_tol = corr_tol;
  const double h = 1.0 / (double)(n + 1);
  G.target = prec_lo == kF16 ? std::ldexp(h * h, 14) / 0.0737 : 1.0;
  G.max_outer = max_outer;
  G.inner_iters = inner_iters > 0 ? inner_iters : mixed_inner_default(n);
  G.phase = kPhResid;
  G.nitems = s.nrb;
  G.rel = NAN;
  G.rinf = NAN;
  G.last_corr = NAN;
}

// Device slot table, queue and ring plus pinned staging, shared by the batch
// and server paths.
struct MixRunner {
  int device = 0;
  int prec_lo = kF32;
  int slots_cap = 0;
  BMGrid *d_grids = nullptr, *h_grids = nullptr;
  BQueue *d_q = nullptr, *h_q = nullptr;
  BItem *d_ring = nullptr, *h_items = nullptr;
  size_t ring_cap = 0, items_cap = 0;
  int *d_list = nullptr, *h_list = nullptr;     // pack / unpack slot lists
  int *d_list2 = nullptr, *h_list2 = nullptr;
  unsigned long long gen = 0;
  int waves = 0;                 // persistent wavefronts of the fixed-depth kernel
  int waves_dyn = 0;             // ... of the run-time-depth kernel
  long long wall_khz = 100000;
  hipStream_t stream = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<long long> sig;
  std::string err;

  ~MixRunner() { release(); }
  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    if (d_grids) (void)hipFree(d_grids);
    if (d_q) (void)hipFree(d_q);
    if (d_ring) (void)hipFree(d_ring);
    if (d_list) (void)hipFree(d_list);
    if (d_list2) (void)hipFree(d_list2);
    if (h_grids) (void)hipHostFree(h_grids);
    if (h_q) (void)hipHostFree(h_q);
    if (h_items) (void)hipHostFree(h_items);
    if (h_list) (void)hipHostFree(h_list);
    if (h_list2) (void)hipHostFree(h_list2);
    if (stream) (void)hipStreamDestroy(stream);
    d_grids = h_grids = nullptr; d_q = h_q = nullptr; d_ring = h_items = nullptr;
    d_list = h_list = d_list2 = h_list2 = nullptr; stream = nullptr;
    slots_cap = 0; ring_cap = items_cap = 0;
  }

  hipError_t init(int dev, int prec, int max_slots, size_t max_items_total) {
    device = dev;
    prec_lo = prec;
    hipError_t e;
    if ((e = hipSetDevice(dev)) != hipSuccess) return e;
    if (!stream && (e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking)) != hipSuccess) return e;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
      wall_khz = khz;
    int cus = 0;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    waves = std::max(1, cus) * mix_waves_per_cu(prec_lo, false);
    waves_dyn = std::max(1, cus) * mix_waves_per_cu(prec_lo, true);
    if (max_slots > slots_cap) {
      if (d_grids) { (void)hipFree(d_grids); d_grids = nullptr; }
      if (h_grids) { (void)hipHostFree(h_grids); h_grids = nullptr; }
      if (d_list) { (void)hipFree(d_list); d_list = nullptr; }
      if (h_list) { (void)hipHostFree(h_list); h_list = nullptr; }
      if (d_list2) { (void)hipFree(d_list2); d_list2 = nullptr; }
      if (h_list2) { (void)hipHostFree(h_list2); h_list2 = nullptr; }
      if ((e = hipMalloc(&d_grids, sizeof(BMGrid) * max_slots)) != hipSuccess) return e;
      if ((e = hipHostMalloc((void **)&h_grids, sizeof(BMGrid) * max_slots, hipHostMallocDefault)) != hipSuccess) return e;
      if ((e = hipMalloc(&d_list, sizeof(int) * max_slots)) != hipSuccess) return e;
      if ((e = hipHostMalloc((void **)&h_list, sizeof(int) * max_slots, hipHostMallocDefault)) != hipSuccess) return e;
      if ((e = hipMalloc(&d_list2, sizeof(int) * max_slots)) != hipSuccess) return e;
      if ((e = hipHostMalloc((void **)&h_list2, sizeof(int) * max_slots, hipHostMallocDefault)) != hipSuccess) return e;
      std::memset(h_grids, 0, sizeof(BMGrid) * max_slots);
      slots_cap = max_slots;
    }
    if (!d_q) {
      if ((e = hipMalloc(&d_q, sizeof(BQueue))) != hipSuccess) return e;
      if ((e = hipHostMalloc((void **)&h_q, sizeof(BQueue), hipHostMallocDefault)) != hipSuccess) return e;
    }
    unsigned long long cap = 1024;
    while (cap < 2ull * (max_items_total + (unsigned long long)std::max(waves, waves_dyn)) + 1024)
      cap <<= 1;
    if (cap > ring_cap) {
      if (d_ring) { (void)hipFree(d_ring); d_ring = nullptr; }
      if ((e = hipMalloc(&d_ring, sizeof(BItem) * cap)) != hipSuccess) return e;
      if ((e = hipMemset(d_ring, 0, sizeof(BItem) * cap)) != hipSuccess) return e;
      ring_cap = cap;
      if (exec) { (void)hipGraphExecDestroy(exec); exec = nullptr; }
    }
    if (max_items_total > items_cap) {
      if (h_items) { (void)hipHostFree(h_items); h_items = nullptr; }
      if ((e = hipHostMalloc((void **)&h_items, sizeof(BItem) * max_items_total, hipHostMallocDefault)) != hipSuccess) return e;
      items_cap = max_items_total;
      if (exec) { (void)hipGraphExecDestroy(exec); exec = nullptr; }
    }
    return hipSuccess;
  }

  // Kernel for a launch over the listed slots: the run-time-depth one when
  // some grid's passes are shallower than the fixed depth (a depth set on
  // the context or tuned for its size class) or its inner iteration count
  // is not a multiple of it, and for binary16 storage (whose fixed-depth
  // kernel holds one wavefront per SIMD, the run-time-depth one two).
  bool need_dyn(const std::vector<int> &active) const {
    if (prec_lo == kF16) return true;
    for (int s : active)
      if (h_grids[s].T != kMixTMax || h_grids[s].inner_iters % kMixTMax != 0) return true;
    return false;
  }

  // Queue the pending items of the listed slots (their descriptors are in
  // h_grids) and set the queue header for a launch whose grids pause after
  // slice_ticks of device wall clock (0: run to completion).
  size_t build_queue(const std::vector<int> &active, long long slice_ticks) {
    const unsigned long long g = (++gen) & 0xffffffull;
    unsigned long long idx = 0;
    for (int s : active)
      for (int t = 0; t < h_grids[s].nitems; ++t, ++idx) {
        h_items[idx].tag = bq_tag(g, idx);
        h_items[idx].payload = ((unsigned long long)s << 32) | (unsigned)t;
      }
    std::memset(h_q, 0, sizeof(BQueue));
    h_q->tail = idx;
    h_q->gen = g;
    h_q->mask = ring_cap - 1;
    h_q->remaining = (int)active.size();
    h_q->deadline_ticks = wall_khz * 1000ll * 20;     // a wait longer than 20 s is a failure
    h_q->t0 = 0;
    h_q->slice_ticks = slice_ticks;
    return idx;
  }
};

}  // namespace
}  // namespace sor

using namespace sor;

// ---------------------------------------------------------------------------
// Batched mixed-precision solves
// ---------------------------------------------------------------------------

namespace sor {
struct MixBatchState {
  MixRunner run;
  DevBuf arena;
};
}  // namespace sor

static std::unordered_map<sor_ctx *, MixBatchState *> g_mix_state;
static std::mutex g_mix_mu;

static MixBatchState *mix_state_for(sor_ctx *c) {
  std::lock_guard<std::mutex> lk(g_mix_mu);
  auto it = g_mix_state.find(c);
  if (it != g_mix_state.end()) return it->second;
  auto *s = new (std::nothrow) MixBatchState;
  if (s) g_mix_state[c] = s;
  return s;
}

namespace sor {
void mix_state_free(sor_ctx *c) {
  std::lock_guard<std::mutex> lk(g_mix_mu);
  auto it = g_mix_state.find(c);
  if (it == g_mix_state.end()) return;
  if (it->second->arena.p) (void)hipFree(it->second->arena.p);
  delete it->second;
  g_mix_state.erase(it);
}
}  // namespace sor

extern "C" sor_status sor_batch_solve_mixed(sor_ctx *c, const sor_mixed_desc *grids,
                                            int32_t count, int32_t inner_bits,
                                            void *stream, sor_result *results) {
  if (!c) return SOR_EINVAL;
  c->err.clear();
  if (!grids || !results || count < 1) return fail(c, SOR_EINVAL, "need grids, results and count >= 1");
  if (inner_bits != 32 && inner_bits != 16) return fail(c, SOR_EINVAL, "inner_bits must be 32 or 16");
  const int plo = inner_bits == 32 ? kF32 : kF16;
  for (int g = 0; g < count; ++g) {
    const sor_mixed_desc &d = grids[g];
    sor_status st = check_common(c, d.u, d.boundary, d.rhs, d.n, d.omega);
    if (st != SOR_OK) return fail(c, st, "grid %d: %s", g, c->err.c_str());
    if (!(d.rel_tol >= 0.0) || !(d.corr_tol >= 0.0) || d.max_outer < 0)
      return fail(c, SOR_EINVAL, "grid %d: rel_tol, corr_tol or max_outer invalid", g);
    if (plo == kF16 && d.n > kMaxN16)
      return fail(c, SOR_EINVAL, "grid %d: binary16 inner storage supports n <= %d (n = %d)", g,
                  kMaxN16, d.n);
  }
  MixBatchState *ms = mix_state_for(c);
  if (!ms) return fail(c, SOR_ENOMEM, "out of host memory");
  MixRunner &R = ms->run;
  // Layout of every grid in one arena.
  std::vector<SlotLayout> lay(count);
  std::vector<size_t> off(count);
  size_t arena = 0, max_items = 0;
  int max_n = 0;
  std::vector<sor_tiling> til(count);
  for (int g = 0; g < count; ++g) {
    lay[g] = slot_layout(grids[g].n, plo, grids[g].rhs != nullptr, false);
    off[g] = arena;
    arena += lay[g].total;
    til[g] = batch_tiling(c, plo == kF32 ? kF32 : kF16, grids[g].n);
    size_t most = (size_t)lay[g].nrb;
    most = std::max(most, (size_t)blocked_ntiles(plo, grids[g].n, kMixTMax, til[g].seg_rows));
    max_items += most;
    max_n = std::max(max_n, grids[g].n);
  }
  hipError_t e = R.init(c->device, plo, count, max_items);
  if (e != hipSuccess) return fail(c, SOR_EDEVICE, "mixed batch set-up: %s", hipGetErrorString(e));
  if (ms->arena.bytes < arena) {
    if (ms->arena.p) (void)hipFree(ms->arena.p);
    ms->arena.p = nullptr;
    ms->arena.bytes = 0;
    if (hipMalloc(&ms->arena.p, arena) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, SOR_ENOMEM, "cannot allocate %zu bytes for the batch", arena);
    }
    HIP_TRY(c, hipMemset(ms->arena.p, 0, arena));
    ms->arena.bytes = arena;
    if (R.exec) { (void)hipGraphExecDestroy(R.exec); R.exec = nullptr; }
  }
  char *base = (char *)ms->arena.p;
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return grids[x].n > grids[y].n; });
  for (int g = 0; g < count; ++g) {
    const sor_mixed_desc &d = grids[g];
    fill_slot(R.h_grids[g], base + off[g], lay[g], plo, d.n, d.u, d.boundary, d.rhs,
              d.omega, d.rel_tol, d.corr_tol, d.max_outer, d.inner_iters, til[g]);
    R.h_list[g] = g;
  }
  const size_t nitems = R.build_queue(order, 0);
  const bool dyn = R.need_dyn(order);
  const int nwaves = dyn ? R.waves_dyn : R.waves;
  const std::vector<long long> sig = {count, (long long)nitems, max_n, plo, nwaves, dyn,
                                      (long long)(uintptr_t)base, (long long)R.ring_cap,
                                      (long long)(uintptr_t)R.h_items};
  hipStream_t s = R.stream;
  hipEvent_t ev;
  HIP_TRY(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  HIP_TRY(c, hipEventRecord(ev, (hipStream_t)stream));
  HIP_TRY(c, hipStreamWaitEvent(s, ev, 0));
  if (!(R.exec && R.sig == sig)) {
    if (R.exec) { (void)hipGraphExecDestroy(R.exec); R.exec = nullptr; }
    hipGraph_t graph = nullptr;
    HIP_TRY(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t er = hipSuccess;
    auto step = [&](hipError_t x) { if (er == hipSuccess) er = x; };
    step(hipMemcpyAsync(R.d_grids, R.h_grids, sizeof(BMGrid) * count, hipMemcpyHostToDevice, s));
    step(hipMemcpyAsync(R.d_list, R.h_list, sizeof(int) * count, hipMemcpyHostToDevice, s));
    step(hipMemcpyAsync(R.d_q, R.h_q, sizeof(BQueue), hipMemcpyHostToDevice, s));
    step(hipMemcpyAsync(R.d_ring, R.h_items, sizeof(BItem) * nitems, hipMemcpyHostToDevice, s));
    step(launch_mix_pack(plo, R.d_grids, R.d_list, count, max_n, s));
    step(launch_mix_batch(plo, dyn, R.d_grids, R.d_q, R.d_ring, nwaves, s));
    step(launch_mix_unpack(R.d_grids, R.d_list, count, max_n, s));
    step(hipMemcpyAsync(R.h_grids, R.d_grids, sizeof(BMGrid) * count, hipMemcpyDeviceToHost, s));
    step(hipMemcpyAsync(R.h_q, R.d_q, sizeof(BQueue), hipMemcpyDeviceToHost, s));
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (er != hipSuccess || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipEventDestroy(ev);
      return fail(c, SOR_EDEVICE, "graph capture: %s", hipGetErrorString(er != hipSuccess ? er : e2));
    }
    er = hipGraphInstantiate(&R.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (er != hipSuccess) {
      R.exec = nullptr;
      (void)hipEventDestroy(ev);
      return fail(c, SOR_EDEVICE, "graph instantiate: %s", hipGetErrorString(er));
    }
    R.sig = sig;
  }
  HIP_TRY(c, hipGraphLaunch(R.exec, s));
  HIP_TRY(c, hipEventRecord(ev, s));
  HIP_TRY(c, hipStreamWaitEvent((hipStream_t)stream, ev, 0));
  HIP_TRY(c, hipStreamSynchronize(s));
  (void)hipEventDestroy(ev);
  if (R.h_q->error) return fail(c, SOR_ETIMEOUT, "a queue wait exceeded its bound");
  sor_status overall = SOR_OK;
  for (int g = 0; g < count; ++g) {
    const BMGrid &G = R.h_grids[g];
    sor_result &r = results[g];
    r = sor_result{};
    r.iterations = G.inner_total;
    r.final_max_delta = G.last_corr;
    r.outer_steps = (int32_t)G.outer;
    r.rel_residual = G.rel;
    r.passes = G.passes;
    r.converged = G.status == 1;
    r.status = G.status == 1 ? SOR_OK : G.status == 2 ? SOR_NOT_CONVERGED
             : G.status == 3 ? SOR_ENONFINITE : SOR_EDEVICE;
    if (r.status == SOR_ENONFINITE) overall = SOR_ENONFINITE;
    else if (r.status == SOR_EDEVICE && overall >= 0) overall = SOR_EDEVICE;
    else if (r.status == SOR_NOT_CONVERGED && overall == SOR_OK) overall = SOR_NOT_CONVERGED;
  }
  if (overall == SOR_EDEVICE) return fail(c, SOR_EDEVICE, "a grid did not finish");
  return overall;
}

// ---------------------------------------------------------------------------
// Serving loop
// ---------------------------------------------------------------------------

namespace {

// First-fit allocator over one device block (the memory budget).
class Arena {
 public:
  bool init(size_t bytes) {
    if (hipMalloc(&base_, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    size_ = bytes;
    free_[0] = bytes;
    return true;
  }
  ~Arena() {
    if (base_) (void)hipFree(base_);
  }
  char *base() const { return (char *)base_; }
  size_t size() const { return size_; }
  size_t in_use() const { return used_; }
  size_t peak() const { return peak_; }
  // Returns an offset, or SIZE_MAX when no free range is large enough.
  size_t alloc(size_t bytes) {
    bytes = align256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return off;
      }
    }
    return SIZE_MAX;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  void *base_ = nullptr;
  size_t size_ = 0;
  size_t used_ = 0, peak_ = 0;      // bytes held by resident requests
  std::map<size_t, size_t> free_;   // offset -> length
};

// A waiting request that does not fit may be overtaken by later ones that do
// (no head-of-line blocking), but at most this many times: then admission
// waits for memory to free up for it.
constexpr int kMaxBypass = 32;

struct Request {
  uint64_t ticket = 0;
  int n = 0;
  std::vector<double> u0, bdy, f;   // host copies
  std::vector<double> out;          // host result
  double omega = 0, rel_tol = 0, corr_tol = 0;
  int64_t max_outer = 0, inner_iters = 0;
  SlotLayout lay;
  size_t off = SIZE_MAX;
  int slot = -1;
  int bypassed = 0;                 // later requests admitted ahead of it
  bool done = false;
  sor_result result{};
  double submit_s = 0, admit_s = 0, done_s = 0;
};

}  // namespace

struct sor_server {
  int device = 0;
  int prec_lo = kF32;
  int max_slots = 0;
  double slice_ms = 2.0;
  sor_ctx *ctx = nullptr;
  MixRunner run;
  Arena arena;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> waiting;
  std::vector<Request *> resident;                  // by slot (nullptr = free)
  std::unordered_map<uint64_t, Request *> by_ticket;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  std::string err;
  int64_t launches = 0, completed = 0;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void loop();
};

void sor_server::loop() {
  (void)hipSetDevice(device);
  std::vector<Request *> fresh, finished;
  std::vector<int> active;
  while (true) {
    fresh.clear();
    {
      std::unique_lock<std::mutex> lk(mu);
      // Admit waiting requests in arrival order while a slot is free; one
      // that does not fit in the free memory is passed over by later ones
      // that do, until it has been passed over kMaxBypass times.
      std::vector<Request *> skipped;
      for (auto it = waiting.begin(); it != waiting.end();) {
        Request *q = *it;
        int slot = -1;
        for (int s = 0; s < max_slots; ++s)
          if (!resident[s]) { slot = s; break; }
        if (slot < 0) break;
        const size_t off = arena.alloc(q->lay.total);
        if (off == SIZE_MAX) {
          skipped.push_back(q);
          if (q->bypassed >= kMaxBypass) break;
          ++it;
          continue;
        }
        it = waiting.erase(it);
        for (Request *p : skipped) ++p->bypassed;
        q->off = off;
        q->slot = slot;
        q->admit_s = now();
        resident[slot] = q;
        fresh.push_back(q);
      }
      active.clear();
      for (int s = 0; s < max_slots; ++s)
        if (resident[s]) active.push_back(s);
      if (active.empty()) {
        if (stop) return;
        cv_work.wait_for(lk, std::chrono::milliseconds(20));
        continue;
      }
      if (stop) return;
    }
    hipStream_t s = run.stream;
    hipError_t e = hipSuccess;
    auto step = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    // Upload new requests and pack them into their slots.
    int nf = 0, max_n = 0;
    for (Request *q : fresh) {
      char *region = arena.base() + q->off;
      double *du = (double *)(region + q->lay.in_u);
      double *db = (double *)(region + q->lay.in_b);
      double *df = q->f.empty() ? nullptr : (double *)(region + q->lay.in_f);
      step(hipMemcpyAsync(du, q->u0.data(), q->u0.size() * 8, hipMemcpyHostToDevice, s));
      step(hipMemcpyAsync(db, q->bdy.data(), q->bdy.size() * 8, hipMemcpyHostToDevice, s));
      if (df) step(hipMemcpyAsync(df, q->f.data(), q->f.size() * 8, hipMemcpyHostToDevice, s));
      sor_tiling t = batch_tiling(ctx, prec_lo, q->n);
      t.seg_rows = std::max(t.seg_rows, kServerMinSeg);
      fill_slot(run.h_grids[q->slot], region, q->lay, prec_lo, q->n, du, db, df, q->omega,
                q->rel_tol, q->corr_tol, q->max_outer, q->inner_iters, t);
      step(hipMemcpyAsync(run.d_grids + q->slot, run.h_grids + q->slot, sizeof(BMGrid),
                          hipMemcpyHostToDevice, s));
      run.h_list[nf++] = q->slot;
      max_n = std::max(max_n, q->n);
    }
    if (nf) {
      step(hipMemcpyAsync(run.d_list, run.h_list, sizeof(int) * nf, hipMemcpyHostToDevice, s));
      step(launch_mix_pack(prec_lo, run.d_grids, run.d_list, nf, max_n, s));
    }
    // One time slice over every resident request: each request's pending
    // phase is queued; grids pause at a phase boundary once the slice is over.
    const long long slice_ticks = std::max(1LL, (long long)(slice_ms * 1e-3 * run.wall_khz * 1000.0));
    const size_t nitems = run.build_queue(active, slice_ticks);
    step(hipMemcpyAsync(run.d_q, run.h_q, sizeof(BQueue), hipMemcpyHostToDevice, s));
    step(hipMemcpyAsync(run.d_ring, run.h_items, sizeof(BItem) * nitems, hipMemcpyHostToDevice, s));
    const bool dyn = run.need_dyn(active);
    step(launch_mix_batch(prec_lo, dyn, run.d_grids, run.d_q, run.d_ring,
                          dyn ? run.waves_dyn : run.waves, s));
    step(hipMemcpyAsync(run.h_grids, run.d_grids, sizeof(BMGrid) * max_slots, hipMemcpyDeviceToHost, s));
    step(hipMemcpyAsync(run.h_q, run.d_q, sizeof(BQueue), hipMemcpyDeviceToHost, s));
    step(hipStreamSynchronize(s));
    ++launches;
    if (e != hipSuccess || run.h_q->error) {
      std::lock_guard<std::mutex> lk(mu);
      err = e != hipSuccess ? hipGetErrorString(e) : "a queue wait exceeded its bound";
      for (int sl : active) {
        Request *q = resident[sl];
        q->result.status = e != hipSuccess ? SOR_EDEVICE : SOR_ETIMEOUT;
        q->done = true;
        q->done_s = now();
        arena.release(q->off, q->lay.total);
        resident[sl] = nullptr;
      }
      cv_done.notify_all();
      continue;
    }
    // Retire finished requests: unpack into their staging, download.
    finished.clear();
    int nd = 0;
    max_n = 0;
    for (int sl : active) {
      const BMGrid &G = run.h_grids[sl];
      if (G.status == 0) continue;
      Request *q = resident[sl];
      finished.push_back(q);
      run.h_list2[nd++] = sl;
      max_n = std::max(max_n, q->n);
    }
    if (nd) {
      step(hipMemcpyAsync(run.d_list2, run.h_list2, sizeof(int) * nd, hipMemcpyHostToDevice, s));
      step(launch_mix_unpack(run.d_grids, run.d_list2, nd, max_n, s));
      for (Request *q : finished) {
        q->out.resize((size_t)q->n * q->n);
        char *region = arena.base() + q->off;
        step(hipMemcpyAsync(q->out.data(), region + q->lay.in_u, q->out.size() * 8,
                            hipMemcpyDeviceToHost, s));
      }
      step(hipStreamSynchronize(s));
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      for (Request *q : finished) {
        const BMGrid &G = run.h_grids[q->slot];
        sor_result &r = q->result;
        r = sor_result{};
        r.iterations = G.inner_total;
        r.final_max_delta = G.last_corr;
        r.outer_steps = (int32_t)G.outer;
        r.rel_residual = G.rel;
        r.passes = G.passes;
        r.converged = G.status == 1;
        r.status = e != hipSuccess ? SOR_EDEVICE
                 : G.status == 1 ? SOR_OK : G.status == 2 ? SOR_NOT_CONVERGED : SOR_ENONFINITE;
        q->done = true;
        q->done_s = now();
        arena.release(q->off, q->lay.total);
        resident[q->slot] = nullptr;
        ++completed;
      }
      if (!finished.empty()) cv_done.notify_all();
    }
  }
}

extern "C" {

sor_status sor_server_create(int device, int32_t inner_bits, size_t hbm_budget,
                             int32_t max_slots, double slice_ms, sor_server **out) {
  if (!out) return SOR_EINVAL;
  *out = nullptr;
  if (inner_bits != 32 && inner_bits != 16) return SOR_EINVAL;
  if (max_slots < 1 || max_slots > 65536 || hbm_budget < (1u << 20) || !(slice_ms > 0.0))
    return SOR_EINVAL;
  sor_server *srv = new (std::nothrow) sor_server;
  if (!srv) return SOR_ENOMEM;
  srv->device = device;
  srv->prec_lo = inner_bits == 32 ? kF32 : kF16;
  srv->max_slots = max_slots;
  srv->slice_ms = slice_ms;
  sor_status st = sor_ctx_create(device, &srv->ctx);
  if (st != SOR_OK) { delete srv; return st; }
  // Ring sized for every slot holding its largest phase at once: sides up to
  // 4096 with tiles of at least kServerMinSeg rows, plus the waiting waves.
  size_t per_slot = (4096 + kMixRows - 1) / kMixRows;
  per_slot = std::max(per_slot, (size_t)blocked_ntiles(srv->prec_lo, 4096, kMixTMax, kServerMinSeg));
  const size_t max_items = (size_t)max_slots * per_slot;
  if (srv->run.init(device, srv->prec_lo, max_slots, max_items) != hipSuccess ||
      !srv->arena.init(hbm_budget)) {
    sor_ctx_destroy(srv->ctx);
    delete srv;
    return SOR_ENOMEM;
  }
  srv->resident.assign(max_slots, nullptr);
  srv->worker = std::thread([srv] { srv->loop(); });
  *out = srv;
  return SOR_OK;
}

sor_status sor_server_submit(sor_server *srv, const sor_request *req, uint64_t *ticket) {
  if (!srv || !req || !ticket || !req->boundary) return SOR_EINVAL;
  const int n = req->n;
  if (n < 1 || n > 4096) return SOR_EINVAL;
  if (srv->prec_lo == kF16 && n > kMaxN16) return SOR_EINVAL;
  if (!(req->rel_tol >= 0.0) || !(req->corr_tol >= 0.0) || req->max_outer < 0) return SOR_EINVAL;
  double omega = req->omega;
  if (!(omega > 0.0)) omega = omega_opt(n);
  if (!(omega < 2.0)) return SOR_EINVAL;
  Request *q = new (std::nothrow) Request;
  if (!q) return SOR_ENOMEM;
  q->n = n;
  q->u0.assign((size_t)n * n, 0.0);
  if (req->u0) std::memcpy(q->u0.data(), req->u0, q->u0.size() * 8);
  q->bdy.assign(req->boundary, req->boundary + 4 * (size_t)n);
  if (req->rhs) q->f.assign(req->rhs, req->rhs + (size_t)n * n);
  q->omega = omega;
  q->rel_tol = req->rel_tol;
  q->corr_tol = req->corr_tol;
  q->max_outer = req->max_outer;
  q->inner_iters = req->inner_iters;
  q->lay = slot_layout(n, srv->prec_lo, req->rhs != nullptr, true);
  if (q->lay.total > srv->arena.size()) {
    delete q;
    return SOR_EBUSY;
  }
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    q->ticket = srv->next_ticket++;
    q->submit_s = srv->now();
    srv->by_ticket[q->ticket] = q;
    srv->waiting.push_back(q);
    *ticket = q->ticket;
  }
  srv->cv_work.notify_one();
  return SOR_OK;
}

sor_status sor_server_poll(sor_server *srv, uint64_t ticket, double wait_ms,
                           sor_request_info *info, double *u_out) {
  if (!srv) return SOR_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->by_ticket.find(ticket);
  if (it == srv->by_ticket.end()) return SOR_EINVAL;
  Request *q = it->second;
  if (!q->done && wait_ms > 0.0)
    srv->cv_done.wait_for(lk, std::chrono::microseconds((long long)(wait_ms * 1000.0)),
                          [q] { return q->done; });
  if (!q->done) return SOR_EBUSY;
  if (info) {
    info->result = q->result;
    info->submit_s = q->submit_s;
    info->admit_s = q->admit_s;
    info->done_s = q->done_s;
  }
  if (u_out && !q->out.empty()) std::memcpy(u_out, q->out.data(), q->out.size() * 8);
  const sor_status st = (sor_status)q->result.status;
  srv->by_ticket.erase(it);
  delete q;
  return st;
}

double sor_server_clock(const sor_server *srv) { return srv ? srv->now() : 0.0; }

sor_status sor_server_stats(sor_server *srv, int64_t *launches, int64_t *completed,
                            int64_t *waiting, int64_t *resident) {
  if (!srv) return SOR_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (launches) *launches = srv->launches;
  if (completed) *completed = srv->completed;
  if (waiting) *waiting = (int64_t)srv->waiting.size();
  if (resident)
    *resident = (int64_t)std::count_if(srv->resident.begin(), srv->resident.end(),
                                       [](Request *q) { return q != nullptr; });
  return SOR_OK;
}

sor_status sor_server_memory(sor_server *srv, size_t *budget, size_t *in_use, size_t *peak) {
  if (!srv) return SOR_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (budget) *budget = srv->arena.size();
  if (in_use) *in_use = srv->arena.in_use();
  if (peak) *peak = srv->arena.peak();
  return SOR_OK;
}

const char *sor_server_last_error(const sor_server *srv) { return srv ? srv->err.c_str() : "null server"; }

void sor_server_destroy(sor_server *srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  for (auto &kv : srv->by_ticket) delete kv.second;
  srv->run.release();
  sor_ctx_destroy(srv->ctx);
  delete srv;
}

}  // extern "C"
