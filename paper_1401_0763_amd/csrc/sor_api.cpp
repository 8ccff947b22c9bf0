// Host runtime of libsor: the C ABI declared in include/sor.h.
//
// Control flow of a plain solve (Algorithm 1 of Mittal 2014, restated):
//   for iter = 1..max_iters: red phase, black phase; on a check iteration
//   (iter % K == 0 or iter == max_iters) stop when the iteration's largest
//   change is strictly below tol.
// On the GPU each "pass" applies T iterations; the last wavefront of a pass
// evaluates the stopping rule for those T iterations on the device and sets a
// stop flag that makes every later pass exit at once.  The host therefore
// enqueues passes in chunks without waiting, and synchronises once per chunk.
// When the rule is met at an iteration inside a pass, that pass's output has
// gone too far: its input grid is still intact (ping-pong, and every later
// pass exited early), so the pass is re-run from its input with exactly the
// iterations needed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <new>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sor_host.h"
#include "sor_3d.h"
#include "sor_variants.h"

using namespace sor;

namespace sor {

sor_status fail(sor_ctx *c, sor_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

sor_status ensure(sor_ctx *c, BufRole role, size_t bytes) {
  DevBuf &b = c->bufs[role];
  if (b.bytes >= bytes) return SOR_OK;
  if (b.p) {
    (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(c, SOR_ENOMEM, "cannot allocate %zu bytes of device memory", bytes);
  }
  // Zero once so margins never hold stale bit patterns.
  e = hipMemset(b.p, 0, bytes);
  if (e != hipSuccess) return fail(c, SOR_EDEVICE, "hipMemset: %s", hipGetErrorString(e));
  b.bytes = bytes;
  return SOR_OK;
}

bool is_device_ptr(sor_ctx *c, const void *p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) &&
         a.device == c->device;
}

sor_status check_common(sor_ctx *c, const void *u, const void *bdy,
                        const void *rhs, int32_t n, double omega) {
  if (!c) return SOR_EINVAL;
  c->err.clear();
  if (n < 1 || n > kMaxN) return fail(c, SOR_EINVAL, "n = %d outside 1..%d", n, kMaxN);
  if (!(omega > 0.0 && omega < 2.0))
    return fail(c, SOR_EINVAL, "omega = %g outside (0, 2)", omega);
  if (!is_device_ptr(c, u)) return fail(c, SOR_EINVAL, "u is not a device pointer on device %d", c->device);
  if (!is_device_ptr(c, bdy)) return fail(c, SOR_EINVAL, "boundary is not a device pointer on device %d", c->device);
  if (rhs && !is_device_ptr(c, rhs)) return fail(c, SOR_EINVAL, "rhs is not a device pointer on device %d", c->device);
  HIP_TRY(c, hipSetDevice(c->device));
  return SOR_OK;
}

int prec_index(int bits) { return bits == 64 ? kF64 : bits == 32 ? kF32 : bits == 16 ? kF16 : -1; }

double omega_opt(int n) {
  if (n < 1) return NAN;
  return 2.0 / (1.0 + std::sin(M_PI / ((double)n + 1.0)));
}

}  // namespace sor

namespace {

template <typename T>
T *origin(sor_ctx *c, BufRole role, const Layout &L) {
  return (T *)c->bufs[role].p + L.origin_off();
}

GridView make_view(const Layout &L, int prec, const sor_tiling &t, const void *in,
                   void *out, const void *F, double omega, int ord = 0) {
  GridView v;
  v.in = in;
  v.out = out;
  v.F = F;
  v.pitch = L.pitch;
  v.n = L.n;
  const BlockGeom g = block_geom(prec, t.iters_per_pass, ord);
  v.nstrips = (L.n + 1 + g.CW - 1) / g.CW;
  v.seg_rows = t.seg_rows;
  v.nseg = (L.n + 1 + t.seg_rows - 1) / t.seg_rows;
  v.omega = omega;
  return v;
}

// The deepest supported pass (1 to 8 iterations) of at most `left`
// iterations and at most T.
int pass_depth(long long left, int T) {
  static const int kDepths[] = {8, 7, 6, 5, 4, 3, 2, 1};
  for (int t : kDepths)
    if (t <= T && t <= left) return t;
  return 1;
}

// The mx of a red-black pass applying iterations it0+1 .. it0+T under sc:
// T when no maximum is read (no check iteration among them, or the pass
// reports nothing), the check iteration's index (from 0) when there is
// exactly one, and -1 when there are several or every iteration's change
// is wanted.
int pass_maxima(long long it0, int T, const Sched &sc, bool every, bool reported) {
  if (!reported) return T;
  if (every) return -1;
  int pos = T, checks = 0;
  for (int t = 0; t < T; ++t) {
    const long long it = it0 + t + 1;
    if (it % sc.check_every == 0 || it == sc.max_iters) {
      pos = t;
      ++checks;
    }
  }
  return checks > 1 ? -1 : pos;
}

GridView view_for(const GridView &base, int prec, int T, int ord = 0) {
  GridView v = base;
  const BlockGeom g = block_geom(prec, T, ord);
  v.nstrips = (v.n + 1 + g.CW - 1) / g.CW;
  v.nseg = (v.n + 1 + v.seg_rows - 1) / v.seg_rows;
  return v;
}

constexpr int kMaxChunk = 64;     // passes enqueued between two host checks

struct PassRec {
  const void *in;
  void *out;
  long long it0;
  int T;
};

// Event pair k of the context's pool (grown on demand).
sor_status prof_events(sor_ctx *c, size_t k, hipEvent_t *a, hipEvent_t *b) {
  while (c->events.size() < 2 * (k + 1)) {
    hipEvent_t e;
    HIP_TRY(c, hipEventCreate(&e));
    c->events.push_back(e);
  }
  *a = c->events[2 * k];
  *b = c->events[2 * k + 1];
  return SOR_OK;
}

// Pass ordering of the blocked tile for a solve ordering (1 four-colour,
// 2 Jacobi, 3 block-parallel), or -1.
int pass_ordering(int32_t ordering) {
  switch (ordering) {
    case SOR_ORDER_FOUR_COLOUR: return 1;
    case SOR_ORDER_JACOBI: return 2;
    case SOR_ORDER_BLOCK_PARALLEL: return 3;
  }
  return -1;
}

// Tiling of a four-colour, Jacobi or block-parallel solve (pass ordering
// ord): the context's setting, with seg_rows from auto_seg_rows when none
// was set.
sor_tiling variant_tiling(sor_ctx *c, int ord, int n, bool pois) {
  sor_tiling t = c->tiling_var[ord == 4 ? 3 : ord];      // both block-parallel kernels
  if (t.seg_rows == 0) t.seg_rows = auto_seg_rows(c, kF64, n, t.iters_per_pass, pois, ord);
  return t;
}

// Run SOR sweeps (red-black; four-colour with ord 1, Jacobi with ord 2 or
// block-parallel red-black with ord 3 or 4 and blocks of shape bs on
// FP64 grids, where the simple kernel is the in-place four-colour one) on the
// packed grids A/B (same layout L) until the stopping rule or max_iters.  On
// return *result_grid is the grid holding the final iterate.  hist (host, may
// be null) receives per-iteration changes.
sor_status run_sweeps(sor_ctx *c, int prec, const Layout &L, void *A, void *B,
                      const void *F, double omega, const Sched &sc,
                      hipStream_t s, sor_result *res, double *hist,
                      void **result_grid, int ord, Ctl *ctl,
                      const BlockShape &bs = BlockShape{}) {
  HIP_TRY(c, launch_ctl_reset(ctl, s));
  const sor_tiling tl = ord ? variant_tiling(c, ord, L.n, F != nullptr)
                            : tuned_tiling(c, prec, L.n, F != nullptr);
  // Jacobi and block-parallel passes read the previous iterate: ping-pong only.
  const bool simple = c->kernel == SOR_KERNEL_SIMPLE && ord <= 1;
  const int T = simple ? 1 : tl.iters_per_pass;
  GridView base = make_view(L, prec, tl, A, B, F, omega, ord);

  PassRec recs[kMaxChunk];          // the passes of the running chunk
  int nrecs = 0;
  long long done = 0;               // iterations enqueued
  long long chunk = 1;              // passes per chunk
  void *cur = A, *oth = B;
  long long reruns = 0;
  *result_grid = A;
  res->converged = 0;
  res->iterations = sc.max_iters;
  res->final_max_delta = NAN;
  for (;;) {
    const long long chunk_it0 = done;
    nrecs = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->prof) {
      sor_status pst = prof_events(c, 0, &e0, &e1);
      if (pst != SOR_OK) return pst;
      HIP_TRY(c, hipEventRecord(e0, s));
    }
    // Enqueue up to `chunk` passes (a truncated pass when < T iterations remain).
    for (long long k = 0; k < chunk && done < sc.max_iters; ++k) {
      const int Tp = pass_depth(sc.max_iters - done, T);
      GridView v = simple ? base : view_for(base, prec, Tp, ord);
      v.in = cur;
      v.out = simple ? cur : oth;
      if (simple && ord == 1) {
        HIP_TRY(c, launch_colour4_iteration((double *)cur, (const double *)F, L.pitch, L.n,
                                            omega, ctl, sc, s));
      } else if (simple) {
        HIP_TRY(c, launch_simple_iteration(prec, v, ctl, sc, s));
      } else {
        const int mx = ord ? -1 : pass_maxima(done, Tp, sc, hist != nullptr, true);
        HIP_TRY(c, launch_blocked_pass(prec, Tp, v, ctl, sc, s, ord, bs, mx));
        std::swap(cur, oth);
      }
      recs[nrecs++] = PassRec{v.in, v.out, done, Tp};
      done += Tp;
      if (done - chunk_it0 >= kHistCap - kTMax) break;
    }
    if (c->prof) HIP_TRY(c, hipEventRecord(e1, s));
    HIP_TRY(c, hipMemcpyAsync(c->host_ctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    const Ctl &h = *c->host_ctl;
    const long long hist_end = h.stop ? h.stop_iter : done;
    if (c->prof) {
      long long worked = 0;                 // passes of the chunk that did not exit early
      for (int k = 0; k < nrecs; ++k)
        if (!(h.stop && recs[k].it0 >= h.stop_iter)) ++worked;
      float ms = 0.f;
      HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
      c->prof_ms += ms;
      c->prof_launches += worked;
    }
    if (hist) {
      for (long long it = chunk_it0 + 1; it <= std::min(hist_end, sc.max_iters); ++it)
        hist[it - 1] = h.hist[(it - 1) % kHistCap];
    }
    if (h.stop) {
      res->iterations = h.stop_iter;
      res->final_max_delta = h.stop_max;
      res->passes = h.passes_done + reruns;
      // Locate the pass in which the rule was met.
      const PassRec *pr = nullptr;
      for (int k = 0; k < nrecs; ++k)
        if (h.stop_iter > recs[k].it0 && h.stop_iter <= recs[k].it0 + recs[k].T) {
          pr = &recs[k];
          break;
        }
      if (!pr) return fail(c, SOR_EDEVICE, "stop iteration %lld outside the chunk", h.stop_iter);
      if (h.stop == 2) {
        *result_grid = pr->out;
        return fail(c, SOR_ENONFINITE, "non-finite value in the grid by iteration %lld", h.stop_iter);
      }
      res->converged = 1;
      if (h.stop_iter == pr->it0 + pr->T || simple) {
        *result_grid = pr->out;
      } else {
        // Rule met inside the pass: redo its first iterations from its intact
        // input, ping-ponging between the pass's two grids.  When the pass
        // also made a non-finite value, the re-run reports its own (a control
        // block whose rule never passes): if one appears within the
        // iterations up to the stop, the solve ends as non-finite instead.
        const bool tentative = h.stop_tentative != 0;
        const long long stop_iter = h.stop_iter;   // h is overwritten below
        Ctl *rctl = tentative ? ctl + 1 : nullptr;
        const Sched rsc{LLONG_MAX, 1, -1.0};
        if (tentative) HIP_TRY(c, launch_ctl_reset(rctl, s));
        void *src = const_cast<void *>(pr->in);
        void *dst = pr->out;
        long long left = h.stop_iter - pr->it0;
        while (left > 0) {
          const int t = pass_depth(left, T);
          GridView v = view_for(base, prec, t, ord);
          v.in = src;
          v.out = dst;
          // The re-run reads no maxima: its rule never passes.
          const int mx = ord ? -1 : t;
          HIP_TRY(c, launch_blocked_pass(prec, t, v, rctl, tentative ? rsc : sc, s, ord, bs, mx));
          ++reruns;
          *result_grid = dst;
          std::swap(src, dst);
          left -= t;
        }
        res->passes = h.passes_done + reruns;
        if (tentative) {
          HIP_TRY(c, hipMemcpyAsync(c->host_ctl, rctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
          HIP_TRY(c, hipStreamSynchronize(s));
          if (c->host_ctl->stop == 2) {
            res->converged = 0;
            return fail(c, SOR_ENONFINITE, "non-finite value in the grid by iteration %lld",
                        stop_iter);
          }
        }
      }
      return SOR_OK;
    }
    if (done >= sc.max_iters) {
      res->iterations = sc.max_iters;
      res->final_max_delta = h.last_max;
      res->passes = h.passes_done;
      *result_grid = cur;
      return SOR_NOT_CONVERGED;
    }
    chunk = std::min<long long>(chunk * 2, kMaxChunk);
  }
}

// Iterations per launch of a 3-D streaming solve.  Two need every check to
// fall at the end of a two-iteration pass (check_every even; an odd max_iters
// ends with a one-iteration pass).  Two by default (with or without a
// source); a context setting of 1 or 2 is honoured under the same condition.
int iters3d_for(sor_ctx *c, int64_t check_every, bool pois) {
  (void)pois;
  const int want = c->tiling3d[0] > 0 ? c->tiling3d[0] : 2;
  return (want == 2 && check_every % 2 == 0) ? 2 : 1;
}

// Tiling of a 3-D solve of side n with T iterations per launch: the
// context's overrides, the rest chosen so the tiles fill the resident
// workgroups.
Tiling3 tiling3_for(sor_ctx *c, int n, bool pois, int T) {
  if (c->cus == 0) {
    hipDeviceProp_t prop;
    c->cus = hipGetDeviceProperties(&prop, c->device) == hipSuccess ? prop.multiProcessorCount
                                                                    : 256;
    (void)hipGetLastError();
  }
  int &occ = c->occ3[T - 1][pois ? 1 : 0];
  if (occ == 0) occ = std::max(1, stream3d_blocks_per_cu(T, pois));
  return tiling3(n, T, c->tiling3d[1], c->tiling3d[2], c->tiling3d[3], occ * c->cus);
}

// Solves whose passes never overshoot a check (the 3-D kernels, the Jacobi
// and four-colour orderings): passes in chunks of 1, 2, 4 ... 64 launches,
// the device verdict read back after each chunk (the 2-D loop without its
// re-run).  launch(done, pass, iters) enqueues the pass that starts after
// `done` iterations (0-based pass number `pass`) on s and sets iters to the
// iterations it applies.  Launches after a stop exit at once, so a ping-pong
// solve's result is in its first grid after an even number of executed
// passes (res->passes), else in its second.
template <class Launch>
sor_status run_iteration_loop(sor_ctx *c, const Sched &sc, hipStream_t s, sor_result *res,
                              double *hist, Launch launch) {
  Ctl *ctl = (Ctl *)c->bufs[kCtlBuf].p;
  HIP_TRY(c, launch_ctl_reset(ctl, s));
  long long done = 0, chunk = 1, npass = 0;
  res->converged = 0;
  res->iterations = sc.max_iters;
  res->final_max_delta = NAN;
  res->passes = 0;
  std::vector<long long> pass_end;        // iteration at the end of each pass of a chunk
  for (;;) {
    const long long chunk_it0 = done;
    long long k = 0;
    pass_end.clear();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->prof) {
      sor_status pst = prof_events(c, 0, &e0, &e1);
      if (pst != SOR_OK) return pst;
      HIP_TRY(c, hipEventRecord(e0, s));
    }
    for (; k < chunk && done < sc.max_iters; ++k) {
      int iters = 1;
      HIP_TRY(c, launch(done, npass, iters));
      done += iters;
      npass += 1;
      pass_end.push_back(done);
      if (done - chunk_it0 >= kHistCap - 2) { ++k; break; }
    }
    if (c->prof) HIP_TRY(c, hipEventRecord(e1, s));
    HIP_TRY(c, hipMemcpyAsync(c->host_ctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    const Ctl &h = *c->host_ctl;
    const long long hist_end = h.stop ? h.stop_iter : done;
    res->passes = h.passes_done;
    if (c->prof) {
      long long worked = 0;                 // passes of the chunk that did not exit early
      for (long long j = 0; j < k; ++j)
        if (!(h.stop && (j == 0 ? chunk_it0 : pass_end[j - 1]) >= h.stop_iter)) ++worked;
      float ms = 0.f;
      HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
      c->prof_ms += ms;
      c->prof_launches += worked;
    }
    if (hist)
      for (long long it = chunk_it0 + 1; it <= std::min(hist_end, sc.max_iters); ++it)
        hist[it - 1] = h.hist[(it - 1) % kHistCap];
    if (h.stop) {
      res->iterations = h.stop_iter;
      res->final_max_delta = h.stop_max;
      if (h.stop == 2)
        return fail(c, SOR_ENONFINITE, "non-finite value in the grid by iteration %lld",
                    h.stop_iter);
      res->converged = 1;
      return SOR_OK;
    }
    if (done >= sc.max_iters) {
      res->final_max_delta = h.last_max;
      return SOR_NOT_CONVERGED;
    }
    chunk = std::min<long long>(chunk * 2, kMaxChunk);
  }
}

// 3-D solve: the streaming kernel alternates A -> B and B -> A (T iterations
// per pass, a one-iteration pass for an odd remainder); the colour kernel
// (t == nullptr) works in place on A, one iteration per pass.
sor_status run_iterations3d(sor_ctx *c, double *A, double *B, const double *F, int n,
                            double omega, const Tiling3 *t, const Tiling3 *t1,
                            const Sched &sc, hipStream_t s, sor_result *res, double *hist,
                            double **result_grid) {
  Ctl *ctl = (Ctl *)c->bufs[kCtlBuf].p;
  const sor_status st = run_iteration_loop(c, sc, s, res, hist,
                                           [&](long long done, long long pass, int &iters) {
    iters = 1;
    if (!t) return launch_sor3d_iteration(A, F, n, omega, ctl, sc, s);
    const bool even = (pass & 1) == 0;
    const bool two = t->T == 2 && sc.max_iters - done >= 2;
    iters = two ? 2 : 1;
    return launch_sor3d_stream(even ? A : B, even ? B : A, F, n, omega, two ? *t : *t1,
                               iters, ctl, sc, s);
  });
  *result_grid = (t && (res->passes & 1)) ? B : A;
  return st;
}


template <typename T>
sor_status solve_plain(sor_ctx *c, int prec, T *u, const T *bdy, const T *rhs,
                       int32_t n, double omega, double tol, int64_t max_iters,
                       int64_t K, void *stream, sor_result *out, double *hist) {
  sor_status st = check_common(c, u, bdy, rhs, n, omega);
  if (st != SOR_OK) return st;
  if (!out) return fail(c, SOR_EINVAL, "out must not be NULL");
  if ((st = check_sched(c, tol, max_iters, K)) != SOR_OK) return st;
  const Layout L = make_layout(n, prec);
  const size_t bytes = (size_t)L.elems() * sizeof(T);
  const BufRole ra = prec == kF64 ? kGridA64 : kGridA32;
  const BufRole rb = prec == kF64 ? kGridB64 : kGridB32;
  const BufRole rf = prec == kF64 ? kF64Buf : kF32Buf;
  if ((st = ensure(c, ra, bytes)) || (st = ensure(c, rb, bytes))) return st;
  if (rhs && (st = ensure(c, rf, bytes))) return st;
  T *A = origin<T>(c, ra, L), *B = origin<T>(c, rb, L);
  T *F = rhs ? origin<T>(c, rf, L) : nullptr;
  return solve_plain_on(c, prec, L, (void *)u, bdy, rhs, A, B, F, (Ctl *)c->bufs[kCtlBuf].p,
                        omega, Sched{max_iters, K, tol}, (hipStream_t)stream, out, hist);
}

}  // namespace

namespace sor {

sor_status check_sched(sor_ctx *c, double tol, int64_t max_iters, int64_t K) {
  if (!(tol >= 0.0)) return fail(c, SOR_EINVAL, "tol = %g must be >= 0", tol);
  if (max_iters < 1) return fail(c, SOR_EINVAL, "max_iters must be >= 1");
  if (K < 1) return fail(c, SOR_EINVAL, "check_every must be >= 1");
  return SOR_OK;
}

sor_status solve_plain_on(sor_ctx *c, int prec, const Layout &L, void *u, const void *bdy,
                          const void *rhs, void *A, void *B, void *F, Ctl *ctl, double omega,
                          const Sched &sc, hipStream_t s, sor_result *out, double *hist) {
  const int n = L.n;
  unsigned *bad = &ctl->input_nonfinite;
  // The input flag must start clear: a reset moves it out of the way (the
  // reset at the start of the sweeps then takes what packing finds).
  HIP_TRY(c, launch_ctl_reset(ctl, s));
  HIP_TRY(c, launch_pack(prec, u, bdy, A, B, L.pitch, n, bad, s));
  if (rhs) HIP_TRY(c, launch_pack_rhs(prec, rhs, F, L.pitch, n, bad, s));
  *out = sor_result{};
  out->rel_residual = NAN;
  void *res_grid = A;
  sor_status st = run_sweeps(c, prec, L, A, B, rhs ? F : nullptr, omega, sc, s, out, hist,
                             &res_grid, 0, ctl);
  if (st == SOR_OK || st == SOR_NOT_CONVERGED || st == SOR_ENONFINITE) {
    HIP_TRY(c, launch_unpack(prec, res_grid, u, L.pitch, n, s));
    HIP_TRY(c, hipStreamSynchronize(s));
  }
  return st;
}

}  // namespace sor

extern "C" {

const char *sor_version(void) { return "sor 0.2.0 gfx950"; }

double sor_omega_opt(int32_t n) { return sor::omega_opt(n); }

sor_status sor_ctx_create(int device, sor_ctx **out) {
  if (!out) return SOR_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) {
    (void)hipGetLastError();
    return SOR_EDEVICE;
  }
  if (device < 0 || device >= count) return SOR_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return SOR_EDEVICE;
  sor_ctx *c = new (std::nothrow) sor_ctx;
  if (!c) return SOR_ENOMEM;
  c->device = device;
  try {
    c->err.reserve(512);        // error messages then fit without reallocation
  } catch (...) {
    delete c;
    return SOR_ENOMEM;
  }
  if (hipHostMalloc((void **)&c->host_ctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&c->host_stats, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    sor_ctx_destroy(c);
    return SOR_ENOMEM;
  }
  // Two control blocks: the solve's, and one for a truncated re-run that
  // must report non-finite values (see run_sweeps).
  if (ensure(c, kCtlBuf, 2 * sizeof(Ctl)) != SOR_OK) {
    sor_ctx_destroy(c);
    return SOR_ENOMEM;
  }
  // Device address of the allocation-free solve's working memory on this
  // device (resolved once per device; a failure is reported by that solve).
  (void)noalloc_init(c);
  *out = c;
  return SOR_OK;
}

void sor_ctx_destroy(sor_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  batch_state_free(c);
  mix_state_free(c);
  for (DevBuf &b : c->bufs)
    if (b.p) (void)hipFree(b.p);
  if (c->host_ctl) (void)hipHostFree(c->host_ctl);
  if (c->host_stats) (void)hipHostFree(c->host_stats);
  delete c;
}

const char *sor_last_error(const sor_ctx *c) { return c ? c->err.c_str() : "null context"; }

sor_status sor_ctx_set_profiling(sor_ctx *c, int32_t on) {
  if (!c) return SOR_EINVAL;
  c->prof = on != 0;
  c->prof_ms = 0.0;
  c->prof_launches = 0;
  return SOR_OK;
}

sor_status sor_ctx_get_profile(const sor_ctx *c, double *kernel_ms, int64_t *launches) {
  if (!c || !kernel_ms || !launches) return SOR_EINVAL;
  *kernel_ms = c->prof_ms;
  *launches = c->prof_launches;
  return SOR_OK;
}

sor_status sor_ctx_set_kernel(sor_ctx *c, int32_t kernel) {
  if (!c) return SOR_EINVAL;
  if (kernel != SOR_KERNEL_BLOCKED && kernel != SOR_KERNEL_SIMPLE)
    return fail(c, SOR_EINVAL, "unknown kernel %d", kernel);
  c->kernel = kernel;
  return SOR_OK;
}

sor_status sor_ctx_set_tiling(sor_ctx *c, int32_t bits, const sor_tiling *t) {
  if (!c || !t) return SOR_EINVAL;
  const int p = prec_index(bits);
  if (p < 0) return fail(c, SOR_EINVAL, "bits must be 64, 32 or 16");
  sor_tiling nt = c->tiling[p];
  if (t->iters_per_pass) {
    if (!blocked_T_supported(t->iters_per_pass))
      return fail(c, SOR_EINVAL, "iters_per_pass must be in 1..%d", kTMax);
    nt.iters_per_pass = t->iters_per_pass;
  }
  if (t->seg_rows) {
    if (t->seg_rows < 8 || t->seg_rows > 1024 || (t->seg_rows & 1))
      return fail(c, SOR_EINVAL, "seg_rows must be even and in 8..1024");
    nt.seg_rows = t->seg_rows;
  }
  c->tiling[p] = nt;
  if (t->iters_per_pass) c->depth_auto[p] = false;
  clear_tuning(c, p);
  return SOR_OK;
}

sor_status sor_ctx_get_tiling(const sor_ctx *c, int32_t bits, sor_tiling *t) {
  if (!c || !t) return SOR_EINVAL;
  const int p = prec_index(bits);
  if (p < 0) return SOR_EINVAL;
  *t = c->tiling[p];
  if (c->depth_auto[p]) t->iters_per_pass = 0;
  return SOR_OK;
}

sor_status sor_ctx_tiling_for(sor_ctx *c, int32_t bits, int32_t n, int32_t has_rhs,
                              sor_tiling *t) {
  if (!c || !t) return SOR_EINVAL;
  const int p = prec_index(bits);
  if (p < 0) return fail(c, SOR_EINVAL, "bits must be 64, 32 or 16");
  if (n < 1 || n > kMaxN) return fail(c, SOR_EINVAL, "n = %d outside 1..%d", n, kMaxN);
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, SOR_EDEVICE, "hipSetDevice failed");
  *t = tuned_tiling(c, p, n, has_rhs != 0);
  return SOR_OK;
}

sor_status sor_solve_f64(sor_ctx *c, double *u, const double *bdy, const double *rhs,
                         int32_t n, double omega, double tol, int64_t max_iters,
                         int64_t check_every, void *stream, sor_result *out,
                         double *max_hist) {
  return solve_plain<double>(c, kF64, u, bdy, rhs, n, omega, tol, max_iters,
                             check_every, stream, out, max_hist);
}

sor_status sor_solve_f32(sor_ctx *c, float *u, const float *bdy, const float *rhs,
                         int32_t n, double omega, double tol, int64_t max_iters,
                         int64_t check_every, void *stream, sor_result *out,
                         double *max_hist) {
  return solve_plain<float>(c, kF32, u, bdy, rhs, n, omega, tol, max_iters,
                            check_every, stream, out, max_hist);
}

sor_status sor_solve3d_f64(sor_ctx *c, double *u, const double *bdy, const double *rhs,
                           int32_t n, double omega, double tol, int64_t max_iters,
                           int64_t check_every, void *stream, sor_result *out,
                           double *hist) {
  if (!c) return SOR_EINVAL;
  c->err.clear();
  if (n < 1 || n > kMaxN3) return fail(c, SOR_EINVAL, "n = %d outside 1..%d", n, kMaxN3);
  sor_status st = check_common(c, u, bdy, rhs, n, omega);
  if (st != SOR_OK) return st;
  if (!out) return fail(c, SOR_EINVAL, "out must not be NULL");
  if ((st = check_sched(c, tol, max_iters, check_every)) != SOR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const bool simple = c->kernel == SOR_KERNEL_SIMPLE;
  Tiling3 t{}, t1{};
  if (!simple) {
    const int T = iters3d_for(c, check_every, rhs != nullptr);
    t = tiling3_for(c, n, rhs != nullptr, T);
    t1 = T == 1 ? t : tiling3_for(c, n, rhs != nullptr, 1);
    if (!t.ok || !t1.ok)
      return fail(c, SOR_EINVAL, "3-D tile region %d x %d exceeds one workgroup's positions",
                  t.ok ? t1.RX : t.RX, t.ok ? t1.RY : t.RY);
  }
  const size_t elems = (size_t)grid3_pitch(n) * (size_t)(n + 2) * (size_t)(n + 2);
  if ((st = ensure(c, kGridA64, elems * sizeof(double)))) return st;
  if (!simple && (st = ensure(c, kGridB64, elems * sizeof(double)))) return st;
  if (rhs && (st = ensure(c, kF64Buf, elems * sizeof(double)))) return st;
  double *A = (double *)c->bufs[kGridA64].p;
  double *B = simple ? nullptr : (double *)c->bufs[kGridB64].p;
  double *F = rhs ? (double *)c->bufs[kF64Buf].p : nullptr;
  unsigned *bad = &((Ctl *)c->bufs[kCtlBuf].p)->input_nonfinite;
  HIP_TRY(c, launch_pack3d(u, bdy, rhs, A, B, F, n, bad, s));
  *out = sor_result{};
  out->rel_residual = NAN;
  const Sched sc{max_iters, check_every, tol};
  double *res_grid = A;
  st = run_iterations3d(c, A, B, F, n, omega, simple ? nullptr : &t, &t1, sc, s, out, hist,
                        &res_grid);
  if (st == SOR_OK || st == SOR_NOT_CONVERGED || st == SOR_ENONFINITE) {
    HIP_TRY(c, launch_unpack3d(res_grid, u, n, s));
    HIP_TRY(c, hipStreamSynchronize(s));
  }
  return st;
}

namespace {

// Jacobi, four-colour or block-parallel solve (arguments checked except the
// ordering's own): pack, run, unpack.
sor_status solve_ordered(sor_ctx *c, int32_t ordering, double *u, const double *bdy,
                         const double *rhs, int32_t n, double omega, int32_t blk_rows,
                         int32_t blk_cols, double tol, int64_t max_iters,
                         int64_t check_every, void *stream, sor_result *out, double *hist) {
  sor_status st = check_common(c, u, bdy, rhs, n, omega);
  if (st != SOR_OK) return st;
  if (!out) return fail(c, SOR_EINVAL, "out must not be NULL");
  if ((st = check_sched(c, tol, max_iters, check_every)) != SOR_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const Layout L = make_layout(n, kF64);
  const size_t bytes = (size_t)L.elems() * sizeof(double);
  const bool jacobi = ordering == SOR_ORDER_JACOBI;
  const bool simple = c->kernel == SOR_KERNEL_SIMPLE;
  if ((st = ensure(c, kGridA64, bytes)) || (st = ensure(c, kGridB64, bytes))) return st;
  if (rhs && (st = ensure(c, kF64Buf, bytes))) return st;
  double *A = origin<double>(c, kGridA64, L), *B = origin<double>(c, kGridB64, L);
  double *F = rhs ? origin<double>(c, kF64Buf, L) : nullptr;
  Ctl *ctl = (Ctl *)c->bufs[kCtlBuf].p;
  unsigned *bad = &ctl->input_nonfinite;
  HIP_TRY(c, launch_pack(kF64, u, bdy, A, B, L.pitch, n, bad, s));
  if (rhs) HIP_TRY(c, launch_pack_rhs(kF64, rhs, F, L.pitch, n, bad, s));
  *out = sor_result{};
  out->rel_residual = NAN;
  const Sched sc{max_iters, check_every, tol};
  void *res_grid = A;
  if (jacobi && simple) {
    st = run_iteration_loop(c, sc, s, out, hist, [&](long long, long long k, int &iters) {
      iters = 1;
      const bool even = (k & 1) == 0;
      return launch_jacobi_iteration(even ? A : B, even ? B : A, F, L.pitch, n, omega, ctl,
                                     sc, s);
    });
    res_grid = (out->passes & 1) ? B : A;
  } else {
    int ord = pass_ordering(ordering);
    // Block-parallel with blocks of even width (or no column edge inside the
    // grid): the kernel without cross-lane old values.
    if (ord == 3 && (blk_cols % 2 == 0 || blk_cols >= n)) ord = 4;
    st = run_sweeps(c, kF64, L, A, B, F, omega, sc, s, out, hist, &res_grid, ord, ctl,
                    BlockShape{blk_rows, blk_cols});
  }
  if (st == SOR_OK || st == SOR_NOT_CONVERGED || st == SOR_ENONFINITE) {
    HIP_TRY(c, launch_unpack(kF64, res_grid, u, L.pitch, n, s));
    HIP_TRY(c, hipStreamSynchronize(s));
  }
  return st;
}

}  // namespace

sor_status sor_solve_variant_f64(sor_ctx *c, int32_t ordering, double *u, const double *bdy,
                                 const double *rhs, int32_t n, double omega, double tol,
                                 int64_t max_iters, int64_t check_every, void *stream,
                                 sor_result *out, double *hist) {
  if (!c) return SOR_EINVAL;
  c->err.clear();
  if (ordering == SOR_ORDER_RED_BLACK)
    return sor_solve_f64(c, u, bdy, rhs, n, omega, tol, max_iters, check_every, stream, out,
                         hist);
  if (ordering == SOR_ORDER_BLOCK_PARALLEL)
    return fail(c, SOR_EINVAL, "the block-parallel ordering needs a block shape: "
                "use sor_solve_blockpar_f64");
  if (ordering != SOR_ORDER_JACOBI && ordering != SOR_ORDER_FOUR_COLOUR)
    return fail(c, SOR_EINVAL, "unknown ordering %d", ordering);
  return solve_ordered(c, ordering, u, bdy, rhs, n, omega, 1, 1, tol, max_iters, check_every,
                       stream, out, hist);
}

sor_status sor_solve_blockpar_f64(sor_ctx *c, double *u, const double *bdy, const double *rhs,
                                  int32_t n, double omega, int32_t block_rows,
                                  int32_t block_cols, double tol, int64_t max_iters,
                                  int64_t check_every, void *stream, sor_result *out,
                                  double *hist) {
  if (!c) return SOR_EINVAL;
  c->err.clear();
  if (block_rows < 1 || block_cols < 1)
    return fail(c, SOR_EINVAL, "block shape %d x %d: both sides must be >= 1", block_rows,
                block_cols);
  // A side of n or more puts every interior row (column) in one block: the
  // same iteration as a side of n, which keeps the kernels' block arithmetic
  // far from overflow.
  if (n > 0) {
    block_rows = std::min(block_rows, n);
    block_cols = std::min(block_cols, n);
  }
  return solve_ordered(c, SOR_ORDER_BLOCK_PARALLEL, u, bdy, rhs, n, omega, block_rows,
                       block_cols, tol, max_iters, check_every, stream, out, hist);
}

sor_status sor_ctx_set_variant_tiling(sor_ctx *c, int32_t ordering, const sor_tiling *t) {
  if (!c || !t) return SOR_EINVAL;
  c->err.clear();
  const int ord = pass_ordering(ordering);
  if (ord < 0) return fail(c, SOR_EINVAL, "ordering %d has no blocked tiling", ordering);
  sor_tiling nt = c->tiling_var[ord];
  if (t->iters_per_pass) {
    if (!blocked_ord_T_supported(ord, t->iters_per_pass))
      return fail(c, SOR_EINVAL, "iters_per_pass must be in 1..%d for this ordering",
                  ord == 1 ? kTMaxC4 : kTMax);
    nt.iters_per_pass = t->iters_per_pass;
  }
  if (t->seg_rows) {
    if (t->seg_rows < 8 || t->seg_rows > 1024 || (t->seg_rows & 1))
      return fail(c, SOR_EINVAL, "seg_rows must be even and in 8..1024");
    nt.seg_rows = t->seg_rows;
  }
  c->tiling_var[ord] = nt;
  return SOR_OK;
}

sor_status sor_ctx_get_variant_tiling(const sor_ctx *c, int32_t ordering, sor_tiling *t) {
  if (!c || !t || pass_ordering(ordering) < 0) return SOR_EINVAL;
  *t = c->tiling_var[pass_ordering(ordering)];
  return SOR_OK;
}

sor_status sor_ctx_set_tiling3d(sor_ctx *c, int32_t iters_per_launch, int32_t cx, int32_t cy,
                                int32_t zs) {
  if (!c) return SOR_EINVAL;
  c->err.clear();
  if (iters_per_launch < 0 || iters_per_launch > 2)
    return fail(c, SOR_EINVAL, "3-D tiling: iters_per_launch = %d not in 0..2", iters_per_launch);
  if (cx < 0 || cy < 0 || zs < 0)
    return fail(c, SOR_EINVAL, "3-D tiling (%d, %d, %d): sizes must be >= 0", cx, cy, zs);
  const int ring = iters_per_launch == 2 ? 4 : 2;
  const int PL = stream3d_positions(iters_per_launch == 2 ? 2 : 1);
  if (cx > 0 && (cx + 2 * ring) * (1 + 2 * ring) > PL)
    return fail(c, SOR_EINVAL, "3-D tiling: cx = %d leaves no room for a row of tiles", cx);
  if (cx > 0 && cy > 0 && (cx + 2 * ring) * (cy + 2 * ring) > PL)
    return fail(c, SOR_EINVAL, "3-D tiling: (%d + %d) x (%d + %d) positions exceed %d", cx,
                2 * ring, cy, 2 * ring, PL);
  c->tiling3d[0] = iters_per_launch;
  c->tiling3d[1] = cx;
  c->tiling3d[2] = cy;
  c->tiling3d[3] = zs;
  return SOR_OK;
}

sor_status sor_ctx_tiling3d_for(sor_ctx *c, int32_t n, int32_t has_rhs, int64_t check_every,
                                int32_t *iters_per_launch, int32_t *cx, int32_t *cy,
                                int32_t *zs) {
  if (!c || !iters_per_launch || !cx || !cy || !zs) return SOR_EINVAL;
  c->err.clear();
  if (n < 1 || n > kMaxN3) return fail(c, SOR_EINVAL, "n = %d outside 1..%d", n, kMaxN3);
  if (check_every < 1) return fail(c, SOR_EINVAL, "check_every must be >= 1");
  HIP_TRY(c, hipSetDevice(c->device));
  const int T = iters3d_for(c, check_every, has_rhs != 0);
  const Tiling3 t = tiling3_for(c, n, has_rhs != 0, T);
  *iters_per_launch = T;
  *cx = t.CX;
  *cy = t.CY;
  *zs = t.Zs;
  return t.ok ? SOR_OK : fail(c, SOR_EINVAL, "3-D tile region %d x %d too large", t.RX, t.RY);
}

sor_status sor_residual_f64(sor_ctx *c, const double *u, const double *bdy,
                            const double *rhs, int32_t n, double *r, double *stats,
                            void *stream) {
  sor_status st = check_common(c, u, bdy, rhs, n, 1.0);
  if (st != SOR_OK) return st;
  if (!stats) return fail(c, SOR_EINVAL, "stats must not be NULL");
  if (r && !is_device_ptr(c, r)) return fail(c, SOR_EINVAL, "r is not a device pointer");
  hipStream_t s = (hipStream_t)stream;
  const Layout L = make_layout(n, kF64);
  const size_t bytes = (size_t)L.elems() * sizeof(double);
  if ((st = ensure(c, kGridA64, bytes))) return st;
  if (rhs && (st = ensure(c, kF64Buf, bytes))) return st;
  if ((st = ensure(c, kPartials, (size_t)residual_partials(n) * 3 * sizeof(double)))) return st;
  if ((st = ensure(c, kStats, 4 * sizeof(double)))) return st;
  double *U = origin<double>(c, kGridA64, L);
  double *F = rhs ? origin<double>(c, kF64Buf, L) : nullptr;
  HIP_TRY(c, launch_pack(kF64, u, bdy, U, nullptr, L.pitch, n, nullptr, s));
  if (rhs) HIP_TRY(c, launch_pack_rhs(kF64, rhs, F, L.pitch, n, nullptr, s));
  double *dstats = (double *)c->bufs[kStats].p;
  HIP_TRY(c, launch_residual(U, F, L.pitch, n, r, (double *)c->bufs[kPartials].p, dstats,
                             nullptr, kF32, 0, 0, s));
  HIP_TRY(c, hipMemcpyAsync(c->host_stats, dstats, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  for (int k = 0; k < 3; ++k) stats[k] = c->host_stats[k];
  return SOR_OK;
}

sor_status sor_solve_mixed(sor_ctx *c, double *u, const double *bdy, const double *rhs,
                           int32_t n, double omega, double rel_tol, int64_t max_outer,
                           int32_t inner_bits, int64_t inner_iters, void *stream,
                           sor_result *out, double *rel_hist) {
  sor_status st = check_common(c, u, bdy, rhs, n, omega);
  if (st != SOR_OK) return st;
  if (!out) return fail(c, SOR_EINVAL, "out must not be NULL");
  if (!(rel_tol >= 0.0)) return fail(c, SOR_EINVAL, "rel_tol must be >= 0");
  if (max_outer < 0) return fail(c, SOR_EINVAL, "max_outer must be >= 0");
  if (inner_bits != 32 && inner_bits != 16) return fail(c, SOR_EINVAL, "inner_bits must be 32 or 16");
  if (inner_bits == 16 && n > kMaxN16)
    return fail(c, SOR_EINVAL, "binary16 inner storage supports n <= %d (n = %d)", kMaxN16, n);
  if (inner_iters <= 0) inner_iters = mixed_inner_default(n);
  hipStream_t s = (hipStream_t)stream;
  const int plo = inner_bits == 32 ? kF32 : kF16;
  const Layout L = make_layout(n, kF64);
  const Layout Llo = make_layout(n, plo);
  const size_t b64 = (size_t)L.elems() * sizeof(double);
  const size_t blo = (size_t)Llo.elems() * (size_t)prec_bytes(plo);
  if ((st = ensure(c, kGridA64, b64))) return st;
  if (rhs && (st = ensure(c, kF64Buf, b64))) return st;
  if ((st = ensure(c, kGridA32, blo)) || (st = ensure(c, kGridB32, blo)) ||
      (st = ensure(c, kLoRhs, blo)))
    return st;
  if ((st = ensure(c, kPartials, (size_t)residual_partials(n) * 3 * sizeof(double)))) return st;
  if ((st = ensure(c, kStats, 4 * sizeof(double)))) return st;
  double *U = origin<double>(c, kGridA64, L);
  double *F = rhs ? origin<double>(c, kF64Buf, L) : nullptr;
  char *EA = (char *)c->bufs[kGridA32].p + Llo.origin_off() * prec_bytes(plo);
  char *EB = (char *)c->bufs[kGridB32].p + Llo.origin_off() * prec_bytes(plo);
  char *R = (char *)c->bufs[kLoRhs].p + Llo.origin_off() * prec_bytes(plo);
  double *dstats = (double *)c->bufs[kStats].p;
  double *partials = (double *)c->bufs[kPartials].p;
  HIP_TRY(c, launch_pack(kF64, u, bdy, U, nullptr, L.pitch, n, nullptr, s));
  if (rhs) HIP_TRY(c, launch_pack_rhs(kF64, rhs, F, L.pitch, n, nullptr, s));
  // The inner right-hand side grid has a zero ring; only its interior changes.
  HIP_TRY(c, launch_fill_zero(plo, R, Llo.pitch, n, s));

  *out = sor_result{};
  const double h = 1.0 / (double)(n + 1);
  const double target = plo == kF16 ? std::ldexp(h * h, 14) / 0.0737 : 1.0;
  long long outer = 0, inner_total = 0, passes = 0;
  double rel = NAN, last_corr = NAN;
  sor_status result = SOR_NOT_CONVERGED;
  for (;;) {
    HIP_TRY(c, launch_residual(U, F, L.pitch, n, nullptr, partials, dstats, nullptr,
                               plo, Llo.pitch, 0, s));
    HIP_TRY(c, hipMemcpyAsync(c->host_stats, dstats, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    const double sr = c->host_stats[0], sb = c->host_stats[1], rinf = c->host_stats[2];
    rel = sb > 0.0 ? std::sqrt(sr) / std::sqrt(sb) : std::sqrt(sr);
    if (rel_hist) rel_hist[outer] = rel;
    if (!std::isfinite(rel)) { result = SOR_ENONFINITE; fail(c, result, "non-finite residual"); break; }
    if (rel <= rel_tol || rinf == 0.0) { result = SOR_OK; break; }
    if (outer == max_outer) break;
    int e2;
    std::frexp(target / rinf, &e2);
    const int p = e2 - 1;
    // r -> inner right-hand side, fl(r * 2^p).
    HIP_TRY(c, launch_residual(U, F, L.pitch, n, nullptr, partials, dstats, R, plo,
                               Llo.pitch, p, s));
    HIP_TRY(c, launch_fill_zero(plo, EA, Llo.pitch, n, s));
    HIP_TRY(c, launch_fill_zero(plo, EB, Llo.pitch, n, s));
    // inner_iters sweeps, no stopping test (tol = 0 never passes).
    const Sched sc{inner_iters, inner_iters, 0.0};
    void *res_grid = EA;
    sor_result ir{};
    st = run_sweeps(c, plo, Llo, EA, EB, R, omega, sc, s, &ir, nullptr, &res_grid, 0,
                    (Ctl *)c->bufs[kCtlBuf].p);
    if (st == SOR_ENONFINITE) { result = st; break; }
    if (st != SOR_NOT_CONVERGED && st != SOR_OK) return st;
    inner_total += inner_iters;
    passes += ir.passes;
    unsigned long long *mb = (unsigned long long *)(dstats + 3);
    HIP_TRY(c, hipMemsetAsync(mb, 0, sizeof(unsigned long long), s));
    HIP_TRY(c, launch_accumulate(U, L.pitch, res_grid, plo, Llo.pitch, n, p, mb, s));
    HIP_TRY(c, hipMemcpyAsync(c->host_stats + 3, mb, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    last_corr = c->host_stats[3];
    ++outer;
  }
  HIP_TRY(c, launch_unpack(kF64, U, u, L.pitch, n, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  out->iterations = inner_total;
  out->final_max_delta = last_corr;
  out->converged = result == SOR_OK;
  out->outer_steps = (int32_t)outer;
  out->rel_residual = rel;
  out->passes = passes;
  return result;
}

}  // extern "C"
