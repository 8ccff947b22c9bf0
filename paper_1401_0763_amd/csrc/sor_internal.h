// Internal declarations shared by the host runtime and the device code of
// libsor.  Not part of the public ABI (include/sor.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sor {

// ---------------------------------------------------------------------------
// Padded working-grid layout (device memory owned by the library)
//
// A grid with n interior nodes per side is stored with its boundary ring
// (rows/columns 0 and n+1) plus kMY margin rows above and below and kMX margin
// columns on the left.  Element (r, c), -kMY <= r <= n+1+kMY and
// -kMX <= c < pitch-kMX, lives at origin[r * pitch + c], where `origin` points
// kMY rows and kMX columns into the allocation.  Rows start on 256-byte
// boundaries.  Margin contents are never read into interior results.
// ---------------------------------------------------------------------------
constexpr int kMX = 16;           // left margin columns (>= widest halo)
constexpr int kMY = 16;           // top and bottom margin rows (>= 2 * kTMax)
constexpr int kTMax = 8;          // most iterations one blocked pass applies
constexpr int kSlots = 64;        // partial-maximum slots per pass
constexpr int kHistCap = 1024;    // per-iteration maxima kept per solve chunk
constexpr int kLanes = 64;        // wavefront width on CDNA
constexpr int kMaxN = 65536;      // largest grid side (32-bit buffer offsets)
constexpr int kMaxSegRows = 1024; // largest rows per tile

// Storage precisions.
enum Prec : int { kF64 = 0, kF32 = 1, kF16 = 2 };

__host__ __device__ inline int prec_bytes(int prec) { return prec == kF64 ? 8 : prec == kF32 ? 4 : 2; }
// Cells held per lane by the blocked kernel (one 16-byte access for FP64 and
// FP32, one 8-byte access for FP16 storage).
__host__ __device__ inline int prec_cells(int prec) { return prec == kF64 ? 2 : 4; }

struct Layout {
  int32_t n = 0;
  int64_t pitch = 0;    // elements per row
  int64_t rows = 0;     // allocated rows (n + 2 + 2*kMY)
  int64_t elems() const { return pitch * rows; }
  int64_t origin_off() const { return (int64_t)kMY * pitch + kMX; }
};
Layout make_layout(int n, int prec);

// Device-resident control block of one solve: partial maxima of the running
// pass, pass bookkeeping and the stopping verdict (Algorithm 1's
// shouldCheckConvergence / maxChange / hasConverged state).
struct alignas(256) Ctl {
  unsigned long long slots[kSlots][kTMax];  // bit patterns of non-negative doubles
  unsigned int counter;     // wavefronts finished in the running pass
  unsigned int nonfinite;   // sticky: a value became NaN or infinite
  int stop;                 // 0 running, 1 converged, 2 non-finite
  unsigned int input_nonfinite;  // set by packing when an input is not finite
  int stop_tentative;       // 1: converged inside a pass that also made a
                            // non-finite value (the truncated re-run decides)
  int pad_;
  long long it_base;        // iterations completed by finished passes
  long long stop_iter;      // iteration whose check passed
  double stop_max;
  long long last_iter;      // last checked iteration
  double last_max;
  long long passes_done;
  double hist[kHistCap];    // change of iteration it at hist[(it-1) % kHistCap]
};

// Stopping schedule (Algorithm 1): check when it % check_every == 0 or
// it == max_iters; converged when the change is strictly below tol.
struct Sched {
  long long max_iters;
  long long check_every;
  double tol;
};

// One grid as seen by the sweep kernels.
struct GridView {
  const void *in;       // origin of the input working grid
  void *out;            // origin of the output working grid (may equal in for SIMPLE)
  const void *F;        // origin of the source grid (h*h*f), or nullptr
  int64_t pitch;
  int32_t n;
  int32_t nstrips;      // column strips of the blocked kernel
  int32_t nseg;         // row segments of the blocked kernel
  int32_t seg_rows;     // output rows per segment (even)
  double omega;
};

// Block shape of a block-parallel pass, in interior cells (>= 1 each).
struct BlockShape {
  int32_t rows = 1;
  int32_t cols = 1;
};

// ---------------------------------------------------------------------------
// Batched solves: many grids advanced by one persistent kernel.
//
// Work items are (grid, tile) pairs of one pass of one grid.  They live in a
// ring buffer; the wave that finishes the last tile of a grid's pass
// evaluates that grid's stopping rule and publishes the tiles of its next
// pass, so an item is only ever published after everything it depends on has
// completed.  Each slot carries a tag (launch generation, index) that the
// consumer waits for.
// ---------------------------------------------------------------------------
constexpr int kBSlots = 8;          // partial-maximum slots per grid

struct alignas(128) BGrid {
  // Set by the host.
  void *A;                 // origin of working grid A (FP64 or storage type)
  void *B;                 // origin of working grid B
  const void *F;           // origin of h*h*f, or nullptr
  double *user_u;          // caller's n*n interior (in: guess, out: result)
  const double *user_bdy;  // caller's 4n boundary
  const double *user_f;    // caller's n*n source, or nullptr
  int64_t pitch;
  int32_t n;
  int32_t T;               // iterations per full pass
  int32_t seg_rows;
  int32_t pad0;
  double omega;
  double tol;
  int64_t max_iters;
  int64_t check_every;
  int64_t pass_budget;     // passes this launch may run before pausing
  // Device state (the host initialises it, the kernel advances it).
  int32_t cur;             // 0: the iterate is in A, 1: in B
  int32_t status;          // 0 running, 1 converged, 2 iteration limit,
                           // 3 non-finite, 4 paused (budget spent)
  int32_t mode;            // 0 normal passes, 1 re-running a truncated pass
  int32_t pass_T;          // depth of the pass whose tiles are queued
  int32_t ntiles;          // tiles of that pass
  uint32_t tiles_done;
  uint32_t nonfinite;
  int32_t pad1;
  int64_t it_base;         // iterations completed
  int64_t rerun_left;      // iterations still to redo in re-run mode
  int64_t stop_iter;
  int64_t passes;          // passes completed (all launches)
  double stop_max;
  double last_max;         // change at the last checked iteration
  int64_t t_done;          // device wall clock when the grid retired
  unsigned long long slots[kBSlots][kTMax];
};

struct alignas(128) BQueue {
  unsigned long long head;   // next index to take
  unsigned long long tail;   // next index to publish
  unsigned long long gen;    // generation of this launch (tag high bits)
  unsigned long long mask;   // ring capacity - 1 (power of two)
  int remaining;             // grids that still have queued work
  int error;                 // 1: a wait timed out
  long long deadline_ticks;  // wait limit in wall-clock ticks
  long long t0;              // wall clock when the launch's first wave began
  long long slice_ticks;     // > 0: grids pause after this long (time slice)
};

struct BItem {
  unsigned long long tag;      // (gen << 40) | (index + 1) once published
  unsigned long long payload;  // (grid << 32) | tile
};

__host__ __device__ inline unsigned long long bq_tag(unsigned long long gen, unsigned long long idx) {
  return (gen << 40) | (idx + 1);
}

// Tiles of one blocked pass of depth T over an n-grid.
__host__ __device__ inline int blocked_ntiles(int prec, int n, int T, int seg_rows) {
  const int V = prec_cells(prec);
  const int S = 2 * T;
  const int A = ((S + V - 1) / V) * V;
  const int CW = kLanes * V - 2 * A;
  return ((n + 1 + CW - 1) / CW) * ((n + 1 + seg_rows - 1) / seg_rows);
}

// Mixed-precision batched solves (FP64 defect correction around low-precision
// sweeps).  Every grid cycles through four phases, each a set of work items:
//   RESID   row blocks: FP64 residual r, partial sums of r^2, b^2 and max|r|
//   CAST    row blocks: inner right-hand side fl(r * 2^p), zero inner iterate
//   SWEEP   blocked-pass tiles of the inner solve (low precision)
//   ACCUM   row blocks: u += e * 2^-p, partial max |correction|
// The wave that completes a phase's last item runs the phase's serial step
// (sums in a fixed order, stopping test, scale choice) and queues the next.
enum MixPhase : int { kPhResid = 0, kPhCast = 1, kPhSweep = 2, kPhAccum = 3 };
constexpr int kMixRows = 8;          // rows per row-block item

struct alignas(128) BMGrid {
  // Set by the host.
  double *U;               // FP64 iterate (padded origin)
  const double *F;         // h*h*f (padded origin) or nullptr
  void *EA;                // inner iterate ping-pong (low precision, padded)
  void *EB;
  void *R;                 // inner right-hand side (low precision, padded)
  double *partials;        // 3 doubles per row block
  double *user_u;
  const double *user_bdy;
  const double *user_f;
  int64_t pitch;           // FP64 grids
  int64_t lo_pitch;        // low-precision grids
  int32_t n;
  int32_t T;               // inner iterations per blocked pass
  int32_t seg_rows;
  int32_t nrb;             // row blocks
  double omega;
  double rel_tol;          // stop when ||r||_2/||b||_2 <= rel_tol
  double corr_tol;         // or when max |correction| < corr_tol (if > 0)
  double target;           // scaling target of the inner right-hand side
  int64_t max_outer;
  int64_t inner_iters;
  // Device state.
  int32_t phase;
  int32_t status;          // 0 running or paused, 1 converged, 2 limit, 3 non-finite
  int32_t cur;             // inner iterate in EA (0) or EB (1)
  int32_t pass_T;
  int32_t nitems;          // items of the queued phase
  int32_t scale_exp;
  uint32_t items_done;
  uint32_t nonfinite;      // an inner sweep produced a non-finite value
  int64_t outer;           // corrections applied
  int64_t inner_left;
  int64_t inner_total;
  int64_t passes;
  double rel;              // latest relative residual
  double rinf;
  double last_corr;        // max |correction| of the latest correction
};

hipError_t launch_mix_pack(int prec_lo, const BMGrid *grids, const int *slots, int count,
                           int max_n, hipStream_t s);
hipError_t launch_mix_unpack(const BMGrid *grids, const int *slots, int count,
                             int max_n, hipStream_t s);
hipError_t launch_mix_batch(int prec_lo, bool dyn, BMGrid *grids, BQueue *q, BItem *ring,
                            int waves, hipStream_t s);
// Persistent wavefronts per CU of the mixed batched kernel: its occupancy,
// capped at one per SIMD.
int mix_waves_per_cu(int prec_lo, bool dyn);

hipError_t launch_batch_pack(BGrid *grids, int count, int max_n,
                             hipStream_t s);
hipError_t launch_batch_unpack(const BGrid *grids, int count, int max_n,
                               hipStream_t s);
// Depth of the persistent batched FP64 sweep (its tile body has a source
// term; grids without one read it as zero).  Measured on 512 grids of sides
// 64-1024, one wavefront per SIMD: depth 7 solves the batch in 0.227 s
// against 0.234 s for depth 6 (with the neighbour exchange through DPP;
// before it, 0.29 s at depth 6 and 7, 0.35 s at depth 5 with two
// wavefronts per SIMD, 0.33 s at depth 8).  A grid's passes all have the
// tile geometry of this depth; shorter passes (re-runs, the last iterations
// before a limit) run in a tail kernel.
constexpr int kBatchT = 7;
// Depth of the inner passes of the mixed-precision persistent kernel
// (batched solves and the request server), measured the same way: the
// 512-grid batch refined with FP32 inner sweeps to each grid's FP64 residual
// takes 0.25 s at depth 6 (one wavefront per SIMD) against 0.35 s at depth 4
// (two), with the same inner iterations.
constexpr int kMixTMax = 6;
// Persistent batched sweep (FP64 storage).  The main kernel (tail false)
// takes its items from q/ring and parks grids that need a shorter pass in
// tq/tring; the tail kernel takes the parked passes from q/ring (pass tq = q,
// tring = ring).  waves: persistent wavefronts.
hipError_t launch_batch_f64(BGrid *grids, BQueue *q, BItem *ring, BQueue *tq, BItem *tring,
                            int waves, bool tail, hipStream_t s);
// Its persistent wavefronts per CU: the occupancy, capped at one per SIMD.
int batch_waves_per_cu_f64(bool tail);

// Geometry of the blocked kernel for a precision, iterations-per-pass T and
// ordering (0: red-black, 1: four-colour): V cells per lane, S stages, H halo
// rows, A halo columns, CW core columns.
struct BlockGeom {
  int V, S, H, A, CW;
  int W;        // steps per chunk of the row walk (window rows)
};
BlockGeom block_geom(int prec, int T, int ord = 0);

// ----------------------------- launchers ----------------------------------
hipError_t launch_ctl_reset(Ctl *ctl, hipStream_t s);
// Packing sets *bad (when bad is not null) if an input value is not finite.
hipError_t launch_pack(int prec, const void *u, const void *bdy, void *gridA,
                       void *gridB, int64_t pitch, int n, unsigned *bad,
                       hipStream_t s);
hipError_t launch_pack_rhs(int prec, const void *f, void *F, int64_t pitch,
                           int n, unsigned *bad, hipStream_t s);
hipError_t launch_unpack(int prec, const void *grid, void *u, int64_t pitch,
                         int n, hipStream_t s);
hipError_t launch_fill_zero(int prec, void *grid, int64_t pitch, int n,
                            hipStream_t s);
// Blocked pass of T iterations from v.in into v.out: red-black (ord 0, T in
// 1..kTMax, every precision), four-colour (ord 1, T in 1..kTMaxC4, FP64),
// Jacobi (ord 2, T in 1..kTMax, FP64) or block-parallel red-black (ord 3, or
// 4 when bs.cols is even or at least n; T in 1..kTMax, FP64, blocks of shape
// bs); the view's nstrips/nseg must match T and the ordering.  ctl ==
// nullptr runs without verdict or early exit.  mx (red-black) names the
// iterations of the pass whose maxima the stopping rule will read: -1 all,
// 0..T-1 that one, T none; a pass that forms more than these (every
// variant not built) reports the same values for them.
constexpr int kTMaxC4 = 5;
hipError_t launch_blocked_pass(int prec, int T, const GridView &v, Ctl *ctl,
                               const Sched &sc, hipStream_t s, int ord = 0,
                               const BlockShape &bs = BlockShape{}, int mx = -1);
bool blocked_T_supported(int T);
bool blocked_ord_T_supported(int ord, int T);
// Pass-kernel workgroups (wavefronts) resident per CU; 0 if the query fails.
int blocked_blocks_per_cu(int prec, int T, bool pois, int ord = 0);
// Simple kernel: one launch per colour, in place on v.in (v.out ignored).
hipError_t launch_simple_iteration(int prec, const GridView &v, Ctl *ctl,
                                   const Sched &sc, hipStream_t s);
// FP64 residual.  partials: device scratch of residual_partials(n) * 3
// doubles; stats: device double[3].  r (nullable): n*n output.  If lo_grid is
// non-null, also writes fl(r * 2^scale_exp) into that padded low-precision
// grid (prec_lo = kF32 or kF16).
int64_t residual_partials(int n);
hipError_t launch_residual(const double *U, const double *F, int64_t pitch,
                           int n, double *r, double *partials, double *stats,
                           void *lo_grid, int prec_lo, int64_t lo_pitch,
                           int scale_exp, hipStream_t s);
// U[interior] += (double)E * 2^-scale_exp; E is the low-precision grid.
// maxabs (device double, may be null) receives max |(double)E * 2^-scale_exp|.
hipError_t launch_accumulate(double *U, int64_t pitch, const void *E,
                             int prec_lo, int64_t lo_pitch, int n,
                             int scale_exp, unsigned long long *maxabs_bits,
                             hipStream_t s);

}  // namespace sor
