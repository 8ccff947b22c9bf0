/*
 * sor.h -- C ABI of libsor, a red-black successive over-relaxation (SOR)
 * solver for AMD Instinct MI355X (gfx950).
 *
 * Problem (Mittal 2014, abstract and Sec. 3.4): 2-D steady-state heat
 * conduction -lap(u) = f on the unit square, discretised with the 5-point
 * stencil on an n x n interior grid (mesh width h = 1/(n+1)), Dirichlet values
 * on the four edges.  f = 0 is the paper's Laplace case.
 *
 * Method (Sec. 2.1 Eq. 1; Sec. 3.1 with Fig. 1-2; Algorithm 1):
 *   every iteration updates the red cells ((i+j) even, full-array indices
 *   with the boundary at index 0) and then the black cells, each with
 *     s  = (N + S) + (W + E)   [+ h*h*f]
 *     dg = fma(0.25, s, -u)               (Gauss-Seidel value minus u, one rounding)
 *     u' = fma(omega, dg, u)              (Eq. 1 in increment form, one rounding)
 *   and the change of one iteration is max |u' - u| over all cells.  A check
 *   runs every check_every iterations and at the last allowed iteration; the
 *   solve stops at the first check whose change is strictly below tol.
 *
 * Array conventions shared by every entry point:
 *   u         n*n interior values, row-major, u[(i-1)*n + (j-1)] = cell (i,j);
 *             row 1 is next to the north edge.
 *   boundary  4*n values: north edge (j = 1..n), south edge (j = 1..n),
 *             west edge (i = 1..n), east edge (i = 1..n).  Corners are never
 *             read by the 5-point stencil and are not part of the interface.
 *   rhs       n*n source f of -lap(u) = f, row-major, or NULL for Laplace.
 *   All three are DEVICE pointers on the context's GPU (e.g. the data of
 *   torch tensors), owned by the caller, and must stay valid until the call
 *   returns.  A host or foreign-device pointer is rejected with SOR_EINVAL.
 *
 * Streams: `stream` is a hipStream_t (NULL for the null stream).  All device
 * work of a call is ordered on it; the call synchronises that stream before
 * it returns, so results are complete on return.
 *
 * Errors: no exception or abort crosses this ABI.  A negative status leaves
 * `u` unspecified; sor_last_error() describes the most recent failure of a
 * context.  A context is not thread-safe: use one per host thread.
 *
 * Ownership: the library owns its padded working grids and scratch, held in
 * the context, grown on demand and released by sor_ctx_destroy().
 */
#ifndef SOR_H
#define SOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sor_status {
    SOR_OK = 0,              /* converged (stopping rule met) / success      */
    SOR_NOT_CONVERGED = 1,   /* ran to the iteration limit; not an error     */
    SOR_EINVAL = -1,         /* invalid argument                             */
    SOR_ENOMEM = -2,         /* device or host allocation failed             */
    SOR_EDEVICE = -3,        /* HIP runtime error                            */
    SOR_ENONFINITE = -4,     /* a NaN or infinity appeared in the grid       */
    SOR_EBUSY = -5,          /* resource limit (e.g. server memory budget)   */
    SOR_ETIMEOUT = -6        /* a device-side wait exceeded its bound        */
} sor_status;

typedef struct sor_ctx sor_ctx;

/* Outcome of a solve. */
typedef struct sor_result {
    int64_t iterations;       /* plain solves: the 1-based iteration whose check
                                 passed, else max_iters.  Mixed: total inner
                                 iterations run.                              */
    double final_max_delta;   /* plain: max |u' - u| of the last checked
                                 iteration.  Mixed: max |correction| of the
                                 last correction (FP64).                      */
    int32_t converged;        /* 1 when the stopping rule was met            */
    int32_t outer_steps;      /* mixed: corrections applied; plain: 0        */
    double rel_residual;      /* mixed: final ||r||_2 / ||b||_2; plain: NaN  */
    int64_t passes;           /* sweep kernel passes that did work           */
    int32_t status;           /* this solve's sor_status (batched solves
                                 report one per grid)                         */
    int32_t reserved;
} sor_result;

/* Library version string, e.g. "sor 0.1.0 gfx950". */
const char *sor_version(void);

/* Young's optimal relaxation factor for the red-black ordering of the 5-point
 * (and 7-point) Dirichlet Laplacian with n interior nodes per side:
 * 2 / (1 + sin(pi h)), h = 1/(n+1), i.e. 2/(1 + sqrt(1 - mu^2)) with the
 * Jacobi spectral radius mu = cos(pi h).  Not in the paper (Sec. 2.1 runs a
 * fixed omega); the solves and the request server use it where the caller
 * passes no omega.  Returns NaN for n < 1.  Host-only, no device access. */
double sor_omega_opt(int32_t n);

/* Create a context bound to HIP device `device`.  Returns SOR_OK and *out, or
 * SOR_EINVAL (bad device / NULL out) or SOR_EDEVICE. */
sor_status sor_ctx_create(int device, sor_ctx **out);

/* Release the context and every device buffer it owns.  NULL is a no-op. */
void sor_ctx_destroy(sor_ctx *ctx);

/* Message of the context's most recent failure ("" if none).  The string is
 * owned by the context and valid until its next call. */
const char *sor_last_error(const sor_ctx *ctx);

/* Sweep kernel family used by the plain solves:
 *   SOR_KERNEL_BLOCKED  (default) one pass per `iters_per_pass` iterations:
 *                       each wavefront streams a column strip of a row segment
 *                       through registers and applies both colours of several
 *                       iterations before writing back (temporal blocking).
 *   SOR_KERNEL_SIMPLE   one launch per colour per iteration, one thread per
 *                       cell of that colour (the paper's red phase, barrier,
 *                       black phase, barrier, as separate launches).        */
enum { SOR_KERNEL_BLOCKED = 0, SOR_KERNEL_SIMPLE = 1 };
sor_status sor_ctx_set_kernel(sor_ctx *ctx, int32_t kernel);

/* Tiling of the blocked kernel for one storage precision (64, 32 or 16 bits):
 * iters_per_pass in 1..8 (iterations applied per HBM pass) and seg_rows, the
 * rows of output per wavefront (even, 8..1024).  0 in a field means "keep".
 * A new context reports both as 0 (chosen per solve).  Until iters_per_pass
 * is set, each plain FP64 or FP32 solve uses 7, and a binary16 one 7 where
 * the 7-deep pass kernel keeps two wavefronts resident per SIMD, else 6
 * (6 on gfx950); batched FP64 solves always
 * run passes of 7 iterations (shorter ones only to finish a solve), and the
 * inner sweeps of batched and served mixed solves use the context's depth
 * capped at 6.  Until seg_rows is set, each plain solve picks it from the
 * grid side, so that a pass has about as many tiles as the device holds
 * resident wavefronts of the pass kernel (2*2*iters_per_pass..768 rows);
 * batched FP64 solves and mixed inner sweeps use 128 rows below n = 512,
 * else 384.  An
 * autotuned entry for the grid's size class (sor_autotune for plain solves,
 * sor_autotune_batch for batched ones) takes precedence.  Results do not
 * depend on the tiling. */
typedef struct sor_tiling {
    int32_t iters_per_pass;
    int32_t seg_rows;
} sor_tiling;
sor_status sor_ctx_set_tiling(sor_ctx *ctx, int32_t bits, const sor_tiling *t);
sor_status sor_ctx_get_tiling(const sor_ctx *ctx, int32_t bits, sor_tiling *t);
/* The tiling a plain solve of a grid with side n at this precision would use
 * now (autotuned entry, else the context's tiling with seg_rows resolved from
 * n); has_rhs != 0 for a Poisson solve (its kernel holds fewer resident
 * wavefronts).  Host-side query (may ask the runtime for the kernel's
 * occupancy); EINVAL for a null argument, bad bits or n outside 1..65536. */
sor_status sor_ctx_tiling_for(sor_ctx *ctx, int32_t bits, int32_t n, int32_t has_rhs,
                              sor_tiling *t);

/* Kernel timing for measurement.  While profiling is on, each run of sweep
 * launches between two host checks of the plain, mixed, 3-D and ordering
 * solves is bracketed by a pair of HIP events on the caller's stream (one
 * pair per run rather than per launch, so that the events add no gaps between
 * launches); the run's duration adds to a running total and its passes that
 * did work to a launch count (passes that exited at once after the stopping
 * rule was met, and the gaps between launches, fall inside the bracket).
 * sor_ctx_get_profile returns the total milliseconds and the number of
 * timed launches since profiling was last switched on. */
sor_status sor_ctx_set_profiling(sor_ctx *ctx, int32_t on);
sor_status sor_ctx_get_profile(const sor_ctx *ctx, double *kernel_ms,
                               int64_t *launches);

/*
 * Plain FP64 red-black SOR (Sec. 2.1 Eq. 1, Sec. 3.1, Algorithm 1).
 *   u           in: initial guess; out: final iterate (device, n*n)
 *   boundary    device, 4*n;  rhs: device n*n or NULL
 *   n           >= 1;  omega in (0, 2) (Sec. 2.1);  tol >= 0
 *   max_iters   >= 1;  check_every >= 1 (Algorithm 1's K)
 *   out         receives the outcome (required)
 *   max_hist    optional HOST array of max_iters doubles: entry k-1 receives
 *               the change of iteration k for k = 1..out->iterations.
 *               Without it, each sweep pass forms only the changes of the
 *               check iterations it holds (one pass variant per position of
 *               the check in the pass, and one forming none), which the
 *               stopping rule reads; results are the same either way.
 * Returns SOR_OK (converged), SOR_NOT_CONVERGED, SOR_ENONFINITE (u holds the
 * non-finite iterate; out->final_max_delta is the change of the last
 * iteration of the pass that found it, or NaN when that pass formed none),
 * SOR_EINVAL, SOR_ENOMEM or SOR_EDEVICE.  A grid value that is not finite is
 * what SOR_ENONFINITE reports; a change that overflows between two finite
 * values is an ordinary (infinite) change, as the oracle counts it.
 */
sor_status sor_solve_f64(sor_ctx *ctx, double *u, const double *boundary,
                         const double *rhs, int32_t n, double omega, double tol,
                         int64_t max_iters, int64_t check_every, void *stream,
                         sor_result *out, double *max_hist);

/*
 * sor_solve_f64 for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, layout, ownership, method, results and errors, bit for
 * bit the same u, result and max_hist, but the working grids and control
 * blocks live in a fixed 64 MiB region of device memory that the library
 * holds on each GPU it runs on until the process ends, so the call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine).
 *   Limit: the working memory of side n must fit the region, which holds
 *   n <= 1951 without a source (rhs NULL) and n <= 1583 with one; larger n
 *   returns SOR_EINVAL before any device work.
 *   Sharing: every call of one process on one GPU uses the same region, so
 *   calls that overlap in time on one GPU (other streams, threads or contexts)
 *   race; serialise them.  Each call initialises what it reads.
 *   The context's kernel and tiling settings apply; its profiling does not
 *   (no events are recorded by this call).
 * SOR_EDEVICE if the region's address could not be obtained when the context
 * was created.
 */
sor_status sor_solve_f64_noalloc(sor_ctx *ctx, double *u, const double *boundary,
                                 const double *rhs, int32_t n, double omega, double tol,
                                 int64_t max_iters, int64_t check_every, void *stream,
                                 sor_result *out, double *max_hist);

/*
 * The same method with float storage and float arithmetic: omega is rounded
 * once to float, the source enters as fl32(h*h*f) with the product formed in
 * double, and changes are compared with tol in double.  Arguments as for
 * sor_solve_f64 with float arrays.
 */
sor_status sor_solve_f32(sor_ctx *ctx, float *u, const float *boundary,
                         const float *rhs, int32_t n, double omega, double tol,
                         int64_t max_iters, int64_t check_every, void *stream,
                         sor_result *out, double *max_hist);

/*
 * FP64 red-black SOR on the 7-point discretisation of the 3-D problem on the
 * unit cube, the extension named as future work in Sec. 5: the same update
 * (Sec. 2.1 Eq. 1 in increment form), colouring (Sec. 3.1 with a third axis:
 * cell (z, y, x) of the (n+2)^3 array is red when z + y + x is even, red
 * first) and stopping rule (Algorithm 1) as sor_solve_f64.  The Gauss-Seidel
 * value is (((W + E) + (N + S)) + (D + U) [+ h*h*f]) * fl(1/6), W/E, N/S and
 * D/U the x-, y- and z-neighbours, then u' = fma(omega, g - u, u).
 *   u         DEVICE n*n*n, index ((z-1)*n + (y-1))*n + (x-1): in initial
 *             guess, out result (caller-owned)
 *   boundary  DEVICE 6*n*n: faces x = 0 and x = n+1 (each indexed
 *             (z-1)*n + (y-1)), y = 0 and y = n+1 ((z-1)*n + (x-1)),
 *             z = 0 and z = n+1 ((y-1)*n + (x-1)), in that order
 *   rhs       DEVICE n*n*n source of -lap(u) = f like u, or NULL
 *   n in 1..1024; other arguments, results and errors as for sor_solve_f64
 *   (out->passes counts iterations; max_hist, if not NULL, HOST max_iters
 *   doubles).
 * With SOR_KERNEL_BLOCKED (default) one launch applies one or two whole
 * iterations from one padded grid into a second (tiles streamed plane by
 * plane, see sor_ctx_set_tiling3d): by default two when check_every is even
 * (every check then falls at the end of a launch; an odd max_iters ends with
 * a one-iteration launch), else one.  The context holds two (n+2)^3 FP64
 * grids plus one for rhs.  With SOR_KERNEL_SIMPLE one launch per colour works in
 * place on one grid.  Results are bit-identical either way; out->passes
 * counts launches of the streaming kernel (iterations of the simple one).
 */
sor_status sor_solve3d_f64(sor_ctx *ctx, double *u, const double *boundary,
                           const double *rhs, int32_t n, double omega, double tol,
                           int64_t max_iters, int64_t check_every, void *stream,
                           sor_result *out, double *max_hist);

/*
 * Orderings of the 2-D FP64 solve.  RED_BLACK is the paper's method
 * (Sec. 3.1).  JACOBI updates every interior cell from the previous iterate
 * (the method Sec. 2.1 contrasts SOR with; omega = 1 is plain Jacobi, other
 * omega the over-relaxed Jacobi iteration).  FOUR_COLOUR is the multi-colour
 * SOR that Sec. 3.1 names, with colour(i, j) = 2 (i mod 2) + (j mod 2) on the
 * full array (boundary at index 0) and the colours swept in the order
 * 0, 1, 2, 3 (colours 1 and 2 never touch, so they are swept together).
 * BLOCK_PARALLEL is the block-parallel SOR that Sec. 3.1 names (solved by
 * sor_solve_blockpar_f64, which takes the block shape; the ordering value
 * selects its tiling in sor_ctx_set_variant_tiling, and sor_solve_variant_f64
 * rejects it with SOR_EINVAL).
 */
enum {
  SOR_ORDER_RED_BLACK = 0,
  SOR_ORDER_JACOBI = 1,
  SOR_ORDER_FOUR_COLOUR = 2,
  SOR_ORDER_BLOCK_PARALLEL = 3
};

/*
 * sor_solve_f64 with the given ordering: same arguments, layout, ownership,
 * update expression ((N+S)+(W+E) [+h*h*f]) * 0.25 in increment form,
 * stopping rule (Algorithm 1), results and errors; SOR_EINVAL for an unknown
 * ordering.  Both follow the context's kernel.  SOR_KERNEL_BLOCKED (default)
 * applies several iterations per HBM pass like the red-black blocked kernel,
 * from one padded grid into a second (FOUR_COLOUR: three colour sweeps per
 * iteration instead of two half-sweeps; JACOBI: one sweep of every cell from
 * the previous iterate per iteration; tiling from
 * sor_ctx_set_variant_tiling).  SOR_KERNEL_SIMPLE runs one iteration per
 * launch for JACOBI (grid to grid) and three launches per iteration in place
 * for FOUR_COLOUR.  Results are bit-identical either way; out->passes counts
 * launches that did work (iterations for the simple kernels).
 */
sor_status sor_solve_variant_f64(sor_ctx *ctx, int32_t ordering, double *u,
                                 const double *boundary, const double *rhs, int32_t n,
                                 double omega, double tol, int64_t max_iters,
                                 int64_t check_every, void *stream, sor_result *out,
                                 double *max_hist);

/*
 * Block-parallel SOR (Sec. 3.1 names it, citing it without a definition;
 * this is the reading the library implements).  The n x n interior is cut
 * into blocks of block_rows x block_cols cells, aligned at interior cell
 * (1, 1) (the last block row and column may be shorter).  One iteration
 * updates every block at once by one red-black iteration of its own cells
 * (red first, same colouring, update expression and increment form of Eq. 1
 * as sor_solve_f64), in which a neighbour lying in another block is always
 * taken at the previous iterate: red cells therefore get the red-black
 * update, and a black cell reads the new value of a red neighbour in its own
 * block and the old value of one across a block edge.  Blocks of at least
 * n x n give sor_solve_f64's iterates bit for bit, blocks of 1 x 1 the
 * over-relaxed Jacobi ones (SOR_ORDER_JACOBI).  Unlike red-black SOR the
 * iteration does not converge for every omega in (0, 2): the bound depends
 * on the block shape (n = 12, 5 x 3 blocks: converges at 1.35, diverges at
 * 1.5); a diverging solve ends with SOR_ENONFINITE or SOR_NOT_CONVERGED like
 * any other.
 *
 * Arguments, layout, ownership, stopping rule (Algorithm 1), results and
 * errors as sor_solve_f64, plus block_rows, block_cols >= 1 (larger than n
 * is allowed; else SOR_EINVAL).  Always runs the blocked kernel (ping-pong
 * between two padded grids, iterations per pass from
 * sor_ctx_set_variant_tiling with SOR_ORDER_BLOCK_PARALLEL), whatever
 * sor_ctx_set_kernel selected; results do not depend on the tiling.
 */
sor_status sor_solve_blockpar_f64(sor_ctx *ctx, double *u, const double *boundary,
                                  const double *rhs, int32_t n, double omega,
                                  int32_t block_rows, int32_t block_cols, double tol,
                                  int64_t max_iters, int64_t check_every, void *stream,
                                  sor_result *out, double *max_hist);

/* Tiling of the blocked kernel of ordering SOR_ORDER_FOUR_COLOUR,
 * SOR_ORDER_JACOBI or SOR_ORDER_BLOCK_PARALLEL (SOR_ORDER_RED_BLACK uses
 * sor_ctx_set_tiling; others: SOR_EINVAL).  iters_per_pass in 1..5 for
 * FOUR_COLOUR (each is 3 colour sweeps, so 5 has 15 stages, about the stage
 * depth of red-black's 7) and 1..8 for JACOBI (one sweep each) and
 * BLOCK_PARALLEL (two half-sweeps each); seg_rows even in 8..1024; 0 in a
 * field means "keep".  A new context uses 5 (FOUR_COLOUR), 8 (JACOBI) and 5
 * (BLOCK_PARALLEL) and picks seg_rows from the grid side as
 * sor_ctx_set_tiling describes.  Results do not depend on the tiling.
 * sor_ctx_get_variant_tiling reports the setting (seg_rows 0 until one is
 * set). */
sor_status sor_ctx_set_variant_tiling(sor_ctx *ctx, int32_t ordering, const sor_tiling *t);
sor_status sor_ctx_get_variant_tiling(const sor_ctx *ctx, int32_t ordering, sor_tiling *t);

/*
 * Tiling of sor_solve3d_f64's streaming kernel (not in the paper; results do
 * not depend on it).  iters_per_launch: 1, 2, or 0 for the default (2 when
 * check_every is even, else 1; a 2 is honoured only when check_every is
 * even).  A tile is a core
 * of cx x cy cells in x and y and zs planes in z, one workgroup of 256
 * threads; the workgroup holds the core plus a ring of 2 cells per
 * iteration: (cx + 4) x (cy + 4) <= 2048 positions for one iteration,
 * (cx + 8) x (cy + 8) <= 2032 for two.  0 for any size picks it per solve:
 * equal strips and bands with the fewest positions per core cell, then zs so
 * that the tiles fill whole rounds of the device's resident workgroups.
 * Errors: SOR_EINVAL for values out of range or a region above the limit (a
 * region check that depends on n is reported by the solve).
 */
sor_status sor_ctx_set_tiling3d(sor_ctx *ctx, int32_t iters_per_launch, int32_t cx,
                                int32_t cy, int32_t zs);

/*
 * The streaming set-up a sor_solve3d_f64 of side n (with a source if has_rhs
 * is non-zero) and the given check_every would use: iterations per launch
 * and the core sizes of its tiles (HOST outputs).
 */
sor_status sor_ctx_tiling3d_for(sor_ctx *ctx, int32_t n, int32_t has_rhs, int64_t check_every,
                                int32_t *iters_per_launch, int32_t *cx, int32_t *cy,
                                int32_t *zs);

/*
 * FP64 residual of the h*h-scaled system 4u - (interior neighbours) = b,
 * b = h*h*f + (boundary neighbours):
 *   r = (h*h*f + ((N + S) + (W + E))) - 4u   at every interior cell.
 *   r      optional DEVICE array of n*n doubles receiving r (NULL: not stored)
 *   stats  HOST array of 3 doubles: { sum r^2, sum b^2, max |r| }; the sums
 *          use a fixed, launch-independent order (deterministic).
 */
sor_status sor_residual_f64(sor_ctx *ctx, const double *u,
                            const double *boundary, const double *rhs,
                            int32_t n, double *r, double *stats, void *stream);

/*
 * Mixed precision: FP64 defect correction around reduced-precision SOR.
 *   repeat: r = b - A u in FP64 (sor_residual_f64's expression);
 *           rel = ||r||_2 / ||b||_2; stop when rel <= rel_tol or after
 *           max_outer corrections;
 *           solve A e = r approximately with inner_iters red-black SOR
 *           iterations from e = 0 under a zero boundary, with e and the
 *           right-hand side stored in `inner_bits` (32: float; 16: IEEE
 *           binary16) and float arithmetic;  u = u + e in FP64.
 *   The inner right-hand side is fl(r * 2^p), p = floor(log2(target/max|r|)),
 *   target = 1 for 32-bit and 2^14*h*h/0.0737 for 16-bit storage (0.0737
 *   bounds the infinity norm of the inverse of the unscaled 5-point operator
 *   on the unit square, keeping the scaled correction below about 2^14);
 *   the correction is added as u + (double)e * 2^-p.
 *   inner_iters <= 0 selects n/2 rounded up to a multiple of 6 (at least 6):
 *   on Poisson problems from 256^2 to 4096^2 about n/2 reaches a relative
 *   residual of 1e-8 in the least time of n/8 .. 2n (each correction lowers
 *   rel about 20-fold); multiples of 6 let batched and served solves run
 *   their faster fixed-depth kernel.
 *   binary16 storage is accepted for n <= 1024 only (SOR_EINVAL above; the
 *   same limit holds for the batched solve and the request server).  Its
 *   11-bit significand cannot hold a smooth correction: once a cell's change
 *   per inner iteration is below half an ulp of its value the sweeps stop
 *   moving it, and the rounding of a smooth field is itself smooth, so the
 *   correction is wrong in the components SOR is slowest to remove.
 *   Measured: the refinement reaches rel 1e-8 within 30 corrections up to
 *   n = 1024; from n = 1536 it stalls near rel 1e2..1e3 whatever the inner
 *   count.  The loop does not stop when rel grows: the first corrections
 *   from a zero correction at omega near 2 raise rel (up to about n/10-fold)
 *   on problems that then converge.
 *   rel_hist: optional HOST array of
 *   max_outer + 1 doubles receiving rel before each correction and at exit.
 *   With ||b||_2 = 0, rel is ||r||_2.  The norms are plain FP64 sums of
 *   squares, so entries of r or b above about 1e150 overflow them.
 * Returns SOR_OK when rel <= rel_tol was reached, else SOR_NOT_CONVERGED,
 * SOR_ENONFINITE when rel is not finite (a non-finite value in the grid or
 * an overflowing norm) or an inner sweep produced one, or an error status.
 */
sor_status sor_solve_mixed(sor_ctx *ctx, double *u, const double *boundary,
                           const double *rhs, int32_t n, double omega,
                           double rel_tol, int64_t max_outer, int32_t inner_bits,
                           int64_t inner_iters, void *stream, sor_result *out,
                           double *rel_hist);

/*
 * One grid of a batched solve.  Arrays follow the conventions above (device
 * pointers, caller-owned); each grid has its own size, omega, tolerance,
 * check cadence and iteration limit.
 */
typedef struct sor_grid_desc {
    double *u;                /* n*n interior: in initial guess, out result  */
    const double *boundary;   /* 4n edge values (north, south, west, east)   */
    const double *rhs;        /* n*n source f, or NULL for Laplace           */
    int32_t n;
    int32_t reserved;
    double omega;             /* in (0, 2)                                   */
    double tol;               /* stop when a checked change is < tol         */
    int64_t max_iters;        /* >= 1                                        */
    int64_t check_every;      /* >= 1                                        */
} sor_grid_desc;

/*
 * Batched FP64 red-black SOR: every grid follows exactly the method of
 * sor_solve_f64 (Sec. 2.1 Eq. 1, Sec. 3.1, Algorithm 1) and gets the result
 * sor_solve_f64 would give it alone, bit for bit.  All grids advance together
 * in one persistent kernel launch: each 64-lane wavefront repeatedly takes a
 * (grid, tile) work item of some grid's current pass from a device queue; the
 * wavefront that completes a grid's pass evaluates that grid's stopping rule
 * and queues its next pass.  The launch sequence (uploads, packing, the
 * persistent kernel, unpacking, result download) is recorded once as a HIP
 * graph and replayed for later batches with the same shapes.
 *   grids    HOST array of `count` descriptors (count >= 1)
 *   results  HOST array of `count` results (status per grid in ->status)
 * Tiles per grid come from the context's batched tuning table
 * (sor_autotune_batch) or a size-based default.  Returns SOR_OK when every grid converged,
 * SOR_NOT_CONVERGED when some reached their limit, SOR_ENONFINITE when some
 * produced a non-finite value, SOR_ETIMEOUT if a device-side queue wait
 * exceeded its bound, or an argument / device error.
 */
sor_status sor_batch_solve_f64(sor_ctx *ctx, const sor_grid_desc *grids,
                               int32_t count, void *stream, sor_result *results);

/*
 * Retire times of the grids of the context's most recent sor_batch_solve_f64
 * (measurement; not in the paper): done_ms[g] (HOST, count doubles) receives
 * the device wall-clock milliseconds from the start of the persistent launch
 * to the moment grid g's stopping rule retired it (NaN for a grid that did not
 * retire).  SOR_EINVAL unless count equals that solve's grid count.
 */
sor_status sor_batch_last_times(const sor_ctx *ctx, int32_t count, double *done_ms);

/*
 * Tiling autotuner for plain solves: times blocked passes of every candidate
 * tiling (1..8 iterations per pass x 16..768 rows per tile) on a scratch
 * n x n Laplace grid of the given storage precision (64 or 32 bits) with HIP
 * events, stores the fastest in the context's plain-solve tuning table for
 * n's size class (side rounded to the nearest half power of two), and returns
 * it in *best (may be NULL).
 * Later plain solves of that precision and class use it.  Only timing is
 * measured: results never depend on the tiling.
 */
sor_status sor_autotune(sor_ctx *ctx, int32_t bits, int32_t n, sor_tiling *best);

/*
 * Tiling autotuner for grids inside batched launches, where many grids share
 * the chip and throughput, not one grid's pass latency, decides: solves a
 * scratch batch of identical n x n grids (enough for about 4096 tiles, at
 * most 256 grids and 1 GiB; 96 iterations each) once per candidate with
 * sor_batch_solve_f64 (bits 64: the fixed depth of 7 x 16..384 rows) or the
 * inner sweeps of sor_batch_solve_mixed (bits 32 or 16: passes of 6
 * iterations x 16..384 rows), keeps the
 * fastest in the context's batched tuning table for n's size class (used by
 * batched solves and by nothing else) and returns it in *best (may be NULL).
 * n in 8..8192.  Results never depend on the tiling.
 */
sor_status sor_autotune_batch(sor_ctx *ctx, int32_t bits, int32_t n, sor_tiling *best);

/*
 * One grid of a mixed-precision batched solve or of a served request: the
 * defect-correction method of sor_solve_mixed, with its parameters per grid.
 */
typedef struct sor_mixed_desc {
    double *u;                /* device n*n: in initial guess, out result   */
    const double *boundary;   /* device 4n                                  */
    const double *rhs;        /* device n*n, or NULL                        */
    int32_t n;
    int32_t reserved;
    double omega;             /* inner SOR relaxation factor, in (0, 2)     */
    double rel_tol;           /* stop when ||r||_2/||b||_2 <= rel_tol       */
    double corr_tol;          /* or (if > 0) when the last correction's max
                                 |e| is below corr_tol                      */
    int64_t max_outer;        /* >= 0 corrections                           */
    int64_t inner_iters;      /* > 0 inner iterations per correction
                                 (<= 0: n/2 rounded up to a multiple of 6)  */
} sor_mixed_desc;

/*
 * Batched mixed-precision solves: each grid gets exactly sor_solve_mixed's
 * arithmetic (FP64 residual, inner right-hand side fl(r*2^p), inner_iters
 * red-black SOR iterations in `inner_bits` storage (32 or 16) from zero,
 * u += e*2^-p), bit for bit whatever else is in the batch; every grid's
 * phases (residual, cast, inner passes, accumulate) are work items of one
 * persistent kernel launch.  The residual-based test of sor_solve_mixed is
 * extended by the optional corr_tol test, evaluated after the residual of
 * the corrected iterate: converged when rel <= rel_tol, or when corr_tol > 0,
 * at least one correction was applied and its max |e| < corr_tol.
 * results[g].outer_steps, .rel_residual, .final_max_delta (last correction)
 * and .iterations (inner iterations) describe each grid.
 */
sor_status sor_batch_solve_mixed(sor_ctx *ctx, const sor_mixed_desc *grids,
                                 int32_t count, int32_t inner_bits, void *stream,
                                 sor_result *results);

/*
 * Serving: a request loop on one GPU.  Requests (host arrays, copied at
 * submission) wait until a slot and enough of the `hbm_budget` bytes of
 * device memory are free (in arrival order, except that a request that does
 * not fit may be overtaken, see sor_server_memory); admitted requests keep their whole state on the device
 * and are advanced together by time-sliced launches of the mixed-precision
 * persistent kernel (each launch runs for about `slice_ms`, then newly
 * arrived requests join and finished ones leave: continuous batching).
 * A background host thread drives the loop; submit/poll are thread-safe.
 */
typedef struct sor_server sor_server;

typedef struct sor_request {
    const double *u0;         /* HOST n*n initial guess (NULL: zeros)       */
    const double *boundary;   /* HOST 4n                                    */
    const double *rhs;        /* HOST n*n or NULL                           */
    int32_t n;
    int32_t reserved;
    double omega;             /* <= 0 selects 2/(1+sin(pi/(n+1)))           */
    double rel_tol;
    double corr_tol;
    int64_t max_outer;
    int64_t inner_iters;      /* <= 0: n/2 rounded up to a multiple of 6    */
} sor_request;

typedef struct sor_request_info {
    sor_result result;
    double submit_s;          /* server clock (seconds) at submission       */
    double admit_s;           /* ... when it got a slot                     */
    double done_s;            /* ... when its result reached the host       */
} sor_request_info;

sor_status sor_server_create(int device, int32_t inner_bits, size_t hbm_budget,
                             int32_t max_slots, double slice_ms, sor_server **out);
/* Copy a request in and queue it; *ticket identifies it.  SOR_EBUSY if the
 * request alone exceeds the memory budget (it could never be admitted);
 * SOR_EINVAL for n outside 1..4096 (1..1024 on a binary16 server) or an
 * invalid parameter. */
sor_status sor_server_submit(sor_server *srv, const sor_request *req, uint64_t *ticket);
/* If the request has finished, fill *info and u_out (HOST n*n, may be NULL),
 * release it and return its status (SOR_OK, SOR_NOT_CONVERGED, SOR_ENONFINITE);
 * SOR_EBUSY while it is still queued or running; SOR_EINVAL for an unknown
 * ticket.  wait_ms > 0 blocks up to that long for completion. */
sor_status sor_server_poll(sor_server *srv, uint64_t ticket, double wait_ms,
                           sor_request_info *info, double *u_out);
/* Server clock now (seconds), and counters: launches, requests completed,
 * requests waiting, requests resident. */
double sor_server_clock(const sor_server *srv);
sor_status sor_server_stats(sor_server *srv, int64_t *launches, int64_t *completed,
                            int64_t *waiting, int64_t *resident);
/* Device memory of the request state (HOST outputs, may be NULL): the
 * budget, the bytes resident requests hold now, and the most they ever held.
 * Admission never lets the held bytes exceed the budget: a waiting request
 * that does not fit is passed over by later ones that do (no head-of-line
 * blocking), but at most 32 times, after which admission waits for it. */
sor_status sor_server_memory(sor_server *srv, size_t *budget, size_t *in_use, size_t *peak);
const char *sor_server_last_error(const sor_server *srv);
/* Stop the loop (unfinished requests are dropped) and free everything. */
void sor_server_destroy(sor_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* SOR_H */
