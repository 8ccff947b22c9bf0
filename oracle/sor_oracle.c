/*
 * Plain, slow, obviously-correct CPU oracle for red-black successive
 * over-relaxation (SOR) on the 5-point discretisation of the 2-D steady-state
 * heat conduction problem with Dirichlet boundaries (Mittal, "A Study of
 * Successive Over-relaxation Method Parallelization Over Modern HPC
 * Languages", 2014), the Jacobi and four-colour alternatives it names
 * (Sec. 2.1, Sec. 3.1), and the 7-point discretisation of its 3-D form (the
 * extension the paper names as future work, Sec. 5; last section below).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this file.  It shares no code,
 * header, table or helper with the GPU library and includes nothing from it.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * (no implicit fused multiply-add, no reassociation: every expression below
 * is evaluated exactly in the order written, one IEEE rounding per operation;
 * the one fused operation, fma(), is written out).
 *
 * Grid convention (the paper's red-black colouring, Sec. 3.1, Fig. 1):
 *   The n x n interior is embedded in an (n+2) x (n+2) array U with the
 *   Dirichlet boundary on the ring.  Row 0 is the north edge, row n+1 the
 *   south edge, column 0 the west edge, column n+1 the east edge.  Corner
 *   cells are never read by the 5-point stencil and are held at 0.
 *   Cell (i, j), both indices into the full array, is red when (i + j) is
 *   even and black when it is odd, so interior cell (1, 1) is red.
 *
 * User-facing arrays:
 *   u    n*n interior values, row-major (u[(i-1)*n + (j-1)] is U[i][j]).
 *   bdy  4*n boundary values in the order north (j = 1..n), south (j = 1..n),
 *        west (i = 1..n), east (i = 1..n).
 *   f    n*n source of -lap(u) = f, row-major, or NULL for Laplace.
 *
 * Readings of the paper this file commits to (each is restated where used):
 *   - h = 1/(n+1); the source enters the update as F = h*h*f, computed once.
 *   - The Gauss-Seidel value of a cell is the average of its four neighbours
 *     (plus F/4 for Poisson); the sum is formed as (N + S) + (W + E), then
 *     + F, then multiplied by 0.25.
 *   - Eq. 1, X = w*Xgs + (1 - w)*Xold, is evaluated in its increment form
 *     Xold + w*(Xgs - Xold), the product and the sum formed with one rounding,
 *     fma(w, d, Xold), where the difference d = Xgs - Xold = 0.25*s - Xold is
 *     also formed with one rounding, fma(0.25, s, -Xold) (the same as rounding
 *     0.25*s and then the difference whenever 0.25*s is a normal number);
 *     algebraically identical, fixed here so that two
 *     implementations can agree bit for bit.
 *   - Red cells are updated first, then black cells using the new red values
 *     (Sec. 3.1).
 *   - The change measured for the stopping rule is max |X_k - X_{k-1}| over
 *     all cells for one whole iteration (Sec. 2.1); it is taken as the max of
 *     the per-update |new - old|, which is the same number because every cell
 *     is written exactly once per iteration.
 *   - The check runs when the iteration number is a multiple of K, and also
 *     at the last allowed iteration; convergence is the strict test
 *     max < tol (Algorithm 1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENONFINITE (-4)

#define AT(i, j) ((size_t)(i) * (size_t)(n + 2) + (size_t)(j))

/* ------------------------------------------------------------------------ */
/* Grid set-up                                                               */
/* ------------------------------------------------------------------------ */

/* Embed interior u and the four boundary edges into the (n+2)^2 array U
 * (grid convention above). */
static void orc_fill_f64(int n, double *U, const double *u, const double *bdy)
{
    memset(U, 0, sizeof(double) * (size_t)(n + 2) * (size_t)(n + 2));
    for (int i = 1; i <= n; ++i)
        for (int j = 1; j <= n; ++j)
            U[AT(i, j)] = u[(size_t)(i - 1) * n + (j - 1)];
    for (int j = 1; j <= n; ++j) {
        U[AT(0, j)] = bdy[j - 1];                /* north */
        U[AT(n + 1, j)] = bdy[n + j - 1];        /* south */
    }
    for (int i = 1; i <= n; ++i) {
        U[AT(i, 0)] = bdy[2 * n + i - 1];        /* west */
        U[AT(i, n + 1)] = bdy[3 * n + i - 1];    /* east */
    }
}

static void orc_extract_f64(int n, const double *U, double *u)
{
    for (int i = 1; i <= n; ++i)
        for (int j = 1; j <= n; ++j)
            u[(size_t)(i - 1) * n + (j - 1)] = U[AT(i, j)];
}

/* Mesh width of the unit square with n interior nodes per side. */
static double orc_h(int n) { return 1.0 / (double)(n + 1); }

/* ------------------------------------------------------------------------ */
/* FP64 red-black SOR (Sec. 2.1 Eq. 1, Sec. 3.1, Algorithm 1)                */
/* ------------------------------------------------------------------------ */

/* One half-sweep over the cells of one colour (0 = red, 1 = black) of U,
 * updated in place.  Returns the max of |new - old| over the updated cells;
 * sets *bad when a non-finite value is produced.  Within one colour no cell
 * reads another cell of the same colour (Sec. 3.1), so the visiting order is
 * immaterial; rows run top to bottom, and within a row the stride-2 walk of
 * Fig. 2 visits only cells of this colour. */
static double orc_half_sweep_f64(int n, double *U, const double *F, double w,
                                 int colour, int i_lo, int i_hi, int *bad)
{
    double m = 0.0;
    for (int i = i_lo; i <= i_hi; ++i) {
        /* first column j >= 1 with (i + j) % 2 == colour */
        int j0 = 1 + ((i + 1 + colour) & 1);
        for (int j = j0; j <= n; j += 2) {
            double old = U[AT(i, j)];
            double s = (U[AT(i - 1, j)] + U[AT(i + 1, j)]) +
                       (U[AT(i, j - 1)] + U[AT(i, j + 1)]);
            if (F) s = s + F[AT(i, j)];
            double dg = fma(0.25, s, -old);     /* Gauss-Seidel value - old */
            double nu = fma(w, dg, old);        /* Eq. 1, increment form */
            double d = fabs(nu - old);
            if (!isfinite(nu)) *bad = 1;
            if (d > m) m = d;
            U[AT(i, j)] = nu;
        }
    }
    return m;
}

/* F = h*h*f on the interior of an (n+2)^2 array (0 on the ring). */
static double *orc_make_F(int n, const double *f)
{
    if (!f) return NULL;
    double *F = calloc((size_t)(n + 2) * (size_t)(n + 2), sizeof(double));
    if (!F) return NULL;
    double h = orc_h(n);
    double h2 = h * h;
    for (int i = 1; i <= n; ++i)
        for (int j = 1; j <= n; ++j)
            F[AT(i, j)] = h2 * f[(size_t)(i - 1) * n + (j - 1)];
    return F;
}

/*
 * Red-black SOR, Algorithm 1: for iter = 1..max_iters do a red half-sweep and
 * then a black half-sweep; on every check iteration (iter % K == 0, or
 * iter == max_iters) compare that iteration's max change with tol and stop
 * when it is strictly smaller.
 *
 * threads > 1 splits the rows of each colour across that many OpenMP workers
 * with an implicit barrier after each colour, which is the paper's P-worker
 * form of Algorithm 1; results are identical for every thread count because
 * a colour's cells are independent and max is exact.
 *
 * Outputs: u holds the final interior; *iters_out the iteration at which the
 * check passed (1-based), or max_iters; *max_out the last checked iteration's
 * max change; mhist (length max_iters, may be NULL) every iteration's max
 * change.  Returns ORC_OK, ORC_NOT_CONVERGED, ORC_ENONFINITE or ORC_EINVAL.
 */
int oracle_sor_f64(int n, double *u, const double *bdy, const double *f,
                   double omega, double tol, int64_t max_iters,
                   int64_t check_every, int threads, int64_t *iters_out,
                   double *max_out, double *mhist)
{
    if (n < 1 || !u || !bdy || !(omega > 0.0 && omega < 2.0) || !(tol >= 0.0) ||
        max_iters < 1 || check_every < 1 || threads < 1)
        return ORC_EINVAL;
    double *U = malloc(sizeof(double) * (size_t)(n + 2) * (size_t)(n + 2));
    if (!U) return ORC_ENOMEM;
    double *F = orc_make_F(n, f);
    if (f && !F) { free(U); return ORC_ENOMEM; }
    orc_fill_f64(n, U, u, bdy);

    int status = ORC_NOT_CONVERGED;
    int64_t it = 0;
    double last = NAN;
    for (it = 1; it <= max_iters; ++it) {
        double m = 0.0;
        int bad = 0;
        for (int colour = 0; colour < 2; ++colour) {
            if (threads == 1) {
                double mc = orc_half_sweep_f64(n, U, F, omega, colour, 1, n, &bad);
                if (mc > m) m = mc;
            } else {
                double mc = 0.0;
                int badc = 0;
#pragma omp parallel for num_threads(threads) schedule(static) reduction(max : mc) reduction(| : badc)
                for (int i = 1; i <= n; ++i) {
                    int b1 = 0;
                    double r = orc_half_sweep_f64(n, U, F, omega, colour, i, i, &b1);
                    if (r > mc) mc = r;
                    badc |= b1;
                }
                if (mc > m) m = mc;
                bad |= badc;
            }
        }
        if (mhist) mhist[it - 1] = m;
        if (bad) { status = ORC_ENONFINITE; last = m; break; }
        if (it % check_every == 0 || it == max_iters) {
            last = m;
            if (m < tol) { status = ORC_OK; break; }
        }
    }
    if (it > max_iters) it = max_iters;
    orc_extract_f64(n, U, u);
    if (iters_out) *iters_out = it;
    if (max_out) *max_out = last;
    free(U);
    free(F);
    return status;
}

/* ------------------------------------------------------------------------ */
/* FP64 variants: Jacobi and the four-colour ordering                        */
/* ------------------------------------------------------------------------ */

/*
 * The two alternatives to the red-black order that the paper names (Sec. 2.1
 * introduces Jacobi as the method that uses only the previous iteration's
 * values; Sec. 3.1 lists multi-colour SOR among the parallel versions).  Both
 * use the same Gauss-Seidel value and increment form of Eq. 1 as
 * oracle_sor_f64 and the same stopping rule (Algorithm 1).
 *
 * ORDER_JACOBI (1): every interior cell is updated from the previous
 *   iterate, X_k = X + w*(avg(neighbours of X) - X) (w = 1 is Jacobi, other
 *   w the over-relaxed Jacobi iteration), computed into a second array.
 * ORDER_FOUR_COLOUR (2): cell (i, j) of the full array has colour
 *   2*(i mod 2) + (j mod 2); an iteration updates colour 0, 1, 2, 3 in that
 *   order, in place, each like a red-black half-sweep (no cell reads a cell
 *   of its own colour, so the visiting order inside a colour is immaterial).
 *
 * Arguments, outputs and statuses as for oracle_sor_f64 (single-threaded).
 */
#define ORC_ORDER_JACOBI 1
#define ORC_ORDER_FOUR_COLOUR 2

/* One Jacobi iteration from U into V (interior only; V's ring is already the
 * boundary).  Returns the max |new - old|. */
static double orc_jacobi_sweep_f64(int n, const double *U, double *V, const double *F,
                                   double w, int *bad)
{
    double m = 0.0;
    for (int i = 1; i <= n; ++i)
        for (int j = 1; j <= n; ++j) {
            double old = U[AT(i, j)];
            double s = (U[AT(i - 1, j)] + U[AT(i + 1, j)]) +
                       (U[AT(i, j - 1)] + U[AT(i, j + 1)]);
            if (F) s = s + F[AT(i, j)];
            double dg = fma(0.25, s, -old);
            double nu = fma(w, dg, old);
            double d = fabs(nu - old);
            if (!isfinite(nu)) *bad = 1;
            if (d > m) m = d;
            V[AT(i, j)] = nu;
        }
    return m;
}

/* Update the cells of colour c (rows i = c/2 mod 2, columns j = c mod 2) of
 * U in place.  Returns the max |new - old| over them. */
static double orc_colour4_sweep_f64(int n, double *U, const double *F, double w, int c,
                                    int *bad)
{
    double m = 0.0;
    int i0 = (c >> 1) ? 1 : 2, j0 = (c & 1) ? 1 : 2;
    for (int i = i0; i <= n; i += 2)
        for (int j = j0; j <= n; j += 2) {
            double old = U[AT(i, j)];
            double s = (U[AT(i - 1, j)] + U[AT(i + 1, j)]) +
                       (U[AT(i, j - 1)] + U[AT(i, j + 1)]);
            if (F) s = s + F[AT(i, j)];
            double dg = fma(0.25, s, -old);
            double nu = fma(w, dg, old);
            double d = fabs(nu - old);
            if (!isfinite(nu)) *bad = 1;
            if (d > m) m = d;
            U[AT(i, j)] = nu;
        }
    return m;
}

int oracle_variant_f64(int ordering, int n, double *u, const double *bdy, const double *f,
                       double omega, double tol, int64_t max_iters, int64_t check_every,
                       int64_t *iters_out, double *max_out, double *mhist)
{
    if ((ordering != ORC_ORDER_JACOBI && ordering != ORC_ORDER_FOUR_COLOUR) || n < 1 ||
        !u || !bdy || !(omega > 0.0 && omega < 2.0) || !(tol >= 0.0) || max_iters < 1 ||
        check_every < 1)
        return ORC_EINVAL;
    size_t cells = (size_t)(n + 2) * (size_t)(n + 2);
    double *U = malloc(sizeof(double) * cells);
    double *V = ordering == ORC_ORDER_JACOBI ? malloc(sizeof(double) * cells) : NULL;
    double *F = orc_make_F(n, f);
    if (!U || (ordering == ORC_ORDER_JACOBI && !V) || (f && !F)) {
        free(U); free(V); free(F);
        return ORC_ENOMEM;
    }
    orc_fill_f64(n, U, u, bdy);
    if (V) memcpy(V, U, sizeof(double) * cells);

    int status = ORC_NOT_CONVERGED;
    int64_t it = 0;
    double last = NAN;
    for (it = 1; it <= max_iters; ++it) {
        double m = 0.0;
        int bad = 0;
        if (ordering == ORC_ORDER_JACOBI) {
            m = orc_jacobi_sweep_f64(n, U, V, F, omega, &bad);
            double *t = U; U = V; V = t;
        } else {
            for (int c = 0; c < 4; ++c) {
                double mc = orc_colour4_sweep_f64(n, U, F, omega, c, &bad);
                if (mc > m) m = mc;
            }
        }
        if (mhist) mhist[it - 1] = m;
        if (bad) { status = ORC_ENONFINITE; last = m; break; }
        if (it % check_every == 0 || it == max_iters) {
            last = m;
            if (m < tol) { status = ORC_OK; break; }
        }
    }
    if (it > max_iters) it = max_iters;
    orc_extract_f64(n, U, u);
    if (iters_out) *iters_out = it;
    if (max_out) *max_out = last;
    free(U);
    free(V);
    free(F);
    return status;
}

/* ------------------------------------------------------------------------ */
/* FP64 block-parallel SOR                                                   */
/* ------------------------------------------------------------------------ */

/*
 * Block-parallel SOR, the third parallel SOR form Sec. 3.1 names (with a
 * citation only; no definition is given).  Reading used here: the n x n
 * interior is cut into blocks of br rows and bc columns, aligned at interior
 * cell (1, 1) (the last block row and column may be shorter); in every
 * iteration all blocks are updated at the same time, each by one red-black
 * SOR iteration of its own cells (red first, same colouring, Gauss-Seidel
 * value and increment form of Eq. 1 as oracle_sor_f64), in which a neighbour
 * that lies in another block is always taken at the previous iterate.  So
 * the red half-sweep is the red-black one (a red cell's neighbours are black
 * and still hold the previous iterate), and a black cell reads the new value
 * of a red neighbour in its own block and the old value of one across a
 * block edge.  Boundary values never change, so either copy serves them.
 *
 * One block of at least n x n cells is red-black SOR; blocks of one cell are
 * the over-relaxed Jacobi iteration (every neighbour from the previous
 * iterate).  Same stopping rule (Algorithm 1) and outputs as oracle_sor_f64.
 */

/* Block coordinate of interior index i (1..n) for blocks of b cells. */
static int orc_block_of(int i, int b) { return (i - 1) / b; }

/* One block-parallel iteration of U in place; P receives the previous
 * iterate first.  Returns the max |new - old| over all updated cells. */
static double orc_blockpar_iter_f64(int n, double *U, double *P, const double *F, double w,
                                    int br, int bc, int *bad)
{
    size_t cells = (size_t)(n + 2) * (size_t)(n + 2);
    memcpy(P, U, sizeof(double) * cells);
    double m = orc_half_sweep_f64(n, U, F, w, 0, 1, n, bad);   /* red: as red-black */
    for (int i = 1; i <= n; ++i) {
        int j0 = 1 + (i & 1);                  /* first black column: (i + j) odd */
        for (int j = j0; j <= n; j += 2) {
            int bi = orc_block_of(i, br), bj = orc_block_of(j, bc);
            /* a neighbour in this block: its current value; else: previous */
            double nn = (i - 1 >= 1 && orc_block_of(i - 1, br) == bi) ? U[AT(i - 1, j)]
                                                                       : P[AT(i - 1, j)];
            double ss = (i + 1 <= n && orc_block_of(i + 1, br) == bi) ? U[AT(i + 1, j)]
                                                                      : P[AT(i + 1, j)];
            double ww = (j - 1 >= 1 && orc_block_of(j - 1, bc) == bj) ? U[AT(i, j - 1)]
                                                                       : P[AT(i, j - 1)];
            double ee = (j + 1 <= n && orc_block_of(j + 1, bc) == bj) ? U[AT(i, j + 1)]
                                                                      : P[AT(i, j + 1)];
            double old = U[AT(i, j)];
            double s = (nn + ss) + (ww + ee);
            if (F) s = s + F[AT(i, j)];
            double dg = fma(0.25, s, -old);
            double nu = fma(w, dg, old);
            double d = fabs(nu - old);
            if (!isfinite(nu)) *bad = 1;
            if (d > m) m = d;
            U[AT(i, j)] = nu;
        }
    }
    return m;
}

int oracle_blockpar_f64(int n, double *u, const double *bdy, const double *f, double omega,
                        int block_rows, int block_cols, double tol, int64_t max_iters,
                        int64_t check_every, int64_t *iters_out, double *max_out,
                        double *mhist)
{
    if (n < 1 || !u || !bdy || !(omega > 0.0 && omega < 2.0) || block_rows < 1 ||
        block_cols < 1 || !(tol >= 0.0) || max_iters < 1 || check_every < 1)
        return ORC_EINVAL;
    size_t cells = (size_t)(n + 2) * (size_t)(n + 2);
    double *U = malloc(sizeof(double) * cells);
    double *P = malloc(sizeof(double) * cells);
    double *F = orc_make_F(n, f);
    if (!U || !P || (f && !F)) {
        free(U); free(P); free(F);
        return ORC_ENOMEM;
    }
    orc_fill_f64(n, U, u, bdy);

    int status = ORC_NOT_CONVERGED;
    int64_t it = 0;
    double last = NAN;
    for (it = 1; it <= max_iters; ++it) {
        int bad = 0;
        double m = orc_blockpar_iter_f64(n, U, P, F, omega, block_rows, block_cols, &bad);
        if (mhist) mhist[it - 1] = m;
        if (bad) { status = ORC_ENONFINITE; last = m; break; }
        if (it % check_every == 0 || it == max_iters) {
            last = m;
            if (m < tol) { status = ORC_OK; break; }
        }
    }
    if (it > max_iters) it = max_iters;
    orc_extract_f64(n, U, u);
    if (iters_out) *iters_out = it;
    if (max_out) *max_out = last;
    free(U);
    free(P);
    free(F);
    return status;
}

/* ------------------------------------------------------------------------ */
/* FP64 residual of the discrete system                                      */
/* ------------------------------------------------------------------------ */

/*
 * For the h*h-scaled system 4u - (sum of interior neighbours) = b with
 * b = F + (sum of boundary neighbours), the residual at an interior cell is
 *   r = (F + ((N + S) + (W + E))) - 4u        (boundary values in N, S, W, E),
 * and b at that cell is F + ((Nb + Sb) + (Wb + Eb)) where a neighbour that is
 * not on the boundary contributes 0.  Laplace (f == NULL) omits the F term.
 * stats receives { sum r^2, sum b^2, max |r| } accumulated in row-major order
 * in FP64; the relative residual is sqrt(stats[0]) / sqrt(stats[1]).
 * r_out (n*n, may be NULL) receives r.  Returns ORC_OK or ORC_EINVAL.
 */
static void orc_residual_core(int n, const double *U, const double *F,
                              double *r_out, double *stats)
{
    double sr = 0.0, sb = 0.0, mr = 0.0;
    for (int i = 1; i <= n; ++i)
        for (int j = 1; j <= n; ++j) {
            double s = (U[AT(i - 1, j)] + U[AT(i + 1, j)]) +
                       (U[AT(i, j - 1)] + U[AT(i, j + 1)]);
            double t = F ? F[AT(i, j)] + s : s;
            double r = t - 4.0 * U[AT(i, j)];
            double nb = (i == 1) ? U[AT(0, j)] : 0.0;
            double sb_ = (i == n) ? U[AT(n + 1, j)] : 0.0;
            double wb = (j == 1) ? U[AT(i, 0)] : 0.0;
            double eb = (j == n) ? U[AT(i, n + 1)] : 0.0;
            double bs = (nb + sb_) + (wb + eb);
            double b = F ? F[AT(i, j)] + bs : bs;
            if (r_out) r_out[(size_t)(i - 1) * n + (j - 1)] = r;
            sr += r * r;
            sb += b * b;
            if (fabs(r) > mr) mr = fabs(r);
        }
    stats[0] = sr;
    stats[1] = sb;
    stats[2] = mr;
}

int oracle_residual_f64(int n, const double *u, const double *bdy,
                        const double *f, double *r_out, double *stats)
{
    if (n < 1 || !u || !bdy || !stats) return ORC_EINVAL;
    double *U = malloc(sizeof(double) * (size_t)(n + 2) * (size_t)(n + 2));
    if (!U) return ORC_ENOMEM;
    double *F = orc_make_F(n, f);
    if (f && !F) { free(U); return ORC_ENOMEM; }
    orc_fill_f64(n, U, u, bdy);
    orc_residual_core(n, U, F, r_out, stats);
    free(U);
    free(F);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Reduced-precision storage                                                 */
/* ------------------------------------------------------------------------ */

/*
 * Round a float to the nearest IEEE 754 binary16 value (ties to even) and
 * return that value as a float.  binary16 has an 11-bit significand, normal
 * exponents -14..15 and subnormal spacing 2^-24; its largest finite value is
 * 65504 and anything at or above 65520 in magnitude (the midpoint to 2^16,
 * which ties to the even neighbour 2^16) overflows to infinity.  The value is
 * snapped to the binade's quantum q with rint() in the default
 * round-to-nearest-even mode; x/q and the product back are exact because q is
 * a power of two.
 */
float oracle_round_half(float x)
{
    if (isnan(x)) return x;
    float ax = fabsf(x);
    if (ax >= 65520.0f) return copysignf(INFINITY, x);
    if (ax == 0.0f) return x;
    int e;
    frexpf(ax, &e);                    /* ax = m * 2^e, m in [0.5, 1) */
    int ulp_exp = (e - 1) - 10;        /* quantum of the binade 2^(e-1) */
    if (e - 1 < -14) ulp_exp = -24;    /* subnormal range */
    float q = ldexpf(1.0f, ulp_exp);
    float y = rintf(x / q) * q;
    return y;
}

/* F in float storage: fl32(h*h*f) with the product formed in double. */
static float *orc_make_F32(int n, const float *f)
{
    if (!f) return NULL;
    float *F = calloc((size_t)(n + 2) * (size_t)(n + 2), sizeof(float));
    if (!F) return NULL;
    double h = orc_h(n);
    double h2 = h * h;
    for (int i = 1; i <= n; ++i)
        for (int j = 1; j <= n; ++j)
            F[AT(i, j)] = (float)(h2 * (double)f[(size_t)(i - 1) * n + (j - 1)]);
    return F;
}

/* One float half-sweep of one colour over rows i_lo..i_hi; half_store != 0
 * rounds every stored value to binary16 (storage in half precision,
 * arithmetic in float). */
static float orc_half_sweep_rows_f32(int n, float *U, const float *F, float w,
                                     int colour, int half_store, int i_lo, int i_hi,
                                     int *bad)
{
    float m = 0.0f;
    for (int i = i_lo; i <= i_hi; ++i) {
        int j0 = 1 + ((i + 1 + colour) & 1);
        for (int j = j0; j <= n; j += 2) {
            float old = U[AT(i, j)];
            float s = (U[AT(i - 1, j)] + U[AT(i + 1, j)]) +
                      (U[AT(i, j - 1)] + U[AT(i, j + 1)]);
            if (F) s = s + F[AT(i, j)];
            float dg = fmaf(0.25f, s, -old);
            /* binary16 storage: the step is rounded to float (product, then
             * sum) before the storage rounding; float storage: one rounding */
            float nu = half_store ? old + w * dg : fmaf(w, dg, old);
            if (half_store) nu = oracle_round_half(nu);
            float d = fabsf(nu - old);
            if (!isfinite(nu)) *bad = 1;
            if (d > m) m = d;
            U[AT(i, j)] = nu;
        }
    }
    return m;
}

/* The same half-sweep over every row; threads > 1 splits the rows across
 * that many OpenMP workers (a colour's cells are independent and max is
 * exact, so the result does not depend on the thread count). */
static float orc_half_sweep_f32(int n, float *U, const float *F, float w,
                                int colour, int half_store, int threads, int *bad)
{
    if (threads <= 1)
        return orc_half_sweep_rows_f32(n, U, F, w, colour, half_store, 1, n, bad);
    float m = 0.0f;
    int badc = 0;
#pragma omp parallel for num_threads(threads) schedule(static) reduction(max : m) reduction(| : badc)
    for (int i = 1; i <= n; ++i) {
        int b1 = 0;
        float r = orc_half_sweep_rows_f32(n, U, F, w, colour, half_store, i, i, &b1);
        if (r > m) m = r;
        badc |= b1;
    }
    if (badc) *bad = 1;
    return m;
}

/*
 * Red-black SOR with float storage and float arithmetic: the same iteration
 * and stopping rule as oracle_sor_f64, with omega rounded once to float and
 * F = fl32(h*h*f).  mhist (may be NULL) receives each iteration's max change.
 */
int oracle_sor_f32(int n, float *u, const float *bdy, const float *f,
                   double omega, double tol, int64_t max_iters,
                   int64_t check_every, int64_t *iters_out, double *max_out,
                   double *mhist)
{
    if (n < 1 || !u || !bdy || !(omega > 0.0 && omega < 2.0) || !(tol >= 0.0) ||
        max_iters < 1 || check_every < 1)
        return ORC_EINVAL;
    size_t cells = (size_t)(n + 2) * (size_t)(n + 2);
    float *U = calloc(cells, sizeof(float));
    if (!U) return ORC_ENOMEM;
    float *F = orc_make_F32(n, f);
    if (f && !F) { free(U); return ORC_ENOMEM; }
    for (int i = 1; i <= n; ++i)
        for (int j = 1; j <= n; ++j)
            U[AT(i, j)] = u[(size_t)(i - 1) * n + (j - 1)];
    for (int j = 1; j <= n; ++j) {
        U[AT(0, j)] = bdy[j - 1];
        U[AT(n + 1, j)] = bdy[n + j - 1];
    }
    for (int i = 1; i <= n; ++i) {
        U[AT(i, 0)] = bdy[2 * n + i - 1];
        U[AT(i, n + 1)] = bdy[3 * n + i - 1];
    }
    float w = (float)omega;
    int status = ORC_NOT_CONVERGED;
    int64_t it;
    double last = NAN;
    for (it = 1; it <= max_iters; ++it) {
        int bad = 0;
        float m0 = orc_half_sweep_f32(n, U, F, w, 0, 0, 1, &bad);
        float m1 = orc_half_sweep_f32(n, U, F, w, 1, 0, 1, &bad);
        double m = (double)(m1 > m0 ? m1 : m0);
        if (mhist) mhist[it - 1] = m;
        if (bad) { status = ORC_ENONFINITE; last = m; break; }
        if (it % check_every == 0 || it == max_iters) {
            last = m;
            if (m < tol) { status = ORC_OK; break; }
        }
    }
    if (it > max_iters) it = max_iters;
    for (int i = 1; i <= n; ++i)
        for (int j = 1; j <= n; ++j)
            u[(size_t)(i - 1) * n + (j - 1)] = U[AT(i, j)];
    if (iters_out) *iters_out = it;
    if (max_out) *max_out = last;
    free(U);
    free(F);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Mixed precision: FP64 defect correction around reduced-precision SOR      */
/* ------------------------------------------------------------------------ */

/*
 * Power-of-two scale for the correction equation's right-hand side:
 * s = 2^floor(log2(target / rinf)), so that max |s*r| lies in [target/2,
 * target).  Scaling and unscaling by a power of two are exact.
 */
static int orc_scale_exp(double target, double rinf)
{
    int e;
    frexp(target / rinf, &e);          /* target/rinf = m * 2^e, m in [0.5,1) */
    return e - 1;
}

/*
 * Defect correction (iterative refinement) with an FP64 outer loop:
 *   r = b - A u in FP64 (oracle_residual_f64's expression), rel = |r|_2/|b|_2;
 *   stop when rel <= rel_tol, or after max_outer corrections;
 *   otherwise solve A e = r approximately by inner_iters red-black SOR
 *   iterations in reduced precision from e = 0 with a zero boundary, then
 *   u = u + e in FP64.
 * inner_bits = 32: e and the right-hand side are floats, arithmetic in float.
 * inner_bits = 16: e and the right-hand side are stored as binary16,
 *   arithmetic in float (each stored value rounded by oracle_round_half).
 * The right-hand side handed to the inner solve is R = fl(r * 2^p) (double to
 * float, then float to binary16 for 16-bit storage) with
 *   p = floor(log2(target / max|r|)), target = 1 for 32-bit storage and
 *   target = 2^14 * h*h / 0.0737 for 16-bit storage (0.0737 bounds the
 *   infinity norm of the inverse of the unscaled 5-point operator on the unit
 *   square, so |e * 2^p| stays below about 2^14, well inside binary16 range);
 * the correction is added as u = u + (double)e * 2^-p.
 * relhist (length max_outer + 1, may be NULL) receives rel before each
 * correction and the final rel.  *outer_out = number of corrections applied.
 * corr_tol > 0 adds a second way to stop, tested after rel: at least one
 * correction applied and the last one's max |e * 2^-p| below corr_tol (the
 * change of u over one outer step).
 * threads > 1 runs each inner half-sweep on that many OpenMP workers (the
 * residual, its sums and the accumulation stay serial, in row-major order);
 * results are identical for every thread count.
 * Returns ORC_OK when a stopping test passed, ORC_ENONFINITE when rel is not
 * finite (a NaN or infinity in the data, or a norm that overflows; the paper
 * says nothing of such values, and every solve here ends on them), else
 * ORC_NOT_CONVERGED.
 */
int oracle_mixed(int n, double *u, const double *bdy, const double *f,
                 double omega, double rel_tol, double corr_tol,
                 int64_t max_outer, int inner_bits, int64_t inner_iters,
                 int threads, int64_t *outer_out, double *rel_out, double *relhist,
                 double *corr_out)
{
    if (n < 1 || !u || !bdy || !(omega > 0.0 && omega < 2.0) ||
        !(rel_tol >= 0.0) || max_outer < 0 || inner_iters < 0 || threads < 1 ||
        (inner_bits != 32 && inner_bits != 16))
        return ORC_EINVAL;
    size_t cells = (size_t)(n + 2) * (size_t)(n + 2);
    double *U = malloc(sizeof(double) * cells);
    double *r = malloc(sizeof(double) * (size_t)n * (size_t)n);
    float *E = malloc(sizeof(float) * cells);
    float *R = calloc(cells, sizeof(float));
    double *F = orc_make_F(n, f);
    if (!U || !r || !E || !R || (f && !F)) {
        free(U); free(r); free(E); free(R); free(F);
        return ORC_ENOMEM;
    }
    orc_fill_f64(n, U, u, bdy);
    double h = orc_h(n);
    double target = (inner_bits == 16) ? ldexp(h * h, 14) / 0.0737 : 1.0;
    float w = (float)omega;
    int half = (inner_bits == 16);

    int status = ORC_NOT_CONVERGED;
    int64_t outer = 0;
    double rel = NAN, last_corr = NAN;
    for (;;) {
        double st[3];
        orc_residual_core(n, U, F, r, st);
        rel = (st[1] > 0.0) ? sqrt(st[0]) / sqrt(st[1]) : sqrt(st[0]);
        if (relhist) relhist[outer] = rel;
        if (!isfinite(rel)) { status = ORC_ENONFINITE; break; }
        if (rel <= rel_tol || st[2] == 0.0) { status = ORC_OK; break; }
        if (corr_tol > 0.0 && outer > 0 && last_corr < corr_tol) { status = ORC_OK; break; }
        if (outer == max_outer) break;
        int p = orc_scale_exp(target, st[2]);
        for (int i = 1; i <= n; ++i)
            for (int j = 1; j <= n; ++j) {
                float v = (float)ldexp(r[(size_t)(i - 1) * n + (j - 1)], p);
                R[AT(i, j)] = half ? oracle_round_half(v) : v;
            }
        memset(E, 0, sizeof(float) * cells);
        for (int64_t k = 0; k < inner_iters; ++k) {
            int bad = 0;
            orc_half_sweep_f32(n, E, R, w, 0, half, threads, &bad);
            orc_half_sweep_f32(n, E, R, w, 1, half, threads, &bad);
        }
        double inv = ldexp(1.0, -p);
        last_corr = 0.0;
        for (int i = 1; i <= n; ++i)
            for (int j = 1; j <= n; ++j) {
                double corr = (double)E[AT(i, j)] * inv;
                U[AT(i, j)] = U[AT(i, j)] + corr;
                if (fabs(corr) > last_corr) last_corr = fabs(corr);
            }
        ++outer;
    }
    orc_extract_f64(n, U, u);
    if (outer_out) *outer_out = outer;
    if (rel_out) *rel_out = rel;
    if (corr_out) *corr_out = last_corr;
    free(U); free(r); free(E); free(R); free(F);
    return status;
}

/* ======================================================================== */
/* 3-D red-black SOR, 7-point stencil (the paper's stated extension, Sec. 5) */
/* ======================================================================== */
/*
 * Grid convention in 3-D: the n x n x n interior of the unit cube is embedded
 * in an (n+2)^3 array V indexed V[z][y][x] (x fastest), with the Dirichlet
 * boundary on the six faces.  Cell (z, y, x), indices into the full array,
 * is red when z + y + x is even (the 2-D rule of Sec. 3.1 with one more
 * axis), so interior cell (1, 1, 1) is black and (1, 1, 2) red; red cells are
 * updated first.
 *
 * User-facing arrays:
 *   u    n^3 interior values, u[((z-1)*n + (y-1))*n + (x-1)] is V[z][y][x].
 *   bdy  6 faces of n*n values in the order x = 0, x = n+1 (indexed [z][y]),
 *        y = 0, y = n+1 (indexed [z][x]), z = 0, z = n+1 (indexed [y][x]),
 *        each row-major over its two indices 1..n.
 *   f    n^3 source of -lap(u) = f, laid out like u, or NULL.
 *
 * The Gauss-Seidel value of a cell is the average of its six neighbours: the
 * sum is formed as ((W + E) + (N + S)) + (D + U) with W/E the x-, N/S the y-
 * and D/U the z-neighbours, then + F with F = h*h*f, then multiplied by
 * SIXTH = fl(1/6) (one rounding; 1/6 is not a power of two, so this product
 * is fixed here as the definition two implementations share).  The update,
 * change and stopping rule are those of the 2-D oracle (Eq. 1 in increment
 * form, Algorithm 1).
 */
#define AT3(z, y, x) (((size_t)(z) * (size_t)(n + 2) + (size_t)(y)) * (size_t)(n + 2) + (size_t)(x))

static const double ORC_SIXTH = 1.0 / 6.0;

static void orc_fill3_f64(int n, double *V, const double *u, const double *bdy)
{
    size_t nn = (size_t)n * (size_t)n;
    memset(V, 0, sizeof(double) * (size_t)(n + 2) * (size_t)(n + 2) * (size_t)(n + 2));
    for (int z = 1; z <= n; ++z)
        for (int y = 1; y <= n; ++y)
            for (int x = 1; x <= n; ++x)
                V[AT3(z, y, x)] = u[((size_t)(z - 1) * n + (y - 1)) * n + (x - 1)];
    for (int a = 1; a <= n; ++a)
        for (int c = 1; c <= n; ++c) {
            size_t k = (size_t)(a - 1) * n + (c - 1);
            V[AT3(a, c, 0)] = bdy[0 * nn + k];          /* x = 0,   [z][y] */
            V[AT3(a, c, n + 1)] = bdy[1 * nn + k];      /* x = n+1, [z][y] */
            V[AT3(a, 0, c)] = bdy[2 * nn + k];          /* y = 0,   [z][x] */
            V[AT3(a, n + 1, c)] = bdy[3 * nn + k];      /* y = n+1, [z][x] */
            V[AT3(0, a, c)] = bdy[4 * nn + k];          /* z = 0,   [y][x] */
            V[AT3(n + 1, a, c)] = bdy[5 * nn + k];      /* z = n+1, [y][x] */
        }
}

/* One half-sweep of one colour over planes z_lo..z_hi, in place. */
static double orc_half_sweep3_f64(int n, double *V, const double *F, double w,
                                  int colour, int z_lo, int z_hi, int *bad)
{
    double m = 0.0;
    for (int z = z_lo; z <= z_hi; ++z)
        for (int y = 1; y <= n; ++y) {
            int x0 = 1 + ((z + y + 1 + colour) & 1);   /* first x with the colour */
            for (int x = x0; x <= n; x += 2) {
                double old = V[AT3(z, y, x)];
                double s = ((V[AT3(z, y, x - 1)] + V[AT3(z, y, x + 1)]) +
                            (V[AT3(z, y - 1, x)] + V[AT3(z, y + 1, x)])) +
                           (V[AT3(z - 1, y, x)] + V[AT3(z + 1, y, x)]);
                if (F) s = s + F[AT3(z, y, x)];
                double gs = ORC_SIXTH * s;
                double nu = fma(w, gs - old, old);
                double d = fabs(nu - old);
                if (!isfinite(nu)) *bad = 1;
                if (d > m) m = d;
                V[AT3(z, y, x)] = nu;
            }
        }
    return m;
}

/*
 * 3-D red-black SOR with Algorithm 1's control (same arguments and outputs as
 * oracle_sor_f64; threads > 1 splits the planes of each colour across OpenMP
 * workers, bitwise identical to one thread).
 */
int oracle_sor3d_f64(int n, double *u, const double *bdy, const double *f,
                     double omega, double tol, int64_t max_iters,
                     int64_t check_every, int threads, int64_t *iters_out,
                     double *max_out, double *mhist)
{
    if (n < 1 || !u || !bdy || !(omega > 0.0 && omega < 2.0) || !(tol >= 0.0) ||
        max_iters < 1 || check_every < 1 || threads < 1)
        return ORC_EINVAL;
    size_t cells = (size_t)(n + 2) * (size_t)(n + 2) * (size_t)(n + 2);
    double *V = malloc(sizeof(double) * cells);
    if (!V) return ORC_ENOMEM;
    double *F = NULL;
    if (f) {
        F = calloc(cells, sizeof(double));
        if (!F) { free(V); return ORC_ENOMEM; }
        double h = orc_h(n);
        double h2 = h * h;
        for (int z = 1; z <= n; ++z)
            for (int y = 1; y <= n; ++y)
                for (int x = 1; x <= n; ++x)
                    F[AT3(z, y, x)] = h2 * f[((size_t)(z - 1) * n + (y - 1)) * n + (x - 1)];
    }
    orc_fill3_f64(n, V, u, bdy);
    int status = ORC_NOT_CONVERGED;
    int64_t it = 0;
    double last = NAN;
    for (it = 1; it <= max_iters; ++it) {
        double m = 0.0;
        int bad = 0;
        for (int colour = 0; colour < 2; ++colour) {
            double mc = 0.0;
            int badc = 0;
            if (threads == 1) {
                mc = orc_half_sweep3_f64(n, V, F, omega, colour, 1, n, &badc);
            } else {
#pragma omp parallel for num_threads(threads) schedule(static) reduction(max : mc) reduction(| : badc)
                for (int z = 1; z <= n; ++z) {
                    int b1 = 0;
                    double r = orc_half_sweep3_f64(n, V, F, omega, colour, z, z, &b1);
                    if (r > mc) mc = r;
                    badc |= b1;
                }
            }
            if (mc > m) m = mc;
            bad |= badc;
        }
        if (mhist) mhist[it - 1] = m;
        if (bad) { status = ORC_ENONFINITE; last = m; break; }
        if (it % check_every == 0 || it == max_iters) {
            last = m;
            if (m < tol) { status = ORC_OK; break; }
        }
    }
    if (it > max_iters) it = max_iters;
    for (int z = 1; z <= n; ++z)
        for (int y = 1; y <= n; ++y)
            for (int x = 1; x <= n; ++x)
                u[((size_t)(z - 1) * n + (y - 1)) * n + (x - 1)] = V[AT3(z, y, x)];
    if (iters_out) *iters_out = it;
    if (max_out) *max_out = last;
    free(V); free(F);
    return status;
}
