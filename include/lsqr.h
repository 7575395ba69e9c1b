/*
 * lsqr.h - C ABI of the MI355X (gfx950) AVU-GSR LSQR library.
 *
 * The library solves the overdetermined sparse system A x = b of the Gaia
 * AVU-GSR solver (Cesare et al., "The MPI + CUDA Gaia AVU-GSR Parallel Solver
 * Toward Next-generation Exascale Infrastructures", Eq. (1)) in the least
 * squares sense with LSQR (Paige & Saunders, ACM TOMS 8, 1982), entirely on
 * one GPU. Each row of A is one observation and holds
 *     n_astro = 5 astrometric coefficients  (columns n_astro*star + j),
 *     n_axes * n_par_axis = 3 * 4 attitude coefficients (axis a, parameter q:
 *         column att_base + a*n_dfa + att_start + q, one att_start per row
 *         shared by the three axes),
 *     n_instr = 6 instrumental coefficients (columns instr_base + instr_idx),
 *     n_glob  = 1 global coefficient (column glob_base + g),
 * the row layout of the paper's Sect. 2 (dense per-row coefficient array A_d
 * with index arrays M_i and I_c); subset layouts (fewer astrometric or
 * instrumental coefficients, no attitude section, up to 5 global columns)
 * are accepted as well. Columns are ordered
 *     astrometric [0, att_base) | attitude [att_base, instr_base) |
 *     instrumental [instr_base, glob_base) | global [glob_base, n)
 * with att_base = n_astro*n_stars, instr_base = att_base + n_axes*n_dfa,
 * glob_base = instr_base + n_instr_cols, n = glob_base + n_glob.
 *
 * All array arguments are DEVICE pointers (memory of the GPU the handle was
 * created on) unless stated otherwise. lsqr_aprod1/lsqr_aprod2 run
 * asynchronously on the stream given in the system descriptor; lsqr_create
 * and the solves first synchronize with that stream, run on a stream owned by
 * the handle and return when done. Calls on one handle must not overlap. No
 * function aborts or exits; each returns an lsqr_status, and on failure
 * lsqr_last_error() describes it.
 */
#ifndef AVUGSR_LSQR_H
#define AVUGSR_LSQR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lsqr_status;
#define LSQR_OK 0
#define LSQR_E_INVALID (-1)     /* bad argument, descriptor or index out of range */
#define LSQR_E_HIP (-2)         /* HIP runtime error                                */
#define LSQR_E_NOMEM (-3)       /* device allocation failed                         */
#define LSQR_E_STATE (-4)       /* call not valid for this handle                   */
#define LSQR_E_UNSUPPORTED (-5) /* descriptor valid but outside what is built       */

#define LSQR_F64 0 /* coefficient values stored as double */
#define LSQR_F32 1 /* coefficient values stored as float  */

/* Sparse system descriptor. The matrix arrays are BORROWED: the library keeps
 * the pointers (zero copy), never frees them, and the caller keeps them alive
 * and unchanged until lsqr_destroy. */
typedef struct lsqr_system {
    int64_t n_rows;       /* m, number of observation rows (> 0)                 */
    int64_t n_stars;      /* stars; astrometric columns = n_astro * n_stars       */
    int32_t n_astro;      /* 0..5 astrometric coefficients per row (5)            */
    int32_t n_axes;       /* 3 attitude axes, or 0: no attitude section           */
    int32_t n_par_axis;   /* 4 attitude parameters per axis (ignored if no axes)  */
    int32_t n_instr;      /* 0..6 instrumental coefficients per row (6)           */
    int64_t n_dfa;        /* attitude degrees of freedom per axis (>= n_par_axis) */
    int64_t n_instr_cols; /* instrumental columns (>= n_instr)                    */
    int32_t n_glob;       /* 0..5 global coefficients per row (1)                 */
    int32_t value_type;   /* LSQR_F64 or LSQR_F32                                 */
    int32_t precondition; /* 1: scale columns to unit norm (Sect. 2), 0: no       */
    int32_t reserved;
    /* [n_par][n_rows] structure of arrays, row i of coefficient c at
     * c*n_rows + i, coefficient order astro(n_astro) | att axis0(4) axis1(4)
     * axis2(4) (if n_axes) | instr(n_instr) | glob(n_glob); n_par = 24 for the
     * full layout. Column order astro | att | instr | glob (Algorithms 2-3):
     * astro n_astro*star + j, att n_astro*n_stars + axis*n_dfa + t + q, instr
     * after the n_axes*n_dfa attitude columns, glob after the n_instr_cols
     * instrumental columns. Layouts other than 5 + 3x4 + 6 + 1 run separate
     * aprod1/aprod2 passes with run-time section sizes and no batched solve. */
    const void* values;
    const int64_t* star_of_row; /* [n_rows], non-decreasing, in [0, n_stars)      */
    const int64_t* att_start;   /* [n_rows], in [0, n_dfa - n_par_axis]; NULL ok
                                   without attitude section                       */
    const int32_t* instr_idx;   /* [n_instr][n_rows] SoA, in [0, n_instr_cols);
                                   NULL ok when n_instr = 0                       */
    void* stream;               /* hipStream_t for all work, NULL = null stream   */
    /* Constraint equations (Sect. 2: extra rows at the bottom of the system,
     * defined outside the paper): n_con rows numbered n_rows .. n_rows +
     * n_con - 1 of A, of b and of aprod1/aprod2's y. Row r holds con_val[e]
     * at column con_col[e] for e in [con_rowptr[r], con_rowptr[r + 1])
     * (CSR; a column repeated within a row adds). FP64 values whatever
     * value_type is; borrowed like the matrix arrays. n_con = 0: none, the
     * pointers are ignored. lsqr_solve_batched returns LSQR_E_UNSUPPORTED
     * on a system with constraint rows. */
    int64_t n_con;              /* 0..2^31                                        */
    const int64_t* con_rowptr;  /* [n_con + 1]: 0, non-decreasing, ends at nnz   */
    const int64_t* con_col;     /* [nnz], in [0, n)                               */
    const double* con_val;      /* [nnz]                                          */
} lsqr_system;

/* Result of a solve. istop follows Paige & Saunders:
 * 0 x = 0 solves (b = 0 or A^T b = 0), 1 residual test S1, 2 normal-equation
 * test S2, 3 condition limit, 4/5/6 the same tests at machine precision,
 * 7 iteration limit. Non-convergence (7) is not an error. */
typedef struct lsqr_info {
    int32_t istop;
    int32_t itn;          /* LSQR iterations (inner iterations summed for refined) */
    int32_t outer_steps;  /* refinement steps (lsqr_solve_refined), else 0         */
    int32_t reserved;
    double rnorm;         /* ||b - A x|| estimate (phibar)                         */
    double arnorm;        /* ||Abar^T r|| estimate                                 */
    double anorm;         /* Frobenius-norm estimate of Abar = A diag(p)           */
    double acond;         /* condition estimate of Abar                            */
    double xnorm;         /* ||diag(p)^-1 x||                                      */
    double bnorm;         /* ||b||                                                 */
} lsqr_info;

typedef struct lsqr_handle lsqr_handle;

/* Create a handle: validates the descriptor and every index (a scan of the
 * index arrays and of the constraint rows' structure on the GPU), computes the column scaling p_j = 1/||A[:,j]||
 * (1 for an empty column; Sect. 2, preconditioning) and allocates the
 * workspace (owned by the handle). Synchronous. */
lsqr_status lsqr_create(const lsqr_system* sys, lsqr_handle** out);

/* Free the workspace. Never touches the borrowed arrays. NULL is a no-op. */
lsqr_status lsqr_destroy(lsqr_handle* h);

/* Options (lsqr_set_option):
 *   LSQR_OPT_CONLIM       condition limit of stopping test 3 (default 1e8; 0 off)
 *   LSQR_OPT_TESTS        1 (default): stopping tests 1..6 on; 0: run exactly
 *                         itn_limit iterations (istop 7)
 *   LSQR_OPT_CHUNK        iterations per HIP-graph launch (default 16, >= 1)
 *   LSQR_OPT_GRAPH        1 (default): iterations replayed from a captured HIP
 *                         graph; 0: launched one by one
 *   LSQR_OPT_PROFILE      1: time every aprod1 / aprod2 launch of a solve with
 *                         HIP events on the handle's stream (forces GRAPH 0);
 *                         read back with lsqr_kernel_times
 *   LSQR_OPT_OUTER_TOL    refinement: stop when ||d||_inf <= tol ||x||_inf, or
 *                         when the corrections contract (||d_k|| <= ||d_k-1|| / 2)
 *                         and the next one, estimated as ||d_k||^2 / ||d_k-1||,
 *                         is below tol ||x||_inf / 100 (default 1e-10)
 *   LSQR_OPT_ATT_MODE     attitude part of aprod2: 1 (default) a pass over the
 *                         rows stably sorted by the bucket of their attitude start
 *                         (W starts per bucket), each bucket's 3 x (W + 3)
 *                         columns accumulated in an LDS histogram (no device
 *                         atomics); costs a copy of the 12 attitude coefficients
 *                         in that order and three int32 per row, built on first
 *                         use, needs n_rows < 2^31; the solver keeps its row
 *                         vector u in bucket order; 0 scatter-add with device
 *                         atomics (no extra memory, about 10x slower)
 *   LSQR_OPT_ASTRO_SCAN   astrometric part of aprod2: 0 (default) running
 *                         per-lane partials reduced only where a star ends;
 *                         1 a segmented scan over every 64-row chunk
 *   LSQR_OPT_ATT_BUCKETS  number of attitude buckets: 0 (default) the fewest
 *                         whose FP64 histogram fits in LDS (16 for 10^5 attitude
 *                         columns per axis), n > 0 that many (raised if they do
 *                         not fit); settable only before the first solve or
 *                         aprod2
 *   LSQR_OPT_ATT_INTERLEAVE  aprod1 reads the 12 attitude values of a row from
 *                         a copy of the attitude section interleaved by axis
 *                         (x3[3 c + axis], rebuilt before every aprod1; the
 *                         values are then consecutive): 1 (default) or 0
 *                         (three 4-value windows straight from the vector)
 *   LSQR_OPT_FUSED        with LSQR_OPT_ATT_MODE 1 on the full row layout:
 *                         1: each LSQR iteration reads A once for aprod1 and
 *                         the astrometric, instrumental and global part of
 *                         aprod2 (u~ = Abar v - alpha u is row-local, so every
 *                         row's new value is scattered as soon as it is
 *                         computed), then runs the attitude pass;
 *                         2 (default): the same, with the attitude part of
 *                         aprod1 computed first by a pass over the rows in
 *                         bucket order (the bucket's attitude columns of v in
 *                         LDS, no gathers from global memory) and folded into
 *                         u~, so the fused pass skips the attitude section;
 *                         3: as 2, but u~ stays in star order: the pre-pass
 *                         writes the attitude part to a separate bucket-order
 *                         vector (8 bytes per row, allocated on first use)
 *                         that the fused pass reads through the permutation,
 *                         and the attitude pass reads u~ through it, so no
 *                         pass writes through the permutation (batched k-tiles
 *                         run mode 2);
 *                         0: separate aprod1 and aprod2
 *   LSQR_OPT_VARIANCE     1: lsqr_solve also accumulates the variance estimate of
 *                         the unknowns, sum over iterations of (w/rho)^2 (Algorithm
 *                         1, variances at the end of each iteration; Paige &
 *                         Saunders' diagonal estimate of (Abar^T Abar)^-1), read
 *                         back re-multiplied by p^2 with lsqr_get_variance;
 *                         0 (default) off. One FP64 update per column per iteration
 *   LSQR_OPT_COMPACT_INDEX 1 (default): on the first solve, build int32 copies of
 *                         star_of_row and uint16 copies of instr_idx for the
 *                         fused passes (16 instead of 32 index bytes per row;
 *                         full row layout, n_instr_cols <= 65536, n_stars <
 *                         2^31) when they take at most 1/32 of the device
 *                         memory; the caller's arrays are used otherwise and
 *                         by every other pass; 0: never (frees the copies)
 *   LSQR_OPT_KTILE        batched solves: right-hand sides advanced together per
 *                         pass over A (1, 2, 4, 8, 16; 16 in fused modes 2 and 3
 *                         with LSQR_OPT_RHS_LANES), 0 (default) = autotune (see
 *                         lsqr_batch_tuning)
 *   LSQR_OPT_ATT_RHS      right-hand sides one sweep of the bucket-order
 *                         attitude passes holds (1 default, 2, 4, 8): the
 *                         buckets narrow until that many LDS windows /
 *                         histograms fit, so a batched k-tile of up to that
 *                         many RHS reads the attitude coefficients once per
 *                         pass instead of once per RHS (single-RHS passes pay
 *                         a few percent for the extra buckets); settable only
 *                         before the first solve or aprod2
 *   LSQR_OPT_PIPELINE     1 (default): each thread of the single-RHS bucket-order
 *                         passes issues the loads of its next row before the
 *                         store (or LDS atomics) of the current one, so that no
 *                         row waits for the previous row's store, and the
 *                         RHS-across-lanes fused pass of 4-RHS tiles (and of
 *                         2-RHS tiles unless both values and vectors are
 *                         FP64) issues the next row step's loads before the
 *                         gathers of the current one; 0: one row at a time
 *                         (same results)
 *   LSQR_OPT_RHS_LANES    batched k-tiles of K >= 2 RHS in fused modes 2 and 3:
 *                         1 (default) the fused pass and the first aprod2 of a
 *                         solve put the K right-hand sides of a row in K lanes
 *                         (a wave covers 64 / K rows, a lane holds one value
 *                         per vector entry); 0: one row per lane with K values
 *                         (K <= 8). Same results up to rounding order; the
 *                         16-RHS tile needs 1
 */
#define LSQR_OPT_CONLIM 1
#define LSQR_OPT_TESTS 2
#define LSQR_OPT_CHUNK 3
#define LSQR_OPT_GRAPH 4
#define LSQR_OPT_PROFILE 5
#define LSQR_OPT_OUTER_TOL 6
#define LSQR_OPT_ATT_MODE 7
#define LSQR_OPT_ASTRO_SCAN 8
#define LSQR_OPT_KTILE 9
#define LSQR_OPT_ATT_BUCKETS 10
#define LSQR_OPT_ATT_INTERLEAVE 11
#define LSQR_OPT_FUSED 12
#define LSQR_OPT_VARIANCE 13
#define LSQR_OPT_COMPACT_INDEX 14
#define LSQR_OPT_ATT_RHS 15
#define LSQR_OPT_PIPELINE 16
#define LSQR_OPT_RHS_LANES 17
lsqr_status lsqr_set_option(lsqr_handle* h, int32_t option, double value);

/* Below, m counts every row: n_rows observation rows plus n_con constraint
 * rows. */

/* aprod mode 1, Eq. (2): y[m] += A x[n] with the raw (unscaled) A.
 * FP64 vectors; float-stored values are widened, accumulation in FP64.
 * Asynchronous on the handle's stream; x and y must not overlap. */
lsqr_status lsqr_aprod1(lsqr_handle* h, const double* x, double* y);

/* Scratch capacity of lsqr_aprod1_noalloc, in doubles: 3 * 2^20 (24 MiB per
 * GPU, so n_dfa <= 2^20 attitude columns per axis). */
#define LSQR_NOALLOC_ATT_MAX (3 * 1048576)

/* For callers that cannot allocate device memory (work recorded under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same y += A x as lsqr_aprod1, and calling no allocating routine. Its only
 * scratch, the attitude section of x interleaved by axis (3 n_dfa doubles),
 * lives in one library-wide device array of LSQR_NOALLOC_ATT_MAX doubles per
 * GPU, held until the process ends and shared by every handle and thread on
 * that GPU: calls that overlap on one GPU (two streams, two threads) race
 * on it. Each call rewrites every element it reads, so nothing needs
 * clearing between calls. Returns LSQR_E_INVALID when 3 n_dfa exceeds
 * LSQR_NOALLOC_ATT_MAX. Asynchronous on the handle's stream, like
 * lsqr_aprod1. */
lsqr_status lsqr_aprod1_noalloc(lsqr_handle* h, const double* x, double* y);

/* aprod mode 2, Eq. (3): x[n] += A^T y[m] with the raw A. Same conventions. */
lsqr_status lsqr_aprod2(lsqr_handle* h, double* x, const double* y);

/* FP32 forms of the two operators for FP32-stored systems (LSQR_F32): Eq. (2)
 * y[m] += A x[n] and Eq. (3) x[n] += A^T y[m] with FP32 vectors, FP32
 * products and FP32 accumulation (the LDS histograms of the instrumental and
 * attitude columns of Eq. (3) add in FP64 and store FP32), the arithmetic of
 * the refined solve's inner iterations. Asynchronous on the handle's stream;
 * x and y must not overlap. LSQR_E_STATE on an LSQR_F64 system. */
lsqr_status lsqr_aprod1_f32(lsqr_handle* h, const float* x, float* y);
lsqr_status lsqr_aprod2_f32(lsqr_handle* h, float* x, const float* y);

/* Variance estimate of the unknowns from the last lsqr_solve run with
 * LSQR_OPT_VARIANCE = 1: var_out[j] = p_j^2 sum_k (w_kj / rho_k)^2 (Algorithm 1,
 * variances re-multiplied by p after the loop), FP64 [n], device. Standard
 * errors follow as sqrt(var_j) times the residual standard deviation. Returns
 * LSQR_E_STATE if the last solve did not compute it (option off, or a refined
 * or batched solve since). Synchronous. */
lsqr_status lsqr_get_variance(lsqr_handle* h, double* var_out);

/* Copy the column scaling p (FP64 [n]) into p_out (device). */
lsqr_status lsqr_get_precond(lsqr_handle* h, double* p_out);

/* Least-squares solve of A x = b by LSQR on Abar = A diag(p), x = p .* y
 * (Sect. 2, Algorithm 1; Paige & Saunders). b: FP64 [m], not modified.
 * x: FP64 [n], output (x_0 = 0). atol/btol: stopping tolerances of tests S1,
 * S2, itn_limit >= 0. On an LSQR_F32 system the float values are widened
 * and every operation is FP64 (the FP64 reference of the refined solve).
 * Synchronous; info may be NULL. */
lsqr_status lsqr_solve(lsqr_handle* h, const double* b, double* x, int32_t itn_limit,
                       double atol, double btol, lsqr_info* info);

/* FP32-stored system: FP64 iterative refinement around an FP32 LSQR.
 * Outer step k: r = b - A x in FP64 (values widened, FP64 accumulation),
 * then an inner LSQR on min ||A d - r|| with FP32 products and FP32
 * accumulation (FP64 norms, Givens scalars and x/w updates), stopped once
 * its normal-equation residual estimate ||Abar^T (r - A d)|| has fallen below
 * atol times its initial value ||Abar^T r|| (btol is unused: the residual of
 * a correction problem is dominated by the irreducible least-squares
 * residual, so the absolute tests S1/S2 cannot measure its progress), or
 * after itn_limit iterations; then x += d in FP64. The outer loop ends when
 * ||d||_inf <= OUTER_TOL ||x||_inf, or when the corrections contract
 * (||d_k||_inf <= ||d_k-1||_inf / 2) and the next one, estimated as
 * ||d_k||^2 / ||d_k-1|| (infinity norms), is below OUTER_TOL ||x||_inf / 100,
 * when r is zero or orthogonal to the range of A, or after outer_limit steps.
 * b: FP64 [m]; x: FP64 [n] output (x_0 = 0). info->itn counts the inner
 * iterations of all steps, info->outer_steps the outer steps, info->istop and
 * the estimates are those of the last inner solve (its rnorm estimates
 * ||b - A x||), info->bnorm is ||b|| (of b rounded to FP32, the first inner
 * solve's start vector). Synchronous; info may be NULL. */
lsqr_status lsqr_solve_refined(lsqr_handle* h, const double* b, double* x, int32_t itn_limit,
                               double atol, double btol, int32_t outer_limit, lsqr_info* info);

/* k right-hand sides at once (noise realisations of b for Monte Carlo error
 * propagation). B: FP64 [m][k] row-interleaved (B[i*k + j] is row i of RHS j),
 * X: FP64 [n][k] output likewise. The RHS are advanced in k-tiles of K (the
 * LSQR_OPT_KTILE option or the autotuner's choice): each pass over A serves K
 * RHS (an SpMM), every RHS keeps its own scalars and stopping tests, and a
 * RHS that has stopped is frozen (its x, w, v, u and estimates no longer
 * change) while the others continue. Each x[:, j] is the result lsqr_solve
 * would give for b[:, j] up to rounding order. infos: host array of k
 * results (may be NULL); outer_steps is 0. Synchronous. */
lsqr_status lsqr_solve_batched(lsqr_handle* h, const double* B, double* X, int32_t k,
                               int32_t itn_limit, double atol, double btol, lsqr_info* infos);

/* k right-hand sides of an FP32-stored system (LSQR_F32), each solved by the
 * FP64 iterative refinement of lsqr_solve_refined, with the FP32 inner LSQR
 * solves of a k-tile advancing together (the SpMM form of
 * lsqr_solve_batched; the FP64 outer residuals r_j = b_j - A x_j are formed
 * for the whole tile in one pass). Per RHS j: outer step r_j in FP64 (FP32
 * values widened, FP64 accumulation, stored as the FP32 start vector), inner
 * LSQR with FP32 products and accumulation and FP64 scalars, stopped once
 * ||Abar^T (r_j - A d_j)|| <= atol ||Abar^T r_j|| or after itn_limit
 * iterations (btol unused), then x_j += d_j in FP64; RHS j stops refining
 * by the outer test of lsqr_solve_refined on its own corrections, when r_j
 * is zero or orthogonal to the range of A, or after outer_limit steps, and
 * is frozen while the
 * others continue. Each x[:, j] is the result lsqr_solve_refined would give
 * for b[:, j] up to rounding order. B: FP64 [m][k], X: FP64 [n][k] output,
 * layouts as in lsqr_solve_batched. infos (host, may be NULL): per RHS, itn
 * = inner iterations of all its steps, outer_steps = its steps, istop and
 * estimates of its last inner solve, bnorm = ||b_j|| (as for
 * lsqr_solve_refined, of b_j rounded to FP32). Returns LSQR_E_STATE on
 * an LSQR_F64 system. Synchronous. */
lsqr_status lsqr_solve_batched_refined(lsqr_handle* h, const double* B, double* X, int32_t k,
                                       int32_t itn_limit, double atol, double btol,
                                       int32_t outer_limit, lsqr_info* infos);

/* Autotuner result of this handle: the k-tile of its last autotuned batched
 * solve (0 if none yet) and the measured milliseconds per RHS-iteration for
 * K = 1, 2, 4, 8, 16 of that tuning (5 host doubles, 0 where not measured). The
 * tuner runs on the first batched call for each precision (FP64 tiles,
 * FP32 inner tiles of the refined form) and each min(k, 8), and again after
 * an option that selects kernels changes. Host pointers; either may be
 * NULL. */
lsqr_status lsqr_batch_tuning(lsqr_handle* h, int32_t* k_tile, double* ms_per_rhs_iter);

/* Per-kernel timing of the last solve run with LSQR_OPT_PROFILE = 1:
 * total milliseconds and launch counts of the aprod1 and aprod2 kernels of
 * the iterations (with LSQR_OPT_FUSED: of the fused pass, which includes the
 * attitude-interleave copy, and of the attitude pass). Host pointers; any may
 * be NULL. */
lsqr_status lsqr_kernel_times(lsqr_handle* h, double* ms_aprod1, int64_t* n_aprod1,
                              double* ms_aprod2, int64_t* n_aprod2);

/* Per-pass timing of the last solve run with LSQR_OPT_PROFILE = 1 (FP64 or
 * refined, not batched): ms[0] the attitude pre-pass of fused mode 2 (with the
 * attitude-interleave copy; only that copy in other modes), ms[1] the rest of
 * the aprod1 window (the fused pass, or aprod1), ms[2] the aprod2 window (the
 * attitude pass, or aprod2); n[i] the iterations timed. Host arrays of 3.
 * mode (may be NULL): the fused mode the last FP64 or refined solve ran
 * (0 to 3, see LSQR_OPT_FUSED); compact (may be NULL): 1 when the fused
 * passes read the compact index copies (LSQR_OPT_COMPACT_INDEX). */
lsqr_status lsqr_pass_times(lsqr_handle* h, double* ms, int64_t* n, int32_t* mode,
                            int32_t* compact);

/* Number of columns n of the handle's system. Host pointer out. */
lsqr_status lsqr_num_cols(lsqr_handle* h, int64_t* n_out);

/* Description of the last error on the calling thread ("" if none). */
const char* lsqr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* AVUGSR_LSQR_H */
