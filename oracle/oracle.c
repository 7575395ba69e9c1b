/*
 * Oracle: plain, slow, sequential FP64 implementation of the AVU-GSR LSQR
 * solve. TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the
 * benchmark's CPU-baseline leg call it; the GPU library never does.
 *
 * What it follows
 *   - System A x = b of the paper's Eq. (1); matrix stored as its nonzeros per
 *     row (the paper's A_d) with the astrometric/attitude column indices M_i
 *     and the instrumental indices I_c (Sect. 2).
 *   - aprod mode 1, b += A x, Eq. (2); aprod mode 2, x += A^T b, Eq. (3);
 *     sections visited per row in the order astrometric, attitude (3 axes x 4
 *     consecutive columns at stride N_DFA, one start per row shared by the
 *     axes), instrumental, global, as in the row loops of Algorithms 2 and 3.
 *   - Preconditioning: every column divided by its 2-norm, the normalisation
 *     factors kept in p, the solution re-multiplied by p after LSQR
 *     (Sect. 2 and Algorithm 1).
 *   - Constraint equations (Sect. 2): extra rows placed after the observation
 *     rows, visited after them in both aprods. Their content is defined
 *     outside the paper; here they are general sparse rows (CSR).
 *   - Norms of the LSQR vectors by the max-scaled sum of squares of Eq. (4).
 *   - LSQR itself: Golub-Kahan bidiagonalisation + Givens QR with the
 *     estimates and stopping rules of Paige & Saunders, ACM TOMS 8 (1982),
 *     Sects. 4 and 6 (the method the paper cites); damping 0.
 *
 * Readings where the paper is silent:
 *   - Columns are ordered astrometric | attitude | instrumental | global;
 *     astrometric column of row i, parameter j: n_astro * star(i) + j.
 *   - A column with zero norm gets p_j = 1.
 *   - x_0 = 0; the "initial solution via aprod 2" is alpha_1 v_1 = A^T u_1.
 *   - xnorm is computed explicitly as ||y_k|| with Eq. (4).
 *   - tests=0 disables the stopping tests 1..6 (fixed iteration count).
 *
 * No code is shared with the GPU library.
 *
 * Builds. The reference build (single thread, -O2, no floating-point
 * contraction) is the pinned oracle. The same source compiled with -fopenmp
 * is the timing build of the CPU baseline: the OpenMP pragmas below only
 * split loops whose iterations are independent (rows of aprod1, elements of
 * the vector updates), reductions, and aprod2 / the column norms, where
 * threads own star-aligned row ranges (so each star's astrometric columns
 * belong to one thread) and accumulate the attitude, instrumental and global
 * columns privately, added up at the end. Without -fopenmp the pragmas are
 * ignored and every loop runs as written, in order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t m;             /* rows (observations) */
    int64_t n_stars;
    int32_t n_astro, n_axes, n_par_axis;
    int64_t n_dfa;
    int32_t n_instr;
    int64_t n_instr_cols;
    int32_t n_glob;
    int32_t value_is_f32;  /* values stored as float: widened on read */
    const void* values;    /* [n_par][m] */
    const int64_t* star;   /* [m] */
    const int64_t* att;    /* [m] */
    const int32_t* instr;  /* [n_instr][m] */
    int64_t n_con;         /* constraint rows m .. m + n_con - 1 */
    const int64_t* con_rowptr; /* [n_con + 1] */
    const int64_t* con_col;    /* [nnz] unknown index */
    const double* con_val;     /* [nnz] */
} orc_system;

typedef struct {
    int32_t istop, itn;
    double rnorm, arnorm, anorm, acond, xnorm, bnorm;
} orc_info;

static int32_t n_par_of(const orc_system* s)
{
    return s->n_astro + s->n_axes * s->n_par_axis + s->n_instr + s->n_glob;
}

int64_t orc_ncols(const orc_system* s)
{
    return (int64_t)s->n_astro * s->n_stars + (int64_t)s->n_axes * s->n_dfa + s->n_instr_cols
           + s->n_glob;
}

/* coefficient c of row i */
static double coef(const orc_system* s, int32_t c, int64_t i)
{
    if (s->value_is_f32) return (double)((const float*)s->values)[(int64_t)c * s->m + i];
    return ((const double*)s->values)[(int64_t)c * s->m + i];
}

/* column in A of coefficient c of row i */
static int64_t column(const orc_system* s, int32_t c, int64_t i)
{
    const int64_t att_base = (int64_t)s->n_astro * s->n_stars;
    const int64_t instr_base = att_base + (int64_t)s->n_axes * s->n_dfa;
    const int64_t glob_base = instr_base + s->n_instr_cols;
    const int32_t n_att = s->n_axes * s->n_par_axis;
    if (c < s->n_astro) return (int64_t)s->n_astro * s->star[i] + c;
    c -= s->n_astro;
    if (c < n_att) {
        int32_t axis = c / s->n_par_axis, q = c % s->n_par_axis;
        return att_base + (int64_t)axis * s->n_dfa + s->att[i] + q;
    }
    c -= n_att;
    if (c < s->n_instr) return instr_base + s->instr[(int64_t)c * s->m + i];
    c -= s->n_instr;
    return glob_base + c;
}

/* Threads of the timing build (1 in the reference build). */
int32_t orc_num_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* Eq. (2): y[i] += sum_c A_d[i][c] * x[col(i,c)], rows in order, then the
 * constraint rows. */
void orc_aprod1(const orc_system* s, const double* x, double* y)
{
    const int32_t np = n_par_of(s);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s->m; ++i) {
        double sum = 0.0;
        for (int32_t c = 0; c < np; ++c) sum += coef(s, c, i) * x[column(s, c, i)];
        y[i] += sum;
    }
    for (int64_t r = 0; r < s->n_con; ++r) {
        double sum = 0.0;
        for (int64_t e = s->con_rowptr[r]; e < s->con_rowptr[r + 1]; ++e)
            sum += s->con_val[e] * x[s->con_col[e]];
        y[s->m + r] += sum;
    }
}

/* Selected observation rows only (rows[k] < m): out[k] = (A x)[rows[k]]. */
void orc_aprod1_rows(const orc_system* s, const double* x, const int64_t* rows, int64_t nr,
                     double* out)
{
    const int32_t np = n_par_of(s);
    for (int64_t k = 0; k < nr; ++k) {
        int64_t i = rows[k];
        double sum = 0.0;
        for (int32_t c = 0; c < np; ++c) sum += coef(s, c, i) * x[column(s, c, i)];
        out[k] = sum;
    }
}

#ifdef _OPENMP
/* Timing build: x[col] += A_d[i][c] * w_i (w_i = y[i], or A_d[i][c] itself
 * when y is NULL: the squared column norms) with threads owning star-aligned
 * row ranges; astrometric columns are written directly (one thread holds all
 * rows of a star), the other columns go to per-thread accumulators that are
 * added to x at the end. */
static int aprod2_threads(const orc_system* s, double* x, const double* y)
{
    const int nt = omp_get_max_threads();
    const int32_t np = n_par_of(s);
    const int64_t att_base = (int64_t)s->n_astro * s->n_stars;
    const int64_t nrest = orc_ncols(s) - att_base;
    double* priv = (double*)calloc((size_t)nt * (size_t)(nrest > 0 ? nrest : 1), sizeof(double));
    if (!priv) return -1;
#pragma omp parallel num_threads(nt)
    {
        const int t = omp_get_thread_num();
        int64_t r0 = s->m * t / nt, r1 = s->m * (t + 1) / nt;
        while (r0 > 0 && r0 < s->m && s->star[r0] == s->star[r0 - 1]) ++r0;
        while (r1 > 0 && r1 < s->m && s->star[r1] == s->star[r1 - 1]) ++r1;
        double* acc = priv + (size_t)t * (size_t)nrest;
        for (int64_t i = r0; i < r1; ++i)
            for (int32_t c = 0; c < np; ++c) {
                const double a = coef(s, c, i);
                const int64_t j = column(s, c, i);
                const double v = a * (y ? y[i] : a);
                if (j < att_base) x[j] += v;
                else acc[j - att_base] += v;
            }
#pragma omp barrier
#pragma omp for schedule(static)
        for (int64_t j = 0; j < nrest; ++j) {
            double sum = 0.0;
            for (int k = 0; k < nt; ++k) sum += priv[(size_t)k * (size_t)nrest + j];
            x[att_base + j] += sum;
        }
    }
    free(priv);
    return 0;
}
#endif

/* Eq. (3): x[col(i,c)] += A_d[i][c] * y[i], rows in order, then the
 * constraint rows. */
void orc_aprod2(const orc_system* s, double* x, const double* y)
{
    const int32_t np = n_par_of(s);
#ifdef _OPENMP
    if (omp_get_max_threads() > 1 && aprod2_threads(s, x, y) == 0) {
        /* done by the threads */
    } else
#endif
    for (int64_t i = 0; i < s->m; ++i)
        for (int32_t c = 0; c < np; ++c) x[column(s, c, i)] += coef(s, c, i) * y[i];
    for (int64_t r = 0; r < s->n_con; ++r)
        for (int64_t e = s->con_rowptr[r]; e < s->con_rowptr[r + 1]; ++e)
            x[s->con_col[e]] += s->con_val[e] * y[s->m + r];
}

/* Eq. (4): max-scaled 2-norm. */
double orc_norm(const double* a, int64_t n)
{
    double mx = 0.0;
#pragma omp parallel for reduction(max : mx) schedule(static)
    for (int64_t i = 0; i < n; ++i) if (fabs(a[i]) > mx) mx = fabs(a[i]);
    if (mx == 0.0) return 0.0;
    double ssq = 0.0;
#pragma omp parallel for reduction(+ : ssq) schedule(static)
    for (int64_t i = 0; i < n; ++i) { double t = a[i] / mx; ssq += t * t; }
    return mx * sqrt(ssq);
}

/* p_j = 1 / ||A[:,j]||_2, or 1 for an empty column. */
void orc_precond(const orc_system* s, double* p)
{
    const int64_t n = orc_ncols(s);
    const int32_t np = n_par_of(s);
    double* ssq = (double*)calloc((size_t)n, sizeof(double));
#ifdef _OPENMP
    if (omp_get_max_threads() > 1 && aprod2_threads(s, ssq, NULL) == 0) {
        /* done by the threads */
    } else
#endif
    for (int64_t i = 0; i < s->m; ++i)
        for (int32_t c = 0; c < np; ++c) {
            double a = coef(s, c, i);
            ssq[column(s, c, i)] += a * a;
        }
    for (int64_t e = 0; e < (s->n_con ? s->con_rowptr[s->n_con] : 0); ++e)
        ssq[s->con_col[e]] += s->con_val[e] * s->con_val[e];
    for (int64_t j = 0; j < n; ++j) p[j] = ssq[j] > 0.0 ? 1.0 / sqrt(ssq[j]) : 1.0;
    free(ssq);
}

/*
 * LSQR on Abar = A diag(p) (p = 1 when precondition == 0), x = p .* y.
 * Returns 0, or -1 on allocation failure. var (optional, [n]) receives the
 * diagonal estimate sum_k (w_k/rho_k)^2, re-multiplied by p^2.
 */
int orc_lsqr(const orc_system* s, const double* b, double* x, int32_t itn_limit, double atol,
             double btol, double conlim, int32_t precondition, int32_t tests, orc_info* info,
             double* var)
{
    const int64_t m_obs = s->m, n = orc_ncols(s);
    const int64_t m = m_obs + s->n_con; /* rows of u and b */
    const int64_t nnz = s->n_con ? s->con_rowptr[s->n_con] : 0;
    const int32_t np = n_par_of(s);
    double* p = (double*)malloc((size_t)n * sizeof(double));
    double* u = (double*)malloc((size_t)m * sizeof(double));
    double* v = (double*)malloc((size_t)n * sizeof(double));
    double* w = (double*)malloc((size_t)n * sizeof(double));
    double* y = (double*)calloc((size_t)n, sizeof(double));
    void* scaled = malloc((size_t)np * (size_t)m_obs * sizeof(double));
    double* con_scaled = (double*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    if (!p || !u || !v || !w || !y || !scaled || !con_scaled) {
        free(p); free(u); free(v); free(w); free(y); free(scaled); free(con_scaled);
        return -1;
    }

    /* Normalise A by p (Algorithm 1, preconditioning). */
    if (precondition) orc_precond(s, p);
    else for (int64_t j = 0; j < n; ++j) p[j] = 1.0;
    double* ad = (double*)scaled;
    for (int32_t c = 0; c < np; ++c)
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < m_obs; ++i)
            ad[(int64_t)c * m_obs + i] = coef(s, c, i) * p[column(s, c, i)];
    for (int64_t e = 0; e < nnz; ++e) con_scaled[e] = s->con_val[e] * p[s->con_col[e]];
    orc_system sb = *s;
    sb.values = ad;
    sb.value_is_f32 = 0;
    sb.con_val = con_scaled;

    if (var) memset(var, 0, (size_t)n * sizeof(double));
    const double ctol = conlim > 0.0 ? 1.0 / conlim : 0.0;

    /* beta_1 u_1 = b ; alpha_1 v_1 = Abar^T u_1 */
    memcpy(u, b, (size_t)m * sizeof(double));
    double beta = orc_norm(u, m);
    double alpha = 0.0;
    memset(v, 0, (size_t)n * sizeof(double));
    if (beta > 0.0) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < m; ++i) u[i] /= beta;
        orc_aprod2(&sb, v, u);
        alpha = orc_norm(v, n);
    }
    if (alpha > 0.0)
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; ++j) v[j] /= alpha;
    memcpy(w, v, (size_t)n * sizeof(double));

    const double bnorm = beta;
    double rhobar = alpha, phibar = beta;
    double anorm = 0.0, acond = 0.0, ddnorm = 0.0, xnorm = 0.0;
    double rnorm = beta, arnorm = alpha * beta;
    int32_t istop = 0, itn = 0;

    if (arnorm == 0.0) goto done; /* b = 0 or A^T b = 0: x = 0 is the solution */

    while (itn < itn_limit) {
        ++itn;
        /* beta_{i+1} u_{i+1} = Abar v_i - alpha_i u_i */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < m; ++i) u[i] = -alpha * u[i];
        orc_aprod1(&sb, v, u);
        beta = orc_norm(u, m);
        if (beta > 0.0) {
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < m; ++i) u[i] /= beta;
            anorm = sqrt(anorm * anorm + alpha * alpha + beta * beta);
            /* alpha_{i+1} v_{i+1} = Abar^T u_{i+1} - beta_{i+1} v_i */
#pragma omp parallel for schedule(static)
            for (int64_t j = 0; j < n; ++j) v[j] = -beta * v[j];
            orc_aprod2(&sb, v, u);
            alpha = orc_norm(v, n);
            if (alpha > 0.0)
#pragma omp parallel for schedule(static)
                for (int64_t j = 0; j < n; ++j) v[j] /= alpha;
        }
        /* plane rotation eliminating beta_{i+1} */
        const double rho = sqrt(rhobar * rhobar + beta * beta);
        const double c = rhobar / rho;
        const double sn = beta / rho;
        const double theta = sn * alpha;
        rhobar = -c * alpha;
        const double phi = c * phibar;
        phibar = sn * phibar;

        /* y_i = y_{i-1} + (phi/rho) w_i ; w_{i+1} = v_{i+1} - (theta/rho) w_i */
        double dd = 0.0;
#pragma omp parallel for reduction(+ : dd) schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            const double dk = w[j] / rho;
            dd += dk * dk;
            if (var) var[j] += dk * dk;
        }
        ddnorm += dd;
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            y[j] += (phi / rho) * w[j];
            w[j] = v[j] - (theta / rho) * w[j];
        }

        /* estimates */
        xnorm = orc_norm(y, n);
        acond = anorm * sqrt(ddnorm);
        rnorm = phibar;
        arnorm = alpha * fabs(c) * phibar;

        /* stopping tests */
        const double test1 = rnorm / bnorm;
        const double test2 = (anorm * rnorm) > 0.0 ? arnorm / (anorm * rnorm) : 0.0;
        const double test3 = acond > 0.0 ? 1.0 / acond : 0.0;
        const double t1 = test1 / (1.0 + anorm * xnorm / bnorm);
        const double rtol = btol + atol * anorm * xnorm / bnorm;
        if (itn >= itn_limit) istop = 7;
        if (tests) {
            if (1.0 + test3 <= 1.0) istop = 6;
            if (1.0 + test2 <= 1.0) istop = 5;
            if (1.0 + t1 <= 1.0) istop = 4;
            if (test3 <= ctol) istop = 3;
            if (test2 <= atol) istop = 2;
            if (test1 <= rtol) istop = 1;
        }
        if (istop != 0) break;
    }

done:
    for (int64_t j = 0; j < n; ++j) x[j] = p[j] * y[j];
    if (var) for (int64_t j = 0; j < n; ++j) var[j] *= p[j] * p[j];
    if (info) {
        info->istop = istop; info->itn = itn;
        info->rnorm = rnorm; info->arnorm = arnorm; info->anorm = anorm;
        info->acond = acond; info->xnorm = xnorm; info->bnorm = bnorm;
    }
    free(p); free(u); free(v); free(w); free(y); free(scaled); free(con_scaled);
    return 0;
}
