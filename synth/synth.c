/*
 * Seeded synthetic inputs for the AVU-GSR astrometric system (host, C).
 *
 * This file is shared input plumbing: it draws the structure, the coefficient
 * values, the true solution and the observation noise of a synthetic system
 * shaped like the one the paper solves (Sect. 2: rows are observations grouped
 * by star, 5 astrometric + 3x4 attitude + 6 instrumental + 1 global nonzeros
 * per row). It contains none of the solver's arithmetic: no products with the
 * matrix, no norms, no LSQR step. The known terms b = A x_true + noise are
 * formed by whoever consumes these arrays.
 *
 * Random numbers come from the counter-based generator Philox4x32-10
 * (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11), implemented here from its published round function. Every draw is
 * addressed by (seed, stream, index, sub-index), so any row range can be
 * produced independently and in parallel with bit-identical results.
 *
 * Streams (key word 1):
 *   0  structure of row i       : attitude start t_i, instrumental columns
 *   1  coefficient values of row i
 *   2  x_true, one draw per column
 *   3+r  observation noise of right-hand side r, one draw per row
 *   4  astrometric column scale (conditioning knob), one draw per astro column
 *   5  observations per star (uneven segment lengths), one draw per star
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

/* One Philox4x32 bijection with 10 rounds: out = F_key(ctr). */
void synth_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        uint64_t p0 = (uint64_t)PHILOX_M0 * x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static inline void draw(uint64_t seed, uint32_t stream, uint64_t idx, uint32_t sub, uint32_t w[4])
{
    uint32_t ctr[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), sub, 0u};
    uint32_t key[2] = {(uint32_t)seed, stream ^ (uint32_t)(seed >> 32)};
    synth_philox4x32_10(ctr, key, w);
}

/* 53-bit uniform in the open interval (0,1). */
static inline double u01(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 0.5) * (1.0 / 9007199254740992.0);
}

/* Uniform integer in [0, n) from a 64-bit draw (multiply-high; bias <= n / 2^64). */
static inline uint64_t below(uint32_t a, uint32_t b, uint64_t n)
{
    uint64_t r = ((uint64_t)a << 32) | b;
    return (uint64_t)(((unsigned __int128)r * n) >> 64);
}

/* Two standard normals from one Philox output, Box-Muller transform. */
static inline void normal2(const uint32_t w[4], double* z0, double* z1)
{
    const double two_pi = 6.283185307179586476925286766559;
    double u1 = u01(w[0], w[1]);
    double u2 = u01(w[2], w[3]);
    double r = sqrt(-2.0 * log(u1));
    *z0 = r * cos(two_pi * u2);
    *z1 = r * sin(two_pi * u2);
}

/* Observations per star: fixed (lo == hi) or uniform in [lo, hi]. */
void synth_star_counts(uint64_t seed, int64_t n_stars, int32_t lo, int32_t hi, int64_t* counts)
{
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n_stars; ++s) {
        if (lo == hi) { counts[s] = lo; continue; }
        uint32_t w[4];
        draw(seed, 5u, (uint64_t)s, 0u, w);
        counts[s] = lo + (int64_t)below(w[0], w[1], (uint64_t)(hi - lo + 1));
    }
}

/* star_of_row for rows [r0, r1) given the exclusive prefix sum of counts
 * (first_row[s] = first row of star s, first_row[n_stars] = total rows). */
void synth_star_of_row(const int64_t* first_row, int64_t n_stars, int64_t r0, int64_t r1,
                       int64_t* star_of_row /* [r1 - r0] */)
{
    /* locate the star of r0 by bisection, then walk */
    int64_t lo = 0, hi = n_stars;
    while (hi - lo > 1) {
        int64_t mid = lo + (hi - lo) / 2;
        if (first_row[mid] <= r0) lo = mid; else hi = mid;
    }
    int64_t s = lo;
    for (int64_t i = r0; i < r1; ++i) {
        while (s + 1 < n_stars && first_row[s + 1] <= i) ++s;
        star_of_row[i - r0] = s;
    }
}

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/*
 * Rows [r0, r1) of the system. Output arrays are structure-of-arrays with row
 * stride `ld` (the caller's leading dimension, usually r1 - r0 or the full m),
 * indexed at (i - r0):
 *   values  [n_par][ld]  as double (value_kind 0) or float (value_kind 1),
 *                        section order astro[0..n_astro) | att axis-major
 *                        [n_axes][n_par_axis] | instr[0..n_instr) | glob[0..n_glob)
 *   att_start [ld]       t_i uniform in [0, n_dfa - n_par_axis]
 *   instr_idx [n_instr][ld]  distinct, ascending, uniform in [0, n_instr_cols)
 * astro_scale_lo/hi: when lo < hi, astrometric coefficient j of row i is
 * multiplied by 10^U(lo,hi) drawn once per astrometric column
 * (n_astro * star + j) before any rounding to float.
 */
void synth_rows(uint64_t seed, int64_t r0, int64_t r1, int64_t ld,
                const int64_t* star_of_row /* [ld], indexed at i - r0 */,
                int32_t n_astro, int32_t n_axes, int32_t n_par_axis, int64_t n_dfa,
                int32_t n_instr, int64_t n_instr_cols, int32_t n_glob,
                double astro_scale_lo, double astro_scale_hi,
                int32_t value_kind, void* values, int64_t* att_start, int32_t* instr_idx)
{
    const int32_t n_par = n_astro + n_axes * n_par_axis + n_instr + n_glob;
    const int do_scale = astro_scale_lo < astro_scale_hi;
    #pragma omp parallel for schedule(static)
    for (int64_t i = r0; i < r1; ++i) {
        const int64_t o = i - r0;
        uint32_t w[4];
        /* structure: attitude start */
        draw(seed, 0u, (uint64_t)i, 0u, w);
        if (att_start) {
            uint64_t span = (uint64_t)(n_dfa - n_par_axis + 1);
            att_start[o] = (int64_t)below(w[0], w[1], span);
        }
        /* structure: n_instr distinct instrumental columns (Floyd's sampling) */
        if (instr_idx && n_instr > 0) {
            int32_t pick[8];
            int32_t k = 0;
            for (int64_t j = n_instr_cols - n_instr; j < n_instr_cols; ++j) {
                uint32_t d = (uint32_t)(j - (n_instr_cols - n_instr)); /* draw number 0.. */
                uint32_t ww[4];
                draw(seed, 0u, (uint64_t)i, 1u + d / 2u, ww);
                uint32_t a = (d & 1u) ? ww[2] : ww[0];
                uint32_t b = (d & 1u) ? ww[3] : ww[1];
                int32_t t = (int32_t)below(a, b, (uint64_t)(j + 1));
                int seen = 0;
                for (int32_t q = 0; q < k; ++q) if (pick[q] == t) { seen = 1; break; }
                pick[k++] = seen ? (int32_t)j : t;
            }
            qsort(pick, (size_t)k, sizeof(int32_t), cmp_i32);
            for (int32_t q = 0; q < k; ++q) instr_idx[(int64_t)q * ld + o] = pick[q];
        }
        /* values: N(0,1), two per Philox call */
        if (values) {
            double z[32];
            for (int32_t g = 0; 2 * g < n_par; ++g) {
                draw(seed, 1u, (uint64_t)i, (uint32_t)g, w);
                normal2(w, &z[2 * g], &z[2 * g + 1]);
            }
            if (do_scale) {
                int64_t s = star_of_row[o];
                for (int32_t j = 0; j < n_astro; ++j) {
                    uint64_t col = (uint64_t)(n_astro * s + j);
                    draw(seed, 4u, col, 0u, w);
                    double e = astro_scale_lo + (astro_scale_hi - astro_scale_lo) * u01(w[0], w[1]);
                    z[j] *= pow(10.0, e);
                }
            }
            if (value_kind == 0) {
                double* v = (double*)values;
                for (int32_t c = 0; c < n_par; ++c) v[(int64_t)c * ld + o] = z[c];
            } else {
                float* v = (float*)values;
                for (int32_t c = 0; c < n_par; ++c) v[(int64_t)c * ld + o] = (float)z[c];
            }
        }
    }
}

/* One N(0, sigma) draw per index in [i0, i1) of stream `stream`. */
void synth_normals(uint64_t seed, uint32_t stream, int64_t i0, int64_t i1, double sigma, double* out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = i0; i < i1; ++i) {
        uint32_t w[4];
        double z0, z1;
        draw(seed, stream, (uint64_t)i, 0u, w);
        normal2(w, &z0, &z1);
        out[i - i0] = sigma * z0;
    }
}
