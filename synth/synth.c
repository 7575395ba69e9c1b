/*
 * Host side of the seeded synthetic-system generator (OpenMP over rows).
 * All draws come from gen_core.h, which the on-GPU generator (synth_gpu.hip)
 * compiles too, so both produce the same bits. See gen_core.h for the
 * streams and counters. Input plumbing only: no arithmetic of the solver.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "gen_core.h"

/* One Philox4x32-10 block (exported for the known-answer test). */
void synth_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    synth_philox(ctr, key, out);
}

void synth_star_counts(uint64_t seed, int64_t n_stars, int32_t lo, int32_t hi, int64_t* counts)
{
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n_stars; ++s) counts[s] = synth_star_count(seed, s, lo, hi);
}

/* star_of_row for rows [r0, r1) from first_row[s] (exclusive prefix sum of
 * the counts, first_row[n_stars] = total rows). */
void synth_star_of_row(const int64_t* first_row, int64_t n_stars, int64_t r0, int64_t r1,
                       int64_t* star_of_row)
{
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

/*
 * Rows [r0, r1) into structure-of-arrays outputs with row stride ld, indexed
 * at (i - r0): values [n_par][ld] as double (value_kind 0) or float (1, one
 * rounding of the double draw), att_start [ld], instr_idx [n_instr][ld].
 */
void synth_rows(uint64_t seed, int64_t r0, int64_t r1, int64_t ld, const int64_t* star_of_row,
                int32_t n_astro, int32_t n_axes, int32_t n_par_axis, int64_t n_dfa,
                int32_t n_instr, int64_t n_instr_cols, int32_t n_glob, double scale_lo,
                double scale_hi, double corr, int32_t value_kind, void* values,
                int64_t* att_start, int32_t* instr_idx)
{
    synth_params P;
    P.n_astro = n_astro; P.n_axes = n_axes; P.n_par_axis = n_par_axis; P.n_instr = n_instr;
    P.n_glob = n_glob; P.value_kind = value_kind; P.n_dfa = n_dfa; P.n_instr_cols = n_instr_cols;
    P.scale_lo = scale_lo; P.scale_hi = scale_hi; P.corr = corr;
    const int32_t n_par = n_astro + n_axes * n_par_axis + n_instr + n_glob;
    #pragma omp parallel for schedule(static)
    for (int64_t i = r0; i < r1; ++i) {
        const int64_t o = i - r0;
        double z[SYNTH_MAX_PAR];
        int32_t ins[SYNTH_MAX_INSTR];
        int64_t t;
        synth_row(seed, i, star_of_row[o], &P, z, &t, ins);
        if (att_start) att_start[o] = t;
        if (instr_idx) for (int32_t q = 0; q < n_instr; ++q) instr_idx[(int64_t)q * ld + o] = ins[q];
        if (values) {
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

void synth_normals(uint64_t seed, uint32_t stream, int64_t i0, int64_t i1, double sigma, double* out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = i0; i < i1; ++i) out[i - i0] = synth_normal_at(seed, stream, i, sigma);
}

/* The generator's own ln and exp, exported for their accuracy test. */
double synth_test_ln(double x) { return synth_ln(x); }
double synth_test_exp(double x) { return synth_exp(x); }
