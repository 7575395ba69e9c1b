/*
 * Core of the seeded synthetic-system generator, compiled twice: by gcc for
 * the host generator (synth.c) and by hipcc for the on-GPU generator
 * (synth_gpu.hip). Every floating-point result is built only from operations
 * IEEE 754 rounds correctly (+, -, *, /, sqrt) in a fixed order with no
 * contraction into fused multiply-adds, plus exact bit manipulation, so both
 * builds produce bit-identical inputs. Input plumbing only: nothing here
 * computes with the coefficient matrix.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written
 * from its published round function. A draw is addressed by
 * key = (seed_lo, stream ^ seed_hi) and counter = (index_lo, index_hi, sub, k).
 * Normals: Marsaglia's polar method; attempt k of draw `sub` uses counter
 * word 3 = k, so the rejection loop stays counter-addressed.
 */
#ifndef AVUGSR_SYNTH_GEN_CORE_H
#define AVUGSR_SYNTH_GEN_CORE_H

#include <stdint.h>
#include <string.h>

#if defined(__HIPCC__)
#define SYNTH_FN __host__ __device__ static inline
#else
#define SYNTH_FN static inline
#endif

#if defined(__clang__)
#pragma clang fp contract(off)
#endif

#define SYNTH_PHILOX_M0 0xD2511F53u
#define SYNTH_PHILOX_M1 0xCD9E8D57u
#define SYNTH_PHILOX_W0 0x9E3779B9u
#define SYNTH_PHILOX_W1 0xBB67AE85u

SYNTH_FN void synth_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += SYNTH_PHILOX_W0;
            k1 += SYNTH_PHILOX_W1;
        }
        const uint64_t p0 = (uint64_t)SYNTH_PHILOX_M0 * x0;
        const uint64_t p1 = (uint64_t)SYNTH_PHILOX_M1 * x2;
        const uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        const uint32_t y1 = (uint32_t)p1;
        const uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        const uint32_t y3 = (uint32_t)p0;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

SYNTH_FN void synth_draw(uint64_t seed, uint32_t stream, uint64_t idx, uint32_t sub, uint32_t k,
                         uint32_t w[4])
{
    const uint32_t ctr[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), sub, k};
    const uint32_t key[2] = {(uint32_t)seed, stream ^ (uint32_t)(seed >> 32)};
    synth_philox(ctr, key, w);
}

/* 53-bit uniform in (0,1). */
SYNTH_FN double synth_u01(uint32_t a, uint32_t b)
{
    const double hi = (double)(a >> 5) * 67108864.0;
    const double lo = (double)(b >> 6) + 0.5;
    return (hi + lo) * (1.0 / 9007199254740992.0);
}

/* floor(r * n / 2^64) for the 64-bit r = (a:b): uniform integer in [0, n). */
SYNTH_FN uint64_t synth_below(uint32_t a, uint32_t b, uint64_t n)
{
    const uint64_t nlo = (uint32_t)n, nhi = n >> 32;
    const uint64_t ll = (uint64_t)b * nlo;
    const uint64_t lh = (uint64_t)b * nhi;
    const uint64_t hl = (uint64_t)a * nlo;
    const uint64_t hh = (uint64_t)a * nhi;
    const uint64_t mid = (ll >> 32) + (uint32_t)lh + (uint32_t)hl;
    return hh + (lh >> 32) + (hl >> 32) + (mid >> 32);
}

SYNTH_FN uint64_t synth_bits(double x)
{
    uint64_t u;
    memcpy(&u, &x, sizeof u);
    return u;
}

SYNTH_FN double synth_from_bits(uint64_t u)
{
    double x;
    memcpy(&x, &u, sizeof x);
    return x;
}

/* Natural logarithm of a positive normal double: x = f 2^e with f in
 * [sqrt(1/2), sqrt(2)), ln f = 2 atanh(z), z = (f-1)/(f+1), odd series to z^25. */
SYNTH_FN double synth_ln(double x)
{
    const uint64_t u = synth_bits(x);
    int64_t e = (int64_t)((u >> 52) & 0x7ff) - 1023;
    double f = synth_from_bits((u & 0x000fffffffffffffull) | 0x3ff0000000000000ull); /* [1,2) */
    if (f > 1.4142135623730951) {
        f = f * 0.5;
        e = e + 1;
    }
    const double z = (f - 1.0) / (f + 1.0);
    const double z2 = z * z;
    double s = 1.0 / 25.0;
    for (int k = 23; k >= 1; k -= 2) s = s * z2 + 1.0 / (double)k;
    return (double)e * 0.6931471805599453 + 2.0 * z * s;
}

/* e^x for |x| < 700: x = k ln2 + r, Taylor series of e^r to r^22, times 2^k. */
SYNTH_FN double synth_exp(double x)
{
    const double ln2_hi = 0.6931471803691238; /* high 32 bits of ln 2 */
    const double ln2_lo = 1.9082149292705877e-10;
    const double kd = x * 1.4426950408889634 + 0.5;
    int64_t k = (int64_t)kd; /* truncation toward zero, corrected to floor */
    if ((double)k > kd) k = k - 1;
    const double r = (x - (double)k * ln2_hi) - (double)k * ln2_lo;
    double s = 1.0;
    for (int j = 22; j >= 1; --j) s = 1.0 + s * r / (double)j;
    return s * synth_from_bits((uint64_t)(k + 1023) << 52);
}

/* Standard normal pair, Marsaglia's polar method. */
SYNTH_FN void synth_normal2(uint64_t seed, uint32_t stream, uint64_t idx, uint32_t sub,
                            double* z0, double* z1)
{
    for (uint32_t k = 0; k < 64; ++k) {
        uint32_t w[4];
        synth_draw(seed, stream, idx, sub, k, w);
        const double u = 2.0 * synth_u01(w[0], w[1]) - 1.0;
        const double v = 2.0 * synth_u01(w[2], w[3]) - 1.0;
        const double s = u * u + v * v;
        if (s < 1.0 && s > 0.0) {
            const double f = sqrt(-2.0 * synth_ln(s) / s);
            *z0 = u * f;
            *z1 = v * f;
            return;
        }
    }
    *z0 = 0.0; /* unreachable in practice: 64 rejections in a row, p < 1e-42 */
    *z1 = 0.0;
}

typedef struct synth_params {
    int32_t n_astro, n_axes, n_par_axis, n_instr, n_glob, value_kind;
    int64_t n_dfa, n_instr_cols;
    double scale_lo, scale_hi; /* astrometric column scale 10^U(lo,hi) when lo < hi */
    double corr;               /* correlation rho in [0, 1) of astrometric coefficients 1.. with 0 */
} synth_params;

#define SYNTH_MAX_PAR 32
#define SYNTH_MAX_INSTR 8

/* Row i of the system (star s): coefficient values z[n_par] in section
 * order, attitude start *t, sorted distinct instrumental columns ins[n_instr]. */
SYNTH_FN void synth_row(uint64_t seed, int64_t i, int64_t s, const synth_params* P, double* z,
                        int64_t* t, int32_t* ins)
{
    uint32_t w[4];
    synth_draw(seed, 0u, (uint64_t)i, 0u, 0u, w);
    *t = (int64_t)synth_below(w[0], w[1], (uint64_t)(P->n_dfa - P->n_par_axis + 1));

    /* Floyd's sampling of n_instr distinct columns, then insertion sort */
    int32_t k = 0;
    for (int64_t j = P->n_instr_cols - P->n_instr; j < P->n_instr_cols; ++j) {
        const uint32_t d = (uint32_t)(j - (P->n_instr_cols - P->n_instr));
        synth_draw(seed, 0u, (uint64_t)i, 1u + d / 2u, 0u, w);
        const uint32_t a = (d & 1u) ? w[2] : w[0];
        const uint32_t b = (d & 1u) ? w[3] : w[1];
        const int32_t c = (int32_t)synth_below(a, b, (uint64_t)(j + 1));
        int seen = 0;
        for (int32_t q = 0; q < k; ++q)
            if (ins[q] == c) seen = 1;
        ins[k++] = seen ? (int32_t)j : c;
    }
    for (int32_t q = 1; q < k; ++q) {
        const int32_t v = ins[q];
        int32_t r = q - 1;
        while (r >= 0 && ins[r] > v) {
            ins[r + 1] = ins[r];
            --r;
        }
        ins[r + 1] = v;
    }

    const int32_t n_par = P->n_astro + P->n_axes * P->n_par_axis + P->n_instr + P->n_glob;
    for (int32_t g = 0; 2 * g < n_par; ++g) {
        double a, b;
        synth_normal2(seed, 1u, (uint64_t)i, (uint32_t)g, &a, &b);
        z[2 * g] = a;
        if (2 * g + 1 < n_par) z[2 * g + 1] = b;
    }
    if (P->corr > 0.0) {
        /* z_j <- rho z_0 + sqrt(1 - rho^2) z_j for the astrometric j >= 1: unit
           variance, correlation rho with z_0 (rho^2 between the others), so the
           per-star blocks become ill-conditioned whatever the column scaling */
        const double c = sqrt((1.0 - P->corr) * (1.0 + P->corr));
        for (int32_t j = 1; j < P->n_astro; ++j) z[j] = P->corr * z[0] + c * z[j];
    }
    if (P->scale_lo < P->scale_hi) {
        for (int32_t j = 0; j < P->n_astro; ++j) {
            synth_draw(seed, 4u, (uint64_t)(P->n_astro * s + j), 0u, 0u, w);
            const double e = P->scale_lo + (P->scale_hi - P->scale_lo) * synth_u01(w[0], w[1]);
            z[j] = z[j] * synth_exp(e * 2.302585092994046);
        }
    }
}

/* Observations of star s: fixed (lo == hi) or uniform in [lo, hi]. */
SYNTH_FN int64_t synth_star_count(uint64_t seed, int64_t s, int32_t lo, int32_t hi)
{
    if (lo == hi) return lo;
    uint32_t w[4];
    synth_draw(seed, 5u, (uint64_t)s, 0u, 0u, w);
    return lo + (int64_t)synth_below(w[0], w[1], (uint64_t)(hi - lo + 1));
}

/* sigma * N(0,1) for index i of `stream` (x_true: stream 2; noise: 3 + rhs). */
SYNTH_FN double synth_normal_at(uint64_t seed, uint32_t stream, int64_t i, double sigma)
{
    double a, b;
    synth_normal2(seed, stream, (uint64_t)i, 0u, &a, &b);
    return sigma * a;
}

#endif /* AVUGSR_SYNTH_GEN_CORE_H */
