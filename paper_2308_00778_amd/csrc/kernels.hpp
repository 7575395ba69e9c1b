// Device code of the AVU-GSR LSQR library for gfx950 (CDNA4, wave64).
//
// The matrix is the paper's dense per-row coefficient array A_d (Sect. 2)
// held as structure-of-arrays: coefficient c of row i at values[c*m + i], so
// that a wave streams 64 consecutive rows of one coefficient as one coalesced
// 512-byte (FP64) or 256-byte (FP32) request. Index arrays follow the same
// layout. All streaming loads carry the nontemporal hint so that the matrix
// does not evict the gathered vector sections from L2.
//
// Kernels:
//   k_aprod1      y = A x (+ mode-specific update), one row per lane, grid
//                 stride, two rows in flight per lane; FP64 sum of squares of
//                 the written y per block (the beta norm of the LSQR step).
//   k_aprod2      x += A^T y over star-aligned per-wave row ranges:
//                   astrometric: segmented reduction over the star key (rows
//                     are sorted by star), plain stores, no atomics;
//                   attitude: left to the bucket-order pass (k_att_hist +
//                     k_att_reduce: rows sorted by the bucket of their
//                     attitude start, per-workgroup FP64 LDS histograms, no
//                     device atomics) by default; scatter-add with device
//                     atomics in the ATT instances (attitude mode 0);
//                   instrumental: workgroup-private LDS histogram, flushed
//                     once per workgroup (k_instr_tail beyond its columns);
//                   global: wave shuffle -> LDS -> per-workgroup partial,
//                     summed in a deterministic second stage (k_glob_sum).
//   k_fused       one sweep doing aprod1 and the non-attitude part of aprod2
//                 of an LSQR step (the attitude dot product optionally first,
//                 by k_att_dot in bucket order).
//   k_col_a/b     column-vector updates of the LSQR step (FP64).
//   k_scalar_*    single-workgroup kernels: norm finishers, Givens rotation,
//                 estimates and stopping tests, all FP64.
//   namespace batched: the same steps for a k-tile of right-hand sides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace avugsr {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

// Row layout of the paper (Sect. 2): 5 astrometric, 3 axes x 4 attitude,
// 6 instrumental, 1 global coefficient.
constexpr int kAstro = 5;
constexpr int kAxes = 3;
constexpr int kParAxis = 4;
constexpr int kInstr = 6;
constexpr int kPar = 24;
constexpr int kOffAtt = kAstro;
constexpr int kOffInstr = kAstro + kAxes * kParAxis;
constexpr int kOffGlob = kOffInstr + kInstr;
static_assert(kOffGlob + 1 == kPar, "row layout");

constexpr int64_t kNoStar = INT64_MAX;

struct SysView {
    const void* val;       // [kPar][m]
    const int64_t* star;   // [m]
    const int64_t* att;    // [m]
    const int32_t* instr;  // [kInstr][m]
    int64_t m;
    int64_t n;
    int64_t n_stars;
    int64_t n_dfa;
    int64_t n_instr_cols;
    int64_t att_base;
    int64_t instr_base;
    int64_t glob_base;
    // section sizes and value-row offsets (general layouts; the full layout
    // is 5, 12, 6, 1 at offsets 5, 17, 23)
    int32_t na, natt, ni, ng;
    int32_t off_att, off_instr, off_glob;
    // compact copies of the star and instrumental indices read by the fused
    // passes (CIDX), or null
    const int32_t* star32;    // [m]
    const uint16_t* instr16;  // [kInstr][m]
};

// Star and instrumental index of row ic, from the compact copies when CIDX.
template <bool CIDX>
__device__ __forceinline__ int64_t star_of(const SysView& s, int64_t ic)
{
    return CIDX ? (int64_t)__builtin_nontemporal_load(&s.star32[ic])
                : __builtin_nontemporal_load(&s.star[ic]);
}
template <bool CIDX>
__device__ __forceinline__ int32_t instr_of(const SysView& s, int j, int64_t ic)
{
    return CIDX ? (int32_t)__builtin_nontemporal_load(&s.instr16[j * s.m + ic])
                : __builtin_nontemporal_load(&s.instr[j * s.m + ic]);
}

// LSQR state kept on the device so that a whole iteration runs without a
// host round trip (and can be captured into a graph).
struct Scalars {
    double alpha, beta, rhobar, phibar, bnorm;
    double anorm, ddnorm, xnorm, rnorm, arnorm, acond;
    double rho, c, s, theta, phi;
    double t1, t2, inv_alpha, coef_u;
    double atol, btol, ctol;
    double dmax, xmax;  // refinement: ||d||_inf, ||x||_inf of the last outer step
    double arnorm0;     // alpha_1 beta_1 = ||Abar^T b||, the initial normal-equation residual
    double rel_ar;      // > 0: also stop (istop 2) once arnorm <= rel_ar * arnorm0
    int32_t itn, itn_limit, istop, done;
    int32_t tests, beta_zero, pad0, pad1;
};

template <typename T>
__device__ __forceinline__ T ldnt(const T* p)
{
    return __builtin_nontemporal_load(p);
}

// A load of a streamed column: nontemporal, or PLAIN where the columns do not
// start on a 128-byte line, so that the line a wave's step shares with its
// next step stays in L2 until that step reads it (nontemporal lines go
// first: at 1e9 rows, m = 8 mod 16, about 2-3 ms less per instrumental tail
// window of 10.7-11.4 ms; with aligned columns plain loads gain nothing).
template <bool PLAIN, typename T>
__device__ __forceinline__ T ld_stream(const T* p)
{
    if constexpr (PLAIN)
        return *p;
    else
        return ldnt(p);
}

// ---------------------------------------------------------------- reductions
// Deterministic block sum of one double per thread; result valid on thread 0.
__device__ __forceinline__ double block_sum(double v, double* lds /* >= kWavesPerBlock */)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kWavesPerBlock; ++k) r += lds[k];
    return r;
}

__device__ __forceinline__ double block_max(double v, double* lds)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off));
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kWavesPerBlock; ++k) r = fmax(r, lds[k]);
    return r;
}

template <int NT>
__device__ __forceinline__ double block_sum_n(double v, double* lds /* >= NT / kWave */)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / kWave; ++k) r += lds[k];
    return r;
}

// Sum of n partials by one block, fixed order (deterministic). Thread 0.
__device__ __forceinline__ double sum_partials(const double* part, int n, double* lds)
{
    double v = 0.0;
    for (int k = threadIdx.x; k < n; k += kBlock) v += part[k];
    return block_sum(v, lds);
}

__device__ __forceinline__ double max_partials(const double* part, int n, double* lds)
{
    double v = 0.0;
    for (int k = threadIdx.x; k < n; k += kBlock) v = fmax(v, part[k]);
    return block_max(v, lds);
}

// ------------------------------------------------------------------- aprod 1
// Eq. (2) for one row: sum over the 24 coefficients in section order.
// xi: the instrumental slice of x (x + instr_base, or its copy in LDS).
// x3 (ATTI): the attitude section interleaved by axis,
// x3[3 c + axis] = x[att_base + axis * n_dfa + c], so that the 12 attitude
// values of a row (columns t..t+3 of the three axes) are 12 consecutive
// elements: about 1.7 cache lines per row instead of 3.6 for three separate
// 4-value windows, with the same footprint.
template <typename T, typename Acc, typename VX, bool ATTI = false>
__device__ __forceinline__ Acc row_dot(const SysView& s, const VX* __restrict__ x,
                                       const VX* __restrict__ xi, int64_t i,
                                       const VX* __restrict__ x3 = nullptr)
{
    const T* __restrict__ val = static_cast<const T*>(s.val);
    const int64_t m = s.m;
    const int64_t st = ldnt(&s.star[i]);
    const int64_t t = ldnt(&s.att[i]);
    T a[kPar];
#pragma unroll
    for (int c = 0; c < kPar; ++c) a[c] = ldnt(&val[c * m + i]);
    int32_t ic[kInstr];
#pragma unroll
    for (int j = 0; j < kInstr; ++j) ic[j] = ldnt(&s.instr[j * m + i]);

    Acc sum = 0;
    const VX* xa = x + kAstro * st;
#pragma unroll
    for (int j = 0; j < kAstro; ++j) sum += (Acc)a[j] * (Acc)xa[j];
#pragma unroll
    for (int ax = 0; ax < kAxes; ++ax) {
        VX xv[kParAxis];
        if (ATTI) {
            const VX* xt = x3 + kAxes * t + ax;
#pragma unroll
            for (int q = 0; q < kParAxis; ++q) xv[q] = xt[kAxes * q];
        } else {
            const VX* xt = x + s.att_base + ax * s.n_dfa + t;
#pragma unroll
            for (int q = 0; q < kParAxis; ++q) xv[q] = xt[q];
        }
#pragma unroll
        for (int q = 0; q < kParAxis; ++q) sum += (Acc)a[kOffAtt + ax * kParAxis + q] * (Acc)xv[q];
    }
#pragma unroll
    for (int j = 0; j < kInstr; ++j) sum += (Acc)a[kOffInstr + j] * (Acc)xi[ic[j]];
    sum += (Acc)a[kOffGlob] * (Acc)x[s.glob_base];
    return sum;
}

enum Aprod1Mode : int {
    A1_ACCUM = 0,  // y += A x
    A1_LSQR = 1,   // y = A x - coef_u * y, coef_u = alpha/beta from the scalars
    A1_RESID = 2,  // y = b - A x
};

// part[blockIdx.x] receives the FP64 sum of squares of the stored y (LSQR,
// RESID modes). NT threads per block. LDSX: the instrumental slice of x
// (n_instr_cols values) is first copied into LDS, so that the six random
// instrumental gathers per row hit LDS instead of L2.
// inv (optional, LSQR and RESID modes): placement of the row vector, the value
// of row i lives at y[inv[i]] (the attitude-bucket order of the solver's work
// vector); nullptr: y[i].
template <typename T, typename Acc, typename VX, typename VY, int MODE, int NT = kBlock,
          bool LDSX = false, bool ATTI = false>
__global__ __launch_bounds__(NT) void k_aprod1(SysView s, const VX* __restrict__ x,
                                                VY* __restrict__ y, const double* __restrict__ b,
                                                const Scalars* __restrict__ sc,
                                                double* __restrict__ part,
                                                const int32_t* __restrict__ inv = nullptr,
                                                const VX* __restrict__ x3 = nullptr)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[NT / kWave];
    if (MODE == A1_LSQR && sc->done) return;
    const VX* xi = x + s.instr_base;
    if (LDSX) {
        VX* xl = reinterpret_cast<VX*>(smem_raw);
        for (int64_t j = threadIdx.x; j < s.n_instr_cols; j += NT) xl[j] = xi[j];
        __syncthreads();
        xi = xl;
    }
    const Acc coef = (MODE == A1_LSQR) ? (Acc)sc->coef_u : (Acc)0;
    const int64_t stride = (int64_t)gridDim.x * NT;
    double ssq = 0.0;
    for (int64_t i0 = (int64_t)blockIdx.x * NT + threadIdx.x; i0 < s.m; i0 += 2 * stride) {
        const int64_t i1 = i0 + stride;
        const bool has1 = i1 < s.m;
        const int64_t i1c = has1 ? i1 : i0;
        const Acc d0 = row_dot<T, Acc, VX, ATTI>(s, x, xi, i0, x3);
        const Acc d1 = row_dot<T, Acc, VX, ATTI>(s, x, xi, i1c, x3);
        if (MODE == A1_ACCUM) {
            y[i0] = (VY)((Acc)y[i0] + d0);
            if (has1) y[i1] = (VY)((Acc)y[i1] + d1);
        } else {
            const int64_t p0 = inv ? (int64_t)ldnt(&inv[i0]) : i0;
            const VY n0 = MODE == A1_LSQR ? (VY)(d0 - coef * (Acc)y[p0]) : (VY)((Acc)b[i0] - d0);
            y[p0] = n0;
            ssq += (double)n0 * (double)n0;
            if (has1) {
                const int64_t p1 = inv ? (int64_t)ldnt(&inv[i1]) : i1;
                const VY n1 =
                    MODE == A1_LSQR ? (VY)(d1 - coef * (Acc)y[p1]) : (VY)((Acc)b[i1] - d1);
                y[p1] = n1;
                ssq += (double)n1 * (double)n1;
            }
        }
    }
    if (MODE != A1_ACCUM) {
        const double r = block_sum_n<NT>(ssq, red);
        if (threadIdx.x == 0) part[blockIdx.x] = r;
    }
}

// x3[3 c + axis] = x[att_base + axis * n_dfa + c]
template <typename V>
__global__ __launch_bounds__(kBlock) void k_interleave_att(const V* __restrict__ x,
                                                            int64_t att_base, int64_t n_dfa,
                                                            V* __restrict__ x3,
                                                            const Scalars* __restrict__ sc)
{
    if (sc != nullptr && sc->done) return;
    const int64_t total = (int64_t)kAxes * n_dfa;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * kBlock) {
        const int64_t c = j / kAxes, ax = j - c * kAxes;
        x3[j] = x[att_base + ax * n_dfa + c];
    }
}

// ------------------------------------------------------------------- aprod 2
// Inclusive segmented scan over the wave of five values keyed by a
// non-decreasing key: equal keys at distance `off` imply the whole span in
// between carries the same key.
template <typename Acc>
__device__ __forceinline__ void seg_scan5(int64_t key, Acc (&v)[kAstro], int lane)
{
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int64_t ko = __shfl_up(key, off);
        Acc vo[kAstro];
#pragma unroll
        for (int j = 0; j < kAstro; ++j) vo[j] = __shfl_up(v[j], off);
        if (lane >= off && ko == key) {
#pragma unroll
            for (int j = 0; j < kAstro; ++j) v[j] += vo[j];
        }
    }
}

// Wave-wide sum, result in every lane.
template <typename Acc>
__device__ __forceinline__ Acc wave_sum(Acc v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Reduction of NV values per row over segments of equal, non-decreasing keys,
// one 64-row chunk at a time. Each lane keeps running partials of the segment
// that is still open at the end of the previous chunk; cross-lane work
// happens only where a segment ends (a wave sum per finished segment), so a
// segment longer than a chunk costs one vector add per lane per chunk.
// Invalid lanes (past the end of the range) carry key kNoStar.
template <typename Acc, int NV>
struct SegAcc {
    int64_t key = -1;  // open segment (wave-uniform), -1: none
    Acc acc[NV];
    __device__ SegAcc()
    {
#pragma unroll
        for (int j = 0; j < NV; ++j) acc[j] = (Acc)0;
    }
};

// emit(key, totals) runs on lane 0 once per finished segment.
template <typename Acc, int NV, typename Emit>
__device__ __forceinline__ void seg_chunk(SegAcc<Acc, NV>& S, int64_t key, const Acc (&v)[NV],
                                          int lane, Emit&& emit)
{
    const bool cont = key == S.key;
#pragma unroll
    for (int j = 0; j < NV; ++j) S.acc[j] += cont ? v[j] : (Acc)0;
    uint64_t rest = __ballot(!cont);
    if (rest == 0) return;  // the whole chunk continues the open segment
    if (S.key >= 0) {       // keys are sorted: the open segment ends here
        Acc t[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) t[j] = wave_sum(S.acc[j]);
        if (lane == 0) emit(S.key, t);
    }
    S.key = -1;
#pragma unroll
    for (int j = 0; j < NV; ++j) S.acc[j] = (Acc)0;
    while (rest != 0) {
        const int l0 = __ffsll((unsigned long long)rest) - 1;
        const int64_t k2 = __shfl(key, l0);
        if (k2 == kNoStar) break;  // only lanes past the end remain
        const bool mine = key == k2;
        const uint64_t same = __ballot(mine);
        if ((same >> (kWave - 1)) & 1ull) {  // reaches the last lane: stays open
            S.key = k2;
#pragma unroll
            for (int j = 0; j < NV; ++j) S.acc[j] = mine ? v[j] : (Acc)0;
            break;
        }
        Acc t[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) t[j] = wave_sum(mine ? v[j] : (Acc)0);
        if (lane == 0) emit(k2, t);
        rest &= ~same;
    }
}

template <typename Acc, int NV, typename Emit>
__device__ __forceinline__ void seg_finish(SegAcc<Acc, NV>& S, int lane, Emit&& emit)
{
    if (S.key < 0) return;
    Acc t[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) t[j] = wave_sum(S.acc[j]);
    if (lane == 0) emit(S.key, t);
    S.key = -1;
}

// Stateless variant: every segment present in the chunk is reduced and
// emitted at once (a segment spanning several chunks is emitted once per
// chunk, so emit must accumulate). Keeps no registers across chunks.
template <typename Acc, int NV, typename Emit>
__device__ __forceinline__ void seg_flush(int64_t key, const Acc (&v)[NV], int lane, Emit&& emit)
{
    uint64_t rest = __ballot(key != kNoStar);
    while (rest != 0) {
        const int l0 = __ffsll((unsigned long long)rest) - 1;
        const int64_t k2 = __shfl(key, l0);
        const bool mine = key == k2;
        const uint64_t same = __ballot(mine);
        Acc t[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) t[j] = wave_sum(mine ? v[j] : (Acc)0);
        if (lane == 0) emit(k2, t);
        rest &= ~same;
    }
}

// x += A^T y (SQUARE: x_j += sum of squared coefficients of column j, used
// for the column norms). wb: star-aligned row boundaries, one range per wave
// (gridDim.x * kWavesPerBlock ranges). Instrumental columns [0, hcols) are
// accumulated in an FP64 LDS histogram (hcols * 8 bytes of dynamic shared
// memory) flushed with one device atomic per column per workgroup; columns
// from hcols on are left to k_instr_tail. gpart[blockIdx.x] gets the
// workgroup's global-column partial; k_glob_sum adds them up.
// ATT = false leaves the attitude columns to the bucket-order pass
// (k_att_hist) and skips loading them. SCAN selects the astrometric
// reduction: a segmented scan every chunk (true) or the accumulate-and-flush
// segments of seg_chunk (false).
// inv (optional): the value of row i is u[inv[i]].
template <typename T, typename Acc, typename VU, bool SQUARE, bool ATT = true, bool SCAN = true,
          int NT = kBlock>
__global__ __launch_bounds__(NT) void k_aprod2(SysView s, const VU* __restrict__ u,
                                                    Acc* __restrict__ q,
                                                    const int64_t* __restrict__ wb,
                                                    Acc* __restrict__ gpart, int64_t hcols,
                                                    const Scalars* __restrict__ sc,
                                                    const int32_t* __restrict__ inv = nullptr)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* lds = reinterpret_cast<double*>(smem_raw);  // FP64 histogram (see k_att_hist)
    __shared__ Acc gred[NT / kWave];
    if (sc != nullptr && (sc->done || sc->beta_zero)) return;

    const T* __restrict__ val = static_cast<const T*>(s.val);
    const int64_t m = s.m;
    for (int64_t j = threadIdx.x; j < hcols; j += NT) lds[j] = 0.0;
    __syncthreads();

    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = (int64_t)blockIdx.x * (NT / kWave) + threadIdx.x / kWave;
    const int64_t rb = wb[wave], re = wb[wave + 1];
    Acc* __restrict__ qatt = q + s.att_base;
    Acc* __restrict__ qins = q + s.instr_base;

    int64_t carry_star = -1;
    Acc carry[kAstro];
#pragma unroll
    for (int j = 0; j < kAstro; ++j) carry[j] = (Acc)0;
    Acc gsum = (Acc)0;
    SegAcc<Acc, kAstro> seg;
    auto astro_emit = [q](int64_t star, const Acc (&tot)[kAstro]) {
#pragma unroll
        for (int j = 0; j < kAstro; ++j) q[kAstro * star + j] += tot[j];
    };

    // Chunks start on 64-row boundaries so that every coefficient stream is
    // read in whole cache lines; lanes before rb (owned by the previous wave)
    // take the first row's star with zero contributions.
    for (int64_t r0 = rb < re ? (rb & ~(int64_t)(kWave - 1)) : re; r0 < re; r0 += kWave) {
        const int64_t i = r0 + lane;
        const bool ok = i >= rb && i < re;
        const int64_t ic = i < rb ? rb : (i < re ? i : re - 1);
        const int64_t st = i < re ? ldnt(&s.star[ic]) : kNoStar;
        const int64_t t = ATT ? ldnt(&s.att[ic]) : 0;
        T a[kPar];
#pragma unroll
        for (int c = 0; c < kPar; ++c)
            a[c] = (ATT || c < kOffAtt || c >= kOffInstr) ? ldnt(&val[c * m + ic]) : (T)0;
        int32_t ix[kInstr];
#pragma unroll
        for (int j = 0; j < kInstr; ++j) ix[j] = ldnt(&s.instr[j * m + ic]);
        Acc ui = (Acc)0;
        if (!SQUARE) ui = ok ? (Acc)u[inv ? (int64_t)ldnt(&inv[ic]) : ic] : (Acc)0;

        Acc contrib[kPar];
#pragma unroll
        for (int c = 0; c < kPar; ++c)
            contrib[c] = SQUARE ? (ok ? (Acc)a[c] * (Acc)a[c] : (Acc)0) : (Acc)a[c] * ui;

        // attitude: 3 axes x 4 consecutive columns from the row's start t
        if (ok) {
            if (ATT) {
#pragma unroll
                for (int ax = 0; ax < kAxes; ++ax) {
                    Acc* dst = qatt + ax * s.n_dfa + t;
#pragma unroll
                    for (int qq = 0; qq < kParAxis; ++qq)
                        atomicAdd(dst + qq, contrib[kOffAtt + ax * kParAxis + qq]);
                }
            }
            // instrumental
#pragma unroll
            for (int j = 0; j < kInstr; ++j)
                if (ix[j] < hcols) atomicAdd(&lds[ix[j]], (double)contrib[kOffInstr + j]);
        }
        gsum += contrib[kOffGlob];

        // astrometric: per-star segmented reduction across chunks
        Acc pa[kAstro];
#pragma unroll
        for (int j = 0; j < kAstro; ++j) pa[j] = contrib[j];
        if (!SCAN) {
            seg_chunk(seg, st, pa, lane, astro_emit);
            continue;
        }
        if (carry_star >= 0) {
            const int64_t st0 = __shfl(st, 0);
            if (lane == 0) {
                if (st0 == carry_star) {
#pragma unroll
                    for (int j = 0; j < kAstro; ++j) pa[j] += carry[j];
                } else {
#pragma unroll
                    for (int j = 0; j < kAstro; ++j) q[kAstro * carry_star + j] += carry[j];
                }
            }
        }
        seg_scan5<Acc>(st, pa, lane);
        const int64_t snext = __shfl_down(st, 1);
        if (ok && lane != kWave - 1 && snext != st) {
#pragma unroll
            for (int j = 0; j < kAstro; ++j) q[kAstro * st + j] += pa[j];
        }
        carry_star = __shfl(st, kWave - 1);
#pragma unroll
        for (int j = 0; j < kAstro; ++j) carry[j] = __shfl(pa[j], kWave - 1);
        if (carry_star == kNoStar) carry_star = -1;
    }
    if (carry_star >= 0 && lane == 0) {
#pragma unroll
        for (int j = 0; j < kAstro; ++j) q[kAstro * carry_star + j] += carry[j];
    }
    if (!SCAN) seg_finish(seg, lane, astro_emit);

    // global column: wave shuffle -> LDS -> one partial per workgroup
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) gsum += __shfl_down(gsum, off);
    if (lane == 0) gred[threadIdx.x / kWave] = gsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        Acc g = (Acc)0;
        for (int k = 0; k < NT / kWave; ++k) g += gred[k];
        gpart[blockIdx.x] = g;
    }
    // instrumental flush: one device atomic per column per workgroup
    for (int64_t j = threadIdx.x; j < hcols; j += NT) {
        const double v = lds[j];
        if (v != 0.0) atomicAdd(&qins[j], (Acc)v);
    }
}

// ------------------------------------------------------ fused iteration pass
// One sweep over the rows in star order doing both operator products of an
// LSQR step (Eq. 2 and Eq. 3). Because u~_{i+1} = Abar v_i - (alpha_i/beta_i) u~_i
// is row-local, each row's new value is known as soon as the row's 24
// coefficients are in registers, and the same registers then feed
// A^T u~_{i+1} for the astrometric (per-star segments), instrumental (LDS
// histogram) and global (per-workgroup partial) columns. beta_{i+1} = ||u~||
// is applied afterwards by the column kernel (v~ = p .* A^T u~ / beta - beta v),
// so A is read once per iteration for these sections; the attitude columns
// are left to the row-reordered pass, which reads u~_{i+1}.
//   x: vp = p .* v (Acc), x3: its interleaved attitude section (kAttX3),
//   u: u~ [m], overwritten (row i at u[inv[i]], or u[i] without inv),
//   part[blockIdx.x]: FP64 sum of squares of the
//   stored u~, q: A^T u~ accumulator (astro, instr, glob sections),
//   gpart[blockIdx.x]: global-column partial, wb: star-aligned wave ranges.
// Dynamic LDS: the FP64 histogram of instrumental columns [0, hcols) (see
// k_att_hist; columns from hcols on are left to k_instr_tail) and, after it,
// the instrumental slice of x (LDSX, n_instr_cols Acc).
// AM, the attitude part of the dot product: kAttX reads three 4-value windows
// of x, kAttX3 one 12-value window of x3, kAttPre none: k_att_dot has already
// replaced u~ by (attitude part of A vp) - coef u~, so the row adds that;
// kAttGather: k_att_dot has written the attitude part of every row to datt in
// bucket order, the row reads it at datt[inv[i]] and keeps u~ in star order
// (u[i]), so that u~ is read and written sequentially and the only permuted
// access is that read.
// us (optional): a star-order copy of the new u~ (us[i]), written
// sequentially for the instrumental tail passes that follow, which then read
// it without the permutation.
enum { kAttX = 0, kAttX3 = 1, kAttPre = 2, kAttGather = 3 };
template <typename T, typename Acc, int NT, bool LDSX, int AM, bool CIDX>
__global__ __launch_bounds__(NT) void k_fused(SysView s, const Acc* __restrict__ x,
                                               const Acc* __restrict__ x3, Acc* __restrict__ u,
                                               Acc* __restrict__ q, const int64_t* __restrict__ wb,
                                               Acc* __restrict__ gpart, double* __restrict__ part,
                                               int64_t hcols, const Scalars* __restrict__ sc,
                                               const int32_t* __restrict__ inv,
                                               const Acc* __restrict__ datt = nullptr,
                                               Acc* __restrict__ us = nullptr)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ Acc gred[NT / kWave];
    __shared__ double sred[NT / kWave];
    if (sc->done) return;

    const T* __restrict__ val = static_cast<const T*>(s.val);
    const int64_t m = s.m;
    const int64_t ninst = s.n_instr_cols;
    double* hist = reinterpret_cast<double*>(smem_raw);
    const Acc* xi = x + s.instr_base;
    for (int64_t j = threadIdx.x; j < hcols; j += NT) hist[j] = 0.0;
    if (LDSX) {
        const int64_t off = (hcols * 8 + 15) & ~(int64_t)15;
        Acc* xl = reinterpret_cast<Acc*>(smem_raw + off);
        for (int64_t j = threadIdx.x; j < ninst; j += NT) xl[j] = xi[j];
        xi = xl;
    }
    __syncthreads();

    const Acc coef = (Acc)sc->coef_u;
    const Acc xg = x[s.glob_base];
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = (int64_t)blockIdx.x * (NT / kWave) + threadIdx.x / kWave;
    const int64_t rb = wb[wave], re = wb[wave + 1];
    Acc* __restrict__ qins = q + s.instr_base;

    double ssq = 0.0;
    Acc gsum = (Acc)0;
    SegAcc<Acc, kAstro> seg;
    auto astro_emit = [q](int64_t star, const Acc (&tot)[kAstro]) {
#pragma unroll
        for (int j = 0; j < kAstro; ++j) q[kAstro * star + j] += tot[j];
    };

    // 64-row aligned chunks, as in k_aprod2; lanes outside [rb, re) compute on
    // a clamped row and contribute nothing.
    for (int64_t r0 = rb < re ? (rb & ~(int64_t)(kWave - 1)) : re; r0 < re; r0 += kWave) {
        const int64_t i = r0 + lane;
        const bool ok = i >= rb && i < re;
        const int64_t ic = i < rb ? rb : (i < re ? i : re - 1);
        const int64_t stc = star_of<CIDX>(s, ic);
        const int64_t st = i < re ? stc : kNoStar;
        constexpr bool kNoAtt = AM == kAttPre || AM == kAttGather;
        const int64_t t = kNoAtt ? 0 : ldnt(&s.att[ic]);
        T a[kPar];
#pragma unroll
        for (int c = 0; c < kPar; ++c)
            if (!kNoAtt || c < kOffAtt || c >= kOffInstr) a[c] = ldnt(&val[c * m + ic]);
        int32_t ix[kInstr];
#pragma unroll
        for (int j = 0; j < kInstr; ++j) ix[j] = instr_of<CIDX>(s, j, ic);
        const int64_t pu = (AM != kAttGather && inv) ? (int64_t)ldnt(&inv[ic]) : ic;
        const Acc dg = AM == kAttGather ? datt[ldnt(&inv[ic])] : (Acc)0;
        const Acc uo = u[pu];

        // Eq. (2): the row's dot product with vp, in section order
        Acc d = (Acc)0;
        const Acc* xa = x + kAstro * stc;
#pragma unroll
        for (int j = 0; j < kAstro; ++j) d += (Acc)a[j] * xa[j];
        if (!kNoAtt) {
#pragma unroll
            for (int ax = 0; ax < kAxes; ++ax) {
#pragma unroll
                for (int qq = 0; qq < kParAxis; ++qq) {
                    const Acc xv = AM == kAttX3 ? x3[kAxes * (t + qq) + ax]
                                                : x[s.att_base + ax * s.n_dfa + t + qq];
                    d += (Acc)a[kOffAtt + ax * kParAxis + qq] * xv;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kInstr; ++j) d += (Acc)a[kOffInstr + j] * xi[ix[j]];
        d += (Acc)a[kOffGlob] * xg;
        if (AM == kAttPre)
            d += uo;
        else if (AM == kAttGather)
            d += dg - coef * uo;
        else
            d -= coef * uo;
        if (ok) u[pu] = d;
        if (ok && us) us[ic] = d;
        if (!ok) d = (Acc)0;
        ssq += (double)d * (double)d;

        // Eq. (3) with the new value, attitude columns excluded
        if (ok) {
#pragma unroll
            for (int j = 0; j < kInstr; ++j) {
                if (ix[j] < hcols) atomicAdd(&hist[ix[j]], (double)((Acc)a[kOffInstr + j] * d));
            }
        }
        gsum += (Acc)a[kOffGlob] * d;
        Acc pa[kAstro];
#pragma unroll
        for (int j = 0; j < kAstro; ++j) pa[j] = (Acc)a[j] * d;
        seg_chunk(seg, st, pa, lane, astro_emit);
    }
    seg_finish(seg, lane, astro_emit);

    // per-workgroup partials: global column and ||u~||^2
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        gsum += __shfl_down(gsum, off);
        ssq += __shfl_down(ssq, off);
    }
    if (lane == 0) {
        gred[threadIdx.x / kWave] = gsum;
        sred[threadIdx.x / kWave] = ssq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Acc g = (Acc)0;
        double r = 0.0;
        for (int k = 0; k < NT / kWave; ++k) {
            g += gred[k];
            r += sred[k];
        }
        gpart[blockIdx.x] = g;
        part[blockIdx.x] = r;
    }
    for (int64_t j = threadIdx.x; j < hcols; j += NT) {
        const double v = hist[j];
        if (v != 0.0) atomicAdd(&qins[j], (Acc)v);
    }
}

// Instrumental columns [c0, c1) of Eq. (3) (or of the squared column norms,
// SQUARE) when the row passes keep only the first columns in LDS: workgroup b
// sweeps rows [b m / G, (b+1) m / G) with an FP64 LDS histogram of the
// window, then flushes it with one device atomic per column. U holds K
// values per row, row i at U[inv[i] K + r] (U[i K + r] without inv); frozen
// RHS (done or beta_zero) are skipped.
// GEN: section sizes from the system view (general layouts); otherwise the
// full layout's constants.
template <typename T, typename Acc, int K, bool SQUARE, int NT, bool GEN, bool PLAIN = false>
__global__ __launch_bounds__(NT) void k_instr_tail(SysView s, const Acc* __restrict__ U,
                                                    const int32_t* __restrict__ inv,
                                                    Acc* __restrict__ Q, int64_t c0, int64_t c1,
                                                    const Scalars* __restrict__ sc)
{
    const int ni = GEN ? s.ni : kInstr, oins = GEN ? s.off_instr : kOffInstr;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* hist = reinterpret_cast<double*>(smem_raw);
    uint32_t live = 0;
#pragma unroll
    for (int r = 0; r < K; ++r)
        live |= (sc != nullptr && (sc[r].done || sc[r].beta_zero)) ? 0u : (1u << r);
    if (live == 0) return;
    const T* __restrict__ val = static_cast<const T*>(s.val);
    const int64_t m = s.m, w = c1 - c0;
    for (int64_t e = threadIdx.x; e < w * K; e += NT) hist[e] = 0.0;
    __syncthreads();
    // the workgroup's rows [r0, r1) as one contiguous range per wave, walked
    // in 64-row steps aligned to 64 rows: a line that two steps share is read
    // by the same wave one step apart (an L2 hit), not by two waves at once
    // (which fetches it twice; also where the caller's columns are not
    // line-aligned)
    static_assert(NT % kWave == 0, "whole waves");
    const int64_t r0 = blockIdx.x * m / gridDim.x, r1 = (blockIdx.x + 1) * m / gridDim.x;
    constexpr int kW = NT / kWave;
    const int wv = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const int64_t rb = r0 + (r1 - r0) * wv / kW, re = r0 + (r1 - r0) * (wv + 1) / kW;
    for (int64_t i0 = rb & ~(int64_t)(kWave - 1); i0 < re; i0 += kWave) {
        const int64_t i = i0 + lane;
        if (i < rb || i >= re) continue;
        int32_t ix[kInstr];
        T a[kInstr];
#pragma unroll
        for (int j = 0; j < kInstr; ++j) {
            ix[j] = j < ni ? ld_stream<PLAIN>(&s.instr[j * m + i]) : -1;
            a[j] = j < ni ? ld_stream<PLAIN>(&val[(oins + j) * m + i]) : (T)0;
        }
        double u[K];
        if (!SQUARE) {
            const int64_t pu = inv ? (int64_t)ldnt(&inv[i]) : i;
#pragma unroll
            for (int r = 0; r < K; ++r) u[r] = ((live >> r) & 1u) ? (double)U[pu * K + r] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kInstr; ++j) {
            const int64_t c = (int64_t)ix[j] - c0;
            if (c < 0 || c >= w) continue;
#pragma unroll
            for (int r = 0; r < K; ++r) {
                if (!((live >> r) & 1u)) continue;
                const double av = (double)(Acc)a[j];
                atomicAdd(&hist[c * K + r], SQUARE ? av * av : (double)((Acc)a[j] * (Acc)u[r]));
            }
        }
    }
    __syncthreads();
    Acc* __restrict__ qins = Q + (s.instr_base + c0) * K;
    for (int64_t e = threadIdx.x; e < w * K; e += NT) {
        const double v = hist[e];
        if (v != 0.0) atomicAdd(&qins[e], (Acc)v);
    }
}

// --------------------------------------------------------- general layouts
// Rows whose sections differ from 5 + 3 x 4 + 6 + 1 (sections absent, fewer
// astrometric or instrumental coefficients, up to kGlobMax global columns):
// section sizes and value-row offsets come from the system view at run time,
// aprod1 and aprod2 run as separate passes, and the attitude columns go
// through the bucket-order pass (or device atomics) as in the full layout.
constexpr int kGlobMax = 5;

// Eq. (2) for a general layout; modes, y placement (inv) and part as k_aprod1.
template <typename T, typename Acc, typename VX, typename VY, int MODE>
__global__ __launch_bounds__(kBlock) void k_gen_aprod1(SysView s, const VX* __restrict__ x,
                                                        VY* __restrict__ y,
                                                        const double* __restrict__ b,
                                                        const Scalars* __restrict__ sc,
                                                        double* __restrict__ part,
                                                        const int32_t* __restrict__ inv)
{
    __shared__ double red[kWavesPerBlock];
    if (MODE == A1_LSQR && sc->done) return;
    const T* __restrict__ val = static_cast<const T*>(s.val);
    const int64_t m = s.m;
    const Acc coef = (MODE == A1_LSQR) ? (Acc)sc->coef_u : (Acc)0;
    double ssq = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * kBlock) {
        Acc d = (Acc)0;
        if (s.na > 0) {
            const VX* xa = x + (int64_t)s.na * ldnt(&s.star[i]);
            for (int j = 0; j < s.na; ++j) d += (Acc)ldnt(&val[j * m + i]) * (Acc)xa[j];
        }
        if (s.natt > 0) {
            const int64_t t = ldnt(&s.att[i]);
#pragma unroll
            for (int ax = 0; ax < kAxes; ++ax)
#pragma unroll
                for (int qq = 0; qq < kParAxis; ++qq)
                    d += (Acc)ldnt(&val[(s.off_att + ax * kParAxis + qq) * m + i]) *
                         (Acc)x[s.att_base + ax * s.n_dfa + t + qq];
        }
        for (int j = 0; j < s.ni; ++j)
            d += (Acc)ldnt(&val[(s.off_instr + j) * m + i]) *
                 (Acc)x[s.instr_base + ldnt(&s.instr[j * m + i])];
        for (int g = 0; g < s.ng; ++g)
            d += (Acc)ldnt(&val[(s.off_glob + g) * m + i]) * (Acc)x[s.glob_base + g];
        if (MODE == A1_ACCUM) {
            y[i] = (VY)((Acc)y[i] + d);
        } else {
            const int64_t p = inv ? (int64_t)ldnt(&inv[i]) : i;
            const VY nv = MODE == A1_LSQR ? (VY)(d - coef * (Acc)y[p]) : (VY)((Acc)b[i] - d);
            y[p] = nv;
            ssq += (double)nv * (double)nv;
        }
    }
    if (MODE != A1_ACCUM) {
        const double r = block_sum(ssq, red);
        if (threadIdx.x == 0) part[blockIdx.x] = r;
    }
}

// Eq. (3) (SQUARE: squared coefficients, the column norms) for a general
// layout over the star-aligned wave ranges: astrometric per-star segments,
// attitude by device atomics when ATT (else left to the bucket-order pass),
// instrumental columns [0, hcols) in an FP64 LDS histogram (the rest to
// k_instr_tail), global columns as per-workgroup partials
// gpart[blockIdx.x * kGlobMax + g].
template <typename T, typename Acc, typename VU, bool SQUARE, bool ATT>
__global__ __launch_bounds__(kBlock) void k_gen_aprod2(SysView s, const VU* __restrict__ u,
                                                        Acc* __restrict__ q,
                                                        const int64_t* __restrict__ wb,
                                                        Acc* __restrict__ gpart, int64_t hcols,
                                                        const Scalars* __restrict__ sc,
                                                        const int32_t* __restrict__ inv)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* lds = reinterpret_cast<double*>(smem_raw);
    __shared__ Acc gred[kGlobMax][kWavesPerBlock];
    if (sc != nullptr && (sc->done || sc->beta_zero)) return;
    const T* __restrict__ val = static_cast<const T*>(s.val);
    const int64_t m = s.m;
    const int na = s.na, ni = s.ni, ng = s.ng;
    for (int64_t j = threadIdx.x; j < hcols; j += kBlock) lds[j] = 0.0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t rb = wb[wave], re = wb[wave + 1];
    Acc gsum[kGlobMax];
#pragma unroll
    for (int g = 0; g < kGlobMax; ++g) gsum[g] = (Acc)0;
    SegAcc<Acc, kAstro> seg;
    auto astro_emit = [q, na](int64_t star, const Acc (&tot)[kAstro]) {
        for (int j = 0; j < na; ++j) q[(int64_t)na * star + j] += tot[j];
    };
    for (int64_t r0 = rb < re ? (rb & ~(int64_t)(kWave - 1)) : re; r0 < re; r0 += kWave) {
        const int64_t i = r0 + lane;
        const bool ok = i >= rb && i < re;
        const int64_t ic = i < rb ? rb : (i < re ? i : re - 1);
        Acc ui = (Acc)0;
        if (!SQUARE) ui = ok ? (Acc)u[inv ? (int64_t)ldnt(&inv[ic]) : ic] : (Acc)0;
        auto contrib = [&](T a) -> Acc {
            return SQUARE ? (ok ? (Acc)a * (Acc)a : (Acc)0) : (Acc)a * ui;
        };
        if (na > 0) {  // uniform: seg_chunk is collective
            const int64_t st = i < re ? ldnt(&s.star[ic]) : kNoStar;
            Acc pa[kAstro];
#pragma unroll
            for (int j = 0; j < kAstro; ++j)
                pa[j] = j < na ? contrib(ldnt(&val[j * m + ic])) : (Acc)0;
            seg_chunk(seg, st, pa, lane, astro_emit);
        }
        if (ATT && s.natt > 0 && ok) {
            const int64_t t = ldnt(&s.att[ic]);
#pragma unroll
            for (int ax = 0; ax < kAxes; ++ax)
#pragma unroll
                for (int qq = 0; qq < kParAxis; ++qq)
                    atomicAdd(&q[s.att_base + ax * s.n_dfa + t + qq],
                              contrib(ldnt(&val[(s.off_att + ax * kParAxis + qq) * m + ic])));
        }
        for (int j = 0; j < ni; ++j) {
            const int32_t ix = ldnt(&s.instr[j * m + ic]);
            const Acc c = contrib(ldnt(&val[(s.off_instr + j) * m + ic]));
            if (ok && ix < hcols) atomicAdd(&lds[ix], (double)c);
        }
        for (int g = 0; g < ng; ++g) {
            const Acc c = contrib(ldnt(&val[(s.off_glob + g) * m + ic]));
            gsum[g] += ok ? c : (Acc)0;
        }
    }
    if (na > 0) seg_finish(seg, lane, astro_emit);
#pragma unroll
    for (int g = 0; g < kGlobMax; ++g) {
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) gsum[g] += __shfl_down(gsum[g], off);
        if (lane == 0) gred[g][threadIdx.x / kWave] = gsum[g];
    }
    __syncthreads();
    if (threadIdx.x < kGlobMax) {
        Acc t = (Acc)0;
        for (int k = 0; k < kWavesPerBlock; ++k) t += gred[threadIdx.x][k];
        gpart[(int64_t)blockIdx.x * kGlobMax + threadIdx.x] = t;
    }
    Acc* __restrict__ qins = q + s.instr_base;
    for (int64_t j = threadIdx.x; j < hcols; j += kBlock) {
        const double v = lds[j];
        if (v != 0.0) atomicAdd(&qins[j], (Acc)v);
    }
}

// q[glob_base + g] += sum over workgroups of gpart[blk * kGlobMax + g], g < ng.
template <typename Acc>
__global__ __launch_bounds__(kBlock) void k_gen_glob_sum(const Acc* __restrict__ gpart, int nblk,
                                                          int ng, Acc* __restrict__ qglob,
                                                          const Scalars* __restrict__ sc)
{
    __shared__ double red[kWavesPerBlock];
    if (sc != nullptr && (sc->done || sc->beta_zero)) return;
    for (int g = 0; g < ng; ++g) {
        double v = 0.0;
        for (int k = threadIdx.x; k < nblk; k += kBlock) v += (double)gpart[(int64_t)k * kGlobMax + g];
        const double r = block_sum(v, red);
        if (threadIdx.x == 0) qglob[g] = (Acc)((double)qglob[g] + r);
    }
}

// --------------------------------------------------------- constraint rows
// Equations appended below the observation rows (Sect. 2): a few long sparse
// rows, in CSR form with FP64 values. One workgroup per row (grid-stride
// over rows); their vector entries sit after the observation rows, unpermuted.

// Eq. (2) on the constraint rows: dot_r = sum_e val[e] x[col[e]], then per
// MODE (as k_aprod1) y[r] += dot, y[r] = dot - coef_u y[r] or
// y[r] = b[r] - dot, and rowssq[r] = y[r]^2 (not in A1_ACCUM).
template <typename Acc, typename VX, typename VY, int MODE>
__global__ __launch_bounds__(kBlock) void k_con_aprod1(int64_t nc,
                                                        const int64_t* __restrict__ rowptr,
                                                        const int64_t* __restrict__ col,
                                                        const double* __restrict__ val,
                                                        const VX* __restrict__ x,
                                                        VY* __restrict__ y,
                                                        const double* __restrict__ b,
                                                        const Scalars* __restrict__ sc,
                                                        double* __restrict__ rowssq)
{
    __shared__ double red[kWavesPerBlock];
    if (MODE == A1_LSQR && sc->done) return;
    const Acc coef = (MODE == A1_LSQR) ? (Acc)sc->coef_u : (Acc)0;
    for (int64_t r = blockIdx.x; r < nc; r += gridDim.x) {
        const int64_t e1 = rowptr[r + 1];
        Acc d = (Acc)0;
        for (int64_t e = rowptr[r] + threadIdx.x; e < e1; e += kBlock)
            d += (Acc)val[e] * (Acc)x[col[e]];
        const double t = block_sum((double)d, red);
        if (threadIdx.x == 0) {
            const Acc dot = (Acc)t;
            if (MODE == A1_ACCUM) {
                y[r] = (VY)((Acc)y[r] + dot);
            } else {
                const VY nv = MODE == A1_LSQR ? (VY)(dot - coef * (Acc)y[r])
                                              : (VY)((Acc)b[r] - dot);
                y[r] = nv;
                rowssq[r] = (double)nv * (double)nv;
            }
        }
    }
}

// part[0] = sum of rowssq[0, nc) in a fixed order: the constraint rows' share
// of ||u||^2, stored after the observation rows' partials.
__global__ __launch_bounds__(kBlock) void k_con_ssq(int64_t nc, const double* __restrict__ rowssq,
                                                     double* __restrict__ part)
{
    __shared__ double red[kWavesPerBlock];
    double v = 0.0;
    for (int64_t k = threadIdx.x; k < nc; k += kBlock) v += rowssq[k];
    const double r = block_sum(v, red);
    if (threadIdx.x == 0) part[0] = r;
}

// Eq. (3) on the constraint rows: q[col[e]] += val[e] u[r] (SQUARE: val[e]^2,
// the column norms), device atomics (a column may appear in several rows).
template <typename Acc, typename VU, bool SQUARE>
__global__ __launch_bounds__(kBlock) void k_con_aprod2(int64_t nc,
                                                        const int64_t* __restrict__ rowptr,
                                                        const int64_t* __restrict__ col,
                                                        const double* __restrict__ val,
                                                        const VU* __restrict__ u,
                                                        Acc* __restrict__ q,
                                                        const Scalars* __restrict__ sc)
{
    if (sc != nullptr && (sc->done || sc->beta_zero)) return;
    for (int64_t r = blockIdx.x; r < nc; r += gridDim.x) {
        const Acc ur = SQUARE ? (Acc)0 : (Acc)u[r];
        const int64_t e1 = rowptr[r + 1];
        for (int64_t e = rowptr[r] + threadIdx.x; e < e1; e += kBlock) {
            const Acc a = (Acc)val[e];
            atomicAdd(&q[col[e]], SQUARE ? a * a : a * ur);
        }
    }
}

// Structure of the constraint rows: rowptr[0] = 0 and non-decreasing (bit 1),
// then, in a second launch once that holds, every column in [0, n) (bit 2).
__global__ __launch_bounds__(kBlock) void k_validate_con_rows(int64_t nc,
                                                               const int64_t* __restrict__ rowptr,
                                                               int32_t* __restrict__ flag)
{
    int32_t bad = 0;
    for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < nc;
         r += (int64_t)gridDim.x * kBlock) {
        if (r == 0 && rowptr[0] != 0) bad |= 1;
        if (rowptr[r + 1] < rowptr[r]) bad |= 1;
    }
    if (bad) atomicOr(flag, bad);
}

__global__ __launch_bounds__(kBlock) void k_validate_con_cols(int64_t nnz,
                                                               const int64_t* __restrict__ col,
                                                               int64_t n,
                                                               int32_t* __restrict__ flag)
{
    int32_t bad = 0;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * kBlock)
        if (col[e] < 0 || col[e] >= n) bad |= 2;
    if (bad) atomicOr(flag, bad);
}

// Second stage of the global-column reduction: q[glob] += sum of partials.
template <typename Acc>
__global__ __launch_bounds__(kBlock) void k_glob_sum(const Acc* __restrict__ gpart, int nblk,
                                                      Acc* __restrict__ qglob,
                                                      const Scalars* __restrict__ sc)
{
    __shared__ double red[kWavesPerBlock];
    if (sc != nullptr && (sc->done || sc->beta_zero)) return;
    double v = 0.0;
    for (int k = threadIdx.x; k < nblk; k += kBlock) v += (double)gpart[k];
    const double r = block_sum(v, red);
    if (threadIdx.x == 0) *qglob = (Acc)((double)*qglob + r);
}

// ---------------------------------------------------------- column vectors
// v~ = p .* q / beta - beta v ; q = 0 ; alpha^2 partials.
template <typename Acc>
__global__ __launch_bounds__(kBlock) void k_col_a(int64_t n, const double* __restrict__ p,
                                                   Acc* __restrict__ q, double* __restrict__ v,
                                                   const Scalars* __restrict__ sc,
                                                   double* __restrict__ part)
{
    __shared__ double red[kWavesPerBlock];
    if (sc->done || sc->beta_zero) return;
    const double beta = sc->beta;
    const double ib = 1.0 / beta;
    double ssq = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock) {
        const double qj = (double)q[j];
        q[j] = (Acc)0;
        const double vt = p[j] * qj * ib - beta * v[j];
        v[j] = vt;
        ssq += vt * vt;
    }
    const double r = block_sum(ssq, red);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// v = v~/alpha ; vp = p .* v ; y += t1 w ; w = v + t2 w ;
// partials of ||w/rho||^2 and ||y||^2 ; var (optional) += (w/rho)^2, the
// per-iteration variance term of Algorithm 1 (diagonal estimate of
// (Abar^T Abar)^-1, rescaled by p^2 after the loop).
template <typename VP>
__global__ __launch_bounds__(kBlock) void k_col_b(int64_t n, const double* __restrict__ p,
                                                   double* __restrict__ v,
                                                   double* __restrict__ w,
                                                   double* __restrict__ y, VP* __restrict__ vp,
                                                   const Scalars* __restrict__ sc,
                                                   double* __restrict__ part_dd,
                                                   double* __restrict__ part_xx,
                                                   double* __restrict__ var)
{
    __shared__ double red[kWavesPerBlock];
    if (sc->done) return;
    const double ia = sc->beta_zero ? 1.0 : sc->inv_alpha;
    const double t1 = sc->t1, t2 = sc->t2, ir = 1.0 / sc->rho;
    double dd = 0.0, xx = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock) {
        const double vj = v[j] * ia;
        v[j] = vj;
        vp[j] = (VP)(p[j] * vj);
        const double wj = w[j];
        const double dk = wj * ir;
        dd += dk * dk;
        if (var) var[j] += dk * dk;
        const double yj = y[j] + t1 * wj;
        y[j] = yj;
        xx += yj * yj;
        w[j] = vj + t2 * wj;
    }
    double r = block_sum(dd, red);
    if (threadIdx.x == 0) part_dd[blockIdx.x] = r;
    r = block_sum(xx, red);
    if (threadIdx.x == 0) part_xx[blockIdx.x] = r;
}

// Initial v = v~/alpha_1 ; vp = p .* v ; w = v ; y = 0.
template <typename VP>
__global__ __launch_bounds__(kBlock) void k_col_init(int64_t n, const double* __restrict__ p,
                                                      double* __restrict__ v,
                                                      double* __restrict__ w,
                                                      double* __restrict__ y,
                                                      VP* __restrict__ vp,
                                                      const Scalars* __restrict__ sc)
{
    const double ia = sc->inv_alpha;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock) {
        const double vj = v[j] * ia;
        v[j] = vj;
        w[j] = vj;
        vp[j] = (VP)(p[j] * vj);
        y[j] = 0.0;
    }
}

// u~ = b (stored as VU, row i at u[inv[i]] or u[i]) ; FP64 sum of squares of
// the stored values.
template <typename VU>
__global__ __launch_bounds__(kBlock) void k_copy_ssq(int64_t m, const double* __restrict__ b,
                                                      VU* __restrict__ u,
                                                      double* __restrict__ part,
                                                      const int32_t* __restrict__ inv)
{
    __shared__ double red[kWavesPerBlock];
    double ssq = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * kBlock) {
        const VU v = (VU)b[i];
        u[inv ? (int64_t)inv[i] : i] = v;
        ssq += (double)v * (double)v;
    }
    const double r = block_sum(ssq, red);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_fill(int64_t n, V* __restrict__ a, V value)
{
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock)
        a[j] = value;
}

// out = p^2 .* var: the variance estimate re-multiplied by the column
// scaling (Algorithm 1 after the loop)
__global__ __launch_bounds__(kBlock) void k_unprecond_var(int64_t n,
                                                           const double* __restrict__ p,
                                                           const double* __restrict__ var,
                                                           double* __restrict__ out)
{
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock)
        out[j] = p[j] * p[j] * var[j];
}

// x = p .* y (un-preconditioning, Algorithm 1 after the loop)
__global__ __launch_bounds__(kBlock) void k_unprecond(int64_t n, const double* __restrict__ p,
                                                       const double* __restrict__ y,
                                                       double* __restrict__ x)
{
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock)
        x[j] = p[j] * y[j];
}

// Refinement: x += p .* y ; partial maxima of |p .* y| and |x|.
__global__ __launch_bounds__(kBlock) void k_refine_update(int64_t n,
                                                           const double* __restrict__ p,
                                                           const double* __restrict__ y,
                                                           double* __restrict__ x,
                                                           double* __restrict__ part_d,
                                                           double* __restrict__ part_x)
{
    __shared__ double red[kWavesPerBlock];
    double dm = 0.0, xm = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock) {
        const double d = p[j] * y[j];
        const double xj = x[j] + d;
        x[j] = xj;
        dm = fmax(dm, fabs(d));
        xm = fmax(xm, fabs(xj));
    }
    double r = block_max(dm, red);
    if (threadIdx.x == 0) part_d[blockIdx.x] = r;
    r = block_max(xm, red);
    if (threadIdx.x == 0) part_x[blockIdx.x] = r;
}

__global__ __launch_bounds__(kBlock) void k_refine_norms(const double* __restrict__ part_d,
                                                          const double* __restrict__ part_x,
                                                          int nblk, Scalars* __restrict__ sc)
{
    __shared__ double red[kWavesPerBlock];
    const double d = max_partials(part_d, nblk, red);
    const double x = max_partials(part_x, nblk, red);
    if (threadIdx.x == 0) {
        sc->dmax = d;
        sc->xmax = x;
    }
}

// ------------------------------------------------------------ scalar kernels
// Start of a solve: beta_1 = ||b||, reset the state.
__global__ __launch_bounds__(kBlock) void k_scalar_init_beta(const double* __restrict__ part,
                                                              int nblk, Scalars* __restrict__ sc)
{
    __shared__ double red[kWavesPerBlock];
    const double ssq = sum_partials(part, nblk, red);
    if (threadIdx.x != 0) return;
    const double beta = sqrt(ssq);
    sc->beta = beta;
    sc->bnorm = beta;
    sc->alpha = 0.0;
    sc->anorm = 0.0;
    sc->ddnorm = 0.0;
    sc->acond = 0.0;
    sc->xnorm = 0.0;
    sc->rnorm = beta;
    sc->arnorm = 0.0;
    sc->itn = 0;
    sc->istop = 0;
    sc->beta_zero = 0;
    sc->done = beta > 0.0 ? 0 : 1;  // b = 0: x = 0 solves it (istop 0)
}

// alpha_1 = ||A^T u_1|| ; rhobar = alpha ; phibar = beta.
__global__ __launch_bounds__(kBlock) void k_scalar_init_alpha(const double* __restrict__ part,
                                                               int nblk, Scalars* __restrict__ sc)
{
    __shared__ double red[kWavesPerBlock];
    const double ssq = sum_partials(part, nblk, red);
    if (threadIdx.x != 0 || sc->done) return;
    const double alpha = sqrt(ssq);
    sc->alpha = alpha;
    sc->rhobar = alpha;
    sc->phibar = sc->beta;
    sc->arnorm = alpha * sc->beta;
    sc->arnorm0 = sc->arnorm;
    sc->inv_alpha = alpha > 0.0 ? 1.0 / alpha : 1.0;
    sc->coef_u = alpha / sc->beta;
    if (sc->arnorm == 0.0) sc->done = 1;  // A^T b = 0: x = 0 (istop 0)
}

// beta_{i+1} = ||u~|| ; anorm update.
__global__ __launch_bounds__(kBlock) void k_scalar_beta(const double* __restrict__ part,
                                                         int nblk, Scalars* __restrict__ sc)
{
    __shared__ double red[kWavesPerBlock];
    if (sc->done) return;
    const double ssq = sum_partials(part, nblk, red);
    if (threadIdx.x != 0) return;
    const double beta = sqrt(ssq);
    sc->beta = beta;
    if (beta > 0.0) {
        const double a = sc->alpha;
        sc->anorm = sqrt(sc->anorm * sc->anorm + a * a + beta * beta);
        sc->beta_zero = 0;
    } else {
        sc->beta_zero = 1;
    }
}

// alpha_{i+1} = ||v~|| and the plane rotation eliminating beta_{i+1}.
__global__ __launch_bounds__(kBlock) void k_scalar_alpha(const double* __restrict__ part,
                                                          int nblk, Scalars* __restrict__ sc)
{
    __shared__ double red[kWavesPerBlock];
    if (sc->done) return;
    const double ssq = sum_partials(part, nblk, red);
    if (threadIdx.x != 0) return;
    double alpha = sc->alpha;
    if (!sc->beta_zero) alpha = sqrt(ssq);
    const double beta = sc->beta;
    const double rhobar = sc->rhobar;
    const double rho = sqrt(rhobar * rhobar + beta * beta);
    const double c = rhobar / rho;
    const double sn = beta / rho;
    const double theta = sn * alpha;
    const double phi = c * sc->phibar;
    sc->alpha = alpha;
    sc->rho = rho;
    sc->c = c;
    sc->s = sn;
    sc->theta = theta;
    sc->rhobar = -c * alpha;
    sc->phi = phi;
    sc->phibar = sn * sc->phibar;
    sc->t1 = phi / rho;
    sc->t2 = -theta / rho;
    sc->inv_alpha = alpha > 0.0 ? 1.0 / alpha : 1.0;
    sc->coef_u = beta > 0.0 ? alpha / beta : 0.0;
    sc->rnorm = sc->phibar;
    sc->arnorm = alpha * fabs(c) * sc->phibar;
}

// ddnorm, xnorm, acond and the stopping tests of Paige & Saunders.
__global__ __launch_bounds__(kBlock) void k_scalar_stop(const double* __restrict__ part_dd,
                                                         const double* __restrict__ part_xx,
                                                         int nblk, Scalars* __restrict__ sc)
{
    __shared__ double red[kWavesPerBlock];
    if (sc->done) return;
    const double dd = sum_partials(part_dd, nblk, red);
    const double xx = sum_partials(part_xx, nblk, red);
    if (threadIdx.x != 0) return;
    const double ddnorm = sc->ddnorm + dd;
    const double xnorm = sqrt(xx);
    const double anorm = sc->anorm;
    const double acond = anorm * sqrt(ddnorm);
    const double rnorm = sc->rnorm, arnorm = sc->arnorm, bnorm = sc->bnorm;
    sc->ddnorm = ddnorm;
    sc->xnorm = xnorm;
    sc->acond = acond;
    const int32_t itn = sc->itn + 1;
    sc->itn = itn;

    const double test1 = rnorm / bnorm;
    const double test2 = (anorm * rnorm) > 0.0 ? arnorm / (anorm * rnorm) : 0.0;
    const double test3 = acond > 0.0 ? 1.0 / acond : 0.0;
    const double t1 = test1 / (1.0 + anorm * xnorm / bnorm);
    const double rtol = sc->btol + sc->atol * anorm * xnorm / bnorm;
    int32_t istop = 0;
    if (itn >= sc->itn_limit) istop = 7;
    if (sc->tests) {
        if (1.0 + test3 <= 1.0) istop = 6;
        if (1.0 + test2 <= 1.0) istop = 5;
        if (1.0 + t1 <= 1.0) istop = 4;
        if (test3 <= sc->ctol) istop = 3;
        if (test2 <= sc->atol) istop = 2;
        if (test1 <= rtol) istop = 1;
    }
    // Relative form of the normal-equation test, for correction problems whose
    // residual is dominated by the irreducible least-squares residual.
    if (sc->rel_ar > 0.0 && arnorm <= sc->rel_ar * sc->arnorm0) istop = 2;
    sc->istop = istop;
    if (istop != 0) sc->done = 1;
}

// ------------------------------------------------------------------- set-up
// Index validation: bit 1 star out of range, 2 stars not sorted,
// 4 attitude start out of range, 8 instrumental index out of range.
__global__ __launch_bounds__(kBlock) void k_validate(SysView s, int32_t* __restrict__ flag)
{
    int32_t bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < s.m;
         i += (int64_t)gridDim.x * kBlock) {
        const int64_t st = s.star[i];
        if (st < 0 || st >= s.n_stars) bad |= 1;
        if (i > 0 && s.star[i - 1] > st) bad |= 2;
        if (s.natt > 0) {
            const int64_t t = s.att[i];
            if (t < 0 || t > s.n_dfa - kParAxis) bad |= 4;
        }
        for (int j = 0; j < s.ni; ++j) {
            const int32_t c = s.instr[j * s.m + i];
            if (c < 0 || (int64_t)c >= s.n_instr_cols) bad |= 8;
        }
    }
    if (bad) atomicOr(flag, bad);
}

// Compact index copies for the fused passes: star as int32, instrumental
// indices as uint16 (the caller checks that they fit).
__global__ __launch_bounds__(kBlock) void k_compact_idx(SysView s, int32_t* __restrict__ star32,
                                                         uint16_t* __restrict__ instr16)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < s.m;
         i += (int64_t)gridDim.x * kBlock) {
        star32[i] = (int32_t)s.star[i];
#pragma unroll
        for (int j = 0; j < kInstr; ++j) instr16[j * s.m + i] = (uint16_t)s.instr[j * s.m + i];
    }
}

// Star-aligned row boundaries: range g starts at the first star boundary at
// or after g*m/nw, so that no star is split between two waves.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_wave_bounds(const K* __restrict__ star,
                                                         int64_t m, int64_t nw,
                                                         int64_t* __restrict__ wb)
{
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g > nw) return;
    if (g == nw) {
        wb[g] = m;
        return;
    }
    int64_t r = g * m / nw;  // g <= nw <= 2^20, m < 2^40: no overflow
    while (r > 0 && r < m && star[r] == star[r - 1]) ++r;
    wb[g] = r;
}

// p_j = 1/sqrt(ssq_j), 1 for an empty column (or for every column when not
// preconditioning); resets ssq.
__global__ __launch_bounds__(kBlock) void k_make_p(int64_t n, double* __restrict__ ssq,
                                                    double* __restrict__ p, int precondition)
{
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock) {
        const double s2 = ssq[j];
        p[j] = (precondition && s2 > 0.0) ? 1.0 / sqrt(s2) : 1.0;
        ssq[j] = 0.0;
    }
}

// ------------------------------------------------ attitude in bucket order
// The attitude columns of a row are 3 windows of 4 consecutive columns at the
// row's start t. Rows stably sorted by the bucket of t (t / W, W starts per
// bucket) put every bucket's rows together while keeping star order inside a
// bucket; the columns one bucket touches are 3 x (W + 3), few enough for an
// LDS histogram, so Eq. (3) for the attitude section becomes a sequential
// sweep with LDS atomics and no device atomics. The solver keeps its row
// vector u~ in this order (row i at u[inv[i]]): the attitude sweep reads it
// sequentially, and the star-order passes reach it through inv, whose targets
// form one run per bucket for any stretch of consecutive rows.
__global__ __launch_bounds__(kBlock) void k_bucket_keys(const int64_t* __restrict__ att, int64_t m,
                                                         int64_t width, int32_t* __restrict__ keys,
                                                         int32_t* __restrict__ rows)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * kBlock) {
        keys[i] = (int32_t)(att[i] / width);
        rows[i] = (int32_t)i;
    }
}

__global__ __launch_bounds__(kBlock) void k_invert_perm(const int32_t* __restrict__ perm, int64_t m,
                                                         int32_t* __restrict__ invperm)
{
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < m;
         k += (int64_t)gridDim.x * kBlock)
        invperm[perm[k]] = (int32_t)k;
}

// bstart[b] = first sorted position of bucket b (b = 0..nb; empty buckets
// included), from the sorted keys.
__global__ __launch_bounds__(kBlock) void k_bucket_starts(const int32_t* __restrict__ skeys,
                                                           int64_t m, int64_t nb,
                                                           int64_t* __restrict__ bstart)
{
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k <= m;
         k += (int64_t)gridDim.x * kBlock) {
        const int64_t prev = k > 0 ? (int64_t)skeys[k - 1] : -1;
        const int64_t cur = k < m ? (int64_t)skeys[k] : nb;
        for (int64_t b = prev + 1; b <= cur; ++b) bstart[b] = k;
    }
}

// att_sorted[c ld + k] = values[off_att + c][perm[k]], c < 12 (ld >= m: the
// column stride of the copy) ; tloc[k] = t of row perm[k] minus its bucket's
// first start.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_att_gather(const T* __restrict__ val,
                                                        const int64_t* __restrict__ att, int64_t m,
                                                        const int32_t* __restrict__ perm,
                                                        int64_t width, int off_att, int64_t ld,
                                                        T* __restrict__ att_sorted,
                                                        int32_t* __restrict__ tloc)
{
    constexpr int kAtt = kAxes * kParAxis;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < m;
         k += (int64_t)gridDim.x * kBlock) {
        const int64_t i = perm[k];
#pragma unroll
        for (int c = 0; c < kAtt; ++c) att_sorted[c * ld + k] = val[(off_att + c) * m + i];
        const int64_t t = att[i];
        tloc[k] = (int32_t)(t - (t / width) * width);
    }
}

// Attitude part of Eq. (2) over the rows in bucket order, folded into the
// row vector: u~[k] <- sum_c a_c x[col_c] - coef_u u~[k] for the 12 attitude
// coefficients of row k (u~ in bucket order, coalesced), for K right-hand
// sides (u~ [m][K] row-interleaved, x3 [3 n_dfa][K]). The G workgroups of a
// bucket share its rows as in k_att_hist; the bucket's attitude columns
// [b W, b W + W + 3) of the interleaved copy x3 are staged in LDS first
// (win[(3 c + axis) KS + j], 3 (W + 3) KS Acc), so no row gathers from global
// memory. KS right-hand sides share one sweep over the rows (one window each);
// K / KS sweeps cover the tile. Frozen RHS (done) keep u~. The fused pass
// (kAttPre) then adds the other sections. SEP: u is a separate bucket-order
// vector that receives the attitude part alone (u[k] <- sum_c a_c x[col_c],
// nothing read), for the fused pass's kAttGather form. att_sorted holds
// coefficient c of bucket-order row k at c ld + k, ld a multiple of 64.
// Row blocks start at the 64-row boundary at or below the bucket's first row
// b0, so every wave reads whole 128-byte lines: a line shared by two waves
// that load at the same time is fetched from memory twice (measured: 1.15x
// the streamed bytes when the blocks started at b0). Lanes below b0 load row
// b0 and store nothing.
// PIPE: each thread issues the loads of its next row before the store of the
// current one. A wave's vector-memory counter retires loads and stores in
// issue order, so a store issued before the next row's loads would be waited
// for together with them (one store round trip per row); after them it is
// not.
template <typename T, typename Acc, int K, int KS, int NT, bool SEP = false, bool PIPE = (K == 1)>
__global__ __launch_bounds__(NT) void k_att_dot(int64_t ld, const T* __restrict__ att_sorted,
                                                 const int32_t* __restrict__ tloc,
                                                 const int64_t* __restrict__ bstart,
                                                 int64_t width, int G, int64_t n_dfa,
                                                 const Acc* __restrict__ x3, Acc* __restrict__ u,
                                                 const Scalars* __restrict__ sc)
{
    static_assert(K % KS == 0, "sweeps of KS right-hand sides cover the tile");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Acc* win = reinterpret_cast<Acc*>(smem_raw);
    const int64_t span = width + kParAxis - 1;
    const int64_t bk = blockIdx.x / G, g = blockIdx.x - bk * G;
    const int64_t c0 = bk * width;
    // columns past n_dfa - 1 are never referenced (t + 3 <= n_dfa - 1)
    const int64_t ncol = span < n_dfa - c0 ? span : n_dfa - c0;
    const int64_t b0 = bstart[bk], r1 = bstart[bk + 1];
    const int64_t a0 = b0 & ~(int64_t)(kWave - 1);
    for (int s0 = 0; s0 < K; s0 += KS) {
        uint32_t live = 0;
        Acc coef[KS];
#pragma unroll
        for (int j = 0; j < KS; ++j) {
            live |= (sc[s0 + j].done ? 0u : 1u) << j;
            coef[j] = (Acc)sc[s0 + j].coef_u;
        }
        if (live == 0) continue;  // uniform over the grid
        if (KS == K) {
            for (int64_t e = threadIdx.x; e < kAxes * ncol * K; e += NT)
                win[e] = x3[kAxes * c0 * K + e];
        } else {
            for (int64_t e = threadIdx.x; e < kAxes * ncol * KS; e += NT) {
                const int64_t col = e / KS;
                win[e] = x3[(kAxes * c0 + col) * K + s0 + (e - col * KS)];
            }
        }
        __syncthreads();
        constexpr int kAtt = kAxes * kParAxis;
        // the attitude dot product of one row from the LDS window
        auto row_dot_win = [&](int64_t tl, const T (&a)[kAtt], Acc (&d)[KS]) {
#pragma unroll
            for (int j = 0; j < KS; ++j) d[j] = (Acc)0;
#pragma unroll
            for (int ax = 0; ax < kAxes; ++ax)
#pragma unroll
                for (int qq = 0; qq < kParAxis; ++qq) {
                    const Acc av = (Acc)a[ax * kParAxis + qq];
                    const Acc* w = win + (kAxes * (tl + qq) + ax) * KS;
#pragma unroll
                    for (int j = 0; j < KS; ++j) d[j] += av * w[j];
                }
        };
        const int64_t stride = (int64_t)G * NT;
        if (PIPE) {
            // Three rows in flight, each in its own registers (no copies,
            // which would wait for the loads): a row's loads are issued two
            // rows before it is finished, so a store is only ever waited for
            // two rows after it was issued. Rows past the end repeat the
            // last row: loaded before that row's store, they store the same
            // value again.
            struct Row {
                int64_t tl;
                T a[kAtt];
                Acc uo[KS];
            };
            auto load = [&](Row& r, int64_t k) {
                const int64_t kk = k < b0 ? b0 : k;
                r.tl = ldnt(&tloc[kk]);
#pragma unroll
                for (int c = 0; c < kAtt; ++c) r.a[c] = ldnt(&att_sorted[c * ld + kk]);
#pragma unroll
                for (int j = 0; j < KS; ++j) r.uo[j] = SEP ? (Acc)0 : u[kk * K + s0 + j];
            };
            auto finish = [&](const Row& r, int64_t k) {
                if (k < b0) return;
                Acc d[KS];
                row_dot_win(r.tl, r.a, d);
#pragma unroll
                for (int j = 0; j < KS; ++j)
                    if (KS == 1 || ((live >> j) & 1u))
                        u[k * K + s0 + j] = SEP ? d[j] : d[j] - coef[j] * r.uo[j];
            };
            int64_t k0 = a0 + g * NT + threadIdx.x;
            if (b0 < r1 && k0 < r1) {
                const int64_t klast = k0 + (r1 - 1 - k0) / stride * stride;
                auto next = [&](int64_t k) { return k < klast ? k + stride : klast; };
                Row A, B, C;
                int64_t k1 = next(k0);
                load(A, k0);
                load(B, k1);
                for (;;) {
                    // scheduling fences keep the issue order of each step:
                    // the loads of the row two ahead, then this row's store
                    const int64_t k2 = next(k1);
                    load(C, k2);
                    __builtin_amdgcn_sched_barrier(0);
                    finish(A, k0);
                    __builtin_amdgcn_sched_barrier(0);
                    const int64_t k3 = next(k2);
                    load(A, k3);
                    __builtin_amdgcn_sched_barrier(0);
                    finish(B, k1);
                    __builtin_amdgcn_sched_barrier(0);
                    const int64_t k4 = next(k3);
                    load(B, k4);
                    __builtin_amdgcn_sched_barrier(0);
                    finish(C, k2);
                    __builtin_amdgcn_sched_barrier(0);
                    if (k2 >= klast) break;  // rows from k3 on repeat the last row
                    k0 = k3;
                    k1 = k4;
                }
            }
        } else {
            for (int64_t k = a0 + g * NT + threadIdx.x; k < r1; k += stride) {
                if (k < b0) continue;
                const int64_t tl = ldnt(&tloc[k]);
                T a[kAtt];
#pragma unroll
                for (int c = 0; c < kAtt; ++c) a[c] = ldnt(&att_sorted[c * ld + k]);
                Acc d[KS];
                row_dot_win(tl, a, d);
#pragma unroll
                for (int j = 0; j < KS; ++j) {
                    if (!((live >> j) & 1u)) continue;
                    Acc* up = u + k * K + s0 + j;
                    *up = SEP ? d[j] : d[j] - coef[j] * *up;
                }
            }
        }
        __syncthreads();  // the next sweep restages the window
    }
}

// Attitude part of Eq. (3) over the rows in bucket order. The G workgroups
// of bucket b share its rows in interleaved blocks of NT (workgroup w = b G +
// g takes blocks g, g + G, ..., so the G streams advance through memory
// together): an LDS histogram hist[axis][W + 3][KS] gets a * u for the 12
// coefficients of each of its rows and the KS right-hand sides of one sweep,
// then is stored as S2[w][r][axis][W + 3]; k_att_reduce adds the slices. The
// histogram and S2 are FP64 whatever Acc is: gfx950's LDS FP64 atomic add
// runs at 7.6x the rate of the FP32 one (measured, random addresses over
// 150 KB: 1550 vs 204 G/s), and the sums are more accurate. U is in bucket
// order ([m][K]); K / KS sweeps cover the tile. Frozen RHS (done or
// beta_zero) are skipped. GATHER: U is in star order instead, and the row at
// bucket position k is read at U[perm[k]] (a read through the permutation,
// whose targets form one increasing run per bucket).
// PIPE: each thread issues the loads of its next row before the atomics of
// the current one (with GATHER, the current row's read through the
// permutation first: its index came with the previous loads).
// att_sorted and the row blocks as in k_att_dot (64-row aligned; lanes below
// the bucket's first row load that row with a zero weight).
template <typename T, typename Acc, int K, int KS, int NT, bool GATHER = false,
          bool PIPE = (K == 1)>
__global__ __launch_bounds__(NT) void k_att_hist(int64_t ld, const T* __restrict__ att_sorted,
                                                  const int32_t* __restrict__ tloc,
                                                  const int64_t* __restrict__ bstart,
                                                  int64_t width, int G, const Acc* __restrict__ U,
                                                  double* __restrict__ S2,
                                                  const Scalars* __restrict__ sc,
                                                  const int32_t* __restrict__ perm = nullptr)
{
    static_assert(K % KS == 0, "sweeps of KS right-hand sides cover the tile");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* hist = reinterpret_cast<double*>(smem_raw);
    const int64_t span = width + kParAxis - 1;
    const int64_t bk = blockIdx.x / G, g = blockIdx.x - bk * G;
    const int64_t b0 = bstart[bk], r1 = bstart[bk + 1];
    const int64_t a0 = b0 & ~(int64_t)(kWave - 1);
    for (int s0 = 0; s0 < K; s0 += KS) {
        uint32_t live = 0;
#pragma unroll
        for (int j = 0; j < KS; ++j)
            live |= (sc != nullptr && (sc[s0 + j].done || sc[s0 + j].beta_zero) ? 0u : 1u) << j;
        if (live == 0) continue;  // uniform over the grid
        for (int64_t e = threadIdx.x; e < kAxes * span * KS; e += NT) hist[e] = 0.0;
        __syncthreads();
        constexpr int kAtt = kAxes * kParAxis;
        auto scatter = [&](int64_t tl, const T (&a)[kAtt], const double (&uk)[KS]) {
#pragma unroll
            for (int ax = 0; ax < kAxes; ++ax)
#pragma unroll
                for (int qq = 0; qq < kParAxis; ++qq)
#pragma unroll
                    for (int j = 0; j < KS; ++j)
                        if ((live >> j) & 1u)
                            atomicAdd(&hist[(ax * span + tl + qq) * KS + j],
                                      (double)a[ax * kParAxis + qq] * uk[j]);
        };
        const int64_t stride = (int64_t)G * NT;
        if (PIPE) {
            // Three rows in flight as in k_att_dot; rows past the end repeat
            // the last row with a zero weight. With GATHER a row's value is
            // read through the permutation one step before the row is
            // scattered (its index came with the row's loads).
            struct Row {
                int64_t tl, ku;
                T a[kAtt];
                double uk[KS];
            };
            auto load = [&](Row& r, int64_t k) {
                const int64_t kk = k < b0 ? b0 : k;
                r.tl = ldnt(&tloc[kk]);
                r.ku = GATHER ? (int64_t)ldnt(&perm[kk]) : kk;
#pragma unroll
                for (int c = 0; c < kAtt; ++c) r.a[c] = ldnt(&att_sorted[c * ld + kk]);
                if (!GATHER)
#pragma unroll
                    for (int j = 0; j < KS; ++j) r.uk[j] = (double)U[kk * K + s0 + j];
            };
            auto value = [&](Row& r, double w) {
#pragma unroll
                for (int j = 0; j < KS; ++j)
                    r.uk[j] = w * (GATHER ? (double)U[r.ku * K + s0 + j] : r.uk[j]);
            };
            int64_t k0 = a0 + g * NT + threadIdx.x;
            if (b0 < r1 && k0 < r1) {
                const int64_t klast = k0 + (r1 - 1 - k0) / stride * stride;
                // next row and its weight (0 for a repeat of the last row;
                // only a thread's first row can lie below b0)
                auto next = [&](int64_t k) { return k < klast ? k + stride : klast; };
                Row A, B, C;
                int64_t k1 = next(k0);
                load(A, k0);
                load(B, k1);
                value(A, k0 >= b0 ? 1.0 : 0.0);
                for (;;) {
                    const int64_t k2 = next(k1);
                    value(B, k1 > k0 ? 1.0 : 0.0);
                    load(C, k2);
                    __builtin_amdgcn_sched_barrier(0);
                    scatter(A.tl, A.a, A.uk);
                    __builtin_amdgcn_sched_barrier(0);
                    const int64_t k3 = next(k2);
                    value(C, k2 > k1 ? 1.0 : 0.0);
                    load(A, k3);
                    __builtin_amdgcn_sched_barrier(0);
                    scatter(B.tl, B.a, B.uk);
                    __builtin_amdgcn_sched_barrier(0);
                    const int64_t k4 = next(k3);
                    value(A, k3 > k2 ? 1.0 : 0.0);
                    load(B, k4);
                    __builtin_amdgcn_sched_barrier(0);
                    scatter(C.tl, C.a, C.uk);
                    __builtin_amdgcn_sched_barrier(0);
                    if (k2 >= klast) break;
                    k0 = k3;
                    k1 = k4;
                }
            }
        } else {
            for (int64_t k = a0 + g * NT + threadIdx.x; k < r1; k += stride) {
                if (k < b0) continue;
                const int64_t tl = ldnt(&tloc[k]);
                const int64_t ku = GATHER ? (int64_t)ldnt(&perm[k]) : k;
                double uk[KS];
#pragma unroll
                for (int j = 0; j < KS; ++j) uk[j] = (double)U[ku * K + s0 + j];
                T a[kAtt];  // all loads issued before the first atomic
#pragma unroll
                for (int c = 0; c < kAtt; ++c) a[c] = ldnt(&att_sorted[c * ld + k]);
                scatter(tl, a, uk);
            }
        }
        __syncthreads();
        for (int j = 0; j < KS; ++j) {
            if (!((live >> j) & 1u)) continue;
            double* out = S2 + ((int64_t)blockIdx.x * K + s0 + j) * kAxes * span;
            for (int64_t e = threadIdx.x; e < kAxes * span; e += NT) out[e] = hist[e * KS + j];
        }
        __syncthreads();
    }
}

// q_att[(axis n_dfa + c) K + r] += sum of the slices of the (at most two)
// buckets whose window holds column c.
template <typename Acc, int K>
__global__ __launch_bounds__(kBlock) void k_att_reduce(const double* __restrict__ S2, int64_t nb,
                                                        int G, int64_t width, int64_t n_dfa,
                                                        Acc* __restrict__ qatt,
                                                        const Scalars* __restrict__ sc)
{
    const int64_t span = width + kParAxis - 1;
    const int64_t total = (int64_t)kAxes * n_dfa * K;
    for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kBlock) {
        const int64_t col = idx / K;
        const int r = (int)(idx - col * K);
        if (sc != nullptr && (sc[r].done || sc[r].beta_zero)) continue;
        const int64_t ax = col / n_dfa, c = col - ax * n_dfa;
        const int64_t bhi = c / width < nb - 1 ? c / width : nb - 1;
        double sum = 0.0;
        for (int64_t bk = bhi; bk >= 0 && c - bk * width < span; --bk) {
            const int64_t off = c - bk * width;
            for (int g = 0; g < G; ++g)
                sum += S2[(((bk * G + g) * K + r) * kAxes + ax) * span + off];
        }
        qatt[idx] = (Acc)((double)qatt[idx] + sum);
    }
}

// ====================================================== batched right-hand sides
// K right-hand sides advance together: one row per lane, K values per lane,
// so every coefficient and index of A is read once per K RHS (an SpMM).
// Layouts of one k-tile: U [m][K] (row-interleaved), column vectors [n][K].
// sc points at the tile's K Scalars; a RHS with sc[r].done set is frozen:
// no kernel changes its vectors or scalars any more.
namespace batched {

// Running masks: bit r set when RHS r is still iterating.
template <int K>
__device__ __forceinline__ uint32_t live_mask(const Scalars* __restrict__ sc)
{
    uint32_t mk = 0;
#pragma unroll
    for (int r = 0; r < K; ++r) mk |= (sc[r].done ? 0u : 1u) << r;
    return mk;
}

// K-wide gather of a column vector row [n][K].
template <typename V, int K>
__device__ __forceinline__ void load_k(const V* __restrict__ p, V (&out)[K])
{
#pragma unroll
    for (int r = 0; r < K; ++r) out[r] = p[r];
}

// Deterministic block sums of K doubles per thread into part[blk*K + r].
template <int K>
__device__ __forceinline__ void block_sums_k(double (&v)[K], double* __restrict__ part,
                                             double* lds /* >= K * kWavesPerBlock */)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int r = 0; r < K; ++r)
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) v[r] += __shfl_down(v[r], off);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int r = 0; r < K; ++r) lds[r * kWavesPerBlock + w] = v[r];
    __syncthreads();
    if (threadIdx.x < K) {
        double s = 0.0;
        for (int k = 0; k < kWavesPerBlock; ++k) s += lds[threadIdx.x * kWavesPerBlock + k];
        part[(int64_t)blockIdx.x * K + threadIdx.x] = s;
    }
}

// U[p(i)][r] = B[i][r] (B row stride ldb; p(i) = inv[i], or i without inv),
// FP64 sums of squares per RHS.
template <typename VU, int K>
__global__ __launch_bounds__(kBlock) void k_copy_ssq(int64_t m, const double* __restrict__ B,
                                                      int64_t ldb, VU* __restrict__ U,
                                                      double* __restrict__ part,
                                                      const int32_t* __restrict__ inv)
{
    __shared__ double red[K * kWavesPerBlock];
    double ssq[K];
#pragma unroll
    for (int r = 0; r < K; ++r) ssq[r] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * kBlock) {
        const int64_t pi = inv ? (int64_t)inv[i] : i;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const VU v = (VU)B[i * ldb + r];
            U[pi * K + r] = v;
            ssq[r] += (double)v * (double)v;
        }
    }
    block_sums_k<K>(ssq, part, red);
}

// U = A VP - coef_r U per live RHS (row i at U[inv[i]] or U[i]); sums of
// squares of the new U per RHS.
template <typename T, typename Acc, int K>
__global__ __launch_bounds__(kBlock) void k_aprod1(SysView s, const Acc* __restrict__ VP,
                                                    Acc* __restrict__ U,
                                                    const Scalars* __restrict__ sc,
                                                    double* __restrict__ part,
                                                    const int32_t* __restrict__ inv)
{
    __shared__ double red[K * kWavesPerBlock];
    const uint32_t live = live_mask<K>(sc);
    if (live == 0) return;
    Acc coef[K];
#pragma unroll
    for (int r = 0; r < K; ++r) coef[r] = (Acc)sc[r].coef_u;
    const T* __restrict__ val = static_cast<const T*>(s.val);
    const int64_t m = s.m;
    double ssq[K];
#pragma unroll
    for (int r = 0; r < K; ++r) ssq[r] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * kBlock) {
        const int64_t st = ldnt(&s.star[i]);
        const int64_t t = ldnt(&s.att[i]);
        T a[kPar];
#pragma unroll
        for (int c = 0; c < kPar; ++c) a[c] = ldnt(&val[c * m + i]);
        int32_t ic[kInstr];
#pragma unroll
        for (int j = 0; j < kInstr; ++j) ic[j] = ldnt(&s.instr[j * m + i]);
        Acc sum[K];
#pragma unroll
        for (int r = 0; r < K; ++r) sum[r] = (Acc)0;
        Acc xv[K];
#pragma unroll
        for (int j = 0; j < kAstro; ++j) {
            load_k<Acc, K>(VP + (kAstro * st + j) * K, xv);
#pragma unroll
            for (int r = 0; r < K; ++r) sum[r] += (Acc)a[j] * xv[r];
        }
#pragma unroll
        for (int ax = 0; ax < kAxes; ++ax)
#pragma unroll
            for (int qq = 0; qq < kParAxis; ++qq) {
                load_k<Acc, K>(VP + (s.att_base + ax * s.n_dfa + t + qq) * K, xv);
#pragma unroll
                for (int r = 0; r < K; ++r) sum[r] += (Acc)a[kOffAtt + ax * kParAxis + qq] * xv[r];
            }
#pragma unroll
        for (int j = 0; j < kInstr; ++j) {
            load_k<Acc, K>(VP + (s.instr_base + ic[j]) * K, xv);
#pragma unroll
            for (int r = 0; r < K; ++r) sum[r] += (Acc)a[kOffInstr + j] * xv[r];
        }
        load_k<Acc, K>(VP + s.glob_base * K, xv);
#pragma unroll
        for (int r = 0; r < K; ++r) sum[r] += (Acc)a[kOffGlob] * xv[r];
        Acc* u = U + (inv ? (int64_t)ldnt(&inv[i]) : i) * K;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            if (!((live >> r) & 1u)) continue;
            const Acc nu = sum[r] - coef[r] * u[r];
            u[r] = nu;
            ssq[r] += (double)nu * (double)nu;
        }
    }
    block_sums_k<K>(ssq, part, red);
}

// Q += A^T U over star-aligned per-wave ranges (astrometric: accumulate-and-
// flush segments, attitude: device atomics, instrumental: LDS histogram
// [hcols][K] of columns [0, hcols), the others left to k_instr_tail, global:
// partials gpart[blk][K]). Frozen RHS contribute nothing.
template <typename T, typename Acc, int K, bool ATT = true, int NT = kBlock>
__global__ __launch_bounds__(NT) void k_aprod2(SysView s, const Acc* __restrict__ U,
                                                    Acc* __restrict__ Q,
                                                    const int64_t* __restrict__ wb,
                                                    Acc* __restrict__ gpart, int64_t hcols,
                                                    const Scalars* __restrict__ sc,
                                                    const int32_t* __restrict__ inv)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* lds = reinterpret_cast<double*>(smem_raw);
    __shared__ Acc gred[K * (NT / kWave)];
    uint32_t live = 0;
#pragma unroll
    for (int r = 0; r < K; ++r) live |= ((sc[r].done || sc[r].beta_zero) ? 0u : 1u) << r;
    if (live == 0) return;
    const T* __restrict__ val = static_cast<const T*>(s.val);
    const int64_t m = s.m;
    for (int64_t j = threadIdx.x; j < hcols * K; j += NT) lds[j] = 0.0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = (int64_t)blockIdx.x * (NT / kWave) + threadIdx.x / kWave;
    const int64_t rb = wb[wave], re = wb[wave + 1];
    Acc* __restrict__ qatt = Q + s.att_base * K;
    Acc* __restrict__ qins = Q + s.instr_base * K;
    Acc gsum[K];
#pragma unroll
    for (int r = 0; r < K; ++r) gsum[r] = (Acc)0;
    SegAcc<Acc, kAstro * K> seg;
    auto astro_emit = [Q](int64_t star, const Acc (&tot)[kAstro * K]) {
        Acc* dst = Q + kAstro * star * K;
#pragma unroll
        for (int j = 0; j < kAstro * K; ++j) dst[j] += tot[j];
    };
    // Chunks start on 64-row boundaries so that every coefficient stream is
    // read in whole cache lines; lanes before rb (owned by the previous wave)
    // take the first row's star with zero contributions.
    for (int64_t r0 = rb < re ? (rb & ~(int64_t)(kWave - 1)) : re; r0 < re; r0 += kWave) {
        const int64_t i = r0 + lane;
        const bool ok = i >= rb && i < re;
        const int64_t ic = i < rb ? rb : (i < re ? i : re - 1);
        const int64_t st = i < re ? ldnt(&s.star[ic]) : kNoStar;
        const int64_t t = ATT ? ldnt(&s.att[ic]) : 0;
        T a[kPar];
#pragma unroll
        for (int c = 0; c < kPar; ++c)
            a[c] = (ATT || c < kOffAtt || c >= kOffInstr) ? ldnt(&val[c * m + ic]) : (T)0;
        int32_t ix[kInstr];
#pragma unroll
        for (int j = 0; j < kInstr; ++j) ix[j] = ldnt(&s.instr[j * m + ic]);
        const int64_t pu = inv ? (int64_t)ldnt(&inv[ic]) : ic;
        Acc u[K];
#pragma unroll
        for (int r = 0; r < K; ++r) u[r] = (ok && ((live >> r) & 1u)) ? U[pu * K + r] : (Acc)0;

        if (ok) {
#pragma unroll
            for (int ax = 0; ax < (ATT ? kAxes : 0); ++ax)
#pragma unroll
                for (int qq = 0; qq < kParAxis; ++qq) {
                    Acc* dst = qatt + (ax * s.n_dfa + t + qq) * K;
                    const Acc av = (Acc)a[kOffAtt + ax * kParAxis + qq];
#pragma unroll
                    for (int r = 0; r < K; ++r)
                        if ((live >> r) & 1u) atomicAdd(dst + r, av * u[r]);
                }
#pragma unroll
            for (int j = 0; j < kInstr; ++j) {
                const Acc av = (Acc)a[kOffInstr + j];
                if (ix[j] >= hcols) continue;
#pragma unroll
                for (int r = 0; r < K; ++r) {
                    if (!((live >> r) & 1u)) continue;
                    atomicAdd(&lds[ix[j] * K + r], (double)(av * u[r]));
                }
            }
        }
#pragma unroll
        for (int r = 0; r < K; ++r) gsum[r] += (Acc)a[kOffGlob] * u[r];
        Acc pa[kAstro * K];
#pragma unroll
        for (int j = 0; j < kAstro; ++j)
#pragma unroll
            for (int r = 0; r < K; ++r) pa[j * K + r] = (Acc)a[j] * u[r];
        seg_chunk(seg, st, pa, lane, astro_emit);
    }
    seg_finish(seg, lane, astro_emit);
#pragma unroll
    for (int r = 0; r < K; ++r) {
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) gsum[r] += __shfl_down(gsum[r], off);
    }
    if (lane == 0)
#pragma unroll
        for (int r = 0; r < K; ++r) gred[r * (NT / kWave) + threadIdx.x / kWave] = gsum[r];
    __syncthreads();
    if (threadIdx.x < K) {
        Acc g = (Acc)0;
        for (int k = 0; k < NT / kWave; ++k) g += gred[threadIdx.x * (NT / kWave) + k];
        gpart[(int64_t)blockIdx.x * K + threadIdx.x] = g;
    }
    for (int64_t j = threadIdx.x; j < hcols * K; j += NT) {
        const double v = lds[j];
        if (v != 0.0) atomicAdd(&qins[j], (Acc)v);
    }
}

// X3[(3 c + axis) K + r] = VP[(att_base + axis n_dfa + c) ld + r]: the
// attitude section interleaved by axis, K values per column kept together
// (ld: row stride of VP, K for a tile's own vectors).
template <typename V, int K>
__global__ __launch_bounds__(kBlock) void k_interleave_att(const V* __restrict__ VP, int64_t ld,
                                                            int64_t att_base, int64_t n_dfa,
                                                            V* __restrict__ X3)
{
    const int64_t total = (int64_t)kAxes * n_dfa * K;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < total;
         j += (int64_t)gridDim.x * kBlock) {
        const int64_t col = j / K, r = j - col * K;
        const int64_t c = col / kAxes, ax = col - c * kAxes;
        X3[j] = VP[(att_base + ax * n_dfa + c) * ld + r];
    }
}

// Refinement residual of a k-tile: U_r = B_r - A X_r for the RHS with bit r
// of `live` set (FP32-stored values widened, FP64 accumulation, stored as
// VU at row i's place inv[i] (or i)), U_r = 0 for the others; FP64 sums of
// squares of the stored values per RHS. X: [n][ldx], B: [m][ldb]; X3: the
// attitude section of X interleaved by axis, K values per column.
template <typename T, typename VU, int K>
__global__ __launch_bounds__(kBlock) void k_resid(SysView s, const double* __restrict__ X,
                                                   int64_t ldx, const double* __restrict__ X3,
                                                   const double* __restrict__ B, int64_t ldb,
                                                   VU* __restrict__ U, double* __restrict__ part,
                                                   const int32_t* __restrict__ inv, uint32_t live)
{
    __shared__ double red[K * kWavesPerBlock];
    const T* __restrict__ val = static_cast<const T*>(s.val);
    const int64_t m = s.m;
    double ssq[K];
#pragma unroll
    for (int r = 0; r < K; ++r) ssq[r] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * kBlock) {
        const int64_t st = ldnt(&s.star[i]);
        const int64_t t = ldnt(&s.att[i]);
        T a[kPar];
#pragma unroll
        for (int c = 0; c < kPar; ++c) a[c] = ldnt(&val[c * m + i]);
        int32_t ic[kInstr];
#pragma unroll
        for (int j = 0; j < kInstr; ++j) ic[j] = ldnt(&s.instr[j * m + i]);
        double d[K];
#pragma unroll
        for (int r = 0; r < K; ++r) d[r] = 0.0;
#pragma unroll
        for (int j = 0; j < kAstro; ++j)
#pragma unroll
            for (int r = 0; r < K; ++r) d[r] += (double)a[j] * X[(kAstro * st + j) * ldx + r];
#pragma unroll
        for (int ax = 0; ax < kAxes; ++ax)
#pragma unroll
            for (int qq = 0; qq < kParAxis; ++qq) {
                const double* xv = X3 + (kAxes * (t + qq) + ax) * K;
                const double av = (double)a[kOffAtt + ax * kParAxis + qq];
#pragma unroll
                for (int r = 0; r < K; ++r) d[r] += av * xv[r];
            }
#pragma unroll
        for (int j = 0; j < kInstr; ++j)
#pragma unroll
            for (int r = 0; r < K; ++r)
                d[r] += (double)a[kOffInstr + j] * X[(s.instr_base + ic[j]) * ldx + r];
#pragma unroll
        for (int r = 0; r < K; ++r) d[r] += (double)a[kOffGlob] * X[s.glob_base * ldx + r];
        VU* u = U + (inv ? (int64_t)ldnt(&inv[i]) : i) * K;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const VU v = ((live >> r) & 1u) ? (VU)(B[i * ldb + r] - d[r]) : (VU)0;
            u[r] = v;
            ssq[r] += (double)v * (double)v;
        }
    }
    block_sums_k<K>(ssq, part, red);
}

// Refinement step of a k-tile: X_r += p .* Y_r for the RHS with bit r of
// `live` set; per-RHS partial maxima of |p .* Y_r| and |X_r|
// (part_d/part_x [nblk][K]).
template <int K>
__global__ __launch_bounds__(kBlock) void k_refine_update(int64_t n, const double* __restrict__ p,
                                                           const double* __restrict__ Y,
                                                           double* __restrict__ X, int64_t ldx,
                                                           uint32_t live,
                                                           double* __restrict__ part_d,
                                                           double* __restrict__ part_x)
{
    __shared__ double red[kWavesPerBlock];
    double dm[K], xm[K];
#pragma unroll
    for (int r = 0; r < K; ++r) dm[r] = xm[r] = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock) {
        const double pj = p[j];
#pragma unroll
        for (int r = 0; r < K; ++r) {
            if (!((live >> r) & 1u)) continue;
            const double d = pj * Y[j * K + r];
            const double xj = X[j * ldx + r] + d;
            X[j * ldx + r] = xj;
            dm[r] = fmax(dm[r], fabs(d));
            xm[r] = fmax(xm[r], fabs(xj));
        }
    }
#pragma unroll
    for (int r = 0; r < K; ++r) {
        double v = block_max(dm[r], red);
        if (threadIdx.x == 0) part_d[(int64_t)blockIdx.x * K + r] = v;
        v = block_max(xm[r], red);
        if (threadIdx.x == 0) part_x[(int64_t)blockIdx.x * K + r] = v;
    }
}

// sc[r].dmax, sc[r].xmax = maxima over the partials of k_refine_update.
template <int K>
__global__ __launch_bounds__(kBlock) void k_refine_norms(const double* __restrict__ part_d,
                                                          const double* __restrict__ part_x,
                                                          int nblk, Scalars* __restrict__ sc)
{
    __shared__ double red[kWavesPerBlock];
    for (int r = 0; r < K; ++r) {
        double v = 0.0, w = 0.0;
        for (int k = threadIdx.x; k < nblk; k += kBlock) {
            v = fmax(v, part_d[(int64_t)k * K + r]);
            w = fmax(w, part_x[(int64_t)k * K + r]);
        }
        const double d = block_max(v, red);
        const double x = block_max(w, red);
        if (threadIdx.x == 0) {
            sc[r].dmax = d;
            sc[r].xmax = x;
        }
    }
}

// X[j][r] = 0 (row stride ldx), r < K
template <int K>
__global__ __launch_bounds__(kBlock) void k_zero_cols(int64_t n, double* __restrict__ X,
                                                       int64_t ldx)
{
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock)
#pragma unroll
        for (int r = 0; r < K; ++r) X[j * ldx + r] = 0.0;
}

// Fused iteration pass of a K-tile (the batched form of the single-RHS fused
// pass): per row, U~_r = Abar VP_r - coef_r U_r for every live RHS r, written
// with its FP64 sum of squares per workgroup (part[blk][K]), and the same
// registers scattered into Q += A^T U~ for the astrometric, instrumental and
// global columns. Frozen RHS keep U and contribute nothing. Dynamic LDS: the
// FP64 histogram [hcols][K] of instrumental columns [0, hcols) (the others
// are left to k_instr_tail), then the instrumental slice of VP (LDSX). In
// 1024-thread workgroups (128 registers per lane) a multi-RHS tile would
// reduce its star segments chunk by chunk instead of carrying 5K running sums;
// the tiles run in 512 or 256 threads, which have the registers. AM as in the single-RHS pass (kAttPre after
// k_att_dot over the tile's K right-hand sides). us (optional): a star-order
// copy of the new U~ (us[i K + r]) for the instrumental tail passes.
template <typename T, typename Acc, int K, int NT, bool LDSX, int AM, bool CIDX>
__global__ __launch_bounds__(NT) void k_fused(SysView s, const Acc* __restrict__ VP,
                                               const Acc* __restrict__ X3, Acc* __restrict__ U,
                                               Acc* __restrict__ Q, const int64_t* __restrict__ wb,
                                               Acc* __restrict__ gpart, double* __restrict__ part,
                                               int64_t hcols, const Scalars* __restrict__ sc,
                                               const int32_t* __restrict__ inv,
                                               Acc* __restrict__ us = nullptr)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ Acc gred[K * (NT / kWave)];
    __shared__ double sred[K * (NT / kWave)];
    const uint32_t live = live_mask<K>(sc);
    if (live == 0) return;
    const T* __restrict__ val = static_cast<const T*>(s.val);
    const int64_t m = s.m;
    const int64_t ninst = s.n_instr_cols;
    double* hist = reinterpret_cast<double*>(smem_raw);
    const Acc* xi = VP + s.instr_base * K;
    for (int64_t j = threadIdx.x; j < hcols * K; j += NT) hist[j] = 0.0;
    if (LDSX) {
        const int64_t off = (hcols * K * 8 + 15) & ~(int64_t)15;
        Acc* xl = reinterpret_cast<Acc*>(smem_raw + off);
        for (int64_t j = threadIdx.x; j < ninst * K; j += NT) xl[j] = xi[j];
        xi = xl;
    }
    __syncthreads();

    Acc coef[K], xg[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
        coef[r] = (Acc)sc[r].coef_u;
        xg[r] = VP[s.glob_base * K + r];
    }
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = (int64_t)blockIdx.x * (NT / kWave) + threadIdx.x / kWave;
    const int64_t rb = wb[wave], re = wb[wave + 1];
    Acc* __restrict__ qins = Q + s.instr_base * K;
    double ssq[K];
    Acc gsum[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
        ssq[r] = 0.0;
        gsum[r] = (Acc)0;
    }
    constexpr bool kChunkFlush = NT > 512 && K > 1;
    SegAcc<Acc, kChunkFlush ? 1 : kAstro * K> seg;
    auto astro_emit = [Q](int64_t star, const Acc (&tot)[kAstro * K]) {
        Acc* dst = Q + kAstro * star * K;
#pragma unroll
        for (int j = 0; j < kAstro * K; ++j) dst[j] += tot[j];
    };
    for (int64_t r0 = rb < re ? (rb & ~(int64_t)(kWave - 1)) : re; r0 < re; r0 += kWave) {
        const int64_t i = r0 + lane;
        const bool ok = i >= rb && i < re;
        const int64_t ic = i < rb ? rb : (i < re ? i : re - 1);
        const int64_t stc = star_of<CIDX>(s, ic);
        const int64_t st = i < re ? stc : kNoStar;
        const int64_t t = AM == kAttPre ? 0 : ldnt(&s.att[ic]);
        T a[kPar];
#pragma unroll
        for (int c = 0; c < kPar; ++c)
            if (AM != kAttPre || c < kOffAtt || c >= kOffInstr) a[c] = ldnt(&val[c * m + ic]);
        int32_t ix[kInstr];
#pragma unroll
        for (int j = 0; j < kInstr; ++j) ix[j] = instr_of<CIDX>(s, j, ic);

        const int64_t pu = inv ? (int64_t)ldnt(&inv[ic]) : ic;
        Acc d[K];
#pragma unroll
        for (int r = 0; r < K; ++r) d[r] = (Acc)0;
        const Acc* xa = VP + kAstro * stc * K;
#pragma unroll
        for (int j = 0; j < kAstro; ++j)
#pragma unroll
            for (int r = 0; r < K; ++r) d[r] += (Acc)a[j] * xa[j * K + r];
        if (AM != kAttPre) {
#pragma unroll
            for (int ax = 0; ax < kAxes; ++ax)
#pragma unroll
                for (int qq = 0; qq < kParAxis; ++qq) {
                    const Acc* xv = AM == kAttX3 ? X3 + (kAxes * (t + qq) + ax) * K
                                                 : VP + (s.att_base + ax * s.n_dfa + t + qq) * K;
                    const Acc av = (Acc)a[kOffAtt + ax * kParAxis + qq];
#pragma unroll
                    for (int r = 0; r < K; ++r) d[r] += av * xv[r];
                }
        }
#pragma unroll
        for (int j = 0; j < kInstr; ++j)
#pragma unroll
            for (int r = 0; r < K; ++r) d[r] += (Acc)a[kOffInstr + j] * xi[ix[j] * K + r];
#pragma unroll
        for (int r = 0; r < K; ++r) {
            d[r] += (Acc)a[kOffGlob] * xg[r];
            const bool on = ok && ((live >> r) & 1u);
            // kAttPre: U already holds the attitude part minus coef U
            const Acc nu = AM == kAttPre ? d[r] + U[pu * K + r] : d[r] - coef[r] * U[pu * K + r];
            if (on) U[pu * K + r] = nu;
            if (on && us) us[ic * K + r] = nu;
            d[r] = on ? nu : (Acc)0;
            ssq[r] += (double)d[r] * (double)d[r];
        }
        if (ok) {
#pragma unroll
            for (int j = 0; j < kInstr; ++j) {
                if (ix[j] >= hcols) continue;
                const Acc av = (Acc)a[kOffInstr + j];
#pragma unroll
                for (int r = 0; r < K; ++r) {
                    if (!((live >> r) & 1u)) continue;
                    atomicAdd(&hist[ix[j] * K + r], (double)(av * d[r]));
                }
            }
        }
#pragma unroll
        for (int r = 0; r < K; ++r) gsum[r] += (Acc)a[kOffGlob] * d[r];
        Acc pa[kAstro * K];
#pragma unroll
        for (int j = 0; j < kAstro; ++j)
#pragma unroll
            for (int r = 0; r < K; ++r) pa[j * K + r] = (Acc)a[j] * d[r];
        if (kChunkFlush) {
            seg_flush(st, pa, lane, astro_emit);
        } else {
            if constexpr (!kChunkFlush) seg_chunk(seg, st, pa, lane, astro_emit);
        }
    }
    if constexpr (!kChunkFlush) seg_finish(seg, lane, astro_emit);
#pragma unroll
    for (int r = 0; r < K; ++r) {
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            gsum[r] += __shfl_down(gsum[r], off);
            ssq[r] += __shfl_down(ssq[r], off);
        }
    }
    if (lane == 0)
#pragma unroll
        for (int r = 0; r < K; ++r) {
            gred[r * (NT / kWave) + threadIdx.x / kWave] = gsum[r];
            sred[r * (NT / kWave) + threadIdx.x / kWave] = ssq[r];
        }
    __syncthreads();
    if (threadIdx.x < K) {
        Acc g = (Acc)0;
        double q2 = 0.0;
        for (int k = 0; k < NT / kWave; ++k) {
            g += gred[threadIdx.x * (NT / kWave) + k];
            q2 += sred[threadIdx.x * (NT / kWave) + k];
        }
        gpart[(int64_t)blockIdx.x * K + threadIdx.x] = g;
        part[(int64_t)blockIdx.x * K + threadIdx.x] = q2;
    }
    for (int64_t j = threadIdx.x; j < hcols * K; j += NT) {
        const double v = hist[j];
        if (v != 0.0) atomicAdd(&qins[j], (Acc)v);
    }
}

// ---- right-hand sides across lanes (k_fused_rl)
// In this layout lane l of a wave handles row slot l / K and right-hand side
// l % K, so a wave steps over R = 64 / K rows at a time and every lane holds
// one RHS value, as in the single-RHS pass (registers do not grow with K).
// Sum over the R row slots of the lanes of one RHS (lanes equal mod K); the
// result is in every lane.
template <int K, typename V>
__device__ __forceinline__ V rhs_sum(V v)
{
#pragma unroll
    for (int off = K; off < kWave; off <<= 1) v += __shfl_xor(v, off);
    return v;
}

// Per-star segmented sums (SegAcc) in the RHS-across-lanes layout: the keys
// of the K lanes of a row slot are equal, segments are runs of row slots;
// emit(key, totals) runs on lanes 0..K-1 (lane j for RHS j) once per
// finished segment.
template <typename Acc, int K, typename Emit>
__device__ __forceinline__ void seg_chunk_rl(SegAcc<Acc, kAstro>& S, int64_t key,
                                             const Acc (&v)[kAstro], int lane, Emit&& emit)
{
    const bool cont = key == S.key;
#pragma unroll
    for (int j = 0; j < kAstro; ++j) S.acc[j] += cont ? v[j] : (Acc)0;
    uint64_t rest = __ballot(!cont);
    if (rest == 0) return;
    if (S.key >= 0) {
        Acc t[kAstro];
#pragma unroll
        for (int j = 0; j < kAstro; ++j) t[j] = rhs_sum<K>(S.acc[j]);
        if (lane < K) emit(S.key, t);
    }
    S.key = -1;
#pragma unroll
    for (int j = 0; j < kAstro; ++j) S.acc[j] = (Acc)0;
    while (rest != 0) {
        const int l0 = __ffsll((unsigned long long)rest) - 1;
        const int64_t k2 = __shfl(key, l0);
        if (k2 == kNoStar) break;
        const bool mine = key == k2;
        const uint64_t same = __ballot(mine);
        if ((same >> (kWave - 1)) & 1ull) {  // reaches the last row slot: stays open
            S.key = k2;
#pragma unroll
            for (int j = 0; j < kAstro; ++j) S.acc[j] = mine ? v[j] : (Acc)0;
            break;
        }
        Acc t[kAstro];
#pragma unroll
        for (int j = 0; j < kAstro; ++j) t[j] = rhs_sum<K>(mine ? v[j] : (Acc)0);
        if (lane < K) emit(k2, t);
        rest &= ~same;
    }
}

template <typename Acc, int K, typename Emit>
__device__ __forceinline__ void seg_finish_rl(SegAcc<Acc, kAstro>& S, int lane, Emit&& emit)
{
    if (S.key < 0) return;
    Acc t[kAstro];
#pragma unroll
    for (int j = 0; j < kAstro; ++j) t[j] = rhs_sum<K>(S.acc[j]);
    if (lane < K) emit(S.key, t);
    S.key = -1;
}

// Lane q of each group of K in {2, 4} lanes broadcast to the group (a quad
// permutation: lane p of a quad reads lane (p & ~(K - 1)) + q), in VALU
// cross-lane moves, without LDS. Every lane of the wave must be active.
template <int K, int Q>
__device__ __forceinline__ int32_t group_bcast(int32_t v)
{
    static_assert((K == 2 || K == 4) && Q < K, "groups of 2 or 4 lanes");
    constexpr int s0 = Q, s1 = Q, s2 = (K == 4 ? 0 : 2) + Q, s3 = s2;
    constexpr int ctrl = s0 | (s1 << 2) | (s2 << 4) | (s3 << 6);
    return __builtin_amdgcn_mov_dpp(v, ctrl, 0xf, 0xf, false);
}
template <int K, int Q, typename V>
__device__ __forceinline__ V group_bcast_v(V v)
{
    if constexpr (sizeof(V) == 8) {
        const int64_t b = __builtin_bit_cast(int64_t, v);
        const int32_t lo = group_bcast<K, Q>((int32_t)(b & 0xffffffff));
        const int32_t hi = group_bcast<K, Q>((int32_t)(b >> 32));
        return __builtin_bit_cast(V, (int64_t)(uint32_t)lo | ((int64_t)hi << 32));
    } else if constexpr (sizeof(V) == 4) {
        return __builtin_bit_cast(V, group_bcast<K, Q>(__builtin_bit_cast(int32_t, v)));
    } else {
        return (V)group_bcast<K, Q>((int32_t)v);
    }
}

constexpr int kNaRl = kAstro + kInstr + 1;  // coefficients outside the attitude section
template <int K>
constexpr int rl_nv() { return kNaRl / K; }                // value loads per lane (K = 2, 4)
template <int K>
constexpr int rl_ni() { return (kInstr + K - 1) / K; }     // index loads per lane
__device__ __forceinline__ constexpr int rl_col(int e)
{
    return e < kAstro ? e : kOffInstr + (e - kAstro);
}

// The loads of load_row_rl for K in {2, 4}, before the broadcast: lane r of a
// row slot loads entries r, r + K, ... of the 12 coefficients and 6 indices.
template <typename T, int K, bool CIDX>
__device__ __forceinline__ void load_raw_rl(const SysView& s, const T* __restrict__ val,
                                            int64_t ic, int rj, T (&tv)[rl_nv<K>()],
                                            int32_t (&ti)[rl_ni<K>()])
{
    static_assert(K == 2 || K == 4, "row slots of 2 or 4 lanes");
    const int64_t m = s.m;
#pragma unroll
    for (int t = 0; t < rl_nv<K>(); ++t) tv[t] = ldnt(&val[rl_col(t * K + rj) * m + ic]);
#pragma unroll
    for (int t = 0; t < rl_ni<K>(); ++t) {
        const int j = t * K + rj < kInstr ? t * K + rj : kInstr - 1;
        ti[t] = instr_of<CIDX>(s, j, ic);
    }
}

// The broadcast of load_row_rl: each loaded entry to the K lanes of its slot.
template <typename T, int K>
__device__ __forceinline__ void bcast_row_rl(const T (&tv)[rl_nv<K>()],
                                             const int32_t (&ti)[rl_ni<K>()], T (&a)[kPar],
                                             int32_t (&ix)[kInstr])
{
    constexpr int nv = rl_nv<K>(), ni = rl_ni<K>();
    auto col = [](int e) { return rl_col(e); };
#pragma unroll
    for (int t = 0; t < nv; ++t) {
        a[col(t * K + 0)] = group_bcast_v<K, 0>(tv[t]);
        a[col(t * K + 1)] = group_bcast_v<K, 1>(tv[t]);
        if constexpr (K == 4) {
            a[col(t * K + 2)] = group_bcast_v<K, 2>(tv[t]);
            a[col(t * K + 3)] = group_bcast_v<K, 3>(tv[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < ni; ++t) {
        if (t * K + 0 < kInstr) ix[t * K + 0] = group_bcast<K, 0>(ti[t]);
        if (t * K + 1 < kInstr) ix[t * K + 1] = group_bcast<K, 1>(ti[t]);
        if constexpr (K == 4) {
            if (t * K + 2 < kInstr) ix[t * K + 2] = group_bcast<K, 2>(ti[t]);
            if (t * K + 3 < kInstr) ix[t * K + 3] = group_bcast<K, 3>(ti[t]);
        }
    }
}

// The 12 coefficients of row ic outside the attitude section (astrometric,
// instrumental, global) and its 6 instrumental indices, loaded by the K lanes
// of its row slot together: lane r of the slot loads entries r, r + K, ...
// and each entry is then broadcast to the K lanes (K in {2, 4}); for other
// K every lane loads all of them.
template <typename T, int K, bool CIDX>
__device__ __forceinline__ void load_row_rl(const SysView& s, const T* __restrict__ val,
                                            int64_t ic, int rj, T (&a)[kPar],
                                            int32_t (&ix)[kInstr])
{
    if constexpr (K == 2 || K == 4) {
        T tv[rl_nv<K>()];
        int32_t ti[rl_ni<K>()];
        load_raw_rl<T, K, CIDX>(s, val, ic, rj, tv, ti);
        bcast_row_rl<T, K>(tv, ti, a, ix);
    } else {
        const int64_t m = s.m;
#pragma unroll
        for (int e = 0; e < kNaRl; ++e) a[rl_col(e)] = ldnt(&val[rl_col(e) * m + ic]);
#pragma unroll
        for (int j = 0; j < kInstr; ++j) ix[j] = instr_of<CIDX>(s, j, ic);
    }
}

// The fused pass of a K-tile after the attitude pre-pass (fused modes 2 and
// 3) with the K right-hand sides of a row in K lanes: per row and live RHS r,
// U~_r = (attitude part already in U) + the other sections' products with
// VP_r, written with its FP64 sum of squares, and the same value scattered
// into Q += A^T U~ for the astrometric (per-star segments), instrumental (LDS
// histogram [hcols][K], the rest to k_instr_tail) and global (partials
// gpart[blk][K]) columns. A2: aprod2 alone (Q += A^T U, U not changed, no
// sums of squares), the start of a tile's solve. U row i at U[inv[i] K + r].
// PIPE (K in {2, 4}, not A2): two row steps in flight per wave. A step waits
// for its coefficient, index, star and permutation loads, then for the
// gathers they address (U through inv, the astrometric and instrumental
// values of VP); the loads of the next step are issued before the gathers of
// the current one, so each step waits one round trip instead of two. Each
// step keeps its loads in its own registers (no copies, which would wait).
template <typename T, typename Acc, int K, int NT, bool LDSX, bool CIDX, bool A2,
          bool PIPE = false>
__global__ __launch_bounds__(NT) void k_fused_rl(SysView s, const Acc* __restrict__ VP,
                                                  Acc* __restrict__ U, Acc* __restrict__ Q,
                                                  const int64_t* __restrict__ wb,
                                                  Acc* __restrict__ gpart,
                                                  double* __restrict__ part, int64_t hcols,
                                                  const Scalars* __restrict__ sc,
                                                  const int32_t* __restrict__ inv)
{
    constexpr int R = kWave / K;  // row slots of a wave
    constexpr int W = NT / kWave;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ Acc gred[W * K];
    __shared__ double sred[W * K];
    uint32_t live = 0;
#pragma unroll
    for (int r = 0; r < K; ++r)
        live |= ((sc[r].done || (A2 && sc[r].beta_zero)) ? 0u : 1u) << r;
    if (live == 0) return;
    const T* __restrict__ val = static_cast<const T*>(s.val);
    const int64_t ninst = s.n_instr_cols;
    double* hist = reinterpret_cast<double*>(smem_raw);
    const Acc* xi = VP + s.instr_base * K;
    for (int64_t e = threadIdx.x; e < hcols * K; e += NT) hist[e] = 0.0;
    if (LDSX && !A2) {
        const int64_t off = (hcols * K * 8 + 15) & ~(int64_t)15;
        Acc* xl = reinterpret_cast<Acc*>(smem_raw + off);
        for (int64_t e = threadIdx.x; e < ninst * K; e += NT) xl[e] = xi[e];
        xi = xl;
    }
    __syncthreads();

    const int lane = threadIdx.x & (kWave - 1);
    const int rj = lane & (K - 1);    // this lane's right-hand side
    const int slot = lane / K;        // and row slot
    const bool lj = (live >> rj) & 1u;
    const Acc xg = A2 ? (Acc)0 : VP[s.glob_base * K + rj];
    const int64_t wave = (int64_t)blockIdx.x * W + threadIdx.x / kWave;
    const int64_t rb = wb[wave], re = wb[wave + 1];
    Acc* __restrict__ qins = Q + s.instr_base * K;
    double ssq = 0.0;
    Acc gsum = (Acc)0;
    SegAcc<Acc, kAstro> seg;
    auto astro_emit = [Q, lane](int64_t star, const Acc (&tot)[kAstro]) {
        Acc* dst = Q + kAstro * star * K + lane;
#pragma unroll
        for (int j = 0; j < kAstro; ++j) dst[j * K] += tot[j];
    };
    // one R-row step: the row of slot `slot` (clamped), its coefficients,
    // indices, star and place in U already loaded
    auto step = [&](int64_t r0, int64_t stc, const T (&a)[kPar], const int32_t (&ix)[kInstr],
                    int64_t pu) {
        const int64_t i = r0 + slot;
        const bool ok = i >= rb && i < re;
        const int64_t st = i < re ? stc : kNoStar;
        const Acc uo = U[pu * K + rj];
        const bool on = ok && lj;
        Acc d;
        if (A2) {
            d = on ? uo : (Acc)0;
        } else {
            // Eq. (2): the row's non-attitude products with VP_r, added to
            // the attitude part the pre-pass left in U
            Acc dot = (Acc)0;
            const Acc* xa = VP + kAstro * stc * K + rj;
#pragma unroll
            for (int j = 0; j < kAstro; ++j) dot += (Acc)a[j] * xa[j * K];
#pragma unroll
            for (int j = 0; j < kInstr; ++j) dot += (Acc)a[kOffInstr + j] * xi[ix[j] * K + rj];
            dot += (Acc)a[kOffGlob] * xg;
            const Acc nu = dot + uo;
            if (on) U[pu * K + rj] = nu;
            d = on ? nu : (Acc)0;
            ssq += (double)d * (double)d;
        }
        // Eq. (3) with the new value, attitude columns excluded
        if (on) {
#pragma unroll
            for (int j = 0; j < kInstr; ++j)
                if (ix[j] < hcols)
                    atomicAdd(&hist[ix[j] * K + rj], (double)((Acc)a[kOffInstr + j] * d));
        }
        gsum += (Acc)a[kOffGlob] * d;
        Acc pa[kAstro];
#pragma unroll
        for (int j = 0; j < kAstro; ++j) pa[j] = (Acc)a[j] * d;
        seg_chunk_rl<Acc, K>(seg, st, pa, lane, astro_emit);
    };
    // R-row steps aligned to R rows (every coefficient stream read in whole
    // R-row pieces); slots outside [rb, re) use a clamped row and contribute
    // nothing
    auto row_of = [&](int64_t r0) {
        const int64_t i = r0 + slot;
        return i < rb ? rb : (i < re ? i : re - 1);
    };
    const int64_t rstart = rb < re ? (rb & ~(int64_t)(R - 1)) : re;
    if constexpr (PIPE && (K == 2 || K == 4) && !A2) {
        struct Raw {
            T tv[rl_nv<K>()];
            int32_t ti[rl_ni<K>()];
            int64_t stc, pu;
        };
        auto load = [&](Raw& w, int64_t r0) {
            const int64_t ic = row_of(r0);
            w.stc = star_of<CIDX>(s, ic);
            load_raw_rl<T, K, CIDX>(s, val, ic, rj, w.tv, w.ti);
            w.pu = inv ? (int64_t)ldnt(&inv[ic]) : ic;
        };
        auto run = [&](const Raw& w, int64_t r0) {
            T a[kPar];
            int32_t ix[kInstr];
            bcast_row_rl<T, K>(w.tv, w.ti, a, ix);
            step(r0, w.stc, a, ix, w.pu);
        };
        // r0, re and R are uniform over the wave, so are the branches
        if (rstart < re) {
            Raw A, B;
            int64_t r0 = rstart;
            load(A, r0);
            for (;;) {
                const int64_t r1 = r0 + R;
                if (r1 < re) load(B, r1);
                __builtin_amdgcn_sched_barrier(0);
                run(A, r0);
                __builtin_amdgcn_sched_barrier(0);
                if (r1 >= re) break;
                const int64_t r2 = r1 + R;
                if (r2 < re) load(A, r2);
                __builtin_amdgcn_sched_barrier(0);
                run(B, r1);
                __builtin_amdgcn_sched_barrier(0);
                if (r2 >= re) break;
                r0 = r2;
            }
        }
    } else {
        for (int64_t r0 = rstart; r0 < re; r0 += R) {
            const int64_t ic = row_of(r0);
            const int64_t stc = star_of<CIDX>(s, ic);
            T a[kPar];
            int32_t ix[kInstr];
            load_row_rl<T, K, CIDX>(s, val, ic, rj, a, ix);
            const int64_t pu = inv ? (int64_t)ldnt(&inv[ic]) : ic;
            step(r0, stc, a, ix, pu);
        }
    }
    seg_finish_rl<Acc, K>(seg, lane, astro_emit);
    gsum = rhs_sum<K>(gsum);
    ssq = rhs_sum<K>(ssq);
    if (lane < K) {
        gred[(threadIdx.x / kWave) * K + lane] = gsum;
        sred[(threadIdx.x / kWave) * K + lane] = ssq;
    }
    __syncthreads();
    if (threadIdx.x < K) {
        Acc g = (Acc)0;
        double q2 = 0.0;
        for (int w = 0; w < W; ++w) {
            g += gred[w * K + threadIdx.x];
            q2 += sred[w * K + threadIdx.x];
        }
        gpart[(int64_t)blockIdx.x * K + threadIdx.x] = g;
        if (!A2) part[(int64_t)blockIdx.x * K + threadIdx.x] = q2;
    }
    for (int64_t e = threadIdx.x; e < hcols * K; e += NT) {
        const double v = hist[e];
        if (v != 0.0) atomicAdd(&qins[e], (Acc)v);
    }
}

template <typename Acc, int K>
__global__ __launch_bounds__(kBlock) void k_glob_sum(const Acc* __restrict__ gpart, int nblk,
                                                      Acc* __restrict__ qglob,
                                                      const Scalars* __restrict__ sc)
{
    __shared__ double red[kWavesPerBlock];
    for (int r = 0; r < K; ++r) {
        if (sc[r].done || sc[r].beta_zero) continue;  // uniform over the block
        double v = 0.0;
        for (int k = threadIdx.x; k < nblk; k += kBlock) v += (double)gpart[(int64_t)k * K + r];
        const double tot = block_sum(v, red);
        if (threadIdx.x == 0) qglob[r] = (Acc)((double)qglob[r] + tot);
    }
}

// V~ = p Q / beta_r - beta_r V ; Q = 0 ; alpha^2 partials per RHS.
template <typename Acc, int K>
__global__ __launch_bounds__(kBlock) void k_col_a(int64_t n, const double* __restrict__ p,
                                                   Acc* __restrict__ Q, double* __restrict__ V,
                                                   const Scalars* __restrict__ sc,
                                                   double* __restrict__ part)
{
    __shared__ double red[K * kWavesPerBlock];
    double beta[K], ib[K], ssq[K];
    uint32_t act = 0;
#pragma unroll
    for (int r = 0; r < K; ++r) {
        beta[r] = sc[r].beta;
        ib[r] = beta[r] > 0.0 ? 1.0 / beta[r] : 0.0;
        ssq[r] = 0.0;
        act |= ((sc[r].done || sc[r].beta_zero) ? 0u : 1u) << r;
    }
    if (act == 0) return;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock) {
        const double pj = p[j];
#pragma unroll
        for (int r = 0; r < K; ++r) {
            if (!((act >> r) & 1u)) continue;
            const double qj = (double)Q[j * K + r];
            Q[j * K + r] = (Acc)0;
            const double vt = pj * qj * ib[r] - beta[r] * V[j * K + r];
            V[j * K + r] = vt;
            ssq[r] += vt * vt;
        }
    }
    block_sums_k<K>(ssq, part, red);
}

template <typename VP, int K>
__global__ __launch_bounds__(kBlock) void k_col_b(int64_t n, const double* __restrict__ p,
                                                   double* __restrict__ V, double* __restrict__ W,
                                                   double* __restrict__ Y, VP* __restrict__ VPv,
                                                   const Scalars* __restrict__ sc,
                                                   double* __restrict__ part_dd,
                                                   double* __restrict__ part_xx)
{
    __shared__ double red[K * kWavesPerBlock];
    double ia[K], t1[K], t2[K], ir[K], dd[K], xx[K];
    uint32_t act = 0;
#pragma unroll
    for (int r = 0; r < K; ++r) {
        ia[r] = sc[r].beta_zero ? 1.0 : sc[r].inv_alpha;
        t1[r] = sc[r].t1;
        t2[r] = sc[r].t2;
        ir[r] = 1.0 / sc[r].rho;
        dd[r] = 0.0;
        xx[r] = 0.0;
        act |= (sc[r].done ? 0u : 1u) << r;
    }
    if (act == 0) return;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock) {
        const double pj = p[j];
#pragma unroll
        for (int r = 0; r < K; ++r) {
            if (!((act >> r) & 1u)) continue;
            const int64_t o = j * K + r;
            const double vj = V[o] * ia[r];
            V[o] = vj;
            VPv[o] = (VP)(pj * vj);
            const double wj = W[o];
            const double dk = wj * ir[r];
            dd[r] += dk * dk;
            const double yj = Y[o] + t1[r] * wj;
            Y[o] = yj;
            xx[r] += yj * yj;
            W[o] = vj + t2[r] * wj;
        }
    }
    block_sums_k<K>(dd, part_dd, red);
    block_sums_k<K>(xx, part_xx, red);
}

template <typename VP, int K>
__global__ __launch_bounds__(kBlock) void k_col_init(int64_t n, const double* __restrict__ p,
                                                      double* __restrict__ V,
                                                      double* __restrict__ W,
                                                      double* __restrict__ Y,
                                                      VP* __restrict__ VPv,
                                                      const Scalars* __restrict__ sc)
{
    double ia[K];
#pragma unroll
    for (int r = 0; r < K; ++r) ia[r] = sc[r].inv_alpha;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock) {
        const double pj = p[j];
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const int64_t o = j * K + r;
            const double vj = V[o] * ia[r];
            V[o] = vj;
            W[o] = vj;
            VPv[o] = (VP)(pj * vj);
            Y[o] = 0.0;
        }
    }
}

// X[j][r] (row stride ldx) = p_j Y[j][r]
template <int K>
__global__ __launch_bounds__(kBlock) void k_unprecond(int64_t n, const double* __restrict__ p,
                                                       const double* __restrict__ Y,
                                                       double* __restrict__ X, int64_t ldx)
{
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock) {
        const double pj = p[j];
#pragma unroll
        for (int r = 0; r < K; ++r) X[j * ldx + r] = pj * Y[j * K + r];
    }
}

// Sum of column r of part[nblk][K], one block, fixed order; thread 0.
template <int K>
__device__ __forceinline__ double sum_col(const double* part, int nblk, int r, double* lds)
{
    double v = 0.0;
    for (int k = threadIdx.x; k < nblk; k += kBlock) v += part[(int64_t)k * K + r];
    return block_sum(v, lds);
}

// The single-RHS scalar steps applied per RHS. Each kernel loops over the K
// RHS of the tile (uniformly over the block) and skips frozen ones.
template <int K>
__global__ __launch_bounds__(kBlock) void k_scalar_init_beta(const double* __restrict__ part,
                                                              int nblk, Scalars* __restrict__ sc)
{
    __shared__ double red[kWavesPerBlock];
    for (int r = 0; r < K; ++r) {
        const double ssq = sum_col<K>(part, nblk, r, red);
        if (threadIdx.x == 0) {
            Scalars& s = sc[r];
            const double beta = sqrt(ssq);
            s.beta = beta;
            s.bnorm = beta;
            s.alpha = s.anorm = s.ddnorm = s.acond = s.xnorm = s.arnorm = 0.0;
            s.rnorm = beta;
            s.inv_alpha = 1.0;
            s.itn = 0;
            s.istop = 0;
            s.beta_zero = 0;
            s.done = beta > 0.0 ? 0 : 1;
        }
    }
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_scalar_init_alpha(const double* __restrict__ part,
                                                               int nblk, Scalars* __restrict__ sc)
{
    __shared__ double red[kWavesPerBlock];
    for (int r = 0; r < K; ++r) {
        const double ssq = sum_col<K>(part, nblk, r, red);
        if (threadIdx.x == 0 && !sc[r].done) {
            Scalars& s = sc[r];
            const double alpha = sqrt(ssq);
            s.alpha = alpha;
            s.rhobar = alpha;
            s.phibar = s.beta;
            s.arnorm = alpha * s.beta;
            s.arnorm0 = s.arnorm;
            s.inv_alpha = alpha > 0.0 ? 1.0 / alpha : 1.0;
            s.coef_u = alpha / s.beta;
            if (s.arnorm == 0.0) s.done = 1;
        }
    }
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_scalar_beta(const double* __restrict__ part, int nblk,
                                                         Scalars* __restrict__ sc)
{
    __shared__ double red[kWavesPerBlock];
    for (int r = 0; r < K; ++r) {
        if (sc[r].done) continue;
        const double ssq = sum_col<K>(part, nblk, r, red);
        if (threadIdx.x == 0) {
            Scalars& s = sc[r];
            const double beta = sqrt(ssq);
            s.beta = beta;
            if (beta > 0.0) {
                s.anorm = sqrt(s.anorm * s.anorm + s.alpha * s.alpha + beta * beta);
                s.beta_zero = 0;
            } else {
                s.beta_zero = 1;
            }
        }
    }
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_scalar_alpha(const double* __restrict__ part,
                                                          int nblk, Scalars* __restrict__ sc)
{
    __shared__ double red[kWavesPerBlock];
    for (int r = 0; r < K; ++r) {
        if (sc[r].done) continue;
        const double ssq = sum_col<K>(part, nblk, r, red);
        if (threadIdx.x == 0) {
            Scalars& s = sc[r];
            double alpha = s.alpha;
            if (!s.beta_zero) alpha = sqrt(ssq);
            const double beta = s.beta;
            const double rho = sqrt(s.rhobar * s.rhobar + beta * beta);
            const double c = s.rhobar / rho;
            const double sn = beta / rho;
            const double theta = sn * alpha;
            const double phi = c * s.phibar;
            s.alpha = alpha;
            s.rho = rho;
            s.c = c;
            s.s = sn;
            s.theta = theta;
            s.rhobar = -c * alpha;
            s.phi = phi;
            s.phibar = sn * s.phibar;
            s.t1 = phi / rho;
            s.t2 = -theta / rho;
            s.inv_alpha = alpha > 0.0 ? 1.0 / alpha : 1.0;
            s.coef_u = beta > 0.0 ? alpha / beta : 0.0;
            s.rnorm = s.phibar;
            s.arnorm = alpha * fabs(c) * s.phibar;
        }
    }
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_scalar_stop(const double* __restrict__ part_dd,
                                                         const double* __restrict__ part_xx,
                                                         int nblk, Scalars* __restrict__ sc)
{
    __shared__ double red[kWavesPerBlock];
    for (int r = 0; r < K; ++r) {
        if (sc[r].done) continue;
        const double dd = sum_col<K>(part_dd, nblk, r, red);
        const double xx = sum_col<K>(part_xx, nblk, r, red);
        if (threadIdx.x == 0) {
            Scalars& s = sc[r];
            const double ddnorm = s.ddnorm + dd;
            const double xnorm = sqrt(xx);
            const double anorm = s.anorm;
            const double acond = anorm * sqrt(ddnorm);
            const double rnorm = s.rnorm, arnorm = s.arnorm, bnorm = s.bnorm;
            s.ddnorm = ddnorm;
            s.xnorm = xnorm;
            s.acond = acond;
            const int32_t itn = s.itn + 1;
            s.itn = itn;
            const double test1 = rnorm / bnorm;
            const double test2 = (anorm * rnorm) > 0.0 ? arnorm / (anorm * rnorm) : 0.0;
            const double test3 = acond > 0.0 ? 1.0 / acond : 0.0;
            const double t1 = test1 / (1.0 + anorm * xnorm / bnorm);
            const double rtol = s.btol + s.atol * anorm * xnorm / bnorm;
            int32_t istop = 0;
            if (itn >= s.itn_limit) istop = 7;
            if (s.tests) {
                if (1.0 + test3 <= 1.0) istop = 6;
                if (1.0 + test2 <= 1.0) istop = 5;
                if (1.0 + t1 <= 1.0) istop = 4;
                if (test3 <= s.ctol) istop = 3;
                if (test2 <= s.atol) istop = 2;
                if (test1 <= rtol) istop = 1;
            }
            // relative normal-equation test of a refinement's inner solve
            if (s.rel_ar > 0.0 && arnorm <= s.rel_ar * s.arnorm0) istop = 2;
            s.istop = istop;
            if (istop != 0) s.done = 1;
        }
    }
}

template <int K>
__global__ void k_all_done(Scalars* __restrict__ sc, int32_t* __restrict__ flag)
{
    if (threadIdx.x != 0) return;
    int32_t all = 1;
    for (int r = 0; r < K; ++r) all &= sc[r].done ? 1 : 0;
    *flag = all;
}

}  // namespace batched
}  // namespace avugsr
