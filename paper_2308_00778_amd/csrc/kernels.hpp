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
//                   attitude: scatter-add with device atomics;
//                   instrumental: workgroup-private LDS histogram, flushed
//                     once per workgroup;
//                   global: wave shuffle -> LDS -> per-workgroup partial,
//                     summed in a deterministic second stage (k_glob_sum).
//   k_col_a/b     column-vector updates of the LSQR step (FP64).
//   k_scalar_*    single-workgroup kernels: norm finishers, Givens rotation,
//                 estimates and stopping tests, all FP64.
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
};

// LSQR state kept on the device so that a whole iteration runs without a
// host round trip (and can be captured into a graph).
struct Scalars {
    double alpha, beta, rhobar, phibar, bnorm;
    double anorm, ddnorm, xnorm, rnorm, arnorm, acond;
    double rho, c, s, theta, phi;
    double t1, t2, inv_alpha, coef_u;
    double atol, btol, ctol;
    double dmax, xmax;  // refinement: ||d||_inf, ||x||_inf of the last outer step
    int32_t itn, itn_limit, istop, done;
    int32_t tests, beta_zero, pad0, pad1;
};

template <typename T>
__device__ __forceinline__ T ldnt(const T* p)
{
    return __builtin_nontemporal_load(p);
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
template <typename T, typename Acc, typename VX>
__device__ __forceinline__ Acc row_dot(const SysView& s, const VX* __restrict__ x, int64_t i)
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
        const VX* xt = x + s.att_base + ax * s.n_dfa + t;
#pragma unroll
        for (int q = 0; q < kParAxis; ++q) sum += (Acc)a[kOffAtt + ax * kParAxis + q] * (Acc)xt[q];
    }
    const VX* xi = x + s.instr_base;
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
// RESID modes).
template <typename T, typename Acc, typename VX, typename VY, int MODE>
__global__ __launch_bounds__(kBlock) void k_aprod1(SysView s, const VX* __restrict__ x,
                                                    VY* __restrict__ y,
                                                    const double* __restrict__ b,
                                                    const Scalars* __restrict__ sc,
                                                    double* __restrict__ part)
{
    __shared__ double red[kWavesPerBlock];
    if (MODE == A1_LSQR && sc->done) return;
    const Acc coef = (MODE == A1_LSQR) ? (Acc)sc->coef_u : (Acc)0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    double ssq = 0.0;
    for (int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x; i0 < s.m; i0 += 2 * stride) {
        const int64_t i1 = i0 + stride;
        const bool has1 = i1 < s.m;
        const int64_t i1c = has1 ? i1 : i0;
        const Acc d0 = row_dot<T, Acc, VX>(s, x, i0);
        const Acc d1 = row_dot<T, Acc, VX>(s, x, i1c);
        if (MODE == A1_ACCUM) {
            y[i0] = (VY)((Acc)y[i0] + d0);
            if (has1) y[i1] = (VY)((Acc)y[i1] + d1);
        } else if (MODE == A1_LSQR) {
            const VY n0 = (VY)(d0 - coef * (Acc)y[i0]);
            y[i0] = n0;
            ssq += (double)n0 * (double)n0;
            if (has1) {
                const VY n1 = (VY)(d1 - coef * (Acc)y[i1]);
                y[i1] = n1;
                ssq += (double)n1 * (double)n1;
            }
        } else {
            const VY n0 = (VY)((Acc)b[i0] - d0);
            y[i0] = n0;
            ssq += (double)n0 * (double)n0;
            if (has1) {
                const VY n1 = (VY)((Acc)b[i1] - d1);
                y[i1] = n1;
                ssq += (double)n1 * (double)n1;
            }
        }
    }
    if (MODE != A1_ACCUM) {
        const double r = block_sum(ssq, red);
        if (threadIdx.x == 0) part[blockIdx.x] = r;
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

// x += A^T y (SQUARE: x_j += sum of squared coefficients of column j, used
// for the column norms). wb: star-aligned row boundaries, one range per wave
// (gridDim.x * kWavesPerBlock ranges). The instrumental columns are
// accumulated in LDS when lds_instr != 0 (n_instr_cols * sizeof(Acc) bytes of
// dynamic shared memory), else by device atomics. gpart[blockIdx.x] gets the
// workgroup's global-column partial; k_glob_sum adds them up.
template <typename T, typename Acc, typename VU, bool SQUARE>
__global__ __launch_bounds__(kBlock) void k_aprod2(SysView s, const VU* __restrict__ u,
                                                    Acc* __restrict__ q,
                                                    const int64_t* __restrict__ wb,
                                                    Acc* __restrict__ gpart, int lds_instr,
                                                    const Scalars* __restrict__ sc)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Acc* lds = reinterpret_cast<Acc*>(smem_raw);
    __shared__ Acc gred[kWavesPerBlock];
    if (sc != nullptr && (sc->done || sc->beta_zero)) return;

    const T* __restrict__ val = static_cast<const T*>(s.val);
    const int64_t m = s.m;
    const int64_t ninst = s.n_instr_cols;
    if (lds_instr) {
        for (int64_t j = threadIdx.x; j < ninst; j += kBlock) lds[j] = (Acc)0;
        __syncthreads();
    }

    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t rb = wb[wave], re = wb[wave + 1];
    Acc* __restrict__ qatt = q + s.att_base;
    Acc* __restrict__ qins = q + s.instr_base;

    int64_t carry_star = -1;
    Acc carry[kAstro];
#pragma unroll
    for (int j = 0; j < kAstro; ++j) carry[j] = (Acc)0;
    Acc gsum = (Acc)0;

    for (int64_t r0 = rb; r0 < re; r0 += kWave) {
        const int64_t i = r0 + lane;
        const bool ok = i < re;
        const int64_t ic = ok ? i : re - 1;
        const int64_t st = ok ? ldnt(&s.star[ic]) : kNoStar;
        const int64_t t = ldnt(&s.att[ic]);
        T a[kPar];
#pragma unroll
        for (int c = 0; c < kPar; ++c) a[c] = ldnt(&val[c * m + ic]);
        int32_t ix[kInstr];
#pragma unroll
        for (int j = 0; j < kInstr; ++j) ix[j] = ldnt(&s.instr[j * m + ic]);
        Acc ui = (Acc)0;
        if (!SQUARE) ui = ok ? (Acc)u[ic] : (Acc)0;

        Acc contrib[kPar];
#pragma unroll
        for (int c = 0; c < kPar; ++c)
            contrib[c] = SQUARE ? (ok ? (Acc)a[c] * (Acc)a[c] : (Acc)0) : (Acc)a[c] * ui;

        // attitude: 3 axes x 4 consecutive columns from the row's start t
        if (ok) {
#pragma unroll
            for (int ax = 0; ax < kAxes; ++ax) {
                Acc* dst = qatt + ax * s.n_dfa + t;
#pragma unroll
                for (int qq = 0; qq < kParAxis; ++qq)
                    atomicAdd(dst + qq, contrib[kOffAtt + ax * kParAxis + qq]);
            }
            // instrumental
#pragma unroll
            for (int j = 0; j < kInstr; ++j) {
                if (lds_instr) atomicAdd(&lds[ix[j]], contrib[kOffInstr + j]);
                else atomicAdd(&qins[ix[j]], contrib[kOffInstr + j]);
            }
        }
        gsum += contrib[kOffGlob];

        // astrometric: per-star segmented reduction across chunks
        Acc pa[kAstro];
#pragma unroll
        for (int j = 0; j < kAstro; ++j) pa[j] = contrib[j];
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

    // global column: wave shuffle -> LDS -> one partial per workgroup
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) gsum += __shfl_down(gsum, off);
    if (lane == 0) gred[threadIdx.x / kWave] = gsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        Acc g = (Acc)0;
        for (int k = 0; k < kWavesPerBlock; ++k) g += gred[k];
        gpart[blockIdx.x] = g;
    }
    // instrumental flush: one device atomic per column per workgroup
    if (lds_instr) {
        for (int64_t j = threadIdx.x; j < ninst; j += kBlock) {
            const Acc v = lds[j];
            if (v != (Acc)0) atomicAdd(&qins[j], v);
        }
    }
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
// partials of ||w/rho||^2 and ||y||^2.
template <typename VP>
__global__ __launch_bounds__(kBlock) void k_col_b(int64_t n, const double* __restrict__ p,
                                                   double* __restrict__ v,
                                                   double* __restrict__ w,
                                                   double* __restrict__ y, VP* __restrict__ vp,
                                                   const Scalars* __restrict__ sc,
                                                   double* __restrict__ part_dd,
                                                   double* __restrict__ part_xx)
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

// u~ = b (stored as VU) ; FP64 sum of squares of the stored values.
template <typename VU>
__global__ __launch_bounds__(kBlock) void k_copy_ssq(int64_t m, const double* __restrict__ b,
                                                      VU* __restrict__ u,
                                                      double* __restrict__ part)
{
    __shared__ double red[kWavesPerBlock];
    double ssq = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * kBlock) {
        const VU v = (VU)b[i];
        u[i] = v;
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
        const int64_t t = s.att[i];
        if (t < 0 || t > s.n_dfa - kParAxis) bad |= 4;
#pragma unroll
        for (int j = 0; j < kInstr; ++j) {
            const int32_t c = s.instr[j * s.m + i];
            if (c < 0 || (int64_t)c >= s.n_instr_cols) bad |= 8;
        }
    }
    if (bad) atomicOr(flag, bad);
}

// Star-aligned row boundaries: range g starts at the first star boundary at
// or after g*m/nw, so that no star is split between two waves.
__global__ __launch_bounds__(kBlock) void k_wave_bounds(const int64_t* __restrict__ star,
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

}  // namespace avugsr
