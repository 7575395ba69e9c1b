// On-GPU twin of the seeded synthetic-system generator: the same gen_core.h
// draws as the host generator (synth.c), one row per thread, written straight
// into the device-resident structure-of-arrays layout. Bit-identical to the
// host output (tests/test_synth_gpu.py). Input plumbing only.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gen_core.h"

namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void k_star_of_row(const int64_t* __restrict__ first_row,
                                                           int64_t n_stars, int64_t m,
                                                           int64_t* __restrict__ star)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * kThreads) {
        int64_t lo = 0, hi = n_stars;  // first_row[lo] <= i < first_row[hi]
        while (hi - lo > 1) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (first_row[mid] <= i) lo = mid;
            else hi = mid;
        }
        star[i] = lo;
    }
}

template <typename V>
__global__ __launch_bounds__(kThreads) void k_rows(uint64_t seed, int64_t r0, int64_t r1,
                                                    int64_t ld, synth_params P,
                                                    const int64_t* __restrict__ star,
                                                    V* __restrict__ values,
                                                    int64_t* __restrict__ att,
                                                    int32_t* __restrict__ instr)
{
    const int32_t n_par = P.n_astro + P.n_axes * P.n_par_axis + P.n_instr + P.n_glob;
    for (int64_t i = r0 + (int64_t)blockIdx.x * kThreads + threadIdx.x; i < r1;
         i += (int64_t)gridDim.x * kThreads) {
        const int64_t o = i - r0;
        double z[SYNTH_MAX_PAR];
        int32_t ins[SYNTH_MAX_INSTR];
        int64_t t;
        synth_row(seed, i, star[o], &P, z, &t, ins);
        att[o] = t;
        for (int32_t q = 0; q < P.n_instr; ++q) instr[(int64_t)q * ld + o] = ins[q];
        for (int32_t c = 0; c < n_par; ++c) values[(int64_t)c * ld + o] = (V)z[c];
    }
}

__global__ __launch_bounds__(kThreads) void k_normals(uint64_t seed, uint32_t stream, int64_t i0,
                                                       int64_t i1, double sigma,
                                                       double* __restrict__ out)
{
    for (int64_t i = i0 + (int64_t)blockIdx.x * kThreads + threadIdx.x; i < i1;
         i += (int64_t)gridDim.x * kThreads)
        out[i - i0] = synth_normal_at(seed, stream, i, sigma);
}

int grid_for(int64_t n)
{
    const int64_t g = (n + kThreads - 1) / kThreads;
    return (int)(g < 65536 ? (g > 0 ? g : 1) : 65536);
}

int status(hipError_t e) { return e == hipSuccess ? 0 : (int)e; }

}  // namespace

extern "C" {

// star[i] for rows [0, m) from first_row[0..n_stars] (device arrays).
int synth_gpu_star_of_row(const int64_t* first_row, int64_t n_stars, int64_t m, int64_t* star,
                          void* stream)
{
    hipLaunchKernelGGL(k_star_of_row, dim3(grid_for(m)), dim3(kThreads), 0,
                       (hipStream_t)stream, first_row, n_stars, m, star);
    return status(hipGetLastError());
}

// Rows [r0, r1) into device SoA arrays with row stride ld, indexed at i - r0;
// star is indexed the same way. value_kind 0: double, 1: float.
int synth_gpu_rows(uint64_t seed, int64_t r0, int64_t r1, int64_t ld, const int64_t* star,
                   int32_t n_astro, int32_t n_axes, int32_t n_par_axis, int64_t n_dfa,
                   int32_t n_instr, int64_t n_instr_cols, int32_t n_glob, double scale_lo,
                   double scale_hi, double corr, int32_t value_kind, void* values, int64_t* att,
                   int32_t* instr, void* stream)
{
    synth_params P;
    P.n_astro = n_astro;
    P.n_axes = n_axes;
    P.n_par_axis = n_par_axis;
    P.n_instr = n_instr;
    P.n_glob = n_glob;
    P.value_kind = value_kind;
    P.n_dfa = n_dfa;
    P.n_instr_cols = n_instr_cols;
    P.scale_lo = scale_lo;
    P.scale_hi = scale_hi;
    P.corr = corr;
    if (n_astro + n_axes * n_par_axis + n_instr + n_glob > SYNTH_MAX_PAR || n_instr > SYNTH_MAX_INSTR)
        return -1;
    const int g = grid_for(r1 - r0);
    if (value_kind == 0)
        hipLaunchKernelGGL((k_rows<double>), dim3(g), dim3(kThreads), 0, (hipStream_t)stream, seed,
                           r0, r1, ld, P, star, (double*)values, att, instr);
    else
        hipLaunchKernelGGL((k_rows<float>), dim3(g), dim3(kThreads), 0, (hipStream_t)stream, seed,
                           r0, r1, ld, P, star, (float*)values, att, instr);
    return status(hipGetLastError());
}

// out[i - i0] = sigma * N(0,1) draw i of `stream_id` for i in [i0, i1).
int synth_gpu_normals(uint64_t seed, uint32_t stream_id, int64_t i0, int64_t i1, double sigma,
                      double* out, void* stream)
{
    hipLaunchKernelGGL(k_normals, dim3(grid_for(i1 - i0)), dim3(kThreads), 0,
                       (hipStream_t)stream, seed, stream_id, i0, i1, sigma, out);
    return status(hipGetLastError());
}

}  // extern "C"
