// Host side of the AVU-GSR LSQR library: handle, workspace, the LSQR
// iteration driven on one GPU, and the C ABI declared in include/lsqr.h.
//
// One LSQR iteration (Paige & Saunders 1982; the paper's Algorithm 1 loop) is
// eight kernels on one stream, with every scalar kept on the device:
//   aprod1      u~ <- A (p.*v) - (alpha/beta) u~      [+ ||u~||^2 partials]
//   beta        beta = ||u~||, anorm
//   aprod2      q  <- A^T u~                           [astro/att/instr/glob]
//   glob_sum    second stage of the global-column reduction
//   col_a       v~ = p.*q/beta - beta v               [+ ||v~||^2 partials]
//   alpha       alpha = ||v~||, plane rotation, estimates
//   col_b       v = v~/alpha, y += (phi/rho) w, w = v - (theta/rho) w
//   stop        ddnorm, xnorm, acond, stopping tests, itn
// u~ is the unnormalised left vector (u = u~/beta); keeping it unnormalised
// saves a pass over the row-sized vector per iteration. Preconditioning
// (column scaling by p, Sect. 2) is applied on the column vectors, so the
// borrowed matrix is never modified.
//
// Iterations are launched in chunks, replayed from a captured HIP graph; a
// finished solve leaves a `done` flag that makes the rest of the chunk a
// sequence of empty kernels. The host reads one flag per chunk.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.hpp"
#include "lsqr.h"

using namespace avugsr;

// Library-wide scratch of the no-allocation entry point (lsqr_aprod1_noalloc):
// the attitude section of x interleaved by axis, LSQR_NOALLOC_ATT_MAX doubles.
// Every GPU the library runs on holds its own copy at its own address until
// the process ends. Host code never passes this name to a kernel (on the host
// it only stands in for the symbol): it uses the per-device address taken
// with hipGetSymbolAddress in lsqr_create.
static __device__ __align__(256) double scratch[LSQR_NOALLOC_ATT_MAX];

namespace {

thread_local std::string g_last_error;

// Device address of `scratch` per device ordinal, taken once per device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

lsqr_status fail(lsqr_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(e_ == hipErrorOutOfMemory ? LSQR_E_NOMEM : LSQR_E_HIP,             \
                        "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__,   \
                        __LINE__);                                                         \
    } while (0)

#define LSQR_TRY(expr)                           \
    do {                                         \
        lsqr_status s_ = (expr);                 \
        if (s_ != LSQR_OK) return s_;            \
    } while (0)

template <typename V>
lsqr_status dalloc(V** p, int64_t count)
{
    *p = nullptr;
    if (count <= 0) count = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), (size_t)count * sizeof(V));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();  // a caller may free memory and try again
        return fail(e == hipErrorOutOfMemory ? LSQR_E_NOMEM : LSQR_E_HIP,
                    "hipMalloc of %lld bytes failed: %s", (long long)(count * sizeof(V)),
                    hipGetErrorString(e));
    }
    return LSQR_OK;
}

template <typename V>
void dfree(V*& p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// bytes of LDS for the instrumental histogram of aprod2 (gfx950 allows 160 KB
// per workgroup; a little is kept for the static arrays)
constexpr int64_t kLdsInstrBudget = 152 * 1024;
constexpr int64_t kLdsXBudget = 64 * 1024;      // bytes of LDS for aprod1's instrumental slice
constexpr int kBlock1 = 512;                    // aprod1 workgroup size
constexpr int kBlock2 = 1024;                   // aprod2 main-pass workgroup size
constexpr int kWavesPerCU = 16;                 // row ranges per compute unit in aprod2
// Rows per block of the two-level attitude sort: the block's slice of an FP64
// row vector (8 B/row) stays well inside the 256 MB last-level cache.
// Attitude buckets: as few as the FP64 LDS histogram of a bucket allows
// (3 x (W + 3) columns within kLdsInstrBudget), because the row-vector
// accesses of the star-order passes through inv cost more the more runs they
// split into (measured on 1e8 rows: +0.17 ms at 16 buckets, +0.65 ms at 25,
// +1.6 ms at 100).
constexpr int kAttBlock = 1024;  // attitude-pass workgroup (one per CU: the histogram fills LDS)
constexpr int kMaxTile = 16;     // right-hand sides of the widest k-tile

// Working vectors of one arithmetic precision of the LSQR loop.
template <typename Acc>
struct Path {
    Acc* u = nullptr;      // [m] unnormalised left vector u~
    Acc* vp = nullptr;     // [n] p .* v, gathered by aprod1
    Acc* q = nullptr;      // [n] aprod2 accumulator (zero between uses)
    Acc* gpart = nullptr;  // [nb2] global-column partials
    Acc* vp3 = nullptr;    // [3 n_dfa] attitude section of vp interleaved by axis
    Acc* datt = nullptr;   // [m] fused mode 3: attitude part of A vp in bucket order
    Acc* ustar = nullptr;  // [m] fused mode 2 with instrumental tail windows: u~ in star order
    int64_t hcols = 0;     // instrumental columns kept in the row passes' LDS histogram
    size_t lds = 0;        // dynamic LDS bytes of aprod2's main pass
    size_t lds_f = 0;      // dynamic LDS bytes of the fused pass
    int f_ldsx = 0;        // fused pass: instrumental slice of vp in LDS
    int64_t f_hcols = 0;   // fused pass: instrumental columns in its histogram
    bool ustar_tried = false;
    hipGraphExec_t graph = nullptr;
    int graph_chunk = 0;
    bool ready = false;
};

}  // namespace

struct lsqr_handle {
    SysView sv{};
    int generic = 0;  // row layout other than 5 + 3x4 + 6 + 1 (k_gen_* kernels)
    int value_type = LSQR_F64;
    int precondition = 1;
    int device = 0;
    int num_cu = 0;
    hipStream_t user_stream = nullptr;  // aprod1/aprod2 entry points
    hipStream_t stream = nullptr;       // solves (capturable, owned)

    int nb1 = 0;  // aprod1 grid
    int64_t nw = 0;  // star-aligned row ranges of aprod2, one per wave (multiple of 16)
    int nb2 = 0;     // aprod2 main-pass grid: nw / 16 workgroups of 1024 threads
    int nba = 0;     // reordered attitude pass grid: nw / 4 workgroups of 256 threads
    int nbc = 0;  // column-kernel grid

    int64_t* wb = nullptr;  // [nw + 1] row boundaries
    double* p = nullptr;    // [n] column scaling
    double* v = nullptr;    // [n]
    double* w = nullptr;    // [n]
    double* y = nullptr;    // [n] iterate in the scaled space
    double* part1 = nullptr;                    // [max(nb1, nb2) + 1]
    double* partc = nullptr;                    // [nbc]
    double* partdd = nullptr;                   // [nbc]
    double* partxx = nullptr;                   // [nbc]
    double* gpart_raw = nullptr;                // [nb2] FP64 partials of lsqr_aprod2
    int32_t* flag = nullptr;                    // validation flags

    // constraint rows (borrowed CSR, FP64 values) below the observation rows
    int64_t nc = 0, con_nnz = 0;
    const int64_t* con_rowptr = nullptr;
    const int64_t* con_col = nullptr;
    const double* con_val = nullptr;
    double* con_ssq = nullptr;  // [nc] squares of the new row-vector entries
    int con_grid = 0;           // workgroups of the constraint kernels
    Scalars* sc = nullptr;                      // device scalars
    Scalars* sc_host = nullptr;                 // pinned mirror

    Path<double> p64;
    Path<float> p32;

    // attitude bucket order (built on first use in attitude mode 1)
    int32_t* perm = nullptr;      // [m] rows in bucket order
    int32_t* invperm = nullptr;   // [m] bucket-order position of each row
    int32_t* tloc = nullptr;      // [m] attitude start minus its bucket's first start
    void* att_sorted = nullptr;   // [12][att_ld] attitude coefficients in bucket order
    int64_t att_ld = 0;           // its column stride: m rounded up to 64 rows
    int64_t* bstart = nullptr;    // [nbk + 1] first position of each bucket
    int64_t nbk = 0;              // buckets
    int64_t bwidth = 0;           // attitude starts per bucket (W)
    int att_g = 1;                // attitude-pass workgroups per bucket
    int64_t att_buckets = 0;      // requested bucket count (0: as few as fit)
    int att_rhs = 1;              // right-hand sides one attitude sweep must hold
    double* S2 = nullptr;         // [nbk att_g][3][W + 3] slices of the attitude pass
    double* x3_raw = nullptr;     // interleaved attitude section of lsqr_aprod1's x
    float* x3_raw32 = nullptr;    // the same for lsqr_aprod1_f32
    float* gpart_raw32 = nullptr; // global-column partials of lsqr_aprod2_f32
    bool att_ready = false;

    // variance estimate of the last lsqr_solve (LSQR_OPT_VARIANCE)
    double* var = nullptr;        // [n] sum of (w/rho)^2 in the scaled space
    int var_on = 0;               // accumulate during solves
    int var_valid = 0;            // var belongs to the last solve

    // batched right-hand sides (tile buffers for the largest K, reused per
    // tile): the FP64 tiles of lsqr_solve_batched and the FP32 inner tiles of
    // lsqr_solve_batched_refined (U, VP, Q, global partials and the
    // interleaved attitude copy in each precision; V, W, Y, partials and
    // scalars shared)
    struct Batch {
        int kmax = 0;
        bool has64 = false, has32 = false;
        double *U = nullptr, *V = nullptr, *W = nullptr, *Y = nullptr, *VP = nullptr, *Q = nullptr;
        double *gpart = nullptr, *part1 = nullptr, *partc = nullptr, *partdd = nullptr,
               *partxx = nullptr, *S2 = nullptr, *X3 = nullptr;
        float *U32 = nullptr, *VP32 = nullptr, *Q32 = nullptr, *gpart32 = nullptr, *X332 = nullptr;
        // 1-RHS tiles whose fused pass leaves instrumental tail windows: the
        // star-order copy of U the tails read (as the single-RHS path's
        // ustar), or null
        double* US1 = nullptr;
        float* US1_32 = nullptr;
        Scalars* sc = nullptr;
        int32_t* flag = nullptr;
        hipGraphExec_t graph[17] = {};    // FP64 tiles, by K
        int graph_chunk[17] = {};
        hipGraphExec_t graph32[17] = {};  // FP32 inner tiles, by K
        int graph32_chunk[17] = {};
        // autotuner: chosen k-tile per precision (0, 1) and per cap min(k, 8)
        // (index log2), and the measured ms per RHS-iteration by K of the last
        // tuning
        int tuned_k[2][5] = {};
        int last_tuned = 0;
        double tuned_ms[17] = {};
    } batch;

    // options
    double conlim = 1e8;
    int tests = 1;
    int chunk = 16;
    int use_graph = 1;
    int profile = 0;
    int att_mode = 1;    // 0: attitude scatter with device atomics, 1: bucket-order pass
    int astro_scan = 0;  // 1: segmented scan per chunk, 0: accumulate-and-flush segments
    int att_il = 1;      // aprod1 gathers attitude values from the interleaved copy
    int fused = 2;       // 1: one pass for aprod1 and the non-attitude part of aprod2;
                         // 2: the same with the attitude part of aprod1 in a bucket-order
                         // pre-pass (k_att_dot); 3: as 2 with the row vector in star
                         // order (pre-pass output gathered); 0: separate aprod1 and aprod2
    int last_mode = 0;   // fused mode of the last single-RHS solve
    int pipe = 1;        // bucket-order passes load the next row before storing the current
    int rhs_lanes = 1;   // k-tiles: the fused pass puts the K RHS of a row in K lanes
    int compact = 1;     // compact index copies for the fused passes when they fit
    int compact_tried = 0;
    int32_t* star32 = nullptr;    // [m] compact star index (or null)
    uint16_t* instr16 = nullptr;  // [6][m] compact instrumental indices (or null)
    double outer_tol = 1e-10;
    int ktile = 0;       // batched k-tile: 0 autotune, else 1, 2, 4 or 8

    // profiling
    std::vector<hipEvent_t> events;
    double ms1 = 0.0, ms2 = 0.0;
    int64_t n1 = 0, n2 = 0;
    double ms_pre = 0.0;  // profile: attitude pre-pass share of ms1 (fused mode 2)
};

namespace {

inline bool att_pass_on(const lsqr_handle* h) { return h->att_mode == 1 && h->sv.natt > 0; }

// The fused pass serves the default attitude mode (bucket-order pass).
inline bool use_fused(const lsqr_handle* h)
{
    return h->fused && att_pass_on(h) && !h->generic;
}

// Effective fused mode of a single-RHS iteration: 0 separate passes, 1 fused
// pass with the attitude dot product, 2 attitude pre-pass + fused pass, 3 the
// same with the row vector kept in star order.
inline int fused_mode(const lsqr_handle* h) { return use_fused(h) ? h->fused : 0; }

// Fused mode 3 keeps the single-RHS row vector in star order: the star-order
// pass reads and writes it sequentially, and the bucket-order passes reach it
// (or the pre-pass's separate output) through the permutation, read-only.
inline bool star_order_u(const lsqr_handle* h) { return fused_mode(h) == 3; }

// k-tiles of K >= 2 after the attitude pre-pass run the fused pass (and the
// first aprod2 of a solve) with the K right-hand sides of a row in K lanes
// (k_fused_rl), which the 16-RHS tile needs
inline bool rhs_lanes_on(const lsqr_handle* h) { return h->rhs_lanes && use_fused(h) && h->fused >= 2; }

// Partials of ||u||^2 that a scalar kernel sums: the row-pass partials plus,
// with constraint rows, their share stored right after them.
inline int n_part(const lsqr_handle* h, int nb) { return nb + (h->nc > 0 ? 1 : 0); }

// Placement of the single-RHS solver's row vector: bucket order in attitude
// mode 1 (row i at u[invperm[i]]) except in fused mode 3.
inline const int32_t* row_map(const lsqr_handle* h)
{
    return (att_pass_on(h) && !star_order_u(h)) ? h->invperm : nullptr;
}

// Placement of a batched k-tile's row vectors: bucket order in attitude mode 1.
inline const int32_t* batch_row_map(const lsqr_handle* h)
{
    return att_pass_on(h) ? h->invperm : nullptr;
}

inline int64_t att_span(const lsqr_handle* h) { return h->bwidth + kParAxis - 1; }
constexpr int kEvIter = 5;  // profile events per single-RHS iteration
inline int64_t att_slices(const lsqr_handle* h) { return h->nbk * h->att_g; }

// ------------------------------------------------------------ launch helpers
// Instrumental columns a row pass keeps in its FP64 LDS histogram for K
// right-hand sides; the remaining columns go to k_instr_tail windows.
inline int64_t instr_hcols(const lsqr_handle* h, int64_t K)
{
    if (h->sv.ni == 0) return 0;
    return std::min<int64_t>(h->sv.n_instr_cols, kLdsInstrBudget / (8 * K));
}

// Tail windows [hcols, n_instr_cols) of the instrumental part of Eq. (3), one
// launch per window of kLdsInstrBudget bytes (nothing when hcols covers all).
template <typename T, typename Acc, int K, bool SQUARE>
void launch_instr_tail(const lsqr_handle* h, const Acc* U, const int32_t* inv, Acc* Q,
                       int64_t hcols, const Scalars* sc, hipStream_t st)
{
    const int64_t ninst = h->sv.ni > 0 ? h->sv.n_instr_cols : 0;
    const int64_t tw = std::max<int64_t>(1, kLdsInstrBudget / (8 * K));
    // plain loads where the caller's instrumental columns are not line-aligned
    const uintptr_t vb = (uintptr_t)h->sv.val, ib = (uintptr_t)h->sv.instr;
    const bool lined = vb % 128 == 0 && ib % 128 == 0 &&
                       (h->sv.m * (int64_t)sizeof(T)) % 128 == 0 && (h->sv.m * 4) % 128 == 0;
    for (int64_t c0 = hcols; c0 < ninst; c0 += tw) {
        const int64_t c1 = std::min(ninst, c0 + tw);
        auto go = [&](auto gen, auto plain) {
            hipLaunchKernelGGL((k_instr_tail<T, Acc, K, SQUARE, kAttBlock, decltype(gen)::value,
                                             decltype(plain)::value>),
                               dim3(h->num_cu), dim3(kAttBlock), (size_t)((c1 - c0) * K * 8), st,
                               h->sv, U, inv, Q, c0, c1, sc);
        };
        using Y = std::true_type;
        using N = std::false_type;
        if (h->generic) {
            if (lined) go(Y(), N());
            else go(Y(), Y());
        } else {
            if (lined) go(N(), N());
            else go(N(), Y());
        }
    }
}

// LDS of a fused pass over K right-hand sides: the FP64 histogram of the
// first *hc instrumental columns and, when it fits beside it, the
// instrumental slice of the vector (vbytes per value and RHS; *ldsx = 1).
// When both do not fit, the histogram shrinks to leave room for the slice
// as long as the columns it leaves out fit two tail windows: gathering the
// slice from L2 costs more than a tail pass over the rows (1e8 rows, 2-RHS
// tiles: 140 -> 155 RHS-iterations/s; 1e9 rows, FP32 values, 30,000 columns:
// 74.7 -> 66.6 ms per pass with one more tail window).
inline size_t fused_lds_plan(const lsqr_handle* h, int64_t K, int64_t vbytes, int64_t* hc,
                             int* ldsx)
{
    *hc = instr_hcols(h, K);
    const int64_t hist = (*hc * K * 8 + 15) & ~(int64_t)15;
    const int64_t xbytes = h->sv.n_instr_cols * K * vbytes;
    *ldsx = 1;
    if (hist + xbytes <= kLdsInstrBudget) return (size_t)(hist + xbytes);
    const int64_t tw = std::max<int64_t>(1, kLdsInstrBudget / (8 * K));
    if (h->sv.ni > 0 && xbytes < kLdsInstrBudget) {
        const int64_t room = std::min<int64_t>(
            *hc, ((kLdsInstrBudget - xbytes) / (K * 8)) & ~(int64_t)63);
        if (room >= 64 && h->sv.n_instr_cols - room <= 2 * tw) {
            *hc = room;
            return (size_t)(room * K * 8 + xbytes);
        }
    }
    *ldsx = 0;
    return (size_t)(*hc * K * 8);
}

// Constraint rows of aprod1 (y, b: their entries, after the observation
// rows) and, except in A1_ACCUM, their share of ||u||^2 into part[0].
template <typename Acc, typename VX, typename VY, int MODE>
void launch_con_aprod1(const lsqr_handle* h, const VX* x, VY* y, const double* b,
                       const Scalars* sc, double* part, hipStream_t st)
{
    if (h->nc == 0) return;
    hipLaunchKernelGGL((k_con_aprod1<Acc, VX, VY, MODE>), dim3(h->con_grid), dim3(kBlock), 0, st,
                       h->nc, h->con_rowptr, h->con_col, h->con_val, x, y, b, sc, h->con_ssq);
    if (MODE != A1_ACCUM)
        hipLaunchKernelGGL(k_con_ssq, dim3(1), dim3(kBlock), 0, st, h->nc,
                           (const double*)h->con_ssq, part);
}

// Constraint rows of aprod2: q += A_con^T u (u: their entries).
template <typename Acc, typename VU>
void launch_con_aprod2(const lsqr_handle* h, const VU* u, Acc* q, const Scalars* sc,
                       hipStream_t st)
{
    if (h->nc == 0) return;
    hipLaunchKernelGGL((k_con_aprod2<Acc, VU, false>), dim3(h->con_grid), dim3(kBlock), 0, st,
                       h->nc, h->con_rowptr, h->con_col, h->con_val, u, q, sc);
}

// aprod1 with the instrumental slice of x staged in LDS when it fits.
// x3 (optional): interleaved attitude section of x, already written
// (k_interleave_att).
// inv (optional): placement of y (row i at y[inv[i]]). Constraint rows follow
// at y[m..] (b[m..]), their ||u||^2 share at part[nb1].
template <typename T, typename Acc, typename VX, typename VY, int MODE>
void launch_aprod1(const lsqr_handle* h, const VX* x, VY* y, const double* b, const Scalars* sc,
                   double* part, hipStream_t st, const int32_t* inv = nullptr,
                   const VX* x3 = nullptr)
{
    const int64_t m = h->sv.m;
    launch_con_aprod1<Acc, VX, VY, MODE>(h, x, y + m, b ? b + m : nullptr, sc,
                                         part ? part + h->nb1 : nullptr, st);
    if (h->generic) {  // any layout: runtime section sizes
        hipLaunchKernelGGL((k_gen_aprod1<T, Acc, VX, VY, MODE>), dim3(h->nb1), dim3(kBlock), 0, st,
                           h->sv, x, y, b, sc, part, inv);
        return;
    }
    const int64_t bytes = h->sv.n_instr_cols * (int64_t)sizeof(VX);
    const dim3 g(h->nb1), b1(kBlock1);
    if (bytes <= kLdsXBudget && x3)
        hipLaunchKernelGGL((k_aprod1<T, Acc, VX, VY, MODE, kBlock1, true, true>), g, b1,
                           (size_t)bytes, st, h->sv, x, y, b, sc, part, inv, x3);
    else if (bytes <= kLdsXBudget)
        hipLaunchKernelGGL((k_aprod1<T, Acc, VX, VY, MODE, kBlock1, true, false>), g, b1,
                           (size_t)bytes, st, h->sv, x, y, b, sc, part, inv, x3);
    else if (x3)
        hipLaunchKernelGGL((k_aprod1<T, Acc, VX, VY, MODE, kBlock1, false, true>), g, b1, 0, st,
                           h->sv, x, y, b, sc, part, inv, x3);
    else
        hipLaunchKernelGGL((k_aprod1<T, Acc, VX, VY, MODE, kBlock1, false, false>), g, b1, 0, st,
                           h->sv, x, y, b, sc, part, inv, x3);
}

template <typename V>
void launch_interleave_att(const lsqr_handle* h, const V* x, V* x3, const Scalars* sc,
                           hipStream_t st)
{
    hipLaunchKernelGGL((k_interleave_att<V>), dim3(h->nbc), dim3(kBlock), 0, st, x,
                       h->sv.att_base, h->sv.n_dfa, x3, sc);
}

// The fused pass (aprod1 and the astrometric, instrumental and global part of
// aprod2 in one sweep) over the main-pass grid.
template <typename T, typename Acc, bool LDSX, int AM>
void launch_fused_as(const lsqr_handle* h, Path<Acc>& P, const Acc* x3, hipStream_t st)
{
    // kAttGather reads the pre-pass output through invperm; u~ is in star order
    const int32_t* inv = AM == kAttGather ? (const int32_t*)h->invperm : row_map(h);
    const Acc* datt = AM == kAttGather ? (const Acc*)P.datt : nullptr;
    if (h->sv.star32)
        hipLaunchKernelGGL((k_fused<T, Acc, kBlock2, LDSX, AM, true>), dim3(h->nb2), dim3(kBlock2),
                           P.lds_f, st, h->sv, (const Acc*)P.vp, x3, P.u, P.q, h->wb, P.gpart,
                           h->part1, P.f_hcols, h->sc, inv, datt, P.ustar);
    else
        hipLaunchKernelGGL((k_fused<T, Acc, kBlock2, LDSX, AM, false>), dim3(h->nb2),
                           dim3(kBlock2), P.lds_f, st, h->sv, (const Acc*)P.vp, x3, P.u, P.q,
                           h->wb, P.gpart, h->part1, P.f_hcols, h->sc, inv, datt, P.ustar);
}

// Attitude part of aprod1 in bucket order (x3 must hold the interleaved
// attitude section of vp): folded into u~ in fused mode 2, written alone to
// the bucket-order vector datt in fused mode 3.
template <typename T, typename Acc, bool SEP, bool PIPE>
void launch_att_dot_as(const lsqr_handle* h, Path<Acc>& P, hipStream_t st)
{
    const size_t lds = (size_t)(kAxes * att_span(h)) * sizeof(Acc);
    hipLaunchKernelGGL((k_att_dot<T, Acc, 1, 1, kAttBlock, SEP, PIPE>), dim3(att_slices(h)),
                       dim3(kAttBlock), lds, st, h->att_ld, (const T*)h->att_sorted,
                       (const int32_t*)h->tloc, (const int64_t*)h->bstart, h->bwidth, h->att_g,
                       h->sv.n_dfa, (const Acc*)P.vp3, SEP ? P.datt : P.u, h->sc);
}

template <typename T, typename Acc>
void launch_att_dot(const lsqr_handle* h, Path<Acc>& P, hipStream_t st)
{
    if (star_order_u(h)) {
        if (h->pipe) launch_att_dot_as<T, Acc, true, true>(h, P, st);
        else launch_att_dot_as<T, Acc, true, false>(h, P, st);
    } else {
        if (h->pipe) launch_att_dot_as<T, Acc, false, true>(h, P, st);
        else launch_att_dot_as<T, Acc, false, false>(h, P, st);
    }
}

// pre: the attitude part of the row products is already in u~ (fused mode 2)
// or in datt (fused mode 3)
template <typename T, typename Acc>
void launch_fused(const lsqr_handle* h, Path<Acc>& P, hipStream_t st, bool pre)
{
    const Acc* x3 = h->att_il ? (const Acc*)P.vp3 : nullptr;
    if (pre && star_order_u(h)) {
        if (P.f_ldsx) launch_fused_as<T, Acc, true, kAttGather>(h, P, nullptr, st);
        else launch_fused_as<T, Acc, false, kAttGather>(h, P, nullptr, st);
    } else if (pre) {
        if (P.f_ldsx) launch_fused_as<T, Acc, true, kAttPre>(h, P, nullptr, st);
        else launch_fused_as<T, Acc, false, kAttPre>(h, P, nullptr, st);
    } else if (P.f_ldsx) {
        if (x3) launch_fused_as<T, Acc, true, kAttX3>(h, P, x3, st);
        else launch_fused_as<T, Acc, true, kAttX>(h, P, x3, st);
    } else {
        if (x3) launch_fused_as<T, Acc, false, kAttX3>(h, P, x3, st);
        else launch_fused_as<T, Acc, false, kAttX>(h, P, x3, st);
    }
    // the tail windows read u~ in star order when the fused pass wrote a copy
    if (P.ustar)
        launch_instr_tail<T, Acc, 1, false>(h, P.ustar, nullptr, P.q, P.f_hcols, h->sc, st);
    else
        launch_instr_tail<T, Acc, 1, false>(h, P.u, row_map(h), P.q, P.f_hcols, h->sc, st);
}

// Attitude part of aprod2 in bucket order: per-workgroup LDS histograms of
// each bucket's columns, then their sum. ub: the row vector in bucket order,
// or (gperm = perm) in star order, read through the permutation.
template <typename T, typename Acc>
void launch_att_pass(lsqr_handle* h, const Acc* ub, Acc* q, const Scalars* sc, hipStream_t st,
                     const int32_t* gperm)
{
    const size_t lds = (size_t)(kAxes * att_span(h) * 8);
    auto go = [&](auto gather, auto pipe) {
        hipLaunchKernelGGL((k_att_hist<T, Acc, 1, 1, kAttBlock, decltype(gather)::value,
                                       decltype(pipe)::value>),
                           dim3(att_slices(h)), dim3(kAttBlock), lds, st, h->att_ld,
                           (const T*)h->att_sorted, (const int32_t*)h->tloc,
                           (const int64_t*)h->bstart, h->bwidth, h->att_g, ub, h->S2, sc, gperm);
    };
    using Y = std::true_type;
    using N = std::false_type;
    if (gperm) {
        if (h->pipe) go(Y(), Y());
        else go(Y(), N());
    } else {
        if (h->pipe) go(N(), Y());
        else go(N(), N());
    }
    hipLaunchKernelGGL((k_att_reduce<Acc, 1>), dim3(h->nbc), dim3(kBlock), 0, st,
                       (const double*)h->S2, h->nbk, h->att_g, h->bwidth, h->sv.n_dfa,
                       q + h->sv.att_base, sc);
}

// q += A^T u for the LSQR loop (and lsqr_aprod2): the constraint rows (u[m..]),
// the main pass over the rows in star order (row i of u at u[inv[i]], or u[i]
// without inv), the
// global-column second stage and, in attitude mode 1, the attitude pass over
// ub, the same vector in bucket order (or in star order, read through gperm).
template <typename T, typename Acc>
void launch_aprod2(lsqr_handle* h, const Acc* u, const int32_t* inv, Acc* q, Acc* gpart,
                   int64_t hcols, const Scalars* sc, hipStream_t st, const Acc* ub,
                   const int32_t* gperm)
{
    const size_t lds = (size_t)(hcols * 8);
    const dim3 g(h->nb2), bm(kBlock2), b(kBlock);
    const bool att = !att_pass_on(h);
    launch_con_aprod2<Acc, Acc>(h, u + h->sv.m, q, sc, st);
    if (h->generic) {  // any layout: runtime section sizes, 256-thread workgroups
        if (att)
            hipLaunchKernelGGL((k_gen_aprod2<T, Acc, Acc, false, true>), dim3(h->nba), b, lds, st,
                               h->sv, u, q, h->wb, gpart, hcols, sc, inv);
        else
            hipLaunchKernelGGL((k_gen_aprod2<T, Acc, Acc, false, false>), dim3(h->nba), b, lds, st,
                               h->sv, u, q, h->wb, gpart, hcols, sc, inv);
        hipLaunchKernelGGL((k_gen_glob_sum<Acc>), dim3(1), b, 0, st, gpart, h->nba, h->sv.ng,
                           q + h->sv.glob_base, sc);
        launch_instr_tail<T, Acc, 1, false>(h, u, inv, q, hcols, sc, st);
        if (!att) launch_att_pass<T, Acc>(h, ub, q, sc, st, gperm);
        return;
    }
    if (att && h->astro_scan)
        hipLaunchKernelGGL((k_aprod2<T, Acc, Acc, false, true, true, kBlock2>), g, bm, lds, st, h->sv,
                           u, q, h->wb, gpart, hcols, sc, inv);
    else if (att)
        hipLaunchKernelGGL((k_aprod2<T, Acc, Acc, false, true, false, kBlock2>), g, bm, lds, st,
                           h->sv, u, q, h->wb, gpart, hcols, sc, inv);
    else if (h->astro_scan)
        hipLaunchKernelGGL((k_aprod2<T, Acc, Acc, false, false, true, kBlock2>), g, bm, lds, st,
                           h->sv, u, q, h->wb, gpart, hcols, sc, inv);
    else
        hipLaunchKernelGGL((k_aprod2<T, Acc, Acc, false, false, false, kBlock2>), g, bm, lds, st,
                           h->sv, u, q, h->wb, gpart, hcols, sc, inv);
    hipLaunchKernelGGL((k_glob_sum<Acc>), dim3(1), b, 0, st, gpart, h->nb2, q + h->sv.glob_base, sc);
    launch_instr_tail<T, Acc, 1, false>(h, u, inv, q, hcols, sc, st);
    if (!att) launch_att_pass<T, Acc>(h, ub, q, sc, st, gperm);
}

// One LSQR iteration; ev (optional) = kEvIter events: [0, 1] around aprod1
// (with the fused pass: the attitude pre-pass, if any, and that pass), [2, 3]
// around aprod2 (the attitude pass), [4] after the pre-pass.
template <typename T, typename Acc>
void launch_iteration(lsqr_handle* h, Path<Acc>& P, hipStream_t st, hipEvent_t* ev)
{
    const int64_t n = h->sv.n;
    if (ev) (void)hipEventRecord(ev[0], st);
    const bool pre = fused_mode(h) >= 2;
    const bool il = (h->att_il || pre) && h->sv.natt > 0 && !h->generic;
    if (il) launch_interleave_att<Acc>(h, P.vp, P.vp3, h->sc, st);
    if (pre) launch_att_dot<T, Acc>(h, P, st);
    if (ev) (void)hipEventRecord(ev[4], st);
    if (use_fused(h)) {
        launch_fused<T, Acc>(h, P, st, pre);
        launch_con_aprod1<Acc, Acc, Acc, A1_LSQR>(h, (const Acc*)P.vp, P.u + h->sv.m, nullptr,
                                                  h->sc, h->part1 + h->nb2, st);
        if (ev) (void)hipEventRecord(ev[1], st);
        hipLaunchKernelGGL(k_scalar_beta, dim3(1), dim3(kBlock), 0, st, h->part1,
                           n_part(h, h->nb2), h->sc);
        if (ev) (void)hipEventRecord(ev[2], st);
        hipLaunchKernelGGL((k_glob_sum<Acc>), dim3(1), dim3(kBlock), 0, st, P.gpart, h->nb2,
                           P.q + h->sv.glob_base, h->sc);
        launch_att_pass<T, Acc>(h, P.u, P.q, h->sc, st,
                                star_order_u(h) ? (const int32_t*)h->perm : nullptr);
        launch_con_aprod2<Acc, Acc>(h, P.u + h->sv.m, P.q, h->sc, st);
    } else {
        launch_aprod1<T, Acc, Acc, Acc, A1_LSQR>(h, (const Acc*)P.vp, P.u, nullptr, h->sc,
                                                h->part1, st, row_map(h),
                                                il ? (const Acc*)P.vp3 : nullptr);
        if (ev) (void)hipEventRecord(ev[1], st);
        hipLaunchKernelGGL(k_scalar_beta, dim3(1), dim3(kBlock), 0, st, h->part1,
                           n_part(h, h->nb1), h->sc);
        if (ev) (void)hipEventRecord(ev[2], st);
        launch_aprod2<T, Acc>(h, P.u, row_map(h), P.q, P.gpart, P.hcols, h->sc, st, P.u,
                              nullptr);
    }
    if (ev) (void)hipEventRecord(ev[3], st);
    hipLaunchKernelGGL((k_col_a<Acc>), dim3(h->nbc), dim3(kBlock), 0, st, n, h->p, P.q, h->v,
                       h->sc, h->partc);
    hipLaunchKernelGGL(k_scalar_alpha, dim3(1), dim3(kBlock), 0, st, h->partc, h->nbc, h->sc);
    hipLaunchKernelGGL((k_col_b<Acc>), dim3(h->nbc), dim3(kBlock), 0, st, n, h->p, h->v, h->w,
                       h->y, P.vp, h->sc, h->partdd, h->partxx,
                       (std::is_same<Acc, double>::value && h->var_on) ? h->var : nullptr);
    hipLaunchKernelGGL(k_scalar_stop, dim3(1), dim3(kBlock), 0, st, h->partdd, h->partxx, h->nbc,
                       h->sc);
}

// Initialisation given u~ (already written, placed by row_map) and ||u~||^2
// partials in part1.
template <typename T, typename Acc>
void launch_init(lsqr_handle* h, Path<Acc>& P, hipStream_t st)
{
    const int64_t n = h->sv.n;
    hipLaunchKernelGGL(k_scalar_init_beta, dim3(1), dim3(kBlock), 0, st, h->part1,
                       n_part(h, h->nb1), h->sc);
    hipLaunchKernelGGL((k_fill<Acc>), dim3(h->nbc), dim3(kBlock), 0, st, n, P.q, (Acc)0);
    hipLaunchKernelGGL((k_fill<double>), dim3(h->nbc), dim3(kBlock), 0, st, n, h->v, 0.0);
    launch_aprod2<T, Acc>(h, P.u, row_map(h), P.q, P.gpart, P.hcols, h->sc, st, P.u,
                          star_order_u(h) ? (const int32_t*)h->perm : nullptr);
    hipLaunchKernelGGL((k_col_a<Acc>), dim3(h->nbc), dim3(kBlock), 0, st, n, h->p, P.q, h->v,
                       h->sc, h->partc);
    hipLaunchKernelGGL(k_scalar_init_alpha, dim3(1), dim3(kBlock), 0, st, h->partc, h->nbc, h->sc);
    hipLaunchKernelGGL((k_col_init<Acc>), dim3(h->nbc), dim3(kBlock), 0, st, n, h->p, h->v, h->w,
                       h->y, P.vp, h->sc);
}

void batch_free(lsqr_handle* h);
template <typename Acc>
void release_path(Path<Acc>& P);

template <typename Acc>
lsqr_status path_alloc(lsqr_handle* h, Path<Acc>& P)
{
    const int64_t m = h->sv.m, n = h->sv.n;
    LSQR_TRY(dalloc(&P.u, m + h->nc));  // observation rows, then constraint rows
    LSQR_TRY(dalloc(&P.vp, n));
    LSQR_TRY(dalloc(&P.q, n));
    LSQR_TRY(dalloc(&P.gpart, std::max<int64_t>(h->nb2, (int64_t)h->nba * kGlobMax)));
    LSQR_TRY(dalloc(&P.vp3, (int64_t)kAxes * h->sv.n_dfa));
    return LSQR_OK;
}

// Working vectors of one precision of the single-RHS loop. When device
// memory runs short, the batched tile buffers are released (a later batched
// solve allocates them again) and the allocation is tried once more.
template <typename T, typename Acc>
lsqr_status prepare_path(lsqr_handle* h, Path<Acc>& P)
{
    if (!P.ready) {
        const int64_t n = h->sv.n;
        lsqr_status rc = path_alloc(h, P);
        if (rc == LSQR_E_NOMEM) {
            release_path(P);
            batch_free(h);
            g_last_error.clear();
            rc = path_alloc(h, P);
        }
        if (rc != LSQR_OK) {
            release_path(P);
            return rc;
        }
        // LDS histograms are FP64 whatever Acc is (k_att_hist)
        P.hcols = instr_hcols(h, 1);
        P.lds = (size_t)(P.hcols * 8);
        P.lds_f = fused_lds_plan(h, 1, (int64_t)sizeof(Acc), &P.f_hcols, &P.f_ldsx);
        hipLaunchKernelGGL((k_fill<Acc>), dim3(h->nbc), dim3(kBlock), 0, h->stream, n, P.q,
                           (Acc)0);
        HIP_TRY(hipGetLastError());
        P.ready = true;
    }
    if (star_order_u(h) && !P.datt) {  // fused mode 3: the pre-pass output
        if (dalloc(&P.datt, h->sv.m) == LSQR_E_NOMEM) {
            batch_free(h);
            g_last_error.clear();
            LSQR_TRY(dalloc(&P.datt, h->sv.m));
        }
    }
    // a fused pass that places u~ through the permutation and leaves
    // instrumental tail windows: a star-order copy of u~ for the tails (an
    // optimisation only: without the memory they read u~ through invperm)
    if (!P.ustar && !P.ustar_tried && use_fused(h) && row_map(h) &&
        P.f_hcols < h->sv.n_instr_cols) {
        P.ustar_tried = true;
        if (dalloc(&P.ustar, h->sv.m) != LSQR_OK) g_last_error.clear();
    }
    return LSQR_OK;
}

// Attitude bucket geometry: the fewest buckets whose FP64 histogram (for
// att_rhs right-hand sides per sweep) fits in LDS, or the requested count
// (raised if needed). Workgroups per bucket G:
// one workgroup fits per CU, so the pass takes ceil(nbk G / CUs) rounds of
// 1/G of a bucket each; G minimises that (up to max(8, CUs / nbk), ties to
// the smaller G, which keeps the slices to add up few).
void att_geometry(lsqr_handle* h)
{
    const int64_t nt = h->sv.n_dfa - kParAxis + 1;
    const int64_t wmax = kLdsInstrBudget / (kAxes * 8 * h->att_rhs) - (kParAxis - 1);
    int64_t nb = h->att_buckets > 0 ? h->att_buckets : cdiv(nt, wmax);
    nb = std::max<int64_t>(1, std::min(nb, nt));
    int64_t w = cdiv(nt, nb);
    if (w > wmax) w = wmax;
    h->bwidth = w;
    h->nbk = cdiv(nt, w);
    const int64_t cu = std::max(1, h->num_cu);
    const int64_t gmax = std::max<int64_t>(8, cu / h->nbk);
    int64_t best = 1;
    double best_cost = 1e300;
    for (int64_t g = 1; g <= gmax; ++g) {
        const double cost = (double)cdiv(h->nbk * g, cu) / (double)g;
        if (cost < best_cost - 1e-12) {
            best_cost = cost;
            best = g;
        }
    }
    h->att_g = (int)best;
}

// Attitude bucket order: a stable radix sort of the rows by t / W, the
// attitude coefficients and local starts gathered into that order, the
// inverse permutation and the bucket boundaries.
template <typename T>
lsqr_status prepare_att_sorted(lsqr_handle* h)
{
    if (h->att_ready) return LSQR_OK;
    const int64_t m = h->sv.m;
    if (m >= ((int64_t)1 << 31) || h->sv.n_dfa >= ((int64_t)1 << 31))
        return fail(LSQR_E_UNSUPPORTED,
                    "the attitude bucket order needs n_rows < 2^31 and n_dfa < 2^31");
    att_geometry(h);
    hipStream_t st = h->stream;
    int32_t *keys = nullptr, *rows = nullptr, *skeys = nullptr;
    void* temp = nullptr;
    size_t temp_bytes = 0;
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) < h->nbk) ++bits;
    LSQR_TRY(dalloc(&h->perm, m));
    LSQR_TRY(dalloc(&h->invperm, m));
    LSQR_TRY(dalloc(&h->tloc, m));
    LSQR_TRY(dalloc(&h->bstart, h->nbk + 1));
    LSQR_TRY(dalloc(&h->S2, att_slices(h) * kAxes * att_span(h)));
    T* att_sorted = nullptr;
    // columns 64-row aligned, so that the bucket-order passes read whole lines
    h->att_ld = cdiv(m, (int64_t)kWave) * kWave;
    LSQR_TRY(dalloc(&att_sorted, (int64_t)kAxes * kParAxis * h->att_ld));
    h->att_sorted = att_sorted;
    LSQR_TRY(dalloc(&keys, m));
    lsqr_status rc = dalloc(&rows, m);
    if (rc == LSQR_OK) rc = dalloc(&skeys, m);
    hipError_t e = hipSuccess;
    const dim3 gm(std::min<int64_t>(cdiv(m, kBlock), 65536)), bb(kBlock);
    if (rc == LSQR_OK) {
        hipLaunchKernelGGL(k_bucket_keys, gm, bb, 0, st, h->sv.att, m, h->bwidth, keys, rows);
        e = rocprim::radix_sort_pairs(nullptr, temp_bytes, keys, skeys, rows, h->perm, (size_t)m,
                                      0, bits, st);
        if (e == hipSuccess) rc = dalloc(reinterpret_cast<char**>(&temp), (int64_t)temp_bytes);
    }
    if (rc == LSQR_OK && e == hipSuccess)
        e = rocprim::radix_sort_pairs(temp, temp_bytes, keys, skeys, rows, h->perm, (size_t)m, 0,
                                      bits, st);
    if (rc == LSQR_OK && e == hipSuccess) {
        hipLaunchKernelGGL((k_att_gather<T>), gm, bb, 0, st, (const T*)h->sv.val, h->sv.att, m,
                           (const int32_t*)h->perm, h->bwidth, h->sv.off_att, h->att_ld,
                           att_sorted, h->tloc);
        hipLaunchKernelGGL(k_invert_perm, gm, bb, 0, st, (const int32_t*)h->perm, m, h->invperm);
        hipLaunchKernelGGL(k_bucket_starts, dim3(std::min<int64_t>(cdiv(m + 1, kBlock), 65536)), bb,
                           0, st, (const int32_t*)skeys, m, h->nbk, h->bstart);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    if (temp) (void)hipFree(temp);
    dfree(keys);
    dfree(rows);
    dfree(skeys);
    if (rc != LSQR_OK) return rc;
    if (e != hipSuccess) return fail(LSQR_E_HIP, "attitude bucket order: %s", hipGetErrorString(e));
    h->att_ready = true;
    return LSQR_OK;
}

lsqr_status ensure_att(lsqr_handle* h)
{
    if (!att_pass_on(h)) return LSQR_OK;
    return h->value_type == LSQR_F64 ? prepare_att_sorted<double>(h) : prepare_att_sorted<float>(h);
}

// Captured iteration graphs bake in the kernel choices: drop them all (single
// solves and every batched k-tile) when an option that selects kernels
// changes.
void drop_graphs(lsqr_handle* h)
{
    for (hipGraphExec_t* g : {&h->p64.graph, &h->p32.graph}) {
        if (*g) (void)hipGraphExecDestroy(*g);
        *g = nullptr;
    }
    for (auto* gs : {h->batch.graph, h->batch.graph32})
        for (int k = 0; k < 17; ++k) {
            if (gs[k]) (void)hipGraphExecDestroy(gs[k]);
            gs[k] = nullptr;
        }
    // the autotuner's choice was made with the kernels these options select
    memset(h->batch.tuned_k, 0, sizeof h->batch.tuned_k);
}

// Compact index copies for the fused passes (int32 star, uint16 instrumental
// index: 16 instead of 32 bytes per row), built once per handle on the first
// solve when the layout allows them and they take at most 1/32 of the
// device's memory; otherwise (or if the allocation fails) the fused passes
// read the caller's arrays.
constexpr int64_t kCompactMemFraction = 32;

lsqr_status ensure_compact(lsqr_handle* h)
{
    if (!h->compact || h->compact_tried || h->generic) return LSQR_OK;
    h->compact_tried = 1;
    const int64_t m = h->sv.m;
    if (h->sv.n_stars > INT32_MAX || h->sv.n_instr_cols > 65536) return LSQR_OK;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return LSQR_OK;
    const int64_t need = m * (int64_t)(sizeof(int32_t) + kInstr * sizeof(uint16_t));
    if (need > (int64_t)(total_b / kCompactMemFraction) || need >= (int64_t)free_b) return LSQR_OK;
    if (dalloc(&h->star32, m) != LSQR_OK || dalloc(&h->instr16, (int64_t)kInstr * m) != LSQR_OK) {
        dfree(h->star32);
        dfree(h->instr16);
        g_last_error.clear();  // not an error: the fused passes use the caller's arrays
        return LSQR_OK;
    }
    hipLaunchKernelGGL(k_compact_idx, dim3(std::min<int64_t>(cdiv(m, kBlock), 8192)), dim3(kBlock),
                       0, h->stream, h->sv, h->star32, h->instr16);
    HIP_TRY(hipGetLastError());
    h->sv.star32 = h->star32;
    h->sv.instr16 = h->instr16;
    drop_graphs(h);
    return LSQR_OK;
}

template <typename Acc>
void release_path(Path<Acc>& P)
{
    if (P.graph) (void)hipGraphExecDestroy(P.graph);
    P.graph = nullptr;
    dfree(P.u);
    dfree(P.vp);
    dfree(P.q);
    dfree(P.gpart);
    dfree(P.vp3);
    dfree(P.datt);
    dfree(P.ustar);
    P.ustar_tried = false;
    P.ready = false;
}

lsqr_status upload_controls(lsqr_handle* h, int32_t itn_limit, double atol, double btol,
                            double rel_ar = 0.0)
{
    // The controls are written into the pinned mirror and copied as one block
    // with the rest of the (reset) state; the kernels then own the state.
    Scalars* s = h->sc_host;
    memset(s, 0, sizeof(Scalars));
    s->atol = atol;
    s->btol = btol;
    s->ctol = h->conlim > 0.0 ? 1.0 / h->conlim : 0.0;
    s->itn_limit = itn_limit;
    s->tests = rel_ar > 0.0 ? 0 : h->tests;
    s->rel_ar = rel_ar;
    s->inv_alpha = 1.0;
    HIP_TRY(hipMemcpyAsync(h->sc, s, sizeof(Scalars), hipMemcpyHostToDevice, h->stream));
    return LSQR_OK;
}

lsqr_status read_scalars(lsqr_handle* h)
{
    HIP_TRY(hipMemcpyAsync(h->sc_host, h->sc, sizeof(Scalars), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LSQR_OK;
}

// Runs chunks of iterations until the device reports done.
template <typename T, typename Acc>
lsqr_status run_iterations(lsqr_handle* h, Path<Acc>& P)
{
    h->last_mode = fused_mode(h);
    const int chunk = std::max(1, h->chunk);
    const bool graph = h->use_graph && !h->profile;
    if (graph && (P.graph == nullptr || P.graph_chunk != chunk)) {
        if (P.graph) (void)hipGraphExecDestroy(P.graph);
        P.graph = nullptr;
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < chunk; ++k) launch_iteration<T, Acc>(h, P, h->stream, nullptr);
        hipError_t e = hipStreamEndCapture(h->stream, &g);
        if (e != hipSuccess) return fail(LSQR_E_HIP, "graph capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&P.graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            P.graph = nullptr;
            return fail(LSQR_E_HIP, "graph instantiate: %s", hipGetErrorString(e));
        }
        P.graph_chunk = chunk;
    }
    if (h->profile && h->events.size() < (size_t)kEvIter * chunk) {
        while (h->events.size() < (size_t)kEvIter * chunk) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            h->events.push_back(e);
        }
    }
    for (;;) {
        const int32_t itn_before = h->sc_host->itn;
        if (graph) {
            HIP_TRY(hipGraphLaunch(P.graph, h->stream));
        } else {
            for (int k = 0; k < chunk; ++k)
                launch_iteration<T, Acc>(h, P, h->stream,
                                         h->profile ? &h->events[kEvIter * k] : nullptr);
            HIP_TRY(hipGetLastError());
        }
        LSQR_TRY(read_scalars(h));
        if (h->profile) {
            const int ran = std::min(chunk, h->sc_host->itn - itn_before);
            for (int k = 0; k < ran; ++k) {
                hipEvent_t* ev = &h->events[kEvIter * k];
                float a = 0.f, b = 0.f, c = 0.f;
                HIP_TRY(hipEventElapsedTime(&a, ev[0], ev[1]));
                HIP_TRY(hipEventElapsedTime(&b, ev[2], ev[3]));
                HIP_TRY(hipEventElapsedTime(&c, ev[0], ev[4]));
                h->ms1 += a;
                h->ms2 += b;
                h->ms_pre += c;
                h->n1 += 1;
                h->n2 += 1;
            }
        }
        if (h->sc_host->done) break;
        // Every chunk either finishes the solve or advances itn; anything else
        // means a launch did not run, and looping would never end.
        if (h->sc_host->itn <= itn_before)
            return fail(LSQR_E_HIP, "LSQR iteration made no progress (itn %d)", h->sc_host->itn);
    }
    return LSQR_OK;
}

void fill_info(const lsqr_handle* h, lsqr_info* info, int32_t itn, int32_t outer, double bnorm)
{
    if (!info) return;
    const Scalars* s = h->sc_host;
    memset(info, 0, sizeof(*info));
    info->istop = s->istop;
    info->itn = itn;
    info->outer_steps = outer;
    info->rnorm = s->rnorm;
    info->arnorm = s->arnorm;
    info->anorm = s->anorm;
    info->acond = s->acond;
    info->xnorm = s->xnorm;
    info->bnorm = bnorm;
}

template <typename T>
lsqr_status solve_fp64(lsqr_handle* h, const double* b, double* x, int32_t itn_limit, double atol,
                       double btol, lsqr_info* info)
{
    LSQR_TRY(ensure_att(h));
    LSQR_TRY(ensure_compact(h));
    LSQR_TRY((prepare_path<T, double>(h, h->p64)));
    Path<double>& P = h->p64;
    const int64_t m = h->sv.m, n = h->sv.n;
    if (h->profile) {
        h->ms1 = h->ms2 = h->ms_pre = 0.0;
        h->n1 = h->n2 = 0;
    }
    LSQR_TRY(upload_controls(h, itn_limit, atol, btol));
    h->var_valid = 0;
    if (h->var_on) {
        if (!h->var) LSQR_TRY(dalloc(&h->var, n));
        hipLaunchKernelGGL((k_fill<double>), dim3(h->nbc), dim3(kBlock), 0, h->stream, n, h->var,
                           0.0);
    }
    hipLaunchKernelGGL((k_copy_ssq<double>), dim3(h->nb1), dim3(kBlock), 0, h->stream, m, b, P.u,
                       h->part1, row_map(h));
    if (h->nc > 0)  // constraint rows: after the observation rows, one partial
        hipLaunchKernelGGL((k_copy_ssq<double>), dim3(1), dim3(kBlock), 0, h->stream, h->nc, b + m,
                           P.u + m, h->part1 + h->nb1, (const int32_t*)nullptr);
    launch_init<T, double>(h, P, h->stream);
    HIP_TRY(hipGetLastError());
    LSQR_TRY(read_scalars(h));
    if (!h->sc_host->done && itn_limit > 0) LSQR_TRY((run_iterations<T, double>(h, P)));
    hipLaunchKernelGGL(k_unprecond, dim3(h->nbc), dim3(kBlock), 0, h->stream, n, h->p, h->y, x);
    HIP_TRY(hipGetLastError());
    LSQR_TRY(read_scalars(h));
    fill_info(h, info, h->sc_host->itn, 0, h->sc_host->bnorm);
    h->var_valid = h->var_on;
    return LSQR_OK;
}

// ------------------------------------------------------------- batched RHS
void batch_free(lsqr_handle* h)
{
    auto& B = h->batch;
    for (auto* gs : {B.graph, B.graph32})
        for (int k = 0; k < 17; ++k) {
            if (gs[k]) (void)hipGraphExecDestroy(gs[k]);
            gs[k] = nullptr;
        }
    dfree(B.U); dfree(B.V); dfree(B.W); dfree(B.Y); dfree(B.VP); dfree(B.Q);
    dfree(B.gpart); dfree(B.part1); dfree(B.partc); dfree(B.partdd); dfree(B.partxx);
    dfree(B.sc); dfree(B.flag); dfree(B.S2); dfree(B.X3);
    dfree(B.U32); dfree(B.VP32); dfree(B.Q32); dfree(B.gpart32); dfree(B.X332);
    dfree(B.US1); dfree(B.US1_32);
    B.kmax = 0;
    B.has64 = B.has32 = false;
}

lsqr_status batch_alloc_once(lsqr_handle* h, int kmax, bool want64, bool want32)
{
    auto& B = h->batch;
    const int64_t m = h->sv.m, n = h->sv.n;
    if (h->att_ready) LSQR_TRY(dalloc(&B.S2, att_slices(h) * kAxes * att_span(h) * kmax));
    LSQR_TRY(dalloc(&B.X3, (int64_t)kAxes * h->sv.n_dfa * kmax));
    LSQR_TRY(dalloc(&B.V, n * kmax));
    LSQR_TRY(dalloc(&B.W, n * kmax));
    LSQR_TRY(dalloc(&B.Y, n * kmax));
    LSQR_TRY(dalloc(&B.gpart, (int64_t)h->nba * kmax));
    LSQR_TRY(dalloc(&B.part1, (int64_t)std::max(h->nb1, h->nba) * kmax));
    LSQR_TRY(dalloc(&B.partc, (int64_t)h->nbc * kmax));
    LSQR_TRY(dalloc(&B.partdd, (int64_t)h->nbc * kmax));
    LSQR_TRY(dalloc(&B.partxx, (int64_t)h->nbc * kmax));
    LSQR_TRY(dalloc(&B.sc, kmax));
    LSQR_TRY(dalloc(&B.flag, 1));
    if (want64) {
        LSQR_TRY(dalloc(&B.U, m * kmax));
        LSQR_TRY(dalloc(&B.VP, n * kmax));
        LSQR_TRY(dalloc(&B.Q, n * kmax));
        hipLaunchKernelGGL((k_fill<double>), dim3(h->nbc), dim3(kBlock), 0, h->stream, n * kmax,
                           B.Q, 0.0);
    }
    if (want32) {
        LSQR_TRY(dalloc(&B.U32, m * kmax));
        LSQR_TRY(dalloc(&B.VP32, n * kmax));
        LSQR_TRY(dalloc(&B.Q32, n * kmax));
        LSQR_TRY(dalloc(&B.gpart32, (int64_t)h->nba * kmax));
        LSQR_TRY(dalloc(&B.X332, (int64_t)kAxes * h->sv.n_dfa * kmax));
        hipLaunchKernelGGL((k_fill<float>), dim3(h->nbc), dim3(kBlock), 0, h->stream, n * kmax,
                           B.Q32, 0.0f);
    }
    // the star-order copy for 1-RHS tiles (an optimisation: when the memory
    // is short the single-RHS working vectors are released for it, as for the
    // tile buffers, and without it the tails read U through the permutation)
    if (use_fused(h) && batch_row_map(h) && h->sv.ni > 0) {
        auto copy = [&](auto** buf, int64_t vbytes) {
            int64_t hc1 = 0;
            int ldsx = 0;
            fused_lds_plan(h, 1, vbytes, &hc1, &ldsx);
            if (hc1 >= h->sv.n_instr_cols || dalloc(buf, m) == LSQR_OK) return;
            release_path(h->p64);
            release_path(h->p32);
            if (dalloc(buf, m) != LSQR_OK) g_last_error.clear();
        };
        if (want64) copy(&B.US1, 8);
        if (want32) copy(&B.US1_32, 4);
    }
    HIP_TRY(hipGetLastError());
    B.kmax = kmax;
    B.has64 = want64;
    B.has32 = want32;
    return LSQR_OK;
}

// Tile buffers for up to kmax right-hand sides in the wanted precision
// (FP64 tiles, FP32 inner tiles). A set too small, or of the other precision
// only, is freed first (the captured graphs go with it). When device memory
// runs short, the single-RHS working vectors are released (a later single
// solve allocates them again) and the allocation is tried once more.
lsqr_status batch_alloc(lsqr_handle* h, int kmax, bool fp32)
{
    auto& B = h->batch;
    if (B.kmax >= kmax && (fp32 ? B.has32 : B.has64) && (B.S2 || !h->att_ready)) return LSQR_OK;
    kmax = std::max(kmax, B.kmax);
    batch_free(h);
    lsqr_status rc = batch_alloc_once(h, kmax, !fp32, fp32);
    if (rc == LSQR_E_NOMEM) {
        batch_free(h);
        release_path(h->p64);
        release_path(h->p32);
        g_last_error.clear();
        rc = batch_alloc_once(h, kmax, !fp32, fp32);
    }
    if (rc != LSQR_OK) batch_free(h);
    return rc;
}

// The buffers of one precision of a k-tile.
template <typename Acc>
struct TileBufs {
    Acc *U, *VP, *Q, *gpart, *X3;
    hipGraphExec_t* graph;
    int* graph_chunk;
    Acc* US1;  // star-order copy of U for 1-RHS tiles with tail windows, or null
};

template <typename Acc>
TileBufs<Acc> tile_bufs(lsqr_handle* h);

template <>
TileBufs<double> tile_bufs<double>(lsqr_handle* h)
{
    auto& B = h->batch;
    return {B.U, B.VP, B.Q, B.gpart, B.X3, B.graph, B.graph_chunk, B.US1};
}

template <>
TileBufs<float> tile_bufs<float>(lsqr_handle* h)
{
    auto& B = h->batch;
    return {B.U32, B.VP32, B.Q32, B.gpart32, B.X332, B.graph32, B.graph32_chunk, B.US1_32};
}

// Workgroup shape of the batched row passes over the star-aligned ranges: K <= 2
// fits the 128 registers a lane has in a 1024-thread workgroup; wider tiles
// use 256-thread workgroups over the same ranges.
template <int K>
constexpr int batch_nt() { return K <= 2 ? kBlock2 : kBlock; }

template <int K>
int batch_grid(const lsqr_handle* h) { return K <= 2 ? h->nb2 : h->nba; }

// Workgroup shape of the fused pass of a K-tile: multi-RHS tiles carry K
// values per gathered vector entry and 5K running star sums, so K = 2 runs
// 512-thread workgroups (256 registers per lane) and wider tiles 256; after
// the attitude pre-pass (kAttPre, no attitude gathers) K = 4 fits 512 too.
template <int K, int AM>
constexpr int fused_nt()
{
    if (K == 1) return kBlock2;
    return K == 2 || (K == 4 && AM == kAttPre) ? kBlock1 : kBlock;
}

template <int K, int AM>
int fused_grid(const lsqr_handle* h) { return (int)(h->nw / (fused_nt<K, AM>() / kWave)); }

// Workgroups (partials) of the fused pass an iteration of a K-tile runs
// (fused mode 3 runs as 2 in k-tiles)
template <int K>
int batch_fused_grid(const lsqr_handle* h)
{
    if (K >= 2 && rhs_lanes_on(h)) return h->nb2;  // k_fused_rl: 1024-thread workgroups
    return h->fused >= 2 ? fused_grid<K, kAttPre>(h) : fused_grid<K, kAttX>(h);
}

// Right-hand sides per sweep of the bucket-order attitude passes of a K-tile:
// the largest power of two up to K whose window or histogram, 3 (W + 3) KS
// values (FP64 for the histograms, vbytes each for the windows), fits in LDS.
// Narrower buckets (more of them) widen the sweeps.
template <int K>
int att_sweep(const lsqr_handle* h, int64_t vbytes = 8)
{
    const int64_t fit = kLdsInstrBudget / (kAxes * att_span(h) * vbytes);
    int ks = 1;
    // at most 4 per sweep: 8 or 16 running dot products per row spill registers
    while (ks * 2 <= K && ks * 2 <= fit && ks * 2 <= 4) ks *= 2;
    return ks;
}

template <int K, typename F>
void by_sweep(int ks, F&& f)
{
    if constexpr (K >= 4)
        if (ks == 4) return f(std::integral_constant<int, 4>());
    if constexpr (K >= 2)
        if (ks == 2) return f(std::integral_constant<int, 2>());
    f(std::integral_constant<int, 1>());
}

template <typename T, typename Acc, int K>
void batch_att_pass(lsqr_handle* h, hipStream_t st)
{
    auto& B = h->batch;
    const TileBufs<Acc> tb = tile_bufs<Acc>(h);
    // at most 2 RHS per histogram sweep: 4 FP64 histograms fill LDS, leave
    // one workgroup per CU and halve the rate of its atomics (1e8 rows, 64
    // buckets: one 4-RHS sweep 6.3 ms, two 2-RHS sweeps 2 x 2.15 ms)
    const int ks = std::min(2, att_sweep<K>(h));
    by_sweep<K>(ks, [&](auto KS) {
        hipLaunchKernelGGL((k_att_hist<T, Acc, K, KS(), kAttBlock>), dim3(att_slices(h)),
                           dim3(kAttBlock), (size_t)(kAxes * att_span(h) * 8 * ks), st, h->att_ld,
                           (const T*)h->att_sorted, (const int32_t*)h->tloc,
                           (const int64_t*)h->bstart, h->bwidth, h->att_g, (const Acc*)tb.U,
                           B.S2, B.sc, (const int32_t*)nullptr);
    });
    hipLaunchKernelGGL((k_att_reduce<Acc, K>), dim3(h->nbc), dim3(kBlock), 0, st,
                       (const double*)B.S2, h->nbk, h->att_g, h->bwidth, h->sv.n_dfa,
                       tb.Q + h->sv.att_base * K, B.sc);
}

template <typename T, typename Acc, int K>
void batch_aprod2(lsqr_handle* h, hipStream_t st)
{
    auto& B = h->batch;
    const TileBufs<Acc> tb = tile_bufs<Acc>(h);
    const int64_t hc = instr_hcols(h, K);
    const size_t lds = (size_t)(hc * K * 8);
    constexpr int NT = batch_nt<K>();
    int grid = batch_grid<K>(h);
    if (K >= 2 && rhs_lanes_on(h)) {
        grid = h->nb2;
        if (h->sv.star32)
            hipLaunchKernelGGL((batched::k_fused_rl<T, Acc, K, kBlock2, false, true, true>),
                               dim3(grid), dim3(kBlock2), lds, st, h->sv, (const Acc*)tb.VP, tb.U,
                               tb.Q, h->wb, tb.gpart, B.part1, hc, B.sc, batch_row_map(h));
        else
            hipLaunchKernelGGL((batched::k_fused_rl<T, Acc, K, kBlock2, false, false, true>),
                               dim3(grid), dim3(kBlock2), lds, st, h->sv, (const Acc*)tb.VP, tb.U,
                               tb.Q, h->wb, tb.gpart, B.part1, hc, B.sc, batch_row_map(h));
    } else if constexpr (K <= 8) {
        if (h->att_mode == 0)
            hipLaunchKernelGGL((batched::k_aprod2<T, Acc, K, true, NT>), dim3(grid), dim3(NT), lds,
                               st, h->sv, (const Acc*)tb.U, tb.Q, h->wb, tb.gpart, hc, B.sc,
                               batch_row_map(h));
        else
            hipLaunchKernelGGL((batched::k_aprod2<T, Acc, K, false, NT>), dim3(grid), dim3(NT),
                               lds, st, h->sv, (const Acc*)tb.U, tb.Q, h->wb, tb.gpart, hc, B.sc,
                               batch_row_map(h));
    }
    hipLaunchKernelGGL((batched::k_glob_sum<Acc, K>), dim3(1), dim3(kBlock), 0, st,
                       (const Acc*)tb.gpart, grid, tb.Q + h->sv.glob_base * K, B.sc);
    launch_instr_tail<T, Acc, K, false>(h, (const Acc*)tb.U, batch_row_map(h), tb.Q, hc, B.sc, st);
    if (h->att_mode != 0) batch_att_pass<T, Acc, K>(h, st);
}

template <typename T, typename Acc, int K, bool LDSX, int AM>
void batch_fused_as(lsqr_handle* h, const Acc* X3, int64_t hc, size_t lds, hipStream_t st)
{
    auto& B = h->batch;
    const TileBufs<Acc> tb = tile_bufs<Acc>(h);
    if constexpr (AM == kAttPre)
        if (K >= 2 && rhs_lanes_on(h)) {  // the K right-hand sides of a row in K lanes
            // two row steps in flight (LSQR_OPT_PIPELINE): K = 4, and K = 2
            // except with FP64 values and vectors, whose second register set
            // would spill
            auto go = [&](auto pipe) {
                constexpr bool P = decltype(pipe)::value;
                if (h->sv.star32)
                    hipLaunchKernelGGL(
                        (batched::k_fused_rl<T, Acc, K, kBlock2, LDSX, true, false, P>),
                        dim3(h->nb2), dim3(kBlock2), lds, st, h->sv, (const Acc*)tb.VP, tb.U,
                        tb.Q, h->wb, tb.gpart, B.part1, hc, B.sc, batch_row_map(h));
                else
                    hipLaunchKernelGGL(
                        (batched::k_fused_rl<T, Acc, K, kBlock2, LDSX, false, false, P>),
                        dim3(h->nb2), dim3(kBlock2), lds, st, h->sv, (const Acc*)tb.VP, tb.U,
                        tb.Q, h->wb, tb.gpart, B.part1, hc, B.sc, batch_row_map(h));
            };
            if constexpr (K == 4 || (K == 2 && (sizeof(T) == 4 || sizeof(Acc) == 4))) {
                if (h->pipe) go(std::true_type());
                else go(std::false_type());
            } else {
                go(std::false_type());
            }
            return;
        }
    if constexpr (K <= 8) {  // 16-RHS tiles are built in the RHS-across-lanes form only
        constexpr int NT = fused_nt<K, AM>();
        Acc* us = K == 1 ? tb.US1 : nullptr;
        if (h->sv.star32)
            hipLaunchKernelGGL((batched::k_fused<T, Acc, K, NT, LDSX, AM, true>),
                               dim3(fused_grid<K, AM>(h)), dim3(NT), lds, st, h->sv,
                               (const Acc*)tb.VP, X3, tb.U, tb.Q, h->wb, tb.gpart, B.part1, hc,
                               B.sc, batch_row_map(h), us);
        else
            hipLaunchKernelGGL((batched::k_fused<T, Acc, K, NT, LDSX, AM, false>),
                               dim3(fused_grid<K, AM>(h)), dim3(NT), lds, st, h->sv,
                               (const Acc*)tb.VP, X3, tb.U, tb.Q, h->wb, tb.gpart, B.part1, hc,
                               B.sc, batch_row_map(h), us);
    }
}

// The fused pass of a k-tile; in fused mode 2 the attitude pre-pass
// (k_att_dot on the tile's U, X3 and Scalars) runs first.
template <typename T, typename Acc, int K>
void batch_fused(lsqr_handle* h, hipStream_t st)
{
    auto& B = h->batch;
    const TileBufs<Acc> tb = tile_bufs<Acc>(h);
    int64_t hc = 0;
    int ldsx = 0;
    const size_t lds = fused_lds_plan(h, K, (int64_t)sizeof(Acc), &hc, &ldsx);
    const bool pre = h->fused >= 2;  // fused mode 3 runs as 2 in k-tiles
    const Acc* X3 = nullptr;
    if (h->att_il || pre) {
        hipLaunchKernelGGL((batched::k_interleave_att<Acc, K>), dim3(h->nbc), dim3(kBlock), 0, st,
                           (const Acc*)tb.VP, (int64_t)K, h->sv.att_base, h->sv.n_dfa, tb.X3);
        X3 = tb.X3;
    }
    if (pre) {
        const int ks = att_sweep<K>(h, (int64_t)sizeof(Acc));
        by_sweep<K>(ks, [&](auto KS) {
            hipLaunchKernelGGL((k_att_dot<T, Acc, K, KS(), kAttBlock>), dim3(att_slices(h)),
                               dim3(kAttBlock), (size_t)(kAxes * att_span(h) * sizeof(Acc) * ks),
                               st, h->att_ld, (const T*)h->att_sorted, (const int32_t*)h->tloc,
                               (const int64_t*)h->bstart, h->bwidth, h->att_g, h->sv.n_dfa, X3,
                               tb.U, (const Scalars*)B.sc);
        });
        if (ldsx) batch_fused_as<T, Acc, K, true, kAttPre>(h, nullptr, hc, lds, st);
        else batch_fused_as<T, Acc, K, false, kAttPre>(h, nullptr, hc, lds, st);
    } else if (ldsx) {
        if (X3) batch_fused_as<T, Acc, K, true, kAttX3>(h, X3, hc, lds, st);
        else batch_fused_as<T, Acc, K, true, kAttX>(h, X3, hc, lds, st);
    } else {
        if (X3) batch_fused_as<T, Acc, K, false, kAttX3>(h, X3, hc, lds, st);
        else batch_fused_as<T, Acc, K, false, kAttX>(h, X3, hc, lds, st);
    }
    // a 1-RHS tile's tail windows read the star-order copy its fused pass wrote
    if (K == 1 && tb.US1)
        launch_instr_tail<T, Acc, K, false>(h, (const Acc*)tb.US1, nullptr, tb.Q, hc, B.sc, st);
    else
        launch_instr_tail<T, Acc, K, false>(h, (const Acc*)tb.U, batch_row_map(h), tb.Q, hc, B.sc,
                                            st);
}

template <typename T, typename Acc, int K>
void batch_iteration(lsqr_handle* h, hipStream_t st, hipEvent_t* ev)
{
    auto& B = h->batch;
    const TileBufs<Acc> tb = tile_bufs<Acc>(h);
    const int64_t n = h->sv.n;
    if (ev) (void)hipEventRecord(ev[0], st);
    if (use_fused(h)) {
        batch_fused<T, Acc, K>(h, st);
        if (ev) (void)hipEventRecord(ev[1], st);
        hipLaunchKernelGGL((batched::k_scalar_beta<K>), dim3(1), dim3(kBlock), 0, st, B.part1,
                           batch_fused_grid<K>(h), B.sc);
        if (ev) (void)hipEventRecord(ev[2], st);
        hipLaunchKernelGGL((batched::k_glob_sum<Acc, K>), dim3(1), dim3(kBlock), 0, st,
                           (const Acc*)tb.gpart, batch_fused_grid<K>(h),
                           tb.Q + h->sv.glob_base * K, B.sc);
        batch_att_pass<T, Acc, K>(h, st);
    } else if constexpr (K <= 8) {
        hipLaunchKernelGGL((batched::k_aprod1<T, Acc, K>), dim3(h->nb1), dim3(kBlock), 0, st,
                           h->sv, (const Acc*)tb.VP, tb.U, B.sc, B.part1, batch_row_map(h));
        if (ev) (void)hipEventRecord(ev[1], st);
        hipLaunchKernelGGL((batched::k_scalar_beta<K>), dim3(1), dim3(kBlock), 0, st, B.part1,
                           h->nb1, B.sc);
        if (ev) (void)hipEventRecord(ev[2], st);
        batch_aprod2<T, Acc, K>(h, st);
    }
    if (ev) (void)hipEventRecord(ev[3], st);
    hipLaunchKernelGGL((batched::k_col_a<Acc, K>), dim3(h->nbc), dim3(kBlock), 0, st, n, h->p,
                       tb.Q, B.V, B.sc, B.partc);
    hipLaunchKernelGGL((batched::k_scalar_alpha<K>), dim3(1), dim3(kBlock), 0, st, B.partc, h->nbc,
                       B.sc);
    hipLaunchKernelGGL((batched::k_col_b<Acc, K>), dim3(h->nbc), dim3(kBlock), 0, st, n, h->p,
                       B.V, B.W, B.Y, tb.VP, B.sc, B.partdd, B.partxx);
    hipLaunchKernelGGL((batched::k_scalar_stop<K>), dim3(1), dim3(kBlock), 0, st, B.partdd,
                       B.partxx, h->nbc, B.sc);
    hipLaunchKernelGGL((batched::k_all_done<K>), dim3(1), dim3(kWave), 0, st, B.sc, B.flag);
}

// Uploads the controls of a tile's K scalar sets (rel_ar > 0: the relative
// normal-equation stop of a refinement's inner solves, tests off).
template <int K>
lsqr_status batch_controls(lsqr_handle* h, int32_t itn_limit, double atol, double btol,
                           double rel_ar = 0.0)
{
    Scalars host[kMaxTile];
    memset(host, 0, sizeof host);
    for (int r = 0; r < K; ++r) {
        host[r].atol = atol;
        host[r].btol = btol;
        host[r].ctol = h->conlim > 0.0 ? 1.0 / h->conlim : 0.0;
        host[r].itn_limit = itn_limit;
        host[r].tests = rel_ar > 0.0 ? 0 : h->tests;
        host[r].rel_ar = rel_ar;
        host[r].inv_alpha = 1.0;
    }
    HIP_TRY(hipMemcpyAsync(h->batch.sc, host, K * sizeof(Scalars), hipMemcpyHostToDevice,
                           h->stream));
    return LSQR_OK;
}

// Start of a tile's LSQR given U (placed by batch_row_map) and its sums of
// squares in part1 (h->nb1 partials): beta_1, alpha_1 v_1 = Abar^T u_1, w, y.
template <typename T, typename Acc, int K>
lsqr_status batch_init(lsqr_handle* h)
{
    auto& B = h->batch;
    const TileBufs<Acc> tb = tile_bufs<Acc>(h);
    hipStream_t st = h->stream;
    const int64_t n = h->sv.n;
    hipLaunchKernelGGL((batched::k_scalar_init_beta<K>), dim3(1), dim3(kBlock), 0, st, B.part1,
                       h->nb1, B.sc);
    hipLaunchKernelGGL((k_fill<Acc>), dim3(h->nbc), dim3(kBlock), 0, st, n * K, tb.Q, (Acc)0);
    hipLaunchKernelGGL((k_fill<double>), dim3(h->nbc), dim3(kBlock), 0, st, n * K, B.V, 0.0);
    batch_aprod2<T, Acc, K>(h, st);
    hipLaunchKernelGGL((batched::k_col_a<Acc, K>), dim3(h->nbc), dim3(kBlock), 0, st, n, h->p,
                       tb.Q, B.V, B.sc, B.partc);
    hipLaunchKernelGGL((batched::k_scalar_init_alpha<K>), dim3(1), dim3(kBlock), 0, st, B.partc,
                       h->nbc, B.sc);
    hipLaunchKernelGGL((batched::k_col_init<Acc, K>), dim3(h->nbc), dim3(kBlock), 0, st, n, h->p,
                       B.V, B.W, B.Y, tb.VP, B.sc);
    hipLaunchKernelGGL((batched::k_all_done<K>), dim3(1), dim3(kWave), 0, st, B.sc, B.flag);
    HIP_TRY(hipGetLastError());
    return LSQR_OK;
}

// Runs the tile's iterations in graph-replayed chunks (one flag read per
// chunk) until every RHS has stopped (or max_chunks chunks, if > 0); host
// receives the K scalar sets at the end.
template <typename T, typename Acc, int K>
lsqr_status batch_run(lsqr_handle* h, int32_t itn_limit, int max_chunks, Scalars* host)
{
    const TileBufs<Acc> tb = tile_bufs<Acc>(h);
    auto& B = h->batch;
    hipStream_t st = h->stream;
    const int chunk = std::max(1, h->chunk);
    const bool graph = h->use_graph && !h->profile;
    if (graph && (tb.graph[K] == nullptr || tb.graph_chunk[K] != chunk)) {
        if (tb.graph[K]) (void)hipGraphExecDestroy(tb.graph[K]);
        tb.graph[K] = nullptr;
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < chunk; ++k) batch_iteration<T, Acc, K>(h, st, nullptr);
        hipError_t e = hipStreamEndCapture(st, &g);
        if (e != hipSuccess) return fail(LSQR_E_HIP, "graph capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&tb.graph[K], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            tb.graph[K] = nullptr;
            return fail(LSQR_E_HIP, "graph instantiate: %s", hipGetErrorString(e));
        }
        tb.graph_chunk[K] = chunk;
    }
    if (h->profile && h->events.size() < (size_t)4 * chunk) {
        while (h->events.size() < (size_t)4 * chunk) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            h->events.push_back(e);
        }
    }
    int32_t done = 0;
    HIP_TRY(hipMemcpyAsync(&done, B.flag, sizeof done, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    int32_t itn_seen = 0;
    for (int c = 0; !done && itn_limit > 0 && (max_chunks <= 0 || c < max_chunks); ++c) {
        if (graph) {
            HIP_TRY(hipGraphLaunch(tb.graph[K], st));
        } else {
            for (int k = 0; k < chunk; ++k)
                batch_iteration<T, Acc, K>(h, st, h->profile ? &h->events[4 * k] : nullptr);
            HIP_TRY(hipGetLastError());
        }
        HIP_TRY(hipMemcpyAsync(host, B.sc, K * sizeof(Scalars), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(&done, B.flag, sizeof done, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        int32_t itn_max = 0;
        for (int r = 0; r < K; ++r) itn_max = std::max(itn_max, host[r].itn);
        if (h->profile) {
            const int ran = std::min(chunk, itn_max - itn_seen);
            for (int k = 0; k < ran; ++k) {
                float a = 0.f, b = 0.f;
                HIP_TRY(hipEventElapsedTime(&a, h->events[4 * k], h->events[4 * k + 1]));
                HIP_TRY(hipEventElapsedTime(&b, h->events[4 * k + 2], h->events[4 * k + 3]));
                h->ms1 += a;
                h->ms2 += b;
                h->n1 += 1;
                h->n2 += 1;
            }
        }
        if (!done && itn_max <= itn_seen)
            return fail(LSQR_E_HIP, "batched LSQR made no progress (itn %d)", itn_max);
        itn_seen = itn_max;
    }
    HIP_TRY(hipMemcpyAsync(host, B.sc, K * sizeof(Scalars), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return LSQR_OK;
}

void fill_batch_info(lsqr_info& in, const Scalars& s, int32_t itn, int32_t outer, double bnorm)
{
    memset(&in, 0, sizeof in);
    in.istop = s.istop;
    in.itn = itn;
    in.outer_steps = outer;
    in.rnorm = s.rnorm;
    in.arnorm = s.arnorm;
    in.anorm = s.anorm;
    in.acond = s.acond;
    in.xnorm = s.xnorm;
    in.bnorm = bnorm;
}

// One FP64 tile of K right-hand sides: B_tile = B[:, j0:j0+K] (row stride
// ldb), X_tile likewise. Per-RHS results in infos (host, may be NULL).
template <typename T, int K>
lsqr_status batch_tile(lsqr_handle* h, const double* Bm, int64_t ldb, double* X, int64_t ldx,
                       int32_t itn_limit, double atol, double btol, lsqr_info* infos,
                       int max_chunks)
{
    auto& B = h->batch;
    hipStream_t st = h->stream;
    const int64_t m = h->sv.m, n = h->sv.n;
    LSQR_TRY(batch_controls<K>(h, itn_limit, atol, btol));
    hipLaunchKernelGGL((batched::k_copy_ssq<double, K>), dim3(h->nb1), dim3(kBlock), 0, st, m, Bm,
                       ldb, B.U, B.part1, batch_row_map(h));
    LSQR_TRY((batch_init<T, double, K>(h)));
    Scalars host[kMaxTile];
    LSQR_TRY((batch_run<T, double, K>(h, itn_limit, max_chunks, host)));
    hipLaunchKernelGGL((batched::k_unprecond<K>), dim3(h->nbc), dim3(kBlock), 0, st, n, h->p,
                       (const double*)B.Y, X, ldx);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    if (infos)
        for (int r = 0; r < K; ++r) fill_batch_info(infos[r], host[r], host[r].itn, 0, host[r].bnorm);
    return LSQR_OK;
}

// Outer test of the refinement after a correction of size d (infinity norm)
// on a solution of size xmax, the previous correction being dprev (0 before
// the second step): stop once d <= tol xmax, or once the corrections contract
// (d <= dprev / 2) fast enough that the next one, estimated as d (d / dprev),
// is below kRefinePredict tol xmax. The second rule spares the step whose
// only effect would be a correction far below the tolerance (the inner solves
// gain a fixed factor per step, so one more step shrinks the error by that
// factor again).
constexpr double kRefinePredict = 1e-2;
inline bool refine_done(double d, double dprev, double xmax, double tol)
{
    if (d <= tol * xmax) return true;
    return dprev > 0.0 && d <= 0.5 * dprev && d * (d / dprev) <= kRefinePredict * tol * xmax;
}

// One tile of the refined form: K right-hand sides of an FP32-stored system,
// each with its own FP64 refinement loop (as lsqr_solve_refined) around FP32
// inner LSQR solves that advance together. Outer step: for every RHS still
// refining, r = b - A x in FP64 (stored as the FP32 start vector), then the
// inner tile solve (relative normal-equation stop atol, itn_limit), then
// x += p .* y. A RHS stops refining by refine_done (its correction against
// its solution and its previous correction), when its residual is zero or
// orthogonal to range(A), or after outer_limit steps; from then on it is
// masked (zero start vector: frozen at once) and its x no longer changes.
template <typename T, int K>
lsqr_status batch_refined_tile(lsqr_handle* h, const double* Bm, int64_t ldb, double* X,
                               int64_t ldx, int32_t itn_limit, double atol, int32_t outer_limit,
                               lsqr_info* infos)
{
    auto& B = h->batch;
    hipStream_t st = h->stream;
    const int64_t n = h->sv.n;
    hipLaunchKernelGGL((batched::k_zero_cols<K>), dim3(h->nbc), dim3(kBlock), 0, st, n, X, ldx);
    uint32_t live = (1u << K) - 1u;
    int32_t total_itn[kMaxTile] = {}, steps[kMaxTile] = {};
    double bnorm[kMaxTile] = {}, dprev[kMaxTile] = {};
    Scalars last[kMaxTile], host[kMaxTile];
    memset(last, 0, sizeof last);
    for (int outer = 1; outer <= outer_limit && live; ++outer) {
        LSQR_TRY(batch_controls<K>(h, itn_limit, 0.0, 0.0, std::max(atol, 1e-300)));
        // FP64 residual of the full problem of every live RHS (B itself at the
        // first step, where X = 0 and every RHS is live)
        if (outer == 1) {
            hipLaunchKernelGGL((batched::k_copy_ssq<float, K>), dim3(h->nb1), dim3(kBlock), 0, st,
                               h->sv.m, Bm, ldb, B.U32, B.part1, batch_row_map(h));
        } else {
            hipLaunchKernelGGL((batched::k_interleave_att<double, K>), dim3(h->nbc), dim3(kBlock),
                               0, st, (const double*)X, ldx, h->sv.att_base, h->sv.n_dfa, B.X3);
            hipLaunchKernelGGL((batched::k_resid<T, float, K>), dim3(h->nb1), dim3(kBlock), 0, st,
                               h->sv, (const double*)X, ldx, (const double*)B.X3, Bm, ldb, B.U32,
                               B.part1, batch_row_map(h), live);
        }
        LSQR_TRY((batch_init<T, float, K>(h)));
        LSQR_TRY((batch_run<T, float, K>(h, itn_limit, 0, host)));
        hipLaunchKernelGGL((batched::k_refine_update<K>), dim3(h->nbc), dim3(kBlock), 0, st, n,
                           h->p, (const double*)B.Y, X, ldx, live, B.partdd, B.partxx);
        hipLaunchKernelGGL((batched::k_refine_norms<K>), dim3(1), dim3(kBlock), 0, st,
                           (const double*)B.partdd, (const double*)B.partxx, h->nbc, B.sc);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(host, B.sc, K * sizeof(Scalars), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int r = 0; r < K; ++r) {
            if (!((live >> r) & 1u)) continue;
            if (outer == 1) bnorm[r] = host[r].bnorm;
            steps[r] = outer;
            total_itn[r] += host[r].itn;
            last[r] = host[r];
            // residual zero or orthogonal to range(A) (stopped at the start),
            // or a correction small against the solution
            if (host[r].itn == 0 ||
                refine_done(host[r].dmax, dprev[r], host[r].xmax, h->outer_tol))
                live &= ~(1u << r);
            dprev[r] = host[r].dmax;
        }
    }
    if (infos)
        for (int r = 0; r < K; ++r) fill_batch_info(infos[r], last[r], total_itn[r], steps[r], bnorm[r]);
    return LSQR_OK;
}

template <typename T>
lsqr_status batch_tile_k(lsqr_handle* h, bool refined, int K, const double* Bm, int64_t ldb,
                         double* X, int64_t ldx, int32_t itn_limit, double atol, double btol,
                         int32_t outer_limit, lsqr_info* infos, int max_chunks)
{
    if (K > 8 && !rhs_lanes_on(h))
        return fail(LSQR_E_UNSUPPORTED, "16-RHS tiles need fused mode 2 or 3, attitude mode 1 "
                                        "and LSQR_OPT_RHS_LANES = 1");
    if (refined) {
        switch (K) {
        case 1: return batch_refined_tile<T, 1>(h, Bm, ldb, X, ldx, itn_limit, atol, outer_limit, infos);
        case 2: return batch_refined_tile<T, 2>(h, Bm, ldb, X, ldx, itn_limit, atol, outer_limit, infos);
        case 4: return batch_refined_tile<T, 4>(h, Bm, ldb, X, ldx, itn_limit, atol, outer_limit, infos);
        case 8: return batch_refined_tile<T, 8>(h, Bm, ldb, X, ldx, itn_limit, atol, outer_limit, infos);
        case 16: return batch_refined_tile<T, 16>(h, Bm, ldb, X, ldx, itn_limit, atol, outer_limit, infos);
        default: return fail(LSQR_E_INVALID, "k-tile must be 1, 2, 4, 8 or 16");
        }
    }
    switch (K) {
    case 1: return batch_tile<T, 1>(h, Bm, ldb, X, ldx, itn_limit, atol, btol, infos, max_chunks);
    case 2: return batch_tile<T, 2>(h, Bm, ldb, X, ldx, itn_limit, atol, btol, infos, max_chunks);
    case 4: return batch_tile<T, 4>(h, Bm, ldb, X, ldx, itn_limit, atol, btol, infos, max_chunks);
    case 8: return batch_tile<T, 8>(h, Bm, ldb, X, ldx, itn_limit, atol, btol, infos, max_chunks);
    case 16: return batch_tile<T, 16>(h, Bm, ldb, X, ldx, itn_limit, atol, btol, infos, max_chunks);
    default: return fail(LSQR_E_INVALID, "k-tile must be 1, 2, 4, 8 or 16");
    }
}

// A few profiled iterations of one tile of K right-hand sides in precision
// Acc (the FP32 inner solve of the refined form, or FP64), from start vector
// B[:, 0:K]: milliseconds per RHS-iteration.
template <typename T, typename Acc, int K>
lsqr_status batch_probe(lsqr_handle* h, const double* Bm, int64_t ldb, double* ms)
{
    auto& B = h->batch;
    const TileBufs<Acc> tb = tile_bufs<Acc>(h);
    LSQR_TRY(batch_controls<K>(h, 1 << 20, 0.0, 0.0));
    hipLaunchKernelGGL((batched::k_copy_ssq<Acc, K>), dim3(h->nb1), dim3(kBlock), 0, h->stream,
                       h->sv.m, Bm, ldb, tb.U, B.part1, batch_row_map(h));
    LSQR_TRY((batch_init<T, Acc, K>(h)));
    Scalars host[kMaxTile];
    h->ms1 = h->ms2 = h->ms_pre = 0.0;
    h->n1 = h->n2 = 0;
    LSQR_TRY((batch_run<T, Acc, K>(h, 1 << 20, 1, host)));
    *ms = (h->ms1 + h->ms2) / std::max<int64_t>(1, h->n1) / K;
    return LSQR_OK;
}

// Autotuner: times a few profiled iterations of the first k-tile for every
// candidate K <= min(k, 8) (in the precision the solve will run) and keeps
// the K with the lowest time per RHS-iteration; the choice is kept per
// precision and per min(k, 8) until an option that selects kernels changes.
template <typename T>
lsqr_status batch_autotune(lsqr_handle* h, bool refined, const double* Bm, int64_t ldb, int32_t k,
                           int* out)
{
    auto& B = h->batch;
    const int saved_profile = h->profile, saved_chunk = h->chunk, saved_tests = h->tests;
    const double saved[5] = {h->ms1, h->ms2, (double)h->n1, (double)h->n2, h->ms_pre};
    int best = 1;
    double best_ms = 1e300;
    lsqr_status rc = LSQR_OK;
    memset(B.tuned_ms, 0, sizeof B.tuned_ms);
    h->profile = 1;
    h->tests = 0;
    h->chunk = 3;
    for (int K = 1; K <= kMaxTile && K <= k; K *= 2) {
        if (K > 8 && !rhs_lanes_on(h)) break;  // 16-RHS tiles need the RHS-across-lanes pass
        double ms = 0.0;
        auto probe = [&](auto KK) {
            constexpr int Kc = decltype(KK)::value;
            return refined ? batch_probe<T, float, Kc>(h, Bm, ldb, &ms)
                           : batch_probe<T, double, Kc>(h, Bm, ldb, &ms);
        };
        switch (K) {
        case 1: rc = probe(std::integral_constant<int, 1>()); break;
        case 2: rc = probe(std::integral_constant<int, 2>()); break;
        case 4: rc = probe(std::integral_constant<int, 4>()); break;
        case 8: rc = probe(std::integral_constant<int, 8>()); break;
        default: rc = probe(std::integral_constant<int, 16>()); break;
        }
        if (rc != LSQR_OK) break;
        B.tuned_ms[K] = ms;
        if (ms < best_ms) {
            best_ms = ms;
            best = K;
        }
    }
    h->profile = saved_profile;
    h->chunk = saved_chunk;
    h->tests = saved_tests;
    h->ms1 = saved[0];
    h->ms2 = saved[1];
    h->n1 = (int64_t)saved[2];
    h->n2 = (int64_t)saved[3];
    h->ms_pre = saved[4];
    if (rc != LSQR_OK) return rc;
    *out = best;
    return LSQR_OK;
}

inline int log2_cap(int32_t k)
{
    return k >= 16 ? 4 : (k >= 8 ? 3 : (k >= 4 ? 2 : (k >= 2 ? 1 : 0)));
}

template <typename T>
lsqr_status solve_batched(lsqr_handle* h, bool refined, const double* Bm, double* X, int32_t k,
                          int32_t itn_limit, double atol, double btol, int32_t outer_limit,
                          lsqr_info* infos)
{
    auto& B = h->batch;
    int K = h->ktile;
    if (K == 0) {
        const int cap = log2_cap(k);
        int& slot = B.tuned_k[refined ? 1 : 0][cap];
        if (slot == 0) {
            LSQR_TRY(batch_alloc(h, 1 << cap, refined));
            int best = 1;
            LSQR_TRY(batch_autotune<T>(h, refined, Bm, k, k, &best));
            slot = best;
        }
        K = slot;
        B.last_tuned = K;
    }
    LSQR_TRY(batch_alloc(h, K, refined));
    if (h->profile) {
        h->ms1 = h->ms2 = h->ms_pre = 0.0;
        h->n1 = h->n2 = 0;
    }
    int32_t j0 = 0;
    while (j0 < k) {
        int kt = K;
        while (kt > k - j0) kt /= 2;  // ragged end: 4, 2, 1
        LSQR_TRY(batch_tile_k<T>(h, refined, kt, Bm + j0, k, X + j0, k, itn_limit, atol, btol,
                                 outer_limit, infos ? infos + j0 : nullptr, 0));
        j0 += kt;
    }
    return LSQR_OK;
}

lsqr_status check_handle(lsqr_handle* h)
{
    if (!h) return fail(LSQR_E_INVALID, "null handle");
    HIP_TRY(hipSetDevice(h->device));
    return LSQR_OK;
}

// Address of the no-allocation scratch on the current device `dev`, taken
// once per device (with that device current) and kept for later calls.
lsqr_status scratch_setup(int dev)
{
    if (dev < 0 || dev >= kMaxDevices)
        return fail(LSQR_E_UNSUPPORTED, "device ordinal %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return LSQR_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
        return fail(LSQR_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
    return LSQR_OK;
}

}  // namespace

// ================================================================== C ABI

extern "C" {

const char* lsqr_last_error(void) { return g_last_error.c_str(); }

lsqr_status lsqr_create(const lsqr_system* sys, lsqr_handle** out)
{
    g_last_error.clear();
    if (!out) return fail(LSQR_E_INVALID, "out is null");
    *out = nullptr;
    if (!sys) return fail(LSQR_E_INVALID, "system descriptor is null");
    if (sys->n_rows <= 0) return fail(LSQR_E_INVALID, "n_rows must be > 0");
    if (sys->n_stars <= 0) return fail(LSQR_E_INVALID, "n_stars must be > 0");
    if (sys->n_astro < 0 || sys->n_astro > kAstro || sys->n_instr < 0 || sys->n_instr > kInstr ||
        sys->n_glob < 0 || sys->n_glob > kGlobMax || sys->n_axes < 0 || sys->n_par_axis < 0)
        return fail(LSQR_E_INVALID, "section sizes out of range (astro 0..5, instr 0..6, "
                                    "glob 0..5)");
    if (sys->n_axes != 0 && (sys->n_axes != kAxes || sys->n_par_axis != kParAxis))
        return fail(LSQR_E_UNSUPPORTED, "the attitude section is 3 axes x 4 parameters or absent "
                                        "(got %dx%d)", sys->n_axes, sys->n_par_axis);
    const int32_t natt = sys->n_axes ? kAxes * kParAxis : 0;
    if (sys->n_astro + natt + sys->n_instr + sys->n_glob < 1)
        return fail(LSQR_E_INVALID, "a row needs at least one coefficient");
    if (natt && sys->n_dfa < sys->n_par_axis)
        return fail(LSQR_E_INVALID, "n_dfa must be >= n_par_axis");
    if (sys->n_dfa < 0 || sys->n_instr_cols < sys->n_instr || sys->n_instr_cols < 0)
        return fail(LSQR_E_INVALID, "n_instr_cols must be >= n_instr and n_dfa >= 0");
    if (sys->n_instr_cols > INT32_MAX) return fail(LSQR_E_INVALID, "n_instr_cols too large");
    if (sys->value_type != LSQR_F64 && sys->value_type != LSQR_F32)
        return fail(LSQR_E_INVALID, "value_type must be LSQR_F64 or LSQR_F32");
    if (!sys->values || !sys->star_of_row || (natt && !sys->att_start) ||
        (sys->n_instr && !sys->instr_idx))
        return fail(LSQR_E_INVALID, "matrix array pointer is null");
    if (sys->n_rows > ((int64_t)1 << 40)) return fail(LSQR_E_INVALID, "n_rows too large");
    if (sys->n_con < 0 || sys->n_con > ((int64_t)1 << 31))
        return fail(LSQR_E_INVALID, "n_con must be in [0, 2^31]");
    if (sys->n_con > 0 && (!sys->con_rowptr || !sys->con_col || !sys->con_val))
        return fail(LSQR_E_INVALID, "constraint array pointer is null");

    lsqr_handle* h = new (std::nothrow) lsqr_handle();
    if (!h) return fail(LSQR_E_NOMEM, "host allocation failed");
    auto bail = [&](lsqr_status st) {
        lsqr_destroy(h);
        return st;
    };

    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) return bail(fail(LSQR_E_HIP, "hipGetDevice: %s", hipGetErrorString(e)));
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, h->device);
    if (e != hipSuccess)
        return bail(fail(LSQR_E_HIP, "hipGetDeviceProperties: %s", hipGetErrorString(e)));
    h->num_cu = prop.multiProcessorCount;
    // device address of the no-allocation scratch, once per device
    if (lsqr_status sst = scratch_setup(h->device); sst != LSQR_OK) return bail(sst);

    SysView& s = h->sv;
    s.val = sys->values;
    s.star = sys->star_of_row;
    s.att = sys->att_start;
    s.instr = sys->instr_idx;
    s.m = sys->n_rows;
    s.n_stars = sys->n_stars;
    s.n_dfa = sys->n_dfa;
    s.n_instr_cols = sys->n_instr_cols;
    // column order astro | att | instr | glob (Algorithms 2-3)
    s.na = sys->n_astro;
    s.natt = natt;
    s.ni = sys->n_instr;
    s.ng = sys->n_glob;
    s.off_att = s.na;
    s.off_instr = s.na + s.natt;
    s.off_glob = s.off_instr + s.ni;
    s.att_base = (int64_t)s.na * sys->n_stars;
    s.instr_base = s.att_base + (int64_t)sys->n_axes * sys->n_dfa;
    s.glob_base = s.instr_base + sys->n_instr_cols;
    s.n = s.glob_base + s.ng;
    h->generic = !(s.na == kAstro && s.natt == kAxes * kParAxis && s.ni == kInstr && s.ng == 1);
    h->nc = sys->n_con;
    if (h->nc > 0) {
        h->con_rowptr = sys->con_rowptr;
        h->con_col = sys->con_col;
        h->con_val = sys->con_val;
    }
    h->value_type = sys->value_type;
    h->precondition = sys->precondition ? 1 : 0;
    h->user_stream = static_cast<hipStream_t>(sys->stream);

    e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(fail(LSQR_E_HIP, "stream: %s", hipGetErrorString(e)));

    // grids
    const int64_t m = s.m, n = s.n;
    {
        // aprod1 grid: resident workgroups of the LDS-staged kernel
        const int64_t bytes = s.n_instr_cols * 8;
        int occ = 0;
        if (bytes <= kLdsXBudget)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &occ, k_aprod1<double, double, double, double, A1_LSQR, kBlock1, true>, kBlock1,
                (size_t)bytes);
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &occ, k_aprod1<double, double, double, double, A1_LSQR, kBlock1, false>, kBlock1, 0);
        if (e != hipSuccess || occ <= 0) occ = 2;
        h->nb1 = (int)std::max<int64_t>(
            1, std::min<int64_t>((int64_t)h->num_cu * occ, cdiv(m, 2 * kBlock1)));
    }
    {
        // aprod2: a fixed number of row ranges (16 waves per compute unit),
        // run by 1024-thread workgroups in the main pass (one per compute
        // unit whatever the LDS histogram size) and by 256-thread workgroups
        // in the attitude pass.
        const int64_t per = kBlock2 / kWave;
        int64_t nw = std::min<int64_t>((int64_t)h->num_cu * kWavesPerCU, cdiv(m, kWave));
        nw = std::max<int64_t>(per, cdiv(nw, per) * per);
        h->nw = nw;
        h->nb2 = (int)(nw / per);
        h->nba = (int)(nw / kWavesPerBlock);
    }
    h->nbc = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)h->num_cu * 4, cdiv(n, kBlock)));

    lsqr_status st;
    const int64_t nw = h->nw;
    if ((st = dalloc(&h->wb, nw + 1)) != LSQR_OK) return bail(st);
    if ((st = dalloc(&h->p, n)) != LSQR_OK) return bail(st);
    if ((st = dalloc(&h->v, n)) != LSQR_OK) return bail(st);
    if ((st = dalloc(&h->w, n)) != LSQR_OK) return bail(st);
    if ((st = dalloc(&h->y, n)) != LSQR_OK) return bail(st);
    if ((st = dalloc(&h->part1, std::max(h->nb1, h->nb2) + 1)) != LSQR_OK) return bail(st);
    if ((st = dalloc(&h->partc, h->nbc)) != LSQR_OK) return bail(st);
    if ((st = dalloc(&h->partdd, h->nbc)) != LSQR_OK) return bail(st);
    if ((st = dalloc(&h->partxx, h->nbc)) != LSQR_OK) return bail(st);
    if ((st = dalloc(&h->gpart_raw, std::max<int64_t>(h->nb2, (int64_t)h->nba * kGlobMax))) !=
        LSQR_OK)
        return bail(st);
    if ((st = dalloc(&h->flag, 1)) != LSQR_OK) return bail(st);
    if ((st = dalloc(&h->sc, 1)) != LSQR_OK) return bail(st);
    e = hipHostMalloc(reinterpret_cast<void**>(&h->sc_host), sizeof(Scalars), hipHostMallocDefault);
    if (e != hipSuccess) return bail(fail(LSQR_E_NOMEM, "pinned scalars: %s", hipGetErrorString(e)));
    memset(h->sc_host, 0, sizeof(Scalars));

    // Work ordered after whatever produced the matrix on the caller's stream.
    e = hipStreamSynchronize(h->user_stream);
    if (e != hipSuccess) return bail(fail(LSQR_E_HIP, "sync: %s", hipGetErrorString(e)));
    hipStream_t st0 = h->stream;

    // 1. validate every index before any kernel gathers or scatters with it
    int32_t zero = 0;
    e = hipMemcpyAsync(h->flag, &zero, sizeof zero, hipMemcpyHostToDevice, st0);
    if (e != hipSuccess) return bail(fail(LSQR_E_HIP, "flag: %s", hipGetErrorString(e)));
    hipLaunchKernelGGL(k_validate, dim3(std::min<int64_t>(cdiv(m, kBlock), 8192)), dim3(kBlock), 0,
                       st0, s, h->flag);
    int32_t bad = 0;
    e = hipMemcpyAsync(&bad, h->flag, sizeof bad, hipMemcpyDeviceToHost, st0);
    if (e == hipSuccess) e = hipStreamSynchronize(st0);
    if (e != hipSuccess) return bail(fail(LSQR_E_HIP, "validate: %s", hipGetErrorString(e)));
    if (bad) {
        return bail(fail(LSQR_E_INVALID,
                         "index validation failed:%s%s%s%s",
                         (bad & 1) ? " star_of_row out of [0,n_stars)" : "",
                         (bad & 2) ? " star_of_row not non-decreasing" : "",
                         (bad & 4) ? " att_start out of [0,n_dfa-4]" : "",
                         (bad & 8) ? " instr_idx out of [0,n_instr_cols)" : ""));
    }
    if (h->nc > 0) {
        // row pointers first (they bound every later read), then the columns
        if ((st = dalloc(&h->con_ssq, h->nc)) != LSQR_OK) return bail(st);
        h->con_grid = (int)std::min<int64_t>(h->nc, 1024);
        hipLaunchKernelGGL(k_validate_con_rows, dim3(std::min<int64_t>(cdiv(h->nc, kBlock), 1024)),
                           dim3(kBlock), 0, st0, h->nc, h->con_rowptr, h->flag);
        int64_t nnz = 0;
        e = hipMemcpyAsync(&bad, h->flag, sizeof bad, hipMemcpyDeviceToHost, st0);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&nnz, h->con_rowptr + h->nc, sizeof nnz, hipMemcpyDeviceToHost, st0);
        if (e == hipSuccess) e = hipStreamSynchronize(st0);
        if (e != hipSuccess)
            return bail(fail(LSQR_E_HIP, "constraint validation: %s", hipGetErrorString(e)));
        if (bad)
            return bail(fail(LSQR_E_INVALID,
                             "constraint rows: con_rowptr must start at 0 and be non-decreasing"));
        h->con_nnz = nnz;
        hipLaunchKernelGGL(k_validate_con_cols,
                           dim3(std::max<int64_t>(1, std::min<int64_t>(cdiv(nnz, kBlock), 8192))),
                           dim3(kBlock), 0, st0, nnz, h->con_col, n, h->flag);
        e = hipMemcpyAsync(&bad, h->flag, sizeof bad, hipMemcpyDeviceToHost, st0);
        if (e == hipSuccess) e = hipStreamSynchronize(st0);
        if (e != hipSuccess)
            return bail(fail(LSQR_E_HIP, "constraint validation: %s", hipGetErrorString(e)));
        if (bad) return bail(fail(LSQR_E_INVALID, "constraint rows: con_col out of [0, n)"));
    }

    // 2. star-aligned row ranges of the aprod2 waves
    hipLaunchKernelGGL((k_wave_bounds<int64_t>), dim3(cdiv(nw + 1, kBlock)), dim3(kBlock), 0, st0,
                       s.star, m, nw, h->wb);

    // 3. column scaling p from the column norms (squared-coefficient aprod2)
    double* ssq = nullptr;
    if ((st = dalloc(&ssq, n)) != LSQR_OK) return bail(st);
    const int64_t hc = instr_hcols(h, 1);
    const size_t lds = (size_t)(hc * 8);
    hipLaunchKernelGGL((k_fill<double>), dim3(h->nbc), dim3(kBlock), 0, st0, n, ssq, 0.0);
    if (h->generic) {
        if (h->value_type == LSQR_F64) {
            hipLaunchKernelGGL((k_gen_aprod2<double, double, double, true, true>), dim3(h->nba),
                               dim3(kBlock), lds, st0, s, (const double*)nullptr, ssq, h->wb,
                               h->gpart_raw, hc, (const Scalars*)nullptr, (const int32_t*)nullptr);
            launch_instr_tail<double, double, 1, true>(h, nullptr, nullptr, ssq, hc, nullptr, st0);
        } else {
            hipLaunchKernelGGL((k_gen_aprod2<float, double, double, true, true>), dim3(h->nba),
                               dim3(kBlock), lds, st0, s, (const double*)nullptr, ssq, h->wb,
                               h->gpart_raw, hc, (const Scalars*)nullptr, (const int32_t*)nullptr);
            launch_instr_tail<float, double, 1, true>(h, nullptr, nullptr, ssq, hc, nullptr, st0);
        }
        hipLaunchKernelGGL((k_gen_glob_sum<double>), dim3(1), dim3(kBlock), 0, st0, h->gpart_raw,
                           h->nba, s.ng, ssq + s.glob_base, (const Scalars*)nullptr);
    } else if (h->value_type == LSQR_F64) {
        hipLaunchKernelGGL((k_aprod2<double, double, double, true, true, true, kBlock2>),
                           dim3(h->nb2), dim3(kBlock2), lds, st0, s, (const double*)nullptr, ssq,
                           h->wb, h->gpart_raw, hc, (const Scalars*)nullptr);
        launch_instr_tail<double, double, 1, true>(h, nullptr, nullptr, ssq, hc, nullptr, st0);
    } else {
        hipLaunchKernelGGL((k_aprod2<float, double, double, true, true, true, kBlock2>),
                           dim3(h->nb2), dim3(kBlock2), lds, st0, s, (const double*)nullptr, ssq,
                           h->wb, h->gpart_raw, hc, (const Scalars*)nullptr);
        launch_instr_tail<float, double, 1, true>(h, nullptr, nullptr, ssq, hc, nullptr, st0);
    }
    if (!h->generic)
        hipLaunchKernelGGL((k_glob_sum<double>), dim3(1), dim3(kBlock), 0, st0, h->gpart_raw,
                           h->nb2, ssq + s.glob_base, (const Scalars*)nullptr);
    if (h->nc > 0)
        hipLaunchKernelGGL((k_con_aprod2<double, double, true>), dim3(h->con_grid), dim3(kBlock), 0,
                           st0, h->nc, h->con_rowptr, h->con_col, h->con_val,
                           (const double*)nullptr, ssq, (const Scalars*)nullptr);
    hipLaunchKernelGGL(k_make_p, dim3(h->nbc), dim3(kBlock), 0, st0, n, ssq, h->p, h->precondition);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st0);
    (void)hipFree(ssq);
    if (e != hipSuccess) return bail(fail(LSQR_E_HIP, "set-up kernels: %s", hipGetErrorString(e)));

    *out = h;
    return LSQR_OK;
}

lsqr_status lsqr_destroy(lsqr_handle* h)
{
    if (!h) return LSQR_OK;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    release_path(h->p64);
    release_path(h->p32);
    batch_free(h);
    dfree(h->wb);
    dfree(h->perm);
    dfree(h->tloc);
    dfree(h->invperm);
    dfree(h->bstart);
    dfree(h->S2);
    dfree(h->var);
    dfree(h->x3_raw);
    dfree(h->x3_raw32);
    dfree(h->gpart_raw32);
    if (h->att_sorted) (void)hipFree(h->att_sorted);
    h->att_sorted = nullptr;
    dfree(h->p);
    dfree(h->v);
    dfree(h->w);
    dfree(h->y);
    dfree(h->part1);
    dfree(h->partc);
    dfree(h->partdd);
    dfree(h->partxx);
    dfree(h->gpart_raw);
    dfree(h->flag);
    dfree(h->con_ssq);
    dfree(h->star32);
    dfree(h->instr16);
    dfree(h->sc);
    if (h->sc_host) (void)hipHostFree(h->sc_host);
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return LSQR_OK;
}

lsqr_status lsqr_set_option(lsqr_handle* h, int32_t option, double value)
{
    if (!h) return fail(LSQR_E_INVALID, "null handle");
    switch (option) {
    case LSQR_OPT_CONLIM:
        if (!(value >= 0.0)) return fail(LSQR_E_INVALID, "conlim must be >= 0");
        h->conlim = value;
        return LSQR_OK;
    case LSQR_OPT_TESTS:
        h->tests = value != 0.0 ? 1 : 0;
        return LSQR_OK;
    case LSQR_OPT_CHUNK:
        if (!(value >= 1.0 && value <= 4096.0)) return fail(LSQR_E_INVALID, "chunk in [1,4096]");
        h->chunk = (int)value;
        return LSQR_OK;
    case LSQR_OPT_GRAPH:
        h->use_graph = value != 0.0 ? 1 : 0;
        return LSQR_OK;
    case LSQR_OPT_PROFILE:
        h->profile = value != 0.0 ? 1 : 0;
        return LSQR_OK;
    case LSQR_OPT_ATT_MODE:
    case LSQR_OPT_ASTRO_SCAN: {
        if (option == LSQR_OPT_ATT_MODE && !(value == 0.0 || value == 1.0))
            return fail(LSQR_E_INVALID, "attitude mode must be 0 or 1");
        const int v = option == LSQR_OPT_ATT_MODE ? (int)value : (value != 0.0 ? 1 : 0);
        int& slot = option == LSQR_OPT_ATT_MODE ? h->att_mode : h->astro_scan;
        if (slot != v) {  // captured graphs bake in the kernel choice
            drop_graphs(h);
        }
        slot = v;
        return LSQR_OK;
    }
    case LSQR_OPT_ATT_INTERLEAVE:
    case LSQR_OPT_FUSED: {
        if (option == LSQR_OPT_FUSED &&
            !(value == 0.0 || value == 1.0 || value == 2.0 || value == 3.0))
            return fail(LSQR_E_INVALID, "fused mode must be 0, 1, 2 or 3");
        const int v = option == LSQR_OPT_FUSED ? (int)value : (value != 0.0 ? 1 : 0);
        int& slot = option == LSQR_OPT_FUSED ? h->fused : h->att_il;
        if (slot != v) {
            drop_graphs(h);
        }
        slot = v;
        return LSQR_OK;
    }
    case LSQR_OPT_KTILE:
        if (!(value == 0.0 || value == 1.0 || value == 2.0 || value == 4.0 || value == 8.0 ||
              value == 16.0))
            return fail(LSQR_E_INVALID, "k-tile must be 0 (autotune), 1, 2, 4, 8 or 16");
        h->ktile = (int)value;
        return LSQR_OK;
    case LSQR_OPT_ATT_RHS:
        if (h->att_ready)
            return fail(LSQR_E_STATE, "attitude sweep width must be set before the first solve");
        if (!(value == 1.0 || value == 2.0 || value == 4.0 || value == 8.0))
            return fail(LSQR_E_INVALID, "attitude sweep width must be 1, 2, 4 or 8");
        h->att_rhs = (int)value;
        return LSQR_OK;
    case LSQR_OPT_ATT_BUCKETS: {
        if (h->att_ready)
            return fail(LSQR_E_STATE, "attitude buckets must be set before the first solve");
        if (!(value >= 0.0 && value <= 2147483647.0))
            return fail(LSQR_E_INVALID, "attitude bucket count must be in [0, 2^31)");
        h->att_buckets = (int64_t)value;
        return LSQR_OK;
    }
    case LSQR_OPT_VARIANCE: {
        const int v = value != 0.0 ? 1 : 0;
        if (h->var_on != v) {  // captured graphs bake in the variance pointer
            drop_graphs(h);
        }
        h->var_on = v;
        return LSQR_OK;
    }
    case LSQR_OPT_COMPACT_INDEX: {
        const int v = value != 0.0 ? 1 : 0;
        if (!v && h->star32) {  // back to the caller's arrays
            drop_graphs(h);
            dfree(h->star32);
            dfree(h->instr16);
            h->sv.star32 = nullptr;
            h->sv.instr16 = nullptr;
        }
        if (v && !h->compact) h->compact_tried = 0;
        h->compact = v;
        return LSQR_OK;
    }
    case LSQR_OPT_RHS_LANES: {
        const int v = value != 0.0 ? 1 : 0;
        if (h->rhs_lanes != v) drop_graphs(h);
        h->rhs_lanes = v;
        return LSQR_OK;
    }
    case LSQR_OPT_PIPELINE: {
        const int v = value != 0.0 ? 1 : 0;
        if (h->pipe != v) drop_graphs(h);
        h->pipe = v;
        return LSQR_OK;
    }
    case LSQR_OPT_OUTER_TOL:
        if (!(value >= 0.0)) return fail(LSQR_E_INVALID, "outer tolerance must be >= 0");
        h->outer_tol = value;
        return LSQR_OK;
    default:
        return fail(LSQR_E_INVALID, "unknown option %d", option);
    }
}

lsqr_status lsqr_aprod1(lsqr_handle* h, const double* x, double* y)
{
    LSQR_TRY(check_handle(h));
    if (!x || !y) return fail(LSQR_E_INVALID, "null vector");
    const double* x3 = nullptr;
    if (h->att_il && h->sv.natt > 0 && !h->generic) {
        if (!h->x3_raw) LSQR_TRY(dalloc(&h->x3_raw, (int64_t)kAxes * h->sv.n_dfa));
        launch_interleave_att<double>(h, x, h->x3_raw, nullptr, h->user_stream);
        x3 = h->x3_raw;
    }
    if (h->value_type == LSQR_F64)
        launch_aprod1<double, double, double, double, A1_ACCUM>(h, x, y, nullptr, nullptr, nullptr,
                                                                h->user_stream, nullptr, x3);
    else
        launch_aprod1<float, double, double, double, A1_ACCUM>(h, x, y, nullptr, nullptr, nullptr,
                                                               h->user_stream, nullptr, x3);
    HIP_TRY(hipGetLastError());
    return LSQR_OK;
}

lsqr_status lsqr_aprod1_noalloc(lsqr_handle* h, const double* x, double* y)
{
    LSQR_TRY(check_handle(h));
    if (!x || !y) return fail(LSQR_E_INVALID, "null vector");
    const double* x3 = nullptr;
    if (h->att_il && h->sv.natt > 0 && !h->generic) {
        const int64_t need = (int64_t)kAxes * h->sv.n_dfa;
        if (need > (int64_t)LSQR_NOALLOC_ATT_MAX)
            return fail(LSQR_E_INVALID,
                        "lsqr_aprod1_noalloc: 3 n_dfa = %lld exceeds the scratch of %lld doubles",
                        (long long)need, (long long)LSQR_NOALLOC_ATT_MAX);
        double* sp = nullptr;
        {
            std::lock_guard<std::mutex> lock(g_scratch_mu);
            sp = g_scratch_ptr[h->device];
        }
        if (!sp) return fail(LSQR_E_STATE, "no-allocation scratch not set up on this device");
        // every element that k_aprod1 reads is rewritten here first
        launch_interleave_att<double>(h, x, sp, nullptr, h->user_stream);
        x3 = sp;
    }
    if (h->value_type == LSQR_F64)
        launch_aprod1<double, double, double, double, A1_ACCUM>(h, x, y, nullptr, nullptr, nullptr,
                                                                h->user_stream, nullptr, x3);
    else
        launch_aprod1<float, double, double, double, A1_ACCUM>(h, x, y, nullptr, nullptr, nullptr,
                                                               h->user_stream, nullptr, x3);
    HIP_TRY(hipGetLastError());
    return LSQR_OK;
}

lsqr_status lsqr_aprod2(lsqr_handle* h, double* x, const double* y)
{
    LSQR_TRY(check_handle(h));
    if (!x || !y) return fail(LSQR_E_INVALID, "null vector");
    LSQR_TRY(ensure_att(h));
    const int64_t hc = instr_hcols(h, 1);
    // y in row order: the attitude pass (where the bucket order exists:
    // attitude section present, mode 1) reads it through the permutation
    const int32_t* gperm = att_pass_on(h) ? (const int32_t*)h->perm : nullptr;
    if (h->value_type == LSQR_F64)
        launch_aprod2<double, double>(h, y, nullptr, x, h->gpart_raw, hc, nullptr,
                                      h->user_stream, y, gperm);
    else
        launch_aprod2<float, double>(h, y, nullptr, x, h->gpart_raw, hc, nullptr,
                                     h->user_stream, y, gperm);
    HIP_TRY(hipGetLastError());
    return LSQR_OK;
}

lsqr_status lsqr_aprod1_f32(lsqr_handle* h, const float* x, float* y)
{
    LSQR_TRY(check_handle(h));
    if (!x || !y) return fail(LSQR_E_INVALID, "null vector");
    if (h->value_type != LSQR_F32)
        return fail(LSQR_E_STATE, "lsqr_aprod1_f32 needs an LSQR_F32 system");
    const float* x3 = nullptr;
    if (h->att_il && h->sv.natt > 0 && !h->generic) {
        if (!h->x3_raw32) LSQR_TRY(dalloc(&h->x3_raw32, (int64_t)kAxes * h->sv.n_dfa));
        launch_interleave_att<float>(h, x, h->x3_raw32, nullptr, h->user_stream);
        x3 = h->x3_raw32;
    }
    launch_aprod1<float, float, float, float, A1_ACCUM>(h, x, y, nullptr, nullptr, nullptr,
                                                        h->user_stream, nullptr, x3);
    HIP_TRY(hipGetLastError());
    return LSQR_OK;
}

lsqr_status lsqr_aprod2_f32(lsqr_handle* h, float* x, const float* y)
{
    LSQR_TRY(check_handle(h));
    if (!x || !y) return fail(LSQR_E_INVALID, "null vector");
    if (h->value_type != LSQR_F32)
        return fail(LSQR_E_STATE, "lsqr_aprod2_f32 needs an LSQR_F32 system");
    LSQR_TRY(ensure_att(h));
    if (!h->gpart_raw32)
        LSQR_TRY(dalloc(&h->gpart_raw32, std::max<int64_t>(h->nb2, (int64_t)h->nba * kGlobMax)));
    const int64_t hc = instr_hcols(h, 1);
    const int32_t* gperm = att_pass_on(h) ? (const int32_t*)h->perm : nullptr;
    launch_aprod2<float, float>(h, y, nullptr, x, h->gpart_raw32, hc, nullptr, h->user_stream, y,
                                gperm);
    HIP_TRY(hipGetLastError());
    return LSQR_OK;
}

lsqr_status lsqr_get_precond(lsqr_handle* h, double* p_out)
{
    LSQR_TRY(check_handle(h));
    if (!p_out) return fail(LSQR_E_INVALID, "null output");
    HIP_TRY(hipMemcpyAsync(p_out, h->p, (size_t)h->sv.n * sizeof(double), hipMemcpyDeviceToDevice,
                           h->user_stream));
    return LSQR_OK;
}

lsqr_status lsqr_get_variance(lsqr_handle* h, double* var_out)
{
    LSQR_TRY(check_handle(h));
    if (!var_out) return fail(LSQR_E_INVALID, "null output");
    if (!h->var_valid || !h->var)
        return fail(LSQR_E_STATE, "no variance: run lsqr_solve with LSQR_OPT_VARIANCE = 1");
    hipLaunchKernelGGL(k_unprecond_var, dim3(h->nbc), dim3(kBlock), 0, h->stream, h->sv.n, h->p,
                       (const double*)h->var, var_out);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LSQR_OK;
}

lsqr_status lsqr_num_cols(lsqr_handle* h, int64_t* n_out)
{
    if (!h || !n_out) return fail(LSQR_E_INVALID, "null argument");
    *n_out = h->sv.n;
    return LSQR_OK;
}

lsqr_status lsqr_solve(lsqr_handle* h, const double* b, double* x, int32_t itn_limit, double atol,
                       double btol, lsqr_info* info)
{
    LSQR_TRY(check_handle(h));
    if (!b || !x) return fail(LSQR_E_INVALID, "null vector");
    if (itn_limit < 0) return fail(LSQR_E_INVALID, "itn_limit must be >= 0");
    if (!(atol >= 0.0) || !(btol >= 0.0)) return fail(LSQR_E_INVALID, "atol, btol must be >= 0");
    HIP_TRY(hipStreamSynchronize(h->user_stream));
    if (h->value_type == LSQR_F64)
        LSQR_TRY(solve_fp64<double>(h, b, x, itn_limit, atol, btol, info));
    else
        LSQR_TRY(solve_fp64<float>(h, b, x, itn_limit, atol, btol, info));
    return LSQR_OK;
}

lsqr_status lsqr_solve_refined(lsqr_handle* h, const double* b, double* x, int32_t itn_limit,
                               double atol, double btol, int32_t outer_limit, lsqr_info* info)
{
    LSQR_TRY(check_handle(h));
    if (!b || !x) return fail(LSQR_E_INVALID, "null vector");
    if (h->value_type != LSQR_F32)
        return fail(LSQR_E_STATE, "lsqr_solve_refined needs an LSQR_F32 system");
    if (itn_limit < 0 || outer_limit < 1)
        return fail(LSQR_E_INVALID, "itn_limit >= 0 and outer_limit >= 1 required");
    if (!(atol >= 0.0) || !(btol >= 0.0)) return fail(LSQR_E_INVALID, "atol, btol must be >= 0");
    HIP_TRY(hipStreamSynchronize(h->user_stream));
    h->var_valid = 0;
    LSQR_TRY(ensure_att(h));
    LSQR_TRY(ensure_compact(h));
    LSQR_TRY((prepare_path<float, float>(h, h->p32)));
    Path<float>& P = h->p32;
    const int64_t n = h->sv.n;
    if (h->profile) {
        h->ms1 = h->ms2 = h->ms_pre = 0.0;
        h->n1 = h->n2 = 0;
    }
    double* part_d = h->partdd;  // reused: not live between outer steps
    double* part_x = h->partxx;
    hipLaunchKernelGGL((k_fill<double>), dim3(h->nbc), dim3(kBlock), 0, h->stream, n, x, 0.0);
    int32_t total_itn = 0, outer = 0;
    double bnorm = 0.0, dprev = 0.0;
    Scalars last{};
    for (outer = 1; outer <= outer_limit; ++outer) {
        // Each correction problem min ||A d - r|| has a residual dominated by the
        // irreducible least-squares residual, so its inner solve stops on the
        // relative decrease of ||Abar^T r|| (tolerance atol) or the itn limit.
        LSQR_TRY(upload_controls(h, itn_limit, 0.0, 0.0, std::max(atol, 1e-300)));
        // FP64 residual of the full problem, stored as the FP32 start vector
        // (b itself at the first step, where x = 0)
        if (outer == 1) {
            hipLaunchKernelGGL((k_copy_ssq<float>), dim3(h->nb1), dim3(kBlock), 0, h->stream,
                               h->sv.m, b, P.u, h->part1, row_map(h));
            if (h->nc > 0)
                hipLaunchKernelGGL((k_copy_ssq<float>), dim3(1), dim3(kBlock), 0, h->stream,
                                   h->nc, b + h->sv.m, P.u + h->sv.m, h->part1 + h->nb1,
                                   (const int32_t*)nullptr);
        } else {
            const double* x3 = nullptr;
            if (h->att_il && h->sv.natt > 0 && !h->generic) {
                if (!h->x3_raw) LSQR_TRY(dalloc(&h->x3_raw, (int64_t)kAxes * h->sv.n_dfa));
                launch_interleave_att<double>(h, x, h->x3_raw, nullptr, h->stream);
                x3 = h->x3_raw;
            }
            launch_aprod1<float, double, double, float, A1_RESID>(
                h, (const double*)x, P.u, b, nullptr, h->part1, h->stream, row_map(h), x3);
        }
        launch_init<float, float>(h, P, h->stream);
        HIP_TRY(hipGetLastError());
        LSQR_TRY(read_scalars(h));
        if (outer == 1) bnorm = h->sc_host->bnorm;
        if (h->sc_host->done) {  // residual zero or orthogonal to range(A)
            last = *h->sc_host;
            break;
        }
        if (itn_limit > 0) LSQR_TRY((run_iterations<float, float>(h, P)));
        last = *h->sc_host;
        total_itn += last.itn;
        hipLaunchKernelGGL(k_refine_update, dim3(h->nbc), dim3(kBlock), 0, h->stream, n, h->p, h->y,
                           x, part_d, part_x);
        hipLaunchKernelGGL(k_refine_norms, dim3(1), dim3(kBlock), 0, h->stream, part_d, part_x,
                           h->nbc, h->sc);
        HIP_TRY(hipGetLastError());
        LSQR_TRY(read_scalars(h));
        if (refine_done(h->sc_host->dmax, dprev, h->sc_host->xmax, h->outer_tol)) break;
        dprev = h->sc_host->dmax;
    }
    if (outer > outer_limit) outer = outer_limit;
    *h->sc_host = last;
    fill_info(h, info, total_itn, outer, bnorm);
    return LSQR_OK;
}

lsqr_status lsqr_solve_batched(lsqr_handle* h, const double* B, double* X, int32_t k,
                               int32_t itn_limit, double atol, double btol, lsqr_info* infos)
{
    LSQR_TRY(check_handle(h));
    if (!B || !X) return fail(LSQR_E_INVALID, "null matrix");
    if (k < 1 || k > 4096) return fail(LSQR_E_INVALID, "k must be in [1, 4096]");
    if (itn_limit < 0) return fail(LSQR_E_INVALID, "itn_limit must be >= 0");
    if (!(atol >= 0.0) || !(btol >= 0.0)) return fail(LSQR_E_INVALID, "atol, btol must be >= 0");
    if (h->generic)
        return fail(LSQR_E_UNSUPPORTED,
                    "batched solves are built for the 5 + 3x4 + 6 + 1 row layout only");
    if (h->nc > 0)
        return fail(LSQR_E_UNSUPPORTED, "batched solves are built without constraint rows");
    HIP_TRY(hipStreamSynchronize(h->user_stream));
    h->var_valid = 0;
    LSQR_TRY(ensure_att(h));
    LSQR_TRY(ensure_compact(h));
    if (h->value_type == LSQR_F64)
        LSQR_TRY(solve_batched<double>(h, false, B, X, k, itn_limit, atol, btol, 0, infos));
    else
        LSQR_TRY(solve_batched<float>(h, false, B, X, k, itn_limit, atol, btol, 0, infos));
    return LSQR_OK;
}

lsqr_status lsqr_solve_batched_refined(lsqr_handle* h, const double* B, double* X, int32_t k,
                                       int32_t itn_limit, double atol, double btol,
                                       int32_t outer_limit, lsqr_info* infos)
{
    LSQR_TRY(check_handle(h));
    if (!B || !X) return fail(LSQR_E_INVALID, "null matrix");
    if (h->value_type != LSQR_F32)
        return fail(LSQR_E_STATE, "lsqr_solve_batched_refined needs an LSQR_F32 system");
    if (k < 1 || k > 4096) return fail(LSQR_E_INVALID, "k must be in [1, 4096]");
    if (itn_limit < 0 || outer_limit < 1)
        return fail(LSQR_E_INVALID, "itn_limit >= 0 and outer_limit >= 1 required");
    if (!(atol >= 0.0) || !(btol >= 0.0)) return fail(LSQR_E_INVALID, "atol, btol must be >= 0");
    if (h->generic)
        return fail(LSQR_E_UNSUPPORTED,
                    "batched solves are built for the 5 + 3x4 + 6 + 1 row layout only");
    if (h->nc > 0)
        return fail(LSQR_E_UNSUPPORTED, "batched solves are built without constraint rows");
    HIP_TRY(hipStreamSynchronize(h->user_stream));
    h->var_valid = 0;
    LSQR_TRY(ensure_att(h));
    LSQR_TRY(ensure_compact(h));
    LSQR_TRY(solve_batched<float>(h, true, B, X, k, itn_limit, atol, btol, outer_limit, infos));
    return LSQR_OK;
}

lsqr_status lsqr_batch_tuning(lsqr_handle* h, int32_t* k_tile, double* ms_per_rhs_iter)
{
    if (!h) return fail(LSQR_E_INVALID, "null handle");
    if (k_tile) *k_tile = h->batch.last_tuned;
    if (ms_per_rhs_iter)
        for (int K = 1, i = 0; K <= kMaxTile; K *= 2, ++i) ms_per_rhs_iter[i] = h->batch.tuned_ms[K];
    return LSQR_OK;
}

lsqr_status lsqr_pass_times(lsqr_handle* h, double* ms, int64_t* n, int32_t* mode,
                            int32_t* compact)
{
    if (!h) return fail(LSQR_E_INVALID, "null handle");
    if (!ms || !n) return fail(LSQR_E_INVALID, "null output");
    if (mode) *mode = h->last_mode;
    if (compact) *compact = h->sv.star32 != nullptr ? 1 : 0;
    ms[0] = h->ms_pre;
    ms[1] = h->ms1 - h->ms_pre;
    ms[2] = h->ms2;
    n[0] = n[1] = h->n1;
    n[2] = h->n2;
    return LSQR_OK;
}

lsqr_status lsqr_kernel_times(lsqr_handle* h, double* ms_aprod1, int64_t* n_aprod1,
                              double* ms_aprod2, int64_t* n_aprod2)
{
    if (!h) return fail(LSQR_E_INVALID, "null handle");
    if (ms_aprod1) *ms_aprod1 = h->ms1;
    if (n_aprod1) *n_aprod1 = h->n1;
    if (ms_aprod2) *ms_aprod2 = h->ms2;
    if (n_aprod2) *n_aprod2 = h->n2;
    return LSQR_OK;
}

}  // extern "C"
