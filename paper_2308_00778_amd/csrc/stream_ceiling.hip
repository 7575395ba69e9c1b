// Streaming kernels that measure the practical HBM ceiling the row passes of
// the solver are compared with: a plain read of large device buffers (what
// a pass that only streams the matrix could reach), a plain write, and a
// copy. Measurement only: the solver never calls them.
//
// Each kernel is a grid-stride loop over 16-byte elements with nontemporal
// loads and stores, the access form of the solver's row passes; the read
// kernel folds what it reads into one value per workgroup so that the loads
// cannot be dropped.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 512;
typedef uint32_t v4u __attribute__((ext_vector_type(4)));  // one 16-byte element

__global__ __launch_bounds__(kThreads) void k_read(const v4u* __restrict__ p, int64_t n,
                                                    double* __restrict__ sink)
{
    uint32_t acc = 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    // four loads in flight per thread
    for (; i + 3 * stride < n; i += 4 * stride) {
        const v4u a = __builtin_nontemporal_load(&p[i]);
        const v4u b = __builtin_nontemporal_load(&p[i + stride]);
        const v4u c = __builtin_nontemporal_load(&p[i + 2 * stride]);
        const v4u d = __builtin_nontemporal_load(&p[i + 3 * stride]);
        acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w;
        acc ^= c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
    }
    for (; i < n; i += stride) {
        const v4u a = __builtin_nontemporal_load(&p[i]);
        acc ^= a.x ^ a.y ^ a.z ^ a.w;
    }
    __shared__ uint32_t red[kThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < kThreads; ++k) t ^= red[k];
        sink[blockIdx.x] = (double)t;
    }
}

__global__ __launch_bounds__(kThreads) void k_write(v4u* __restrict__ p, int64_t n, uint32_t v)
{
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    const v4u w = {v, v, v, v};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(w, &p[i]);
}

__global__ __launch_bounds__(kThreads) void k_copy(const v4u* __restrict__ s,
                                                    v4u* __restrict__ d, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(&s[i]), &d[i]);
}

int grid_size()
{
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 1024;
    return cu * 8;
}

}  // namespace

extern "C" {

// Workgroups of every launch: the size the sink of sc_read must have.
int sc_grid(void) { return grid_size(); }

// Reads `bytes` (a multiple of 16, 16-byte aligned) at p; sink: device
// array of sc_grid() doubles. Asynchronous on `stream`. 0, or -1 on a bad
// argument, or the HIP error code of the launch.
int sc_read(const void* p, int64_t bytes, double* sink, void* stream)
{
    if (!p || !sink || bytes <= 0 || (bytes & 15) || ((uintptr_t)p & 15)) return -1;
    hipLaunchKernelGGL(k_read, dim3(grid_size()), dim3(kThreads), 0, (hipStream_t)stream,
                       (const v4u*)p, bytes / 16, sink);
    return (int)hipGetLastError();
}

// Writes `bytes` at p (same conditions).
int sc_write(void* p, int64_t bytes, void* stream)
{
    if (!p || bytes <= 0 || (bytes & 15) || ((uintptr_t)p & 15)) return -1;
    hipLaunchKernelGGL(k_write, dim3(grid_size()), dim3(kThreads), 0, (hipStream_t)stream,
                       (v4u*)p, bytes / 16, 0x3ff00000u);
    return (int)hipGetLastError();
}

// Copies `bytes` from src to dst (same conditions, no overlap).
int sc_copy(const void* src, void* dst, int64_t bytes, void* stream)
{
    if (!src || !dst || bytes <= 0 || (bytes & 15) || (((uintptr_t)src | (uintptr_t)dst) & 15))
        return -1;
    hipLaunchKernelGGL(k_copy, dim3(grid_size()), dim3(kThreads), 0, (hipStream_t)stream,
                       (const v4u*)src, (v4u*)dst, bytes / 16);
    return (int)hipGetLastError();
}

}  // extern "C"
