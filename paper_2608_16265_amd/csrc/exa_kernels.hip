// Fixed kernels compiled ahead of time: the deterministic reductions that
// follow the generated evaluation kernels.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "exa_kernels.h"

namespace {

constexpr int kSegBlock = 256;

// out[s] (+)= sum of buf[idx[j]] for j in [ptr[s], ptr[s+1]), in ascending j:
// the sparse-to-dense compression of Sec. 7.2.3, one lane per segment, with
// a fixed summation order so the result does not depend on scheduling.
template <class I>
__global__ void __launch_bounds__(kSegBlock)
k_segsum(const I* __restrict__ ptr, const I* __restrict__ idx, const double* __restrict__ buf,
         double* __restrict__ out, int64_t nseg, int accumulate) {
    const int64_t s = (int64_t)blockIdx.x * kSegBlock + threadIdx.x;
    if (s >= nseg) return;
    const int64_t b = ptr[s], e = ptr[s + 1];
    double acc = accumulate ? out[s] : 0.0;
    int64_t j = b;
    // four entries at a time: their index and value loads are issued
    // together, the additions stay in ascending order
    for (; j + 4 <= e; j += 4) {
        const I i0 = idx[j], i1 = idx[j + 1], i2 = idx[j + 2], i3 = idx[j + 3];
        const double v0 = buf[i0], v1 = buf[i1], v2 = buf[i2], v3 = buf[i3];
        acc += v0;
        acc += v1;
        acc += v2;
        acc += v3;
    }
    for (; j < e; ++j) acc += buf[idx[j]];
    out[s] = acc;
}

// Sum of n partials in a fixed order: strided per-lane sums, then a tree.
__global__ void __launch_bounds__(256) k_sum(const double* __restrict__ part, int64_t n,
                                             double* __restrict__ out) {
    __shared__ double lds[256];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc += part[i];
    lds[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = lds[0];
}

__global__ void __launch_bounds__(256) k_fill(double* __restrict__ p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

hipError_t exa_launch_segsum(const void* ptr, const void* idx, int wide, const double* buf, double* out,
                             int64_t nseg, int accumulate, hipStream_t s) {
    if (nseg <= 0) return hipSuccess;
    const int64_t grid = (nseg + kSegBlock - 1) / kSegBlock;
    if (wide)
        hipLaunchKernelGGL(k_segsum<int64_t>, dim3((unsigned)grid), dim3(kSegBlock), 0, s,
                           (const int64_t*)ptr, (const int64_t*)idx, buf, out, nseg, accumulate);
    else
        hipLaunchKernelGGL(k_segsum<int32_t>, dim3((unsigned)grid), dim3(kSegBlock), 0, s,
                           (const int32_t*)ptr, (const int32_t*)idx, buf, out, nseg, accumulate);
    return hipGetLastError();
}

hipError_t exa_launch_sum(const double* part, int64_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, part, n, out);
    return hipGetLastError();
}

hipError_t exa_launch_fill(double* p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t grid = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)grid), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
