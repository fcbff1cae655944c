// Fixed kernels compiled ahead of time: the deterministic reductions that
// follow the generated evaluation kernels.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "exa_kernels.h"

namespace {

constexpr int kSegBlock = 256;

// Workgroup b runs on XCD b % 8.  Launches of these kernels have 8 * per_xcd
// workgroups, and workgroup b takes logical block (b % 8) * per_xcd + b / 8,
// so each XCD sums a contiguous range of segments and keeps its part of the
// buffers in its own L2.
__device__ __forceinline__ int64_t xcd_block(int64_t per_xcd) {
    return (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
}

// A segment's result: out[s] = acc, or with the epilogue out[s] = alpha *
// out[s] + acc, the product rounded before the sum (as two separate
// elementwise operations would give).
__device__ __forceinline__ void put(double* __restrict__ out, int64_t s, double acc, bool ep, double alpha) {
#pragma clang fp contract(off)
    if (ep) {
        const double p = alpha * out[s];
        out[s] = p + acc;
    } else {
        out[s] = acc;
    }
}

// Value of map position i: buf[i], or for a weight entry i = ~(2 row + neg)
// the weight w[row], negated when neg is set.  One load either way (the
// base and offset are selected), so lanes that mix both kinds issue one
// load instruction, not two.
template <class I>
__device__ __forceinline__ double entry(const double* __restrict__ buf, const double* __restrict__ w, I i) {
    const bool wt = i < 0;
    const I e = ~i;
    const double* base = wt ? w : buf;
    const double v = base[wt ? (e >> 1) : i];
    return wt && (e & 1) ? -v : v;
}

// out[s] = sum of buf[idx[j]] for j in [ptr[s], ptr[s+1]), in ascending j:
// the sparse-to-dense compression of Sec. 7.2.3, one lane per segment, with
// a fixed summation order so the result does not depend on scheduling.  A
// negative end (~end) marks a segment whose output the evaluation kernel
// writes itself: it is left alone.
template <class I>
__device__ __forceinline__ void seg_body(const I* __restrict__ ptr, const I* __restrict__ idx,
                                         const double* __restrict__ buf, const double* __restrict__ w,
                                         double* __restrict__ out, int64_t s, bool parts, bool ep, double alpha) {
    const I pb = ptr[s], pe = ptr[s + 1];
    if (pe < 0) return;
    const int64_t b = pb < 0 ? ~pb : pb, e = pe;
    if (parts && e - b > kExaLongSeg) return;  // summed in parts
    double acc = 0.0;
    int64_t j = b;
    // four entries at a time: their index and value loads are issued
    // together, the additions stay in ascending order
    for (; j + 4 <= e; j += 4) {
        const I i0 = idx[j], i1 = idx[j + 1], i2 = idx[j + 2], i3 = idx[j + 3];
        const double v0 = entry(buf, w, i0), v1 = entry(buf, w, i1), v2 = entry(buf, w, i2), v3 = entry(buf, w, i3);
        acc += v0;
        acc += v1;
        acc += v2;
        acc += v3;
    }
    for (; j < e; ++j) acc += entry(buf, w, idx[j]);
    put(out, s, acc, ep, alpha);
}

// The same sums for maps with long segments: lane l of the job adds one
// chunk of at most kExaChunk entries, whose positions sit in its own lane
// record, so the record, the positions and then the values are two
// dependent loads; the segment's first lane adds the chunk sums of its
// segment, which lie in the same workgroup, in chunk order.  The order
// depends on the map only.  Called by every lane of the workgroup, with
// l < J.nlanes (launches cover whole 256-lane blocks).
__device__ __forceinline__ void chunk_body(const ExaSegJob& J, int64_t l, double* lds, bool ep, double alpha) {
    static_assert(kExaChunk == 4, "one int4 of positions per lane");
    const double* __restrict__ buf = J.buf;
    const int2 m = ((const int2*)J.lanes)[l];
    const int4 ix = ((const int4*)J.lidx)[l];
    const double* __restrict__ w = J.w;
    const double v0 = entry(buf, w, ix.x), v1 = entry(buf, w, ix.y), v2 = entry(buf, w, ix.z), v3 = entry(buf, w, ix.w);
    const int seg = m.x, cnt = m.y & 15, nl = m.y >> 4;
    double part = 0.0;
    if (cnt > 0) part += v0;
    if (cnt > 1) part += v1;
    if (cnt > 2) part += v2;
    if (cnt > 3) part += v3;
    lds[threadIdx.x] = part;
    __syncthreads();
    if (seg >= 0 && nl > 0) {
        double acc = lds[threadIdx.x];
        for (int i = 1; i < nl; ++i) acc += lds[threadIdx.x + i];
        put(J.out, seg, acc, ep, alpha);
    }
    __syncthreads();
}

// Sum of the 256 lane values v by a fixed tree; every lane gets the sum.
// Called by every lane of the workgroup; lds is free again on return.
__device__ __forceinline__ double block_sum(double v, double* lds) {
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}

// Part block r (see ExaSegJob): part q of long segment ls, lane t adds
// entries 4t .. 4t+3 of the part and the block adds the lanes by block_sum
// into lsum[q].  Called by every lane of the workgroup.
__device__ __forceinline__ void long_part_body(const ExaSegJob& J, int64_t r, double* lds) {
#pragma clang fp contract(off)
    const int32_t* __restrict__ idx = (const int32_t*)J.idx;
    const double* __restrict__ buf = J.buf;
    const int2 lq = ((const int2*)J.lpart)[r];
    const int32_t ls = lq.x, q = lq.y;
    const int32_t beg = J.longs[5 * ls + 1], len = J.longs[5 * ls + 2], part0 = J.longs[5 * ls + 3];
    const int32_t pb = beg + ((int32_t)q - part0) * kExaLongSeg;
    const int32_t pe = min(beg + len, pb + kExaLongSeg);
    const int32_t j0 = pb + kExaChunk * (int32_t)threadIdx.x;
    double part = 0.0;
    if (j0 < pe) {
        const int cnt = min(kExaChunk, pe - j0);
        int32_t ix[kExaChunk];
#pragma unroll
        for (int u = 0; u < kExaChunk; ++u) ix[u] = idx[j0 + (u < cnt ? u : cnt - 1)];
        double v[kExaChunk];
#pragma unroll
        for (int u = 0; u < kExaChunk; ++u) v[u] = entry(buf, J.w, ix[u]);
#pragma unroll
        for (int u = 0; u < kExaChunk; ++u)
            if (u < cnt) part += v[u];
    }
    const double s = block_sum(part, lds);
    if (threadIdx.x == 0) J.lsum[q] = s;
}

// Sum of n partials in a fixed order by one 256-wide workgroup: strided
// per-lane sums, then a tree.
__device__ __forceinline__ void sum_body(const double* __restrict__ part, int64_t n, double* __restrict__ out,
                                         double* lds) {
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc += part[i];
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) out[0] = s;
}

__global__ void __launch_bounds__(256) k_sum(const double* __restrict__ part, int64_t n,
                                             double* __restrict__ out) {
    __shared__ double lds[256];
    sum_body(part, n, out, lds);
}

// Several reductions in one launch: the segment sums of each job over
// consecutive block ranges (one block per 256 segments; for a chunked job,
// one per 256 lanes, then one per part of a long segment), then (when
// R.part is set) one block for the objective partials, summed as k_sum
// does.
__host__ __device__ inline int64_t job_blocks(const ExaSegJob& J) {
    return (J.chunked ? J.nlanes / kSegBlock : (J.nseg + kSegBlock - 1) / kSegBlock) + J.nparts;
}

__global__ void __launch_bounds__(kSegBlock) k_reduce(ExaReduce R, int64_t per_xcd) {
    __shared__ double lds[256];
    const int64_t b0 = xcd_block(per_xcd);
    // the job from the block ranges (one cache line of arguments), then the
    // job's fields in one burst, before anything depends on them
    static_assert(kExaReduceJobs == 3, "the job lookup below reads three block ranges");
    const int64_t e0 = R.bend[0], e1 = R.bend[1], e2 = R.bend[2];
    const int k = b0 < e0 ? 0 : b0 < e1 ? 1 : b0 < e2 ? 2 : 3;
    if (k >= R.njobs) {  // ends past the last job equal the total
        if (R.part && b0 == e2) sum_body(R.part, R.npart, R.f, lds);
        return;
    }
    const ExaSegJob J = R.job[k];
    const int64_t b = b0 - (k == 0 ? 0 : k == 1 ? e0 : e1);
    const bool ep = k == R.ep_job;
    if (J.chunked) {
        const int64_t nlb = J.nlanes / kSegBlock;
        if (b < nlb)
            chunk_body(J, b * kSegBlock + threadIdx.x, lds, ep, R.ax_alpha);
        else
            long_part_body(J, b - nlb, lds);
        return;
    }
    const int64_t nsb = (J.nseg + kSegBlock - 1) / kSegBlock;
    if (b >= nsb) {
        long_part_body(J, b - nsb, lds);
        return;
    }
    const int64_t s = b * kSegBlock + threadIdx.x;
    if (s < J.nseg) {
        if (J.wide)
            seg_body((const int64_t*)J.ptr, (const int64_t*)J.idx, J.buf, J.w, J.out, s, false, ep, R.ax_alpha);
        else
            seg_body((const int32_t*)J.ptr, (const int32_t*)J.idx, J.buf, J.w, J.out, s, J.nparts > 0, ep,
                     R.ax_alpha);
    }
}

// Second launch for jobs with long segments: block b adds the part sums of
// one long segment (the jobs' long segments in job order), strided per lane
// and then by block_sum.
__global__ void __launch_bounds__(kSegBlock) k_reduce_long(ExaReduce R) {
    __shared__ double lds[256];
    int64_t b = blockIdx.x;
    for (int k = 0; k < R.njobs; ++k) {
        const ExaSegJob& J = R.job[k];
        if (b < J.nlong) {
            const int32_t* L = J.longs + 5 * b;
            const int32_t seg = L[0], part0 = L[3], nparts = L[4];
            // lane t adds parts t, t + 256, ... in that order; eight loads
            // are issued before their adds, so a segment of thousands of
            // parts is a few dependent round trips deep, not one per part
            double acc = 0.0;
            for (int32_t i0 = threadIdx.x; i0 < nparts; i0 += 256 * 8) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = i0 + 256 * u < nparts ? J.lsum[part0 + i0 + 256 * u] : 0.0;
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (i0 + 256 * u < nparts) acc += v[u];
            }
            const double tot = block_sum(acc, lds);
            if (threadIdx.x == 0) put(J.out, seg, tot, k == R.ep_job, R.ax_alpha);
            return;
        }
        b -= J.nlong;
    }
}

// The segment-sum job of a batched job, with its buffer and output resolved.
__device__ __forceinline__ ExaSegJob batch_seg(const ExaBatchReduce& R, const ExaBatchJob& B) {
    ExaSegJob J;
    J.ptr = B.ptr;
    J.idx = B.idx;
    J.buf = R.bufs[B.buf] + B.buf_off;
    J.w = R.w ? R.w + B.w_off : nullptr;
    J.out = R.outs[B.out] + B.out_off;
    J.nseg = B.nseg;
    J.lanes = B.lanes;
    J.lidx = B.lidx;
    J.nlanes = B.nlanes;
    J.longs = B.longs;
    J.lpart = B.lpart;
    J.nparts = B.nparts;
    J.nlong = B.nlong;
    J.lsum = B.lsum;
    J.wide = B.wide;
    J.chunked = B.chunked;
    return J;
}

// Batched reductions: every block runs one block of one instance's job, the
// same block k_reduce would run for that job alone, so each instance's sums
// come out bit for bit as its own reduction gives them.
__global__ void __launch_bounds__(kSegBlock) k_reduce_batch(ExaBatchReduce R) {
    __shared__ double lds[256];
    const int64_t per_xcd = R.nblocks / 8;
    const int64_t b0 = xcd_block(per_xcd);
    const int2 jb = ((const int2*)R.blocks)[b0];
    if (jb.x < 0) return;
    const ExaBatchJob& B = R.jobs[jb.x];
    if (B.kind == 1) {
        // objective partials: none -> 0, one -> itself (the value a single
        // tile writes directly), several -> the fixed-order sum
        const double* part = R.bufs[B.buf] + B.buf_off;
        double* f = R.outs[B.out] + B.out_off;
        if (B.nseg > 1) {
            sum_body(part, B.nseg, f, lds);
        } else if (threadIdx.x == 0) {
            f[0] = B.nseg == 1 ? part[0] : 0.0;
        }
        return;
    }
    const ExaSegJob J = batch_seg(R, B);
    const int64_t b = jb.y;
    const bool ep = B.ep != 0;
    if (J.chunked) {
        const int64_t nlb = J.nlanes / kSegBlock;
        if (b < nlb)
            chunk_body(J, b * kSegBlock + threadIdx.x, lds, ep, R.alpha);
        else
            long_part_body(J, b - nlb, lds);
        return;
    }
    const int64_t nsb = (J.nseg + kSegBlock - 1) / kSegBlock;
    if (b >= nsb) {
        long_part_body(J, b - nsb, lds);
        return;
    }
    const int64_t s = b * kSegBlock + threadIdx.x;
    if (s < J.nseg) {
        if (J.wide)
            seg_body((const int64_t*)J.ptr, (const int64_t*)J.idx, J.buf, J.w, J.out, s, false, ep, R.alpha);
        else
            seg_body((const int32_t*)J.ptr, (const int32_t*)J.idx, J.buf, J.w, J.out, s, J.nparts > 0, ep, R.alpha);
    }
}

// Second batched launch: the part sums of one long segment of one job per
// block, added as k_reduce_long adds them.
__global__ void __launch_bounds__(kSegBlock) k_reduce_batch_long(ExaBatchReduce R) {
    __shared__ double lds[256];
    const int2 jl = ((const int2*)R.lblocks)[blockIdx.x];
    const ExaBatchJob& B = R.jobs[jl.x];
    const ExaSegJob J = batch_seg(R, B);
    const int32_t* L = J.longs + 5 * jl.y;
    const int32_t seg = L[0], part0 = L[3], nparts = L[4];
    double acc = 0.0;
    for (int32_t i0 = threadIdx.x; i0 < nparts; i0 += 256 * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = i0 + 256 * u < nparts ? J.lsum[part0 + i0 + 256 * u] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i0 + 256 * u < nparts) acc += v[u];
    }
    const double tot = block_sum(acc, lds);
    if (threadIdx.x == 0) put(J.out, seg, tot, B.ep != 0, R.alpha);
}

// Streaming copy with 16-byte non-temporal loads and stores, one vector per
// lane: the access pattern of the evaluation kernels' final outputs, used to
// measure the device's practical bandwidth.
typedef double exa_d2 __attribute__((ext_vector_type(2)));
__global__ void __launch_bounds__(256) k_copy16(const exa_d2* __restrict__ src, exa_d2* __restrict__ dst, int64_t n2) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n2) __builtin_nontemporal_store(__builtin_nontemporal_load(&src[i]), &dst[i]);
}

__global__ void __launch_bounds__(256) k_copy1(const char* __restrict__ src, char* __restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// out[i] = a * out[i] + add[i], the product rounded before the sum (no
// fused multiply-add), as two separate elementwise operations would give
__global__ void __launch_bounds__(256) k_axpy(double* __restrict__ out, const double* __restrict__ add, double a,
                                              int64_t n) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        const double p = a * out[i];
        out[i] = p + add[i];
    }
}

__global__ void __launch_bounds__(256) k_fill(double* __restrict__ p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

hipError_t exa_launch_sum(const double* part, int64_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, part, n, out);
    return hipGetLastError();
}

hipError_t exa_launch_reduce(const ExaReduce& r, hipStream_t s) {
    if (r.njobs < 0 || r.njobs > kExaReduceJobs) return hipErrorInvalidValue;
    int64_t blocks = r.part ? 1 : 0, nlong = 0;
    for (int k = 0; k < r.njobs; ++k) {
        const ExaSegJob& J = r.job[k];
        if (J.chunked && (J.nlanes % kSegBlock || J.wide || (J.nlanes && !(J.lanes && J.lidx))))
            return hipErrorInvalidValue;
        if (J.nparts && (J.wide || !(J.longs && J.lpart && J.lsum && J.nlong > 0))) return hipErrorInvalidValue;
        blocks += job_blocks(J);
        nlong += J.nparts ? J.nlong : 0;
    }
    if (r.ax_out && (!r.ax_add || r.ax_n < 0)) return hipErrorInvalidValue;
    if (r.ep_job >= r.njobs) return hipErrorInvalidValue;
    if (blocks > 0) {
        ExaReduce rr = r;
        int64_t end = 0;
        for (int k = 0; k < kExaReduceJobs; ++k) {
            if (k < r.njobs) end += job_blocks(r.job[k]);
            rr.bend[k] = end;
        }
        const int64_t per_xcd = (blocks + 7) / 8;
        hipLaunchKernelGGL(k_reduce, dim3((unsigned)(8 * per_xcd)), dim3(kSegBlock), 0, s, rr, per_xcd);
    }
    if (nlong > 0) hipLaunchKernelGGL(k_reduce_long, dim3((unsigned)nlong), dim3(kSegBlock), 0, s, r);
    if (r.ax_out && r.ax_n > 0)
        hipLaunchKernelGGL(k_axpy, dim3((unsigned)((r.ax_n + 255) / 256)), dim3(256), 0, s, r.ax_out, r.ax_add,
                           r.ax_alpha, r.ax_n);
    return hipGetLastError();
}

int64_t exa_job_blocks(const ExaSegJob& J) { return job_blocks(J); }

hipError_t exa_launch_reduce_batch(const ExaBatchReduce& r, hipStream_t s) {
    if (r.nblocks % 8 || r.nblocks < 0 || r.nlblocks < 0) return hipErrorInvalidValue;
    if ((r.nblocks && !(r.jobs && r.blocks)) || (r.nlblocks && !(r.jobs && r.lblocks))) return hipErrorInvalidValue;
    if (r.nblocks > 0) hipLaunchKernelGGL(k_reduce_batch, dim3((unsigned)r.nblocks), dim3(kSegBlock), 0, s, r);
    if (r.nlblocks > 0) hipLaunchKernelGGL(k_reduce_batch_long, dim3((unsigned)r.nlblocks), dim3(kSegBlock), 0, s, r);
    return hipGetLastError();
}

hipError_t exa_launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t s) {
    if (bytes <= 0) return hipSuccess;
    const bool aligned = ((uintptr_t)src % 16 == 0) && ((uintptr_t)dst % 16 == 0);
    const int64_t n2 = aligned ? bytes / 16 : 0, tail = bytes - 16 * n2;
    if (n2 > 0)
        hipLaunchKernelGGL(k_copy16, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, (const exa_d2*)src,
                           (exa_d2*)dst, n2);
    if (tail > 0)
        hipLaunchKernelGGL(k_copy1, dim3((unsigned)((tail + 255) / 256)), dim3(256), 0, s,
                           (const char*)src + 16 * n2, (char*)dst + 16 * n2, tail);
    return hipGetLastError();
}

hipError_t exa_launch_fill(double* p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t grid = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)grid), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
