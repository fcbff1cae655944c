// Host entry points of the ahead-of-time kernels (exa_kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstdint>

hipError_t exa_launch_sum(const double* part, int64_t n, double* out, hipStream_t s);
hipError_t exa_launch_fill(double* p, int64_t n, double v, hipStream_t s);
hipError_t exa_launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t s);

// One segment-sum job: out[s] = sum of buf[idx[j]], j in [ptr[s], ptr[s+1]),
// in a summation order fixed by the map:
// * segments longer than kExaLongSeg, when the job has parts (nparts > 0;
//   int32 maps only): one block per part of kExaLongSeg entries adds its
//   entries (4 per lane) by a fixed tree into lsum[part], and a second
//   launch adds each segment's part sums, again in a fixed order.
//   longs[5i..5i+4] = {segment, first entry, length, first part, parts} of
//   long segment i; part block r adds part lpart[2r+1] of long segment
//   lpart[2r] (the segment's parts are numbered from its first part up).
//   Part blocks are interleaved over the segments (the i-th part of every
//   long segment before any (i+1)-th), so a contiguous range of part blocks
//   covers the same range of points for every long segment;
// * the other segments, unless chunked is set: one lane per segment, entries
//   in ascending j;
// A position below zero is a weight entry ~(2 row + neg): the value is
// w[row], negated when neg is set (an augmentation term that is plus or
// minus one variable adds plus or minus its row's weight to J^T w).
// * with chunked set (int32 maps only): lane l adds one chunk of at most
//   kExaChunk consecutive entries, with lanes[2l] = segment (-1 for
//   padding), lanes[2l+1] = count | (number of chunks of the segment << 4)
//   on the segment's first chunk, and lidx[4l .. 4l+3] = the chunk's buffer
//   positions (the last one repeated past the count; 0 for padding); a
//   segment's chunks lie in one 256-lane block, and its first lane adds the
//   chunk sums in chunk order.
constexpr int kExaChunk = 4;
constexpr int kExaLongSeg = 256 * kExaChunk;
constexpr int kExaShortSeg = 16;
struct ExaSegJob {
    const void* ptr;
    const void* idx;
    const double* buf;
    const double* w;  // weights of the weight entries (maps without any: unused)
    double* out;
    int64_t nseg;
    const int32_t* lanes;
    const int32_t* lidx;
    int64_t nlanes;  // a multiple of 256
    const int32_t* longs;
    const int32_t* lpart;
    int64_t nparts, nlong;
    double* lsum;
    int32_t wide;    // ptr/idx are int64 when set, else int32
    int32_t chunked;
};
constexpr int kExaReduceJobs = 3;
// Up to three segment-sum jobs and, when part is not null, the sum of the
// npart objective partials into f[0], in one launch (one more when a job
// has long segments, and one more for the ax_* update).
struct ExaReduce {
    ExaSegJob job[kExaReduceJobs];
    // first block after job k (cumulative); set by exa_launch_reduce
    int64_t bend[kExaReduceJobs];
    int32_t njobs;
    // job whose sums are added to ax_alpha times its output's old values
    // (out[s] = ax_alpha * out[s] + sum, the product rounded first), or -1
    int32_t ep_job;
    const double* part;
    int64_t npart;
    double* f;
    // when ax_out is set, after the sums: ax_out[i] = ax_alpha * ax_out[i] +
    // ax_add[i] for i < ax_n, each operation rounded on its own
    double* ax_out;
    const double* ax_add;
    double ax_alpha;
    int64_t ax_n;
};
hipError_t exa_launch_reduce(const ExaReduce& r, hipStream_t s);

// Segment sums and objective sums of many instances in one launch (the
// batched reductions).  Job j sums one instance's map, exactly as a single
// ExaSegJob over the same map would (same chunking, same parts, same order),
// or adds one instance's objective partials as the objective's own
// reduction does (one partial: copied; none: 0).  Buffers and outputs are
// named by index and offset, so the job table does not depend on the
// caller's pointers: bufs[buf] + buf_off is the job's buffer and
// outs[out] + out_off its output.
// first-order, H v, parameter, objective partials
constexpr int kExaBatchBufs = 4;
constexpr int kExaBatchOuts = 8;
struct ExaBatchJob {
    const void* ptr;
    const void* idx;
    const int32_t* lanes;
    const int32_t* lidx;
    const int32_t* longs;
    const int32_t* lpart;
    double* lsum;
    int64_t nseg, nlanes, nparts, nlong;
    int64_t buf_off, out_off;
    int64_t w_off;  // the instance's first row in the call's weights
    int32_t wide, chunked;
    int32_t buf, out;
    int32_t kind;  // 0: segment sums; 1: objective partials (nseg of them) into one value
    int32_t ep;    // 1: out = alpha * out + sum, the product rounded first
};
struct ExaBatchReduce {
    const ExaBatchJob* jobs;
    // block b of the first launch runs (job, block within the job) =
    // blocks[b] (job -1: nothing); nblocks is a multiple of 8, and XCD j
    // takes blocks [j * nblocks / 8, (j + 1) * nblocks / 8)
    const int32_t* blocks;
    int64_t nblocks;
    // block b of the second launch adds the part sums of long segment
    // lblocks[2b + 1] of job lblocks[2b]
    const int32_t* lblocks;
    int64_t nlblocks;
    const double* bufs[kExaBatchBufs];
    double* outs[kExaBatchOuts];
    const double* w;  // weights of the J^T w (or J^T y) weight entries
    double alpha;
};
hipError_t exa_launch_reduce_batch(const ExaBatchReduce& r, hipStream_t s);
int64_t exa_job_blocks(const ExaSegJob& J);

