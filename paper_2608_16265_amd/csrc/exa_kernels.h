// Host entry points of the ahead-of-time kernels (exa_kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstdint>

hipError_t exa_launch_sum(const double* part, int64_t n, double* out, hipStream_t s);
hipError_t exa_launch_fill(double* p, int64_t n, double v, hipStream_t s);
hipError_t exa_launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t s);

// One segment-sum job: out[s] = sum of buf[idx[j]], j in [ptr[s], ptr[s+1]).
// With lanes == nullptr one lane sums one segment in ascending j.  With
// lanes set, lane l sums a chunk of at most kExaChunk consecutive entries:
// lanes[3l] = segment (-1 for padding), lanes[3l+1] = first entry,
// lanes[3l+2] = count | (number of chunks of the segment << 4) on the
// segment's first chunk; a segment's chunks lie in one 256-lane block, and
// its first lane adds the chunk sums in chunk order.
constexpr int kExaChunk = 4;
struct ExaSegJob {
    const void* ptr;
    const void* idx;
    const double* buf;
    double* out;
    int64_t nseg;
    const int32_t* lanes;
    int64_t nlanes;  // a multiple of 256 when lanes is set
    int32_t wide;    // ptr/idx are int64 when set, else int32
    int32_t pad;
};
constexpr int kExaReduceJobs = 3;
// Up to three segment-sum jobs and, when part is not null, the sum of the
// npart objective partials into f[0], all in one launch.
struct ExaReduce {
    ExaSegJob job[kExaReduceJobs];
    int32_t njobs;
    int32_t pad;
    const double* part;
    int64_t npart;
    double* f;
};
hipError_t exa_launch_reduce(const ExaReduce& r, hipStream_t s);
