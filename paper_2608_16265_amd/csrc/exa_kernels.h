// Host entry points of the ahead-of-time kernels (exa_kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstdint>

// ptr/idx are int64 when wide != 0, else int32
hipError_t exa_launch_segsum(const void* ptr, const void* idx, int wide, const double* buf, double* out,
                             int64_t nseg, int accumulate, hipStream_t s);
hipError_t exa_launch_sum(const double* part, int64_t n, double* out, hipStream_t s);
hipError_t exa_launch_fill(double* p, int64_t n, double v, hipStream_t s);

// One segment-sum job: out[s] = sum of buf[idx[j]], j in [ptr[s], ptr[s+1]).
struct ExaSegJob {
    const void* ptr;
    const void* idx;
    const double* buf;
    double* out;
    int64_t nseg;
    int32_t wide;  // ptr/idx are int64 when set, else int32
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
