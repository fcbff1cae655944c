// Host entry points of the ahead-of-time kernels (exa_kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstdint>

// ptr/idx are int64 when wide != 0, else int32
hipError_t exa_launch_segsum(const void* ptr, const void* idx, int wide, const double* buf, double* out,
                             int64_t nseg, int accumulate, hipStream_t s);
hipError_t exa_launch_sum(const double* part, int64_t n, double* out, hipStream_t s);
hipError_t exa_launch_fill(double* p, int64_t n, double v, hipStream_t s);
