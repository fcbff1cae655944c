// Host entry points of the ahead-of-time kernels (exa_kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstdint>

hipError_t exa_launch_segsum(const int64_t* ptr, const int64_t* idx, const double* buf, double* out,
                             int64_t nseg, int accumulate, hipStream_t s);
hipError_t exa_launch_sum(const double* part, int64_t n, double* out, hipStream_t s);
hipError_t exa_launch_fill(double* p, int64_t n, double v, hipStream_t s);
