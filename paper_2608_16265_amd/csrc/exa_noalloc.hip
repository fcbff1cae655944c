// An H v entry point that allocates nothing, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).
//
// exa_hprod evaluates the local (w H) v contributions of every curved slot
// and data point into the model's H v work buffer and sums them per
// variable by the deterministic segment sums (plus part sums for segments
// longer than 1024 entries).  exa_hprod_noalloc runs the same kernels in the
// same order, with those two work arrays placed in `scratch`, a fixed array
// in device memory that every GPU the library runs on holds until the
// process ends; the call itself allocates nothing and never tunes.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>

#include "exa_internal.h"
#include "exa_runtime.h"

using namespace exa;

namespace {

// 32 MiB: the H v work buffer of a model with up to about 4.19 million
// curved-slot contributions (the 10,000-bus ACOPF model needs about 0.3
// million, the 1000 x 1000 PDE model about 3 million), plus its part sums.
constexpr int64_t kScratchDoubles = (int64_t)1 << 22;

static __device__ __align__(256) double scratch[kScratchDoubles];

// Device address of `scratch` on each device, looked up once per device
// (hipGetSymbolAddress with that device current): the array's name in host
// code is only a host-side stand-in.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

double* scratch_on(int dev) {
    if (dev < 0 || dev >= kMaxDevices) fail(EXA_EINVAL, "device ordinal out of range for the scratch table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
        if (!p) fail(EXA_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_ptr[dev] = (double*)p;
    }
    return g_ptr[dev];
}

}  // namespace

extern "C" {

exa_status exa_hprod_noalloc(exa_model* m, const double* x, const double* y, double obj_weight, const double* v,
                             double* Hv, exa_stream_t stream) {
    return guard_status([&] {
        Model& M = live_model(m);
        auto need = [](const void* p, int64_t n, const char* what) {
            if (n > 0 && !p) fail(EXA_EINVAL, std::string("null pointer: ") + what);
        };
        need(x, M.nvar, "x");
        need(y, M.ncon, "y");
        need(v, M.nvar, "v");
        need(Hv, M.nvar, "Hv");
        DeviceState& D = *M.dev;
        // the H v buffer, then the part sums of long segments (a 128-byte line apart)
        const int64_t hv_len = (M.hv_len + 15) / 16 * 16;
        const int64_t need_len = hv_len + D.h_map.nparts;
        if (need_len > kScratchDoubles)
            fail(EXA_EINVAL, "exa_hprod_noalloc: the model needs " + std::to_string(need_len) +
                                 " doubles of work space, more than its fixed " + std::to_string(kScratchDoubles) +
                                 " (use exa_hprod)");
        int dev = 0;
        hip_check(hipGetDevice(&dev), "hipGetDevice");
        if (dev != D.device) fail(EXA_EINVAL, "the model lives on another device than the current one");
        double* sp = scratch_on(dev);
        hipStream_t s = (hipStream_t)stream;
        ExaCall c;
        std::memset(&c, 0, sizeof c);
        c.x = x;
        c.y = y;
        c.v = v;
        c.sigma = obj_weight;
        c.out0 = sp;
        c.out1 = Hv;
        launch_mode_untuned(M, M_HPROD, c, s);
        DevMap map = D.h_map;
        if (map.nparts > 0) map.lsum = sp + hv_len;
        segsum(map, sp, Hv, s);
        M.counters[7]++;
    });
}

}  // extern "C"
