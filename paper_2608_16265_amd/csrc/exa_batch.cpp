// Batched evaluation of many instances of one formulation (Sec. 7.4.3 batch
// models, generalised to instances of different sizes).
//
// All instances share the generated code; their data stays where each model
// put it, and their sizes and offsets are table data.  A tile list spans
// (instance, unit, data range); ONE persistent launch walks it and the launch
// is recorded once into a HIP graph and replayed.  For the Jacobian and the
// Hessian together the tiles are either combined units (both sweeps of a data
// point in one pass over one set of loads) or separate Jacobian and Hessian
// tiles.  With xcd_aware, instances are binned over the 8 XCDs by estimated
// cost and each XCD walks its bin instance by instance, so an instance's x
// stays in that XCD's L2.  Points per tile, grid size and combined/separate
// are picked by timing candidates at the first evaluation; results do not
// depend on the schedule because every data point is evaluated by the same
// code and written to its own slice.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>

#include "exa_internal.h"
#include "exa_runtime.h"

using namespace exa;

struct exa_batch {
    std::vector<exa_model*> models;
    int B = 0;
    int block = 256;
    std::shared_ptr<Module> module;
    DeviceState mem;                       // owns the tables below
    ExaInstDev* inst = nullptr;
    std::vector<int64_t> offsets;          // 4 * (B + 1): x, y, jac, hess
    // schedule
    bool autotune = true, use_graph = true, tuned = false, fuse = true, xcd_aware = true;
    bool combined = true;                  // Jacobian + Hessian units (mask 3)
    int epl = 4;
    int64_t grid = 0;
    int64_t tuned_ns = 0;
    // tile lists per mask value (1: jac, 2: hess, 3: both) for (epl, combined)
    ExaTile* tiles[4] = {};
    long long* xcd_ranges[4] = {};
    int64_t ntiles[4] = {};
    int64_t per_xcd[4] = {};               // tiles per XCD range of the list
    int tiles_epl = -1, tiles_block = -1;
    bool tiles_combined = true;
    // graph for the last call signature
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    struct Key {
        uint32_t mask;
        const void *x, *y, *j, *h;
        double sigma;
        int epl, block;
        int64_t grid;
        bool combined;
        bool operator==(const Key& o) const {
            return mask == o.mask && x == o.x && y == o.y && j == o.j && h == o.h && sigma == o.sigma &&
                   epl == o.epl && block == o.block && grid == o.grid && combined == o.combined;
        }
    } key{};
    bool have_graph = false;
    int cus = 256;

    ~exa_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

namespace {

// Estimated cost of one data point of pattern P (in 8-byte words moved).
int64_t point_cost(const Pattern& P, int mode) {
    const int64_t loads = P.n_icols / 2 + P.n_fcols + P.o1step() + 1;
    if (mode == M_JH) return loads + P.o1step() + P.o2step();
    return loads + (mode == M_JAC ? P.o1step() : P.o2step());
}

// Modes whose tiles a mask launches: (mode, tile code offset).
std::vector<std::pair<int, int>> mask_modes(uint32_t mask, bool combined) {
    if (mask == 1) return {{M_JAC, 0}};
    if (mask == 2) return {{M_HESS, 0}};
    if (combined) return {{M_JH, 0}};
    return {{M_JAC, 0}, {M_HESS, 64}};
}

void build_tiles(exa_batch& b, int epl, bool combined) {
    if (b.tiles_epl == epl && b.tiles_block == b.block && b.tiles_combined == combined) return;
    const int64_t tp = (int64_t)b.block * epl;
    for (int m = 1; m <= 3; ++m) {
        // per instance: its tiles and their total cost
        std::vector<std::vector<std::pair<int64_t, ExaTile>>> per(b.B);
        std::vector<int64_t> cost(b.B, 0);
        for (int i = 0; i < b.B; ++i) {
            const Model& M = b.models[i]->impl;
            for (auto mc : mask_modes((uint32_t)m, combined)) {
                for (const Unit& u : units_for(M, mc.first, b.fuse)) {
                    int64_t pc = 0;
                    for (int p : u.members) pc += point_cost(M.pats[p], mc.first);
                    for (int64_t s = 0; s < u.ndata; s += tp) {
                        ExaTile t{};
                        t.pat = u.code + mc.second;
                        t.inst = i;
                        t.start = s;
                        t.count = std::min(tp, u.ndata - s);
                        per[i].emplace_back(t.count * pc, t);
                        cost[i] += t.count * pc;
                    }
                }
            }
        }
        std::vector<ExaTile> v;
        std::vector<long long> range(9, 0);
        if (b.xcd_aware) {
            // instances to 8 bins, largest first into the lightest bin; each
            // bin lists its instances one after another
            std::vector<int> order(b.B);
            std::iota(order.begin(), order.end(), 0);
            std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] > cost[c]; });
            std::vector<std::vector<int>> bins(8);
            std::vector<int64_t> load(8, 0);
            for (int i : order) {
                const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                bins[j].push_back(i);
                load[j] += cost[i];
            }
            // every bin padded with no-op tiles to the longest, so that bin j
            // is exactly tiles [j * per_xcd, (j + 1) * per_xcd): the XCD
            // ranges of both the persistent walk and a one-tile-per-workgroup
            // launch
            int64_t longest = 0;
            for (int j = 0; j < 8; ++j) {
                int64_t n = 0;
                for (int i : bins[j]) n += (int64_t)per[i].size();
                longest = std::max(longest, n);
            }
            for (int j = 0; j < 8; ++j) {
                range[j] = (long long)v.size();
                for (int i : bins[j])
                    for (auto& e : per[i]) v.push_back(e.second);
                ExaTile pad{};
                pad.pat = EXA_PAD_TILE;
                while ((int64_t)v.size() < (j + 1) * longest) v.push_back(pad);
            }
            range[8] = (long long)v.size();
            b.per_xcd[m] = longest;
        } else {
            // all tiles, largest first, so the grid-stride walk of the
            // persistent grid approximates longest-processing-time-first
            std::vector<std::pair<int64_t, ExaTile>> all;
            for (auto& pi : per) all.insert(all.end(), pi.begin(), pi.end());
            std::stable_sort(all.begin(), all.end(),
                             [](const auto& a, const auto& c) { return a.first > c.first; });
            for (auto& e : all) v.push_back(e.second);
            b.per_xcd[m] = ((int64_t)v.size() + 7) / 8;
        }
        for (size_t i = 0; i < v.size(); ++i) v[i].slot = (int64_t)i;
        b.mem.release(b.tiles[m]);
        b.mem.release(b.xcd_ranges[m]);
        b.tiles[m] = (ExaTile*)b.mem.upload(v.data(), v.size() * sizeof(ExaTile));
        b.ntiles[m] = (int64_t)v.size();
        b.xcd_ranges[m] =
            b.xcd_aware ? (long long*)b.mem.upload(range.data(), range.size() * sizeof(long long)) : nullptr;
    }
    b.tiles_epl = epl;
    b.tiles_block = b.block;
    b.tiles_combined = combined;
}

void launch(exa_batch& b, uint32_t mask, const double* x, const double* y, double sigma, double* j, double* h,
            hipStream_t s) {
    const int64_t nt = b.ntiles[mask];
    if (nt == 0) return;
    ExaCall c;
    std::memset(&c, 0, sizeof c);
    c.tiles = b.tiles[mask];
    c.ntiles = nt;
    c.inst = b.inst;
    c.x = x;
    c.y = y;
    c.sigma = sigma;
    c.persistent = b.grid < 0 ? 0 : 1;
    c.xcd_range = b.grid < 0 ? nullptr : b.xcd_ranges[mask];
    c.per_xcd = b.per_xcd[mask];
    hipFunction_t fn;
    if (mask == 1) {
        fn = b.module->fn[M_JAC];
        c.out0 = j;
    } else if (mask == 2) {
        fn = b.module->fn[M_HESS];
        c.out0 = h;
    } else {
        fn = b.tiles_combined ? b.module->fn[M_JH] : b.module->fn_sep;
        c.out0 = j;
        c.out1 = h;
    }
    // b.grid < 0: one workgroup per tile (workgroup w takes tile
    // (w % 8) * per_xcd + w / 8); else a persistent grid, a multiple of 8
    // (one share per XCD)
    int64_t grid = 8 * b.per_xcd[mask];
    if (b.grid >= 0) {
        grid = std::max<int64_t>(8, std::min<int64_t>(b.grid, nt));
        grid = (grid + 7) / 8 * 8;
    }
    void* args[] = {&c};
    hip_check(hipModuleLaunchKernel(fn, (unsigned)grid, 1, 1, (unsigned)b.block, 1, 1, 0, s, args, nullptr),
              "hipModuleLaunchKernel");
}

void tune(exa_batch& b, uint32_t mask, const double* x, const double* y, double sigma, double* j, double* h,
          hipStream_t s) {
    const int blocks[] = {64, 128, 256};
    const int epls[] = {1, 2, 4, 8, 16};
    const int64_t grids[] = {-1, b.cus * 2, b.cus * 4, b.cus * 8, b.cus * 16};
    std::vector<int> combos = {1};
    if (mask == 3) combos.push_back(0);
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    struct Cand {
        float ms;
        int block, epl, comb;
        int64_t grid;
    };
    // average of `reps` back-to-back launches of the current schedule
    auto time_it = [&](int reps) {
        launch(b, mask, x, y, sigma, j, h, s);  // warm
        hip_check(hipEventRecord(e0, s), "hipEventRecord");
        for (int r = 0; r < reps; ++r) launch(b, mask, x, y, sigma, j, h, s);
        hip_check(hipEventRecord(e1, s), "hipEventRecord");
        hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        return ms / reps;
    };
    std::vector<Cand> cands;
    try {
        for (int bk : blocks)
        for (int comb : combos)
            for (int epl : epls) {
                b.block = bk;
                build_tiles(b, epl, comb != 0);
                for (int64_t g : grids) {
                    b.grid = g;
                    cands.push_back({time_it(3), bk, epl, comb, g});
                }
            }
        // candidates within a few percent differ by less than one run's
        // noise: the fastest few are timed again, longer, in turns, and the
        // best of their rounds decides
        std::sort(cands.begin(), cands.end(), [](const Cand& a, const Cand& c) { return a.ms < c.ms; });
        cands.resize(std::min<size_t>(cands.size(), 6));
        for (auto& c : cands) c.ms = 1e30f;
        for (int round = 0; round < 3; ++round)
            for (auto& c : cands) {
                b.block = c.block;
                b.grid = c.grid;
                build_tiles(b, c.epl, c.comb != 0);
                c.ms = std::min(c.ms, time_it(8));
            }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const Cand& w = *std::min_element(cands.begin(), cands.end(), [](const Cand& a, const Cand& c) { return a.ms < c.ms; });
    b.epl = w.epl;
    b.block = w.block;
    b.grid = w.grid;
    b.combined = w.comb != 0;
    b.tuned_ns = (int64_t)(w.ms * 1e6);
    build_tiles(b, b.epl, b.combined);
    b.tuned = true;
}

template <class F>
exa_status guard(F&& f) {
    try {
        f();
        set_last_error("");
        return EXA_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return EXA_ENOMEM;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return EXA_EINVAL;
    }
}

}  // namespace

extern "C" {

exa_status exa_batch_create(exa_model* const* models, int32_t B, const exa_batch_options* opt,
                            exa_batch** out) {
    return guard([&] {
        if (!out) fail(EXA_EINVAL, "null output handle");
        *out = nullptr;
        if (B < 1 || !models) fail(EXA_EINVAL, "a batch needs at least one model");
        std::unique_ptr<exa_batch> b(new exa_batch());
        b->B = B;
        b->models.assign(models, models + B);
        for (int i = 0; i < B; ++i) {
            if (!models[i]) fail(EXA_EINVAL, "null model in batch");
            if (models[i]->impl.host_only || !models[i]->impl.dev)
                fail(EXA_ESTATE, "batched models need a device");
            if (models[i]->impl.signature != models[0]->impl.signature)
                fail(EXA_EINVAL, "model " + std::to_string(i) + " does not share the pattern trees of model 0");
        }
        if (opt) {
            b->autotune = opt->autotune != 0;
            if (opt->block) b->block = opt->block;
            if (opt->epl) b->epl = opt->epl;
            b->grid = opt->grid;
            b->use_graph = opt->use_graph != 0;
            b->fuse = opt->fuse != 0;
            b->xcd_aware = opt->xcd_aware != 0;
            b->combined = opt->separate == 0;
        }
        if (b->block != 64 && b->block != 128 && b->block != 256) fail(EXA_EINVAL, "block must be 64, 128 or 256");
        if (b->epl < 1 || b->epl > 16) fail(EXA_EINVAL, "epl must be in 1..16");
        int dev = 0;
        hip_check(hipGetDevice(&dev), "hipGetDevice");
        hipDeviceProp_t prop;
        hip_check(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
        b->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
        if (b->grid == 0 || b->grid < -1) b->grid = (int64_t)b->cus * 8;
        b->module = models[0]->impl.dev->module;  // every instance runs the same generated code

        std::vector<ExaInstDev> inst(B);
        b->offsets.assign(4 * (B + 1), 0);
        for (int i = 0; i < B; ++i) {
            const Model& M = models[i]->impl;
            inst[i] = M.dev->inst_host;
            std::memset(inst[i].off, 0, sizeof inst[i].off);
            int64_t* o = &b->offsets[4 * i];
            inst[i].off[EXA_OFF_X] = o[0];
            inst[i].off[EXA_OFF_Y] = o[1];
            inst[i].off[EXA_OFF_JAC] = o[2];
            inst[i].off[EXA_OFF_HESS] = o[3];
            o[4] = o[0] + M.nvar;
            o[5] = o[1] + M.ncon;
            o[6] = o[2] + M.nnzj;
            o[7] = o[3] + M.nnzh;
        }
        b->inst = (ExaInstDev*)b->mem.upload(inst.data(), inst.size() * sizeof(ExaInstDev));
        build_tiles(*b, b->epl, b->combined);
        hip_check(hipStreamCreate(&b->cap), "hipStreamCreate");
        *out = b.release();
    });
}

exa_status exa_batch_destroy(exa_batch* b) {
    return guard([&] { delete b; });
}

exa_status exa_batch_offsets(const exa_batch* b, int64_t* offsets) {
    return guard([&] {
        if (!b || !offsets) fail(EXA_EINVAL, "null argument");
        std::copy(b->offsets.begin(), b->offsets.end(), offsets);
    });
}

exa_status exa_batch_schedule(const exa_batch* b, int64_t* out6) {
    return guard([&] {
        if (!b || !out6) fail(EXA_EINVAL, "null argument");
        out6[0] = b->block;
        out6[1] = b->epl;
        out6[2] = b->grid;
        out6[3] = b->ntiles[3];
        out6[4] = b->tuned_ns;
        out6[5] = b->combined ? 1 : 0;
    });
}

exa_status exa_batch_bytes(const exa_batch* b, uint32_t mask, int64_t* read_bytes, int64_t* write_bytes) {
    return guard([&] {
        if (!b) fail(EXA_EINVAL, "null batch");
        if (mask == 0 || mask > 3) fail(EXA_EINVAL, "mask must be EXA_CB_JAC, EXA_CB_HESS or both");
        std::vector<int> modes;
        for (auto mc : mask_modes(mask, b->combined)) modes.push_back(mc.first);
        int64_t rd = 0, wr = 0;
        for (int i = 0; i < b->B; ++i) {
            int64_t r = 0, w = 0;
            kernel_bytes(b->models[i]->impl, modes, b->fuse, r, w);
            rd += r;
            wr += w;
        }
        if (read_bytes) *read_bytes = rd;
        if (write_bytes) *write_bytes = wr;
    });
}

exa_status exa_batch_eval(exa_batch* b, uint32_t mask, const double* x, const double* y, double sigma,
                          double* jac, double* hess, exa_stream_t stream) {
    return guard([&] {
        if (!b) fail(EXA_EINVAL, "null batch");
        if (mask == 0 || mask > 3) fail(EXA_EINVAL, "mask must be EXA_CB_JAC, EXA_CB_HESS or both");
        const int64_t* tot = &b->offsets[4 * b->B];
        if (!x && tot[0]) fail(EXA_EINVAL, "null x");
        if ((mask & EXA_CB_HESS) && !y && tot[1]) fail(EXA_EINVAL, "null y");
        if ((mask & EXA_CB_JAC) && !jac && tot[2]) fail(EXA_EINVAL, "null jac output");
        if ((mask & EXA_CB_HESS) && !hess && tot[3]) fail(EXA_EINVAL, "null hess output");
        hipStream_t s = (hipStream_t)stream;
        if (b->autotune && !b->tuned) {
            tune(*b, mask, x, y, sigma, jac, hess, s);
            b->have_graph = false;
        }
        build_tiles(*b, b->epl, b->combined);
        if (!b->use_graph) {
            launch(*b, mask, x, y, sigma, jac, hess, s);
            return;
        }
        exa_batch::Key k{mask, x, y, jac, hess, sigma, b->epl, b->block, b->grid, b->combined};
        if (!b->have_graph || !(k == b->key)) {
            if (b->exec) (void)hipGraphExecDestroy(b->exec);
            if (b->graph) (void)hipGraphDestroy(b->graph);
            b->exec = nullptr;
            b->graph = nullptr;
            hip_check(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            try {
                launch(*b, mask, x, y, sigma, jac, hess, b->cap);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(b->cap, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            hip_check(hipStreamEndCapture(b->cap, &b->graph), "hipStreamEndCapture");
            hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
            b->key = k;
            b->have_graph = true;
        }
        hip_check(hipGraphLaunch(b->exec, s), "hipGraphLaunch");
    });
}

}  // extern "C"
