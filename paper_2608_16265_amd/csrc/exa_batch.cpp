// Batched evaluation of many instances of one formulation (Sec. 7.4.3 batch
// models, generalised to instances of different sizes and to every
// callback).
//
// All instances share the generated code; their data stays where each model
// put it, and their sizes and offsets are table data (one ExaInstDev per
// instance, whose offsets place the instance in the concatenated inputs,
// outputs and work buffers).  A call is
//   * ONE evaluation launch over a tile list of (instance, unit, data range)
//     tiles of every selected callback, one workgroup per tile (the kernels
//     and units of exa_eval: per-callback tiles, Jacobian + Hessian units or
//     one pass per point), or one launch per callback (each kernel with the
//     register budget of its own units), plus a launch for the parameter
//     adjoint;
//   * ONE launch of every instance's deterministic reductions (the same
//     segment sums, chunks and parts as the instance's own reduction, and
//     its objective partials), plus one small launch for the part sums of
//     segments longer than 1024 entries;
// recorded once into a HIP graph and replayed.  With xcd_aware, instances are
// binned over the 8 XCDs by algorithmic bytes (largest first into the
// lightest bin) and XCD j takes bin j's tiles and reduction blocks, so an
// instance's x and work buffers stay in that XCD's L2.  Workgroup size,
// points per lane, fused or separate patterns and the units are picked by
// timing candidates at a mask's first call; results do not depend on the
// schedule because every data point is evaluated by the same code and every
// reduction sums the same entries in the same order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <numeric>

#include "exa_internal.h"
#include "exa_kernels.h"
#include "exa_runtime.h"

using namespace exa;

namespace {
// work buffers of the batch (ExaBatchReduce::bufs)
constexpr int kBufFo = 0, kBufHv = 1, kBufPar = 2, kBufTile = 3;
constexpr int kWorkBufs = 4;  // the batch's own buffers (the others are the caller's)
// outputs of the reduction launch (ExaBatchReduce::outs)
constexpr int kOutF = 0, kOutG = 1, kOutJtw = 2, kOutHv = 3, kOutLag = 4, kOutLagTmp = 5, kOutThetaBar = 6;
constexpr int kOffX = 0, kOffY = 1, kOffJac = 2, kOffHess = 3, kOffTheta = 4, kNoff = 5;
constexpr int64_t kAlign = 16;  // entries: 128-byte lines
int64_t aligned(int64_t n) { return (n + kAlign - 1) / kAlign * kAlign; }
}  // namespace

struct exa_batch {
    std::vector<exa_model*> models;
    int B = 0;
    std::shared_ptr<Module> module;
    // code of the batch's own when the instances disagree on which index
    // columns are 0, 1, ..., n-1 (then only the columns that are so in every
    // instance use the data point itself), with its liveness records
    bool own_code = false;
    std::map<std::pair<int, int>, UnitLive> live;
    DeviceState mem;                   // owns every device array below
    ExaInstDev* inst = nullptr;        // per-instance tables (device)
    std::vector<int64_t> offsets;      // kNoff * (B + 1)
    double* theta = nullptr;           // the batch's parameters
    // work buffers, allocated on first use; instance i's block starts at
    // entry base[k][i] (a 128-byte line)
    double* buf[kWorkBufs] = {};
    std::vector<int64_t> base[kWorkBufs];
    int64_t buf_len[kWorkBufs] = {};
    double* lag_tmp = nullptr;         // J^T y of EXA_EV_LAG when the gradient is reduced
    // per instance: its models' device maps, with part sums of the batch's own
    struct Maps {
        DevMap grad, jt, h, par;
    };
    std::vector<Maps> maps;
    std::vector<int64_t> nobj;         // objective tiles per instance
    bool grad_direct_all = true, grad_direct_any = false;
    // options
    bool autotune = true, use_graph = true, xcd_aware = true, fuse = true;
    int block = 256, epl = 4, units = EXA_UNITS_JAC_HESS;
    // per mask: schedule, tile lists, reduction table
    struct Sched {
        int block = 256, epl = 4, units = EXA_UNITS_PER_CALLBACK;
        bool fused = true, tuned = false;
        bool unstaged = false;               // each lane's own output stores (EXA_UNSTAGED)
        std::vector<std::vector<int>> bins;  // instances per XCD
        ExaTile* tiles = nullptr;
        int64_t ntiles = 0;
        ExaTile* atiles = nullptr;           // parameter adjoint launch
        int64_t antiles = 0;
        // EXA_UNITS_SEPARATE: one launch per callback (mode, tiles, count)
        struct Part {
            int mode;
            ExaTile* tiles;
            int64_t ntiles;
        };
        std::vector<Part> parts;
        int64_t tuned_ns = 0;
        ExaBatchJob* jobs = nullptr;
        int32_t* blocks = nullptr;
        int64_t nblocks = 0;
        int32_t* lblocks = nullptr;
        int64_t nlblocks = 0;
        bool axpy = false, reduce_built = false;
    };
    std::map<uint32_t, Sched> sched;
    // graph of the last call
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    struct Key {
        uint32_t mask = 0;
        exa_batch_io io;
        int block = 0, epl = 0, units = 0;
        bool fused = false;
        bool operator==(const Key& o) const {
            return mask == o.mask && std::memcmp(&io, &o.io, sizeof io) == 0 && block == o.block && epl == o.epl &&
                   units == o.units && fused == o.fused;
        }
    } key, last;  // the graph's call; the previous call
    bool have_graph = false, have_last = false;
    // launch timing (exa_batch_timing)
    struct Timing {
        bool on = false;
        std::vector<hipEvent_t> ev;
        std::vector<char> reduced;
        int64_t used = 0;
    } timing;

    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        have_graph = false;
    }
    void timing_off() {
        for (hipEvent_t e : timing.ev) (void)hipEventDestroy(e);
        timing = Timing();
    }
    ~exa_batch() {
        drop_graph();
        timing_off();
        if (cap) (void)hipStreamDestroy(cap);
    }
};

namespace {

// The exa_eval mask whose tiles a batch mask launches (the Lagrangian
// gradient is the gradient and J^T y tiles; the adjoint has a launch of its
// own).
uint32_t eval_mask(uint32_t mask) {
    uint32_t e = mask & EXA_EV_ALL;
    if (mask & EXA_EV_LAG) e |= EXA_EV_GRAD | EXA_EV_JTPROD;
    return e;
}

// The units a batch mask can run as asked: EXA_UNITS_SEPARATE needs two
// callbacks or more; the others as exa_eval allows them.
int batch_units(uint32_t em, int units) {
    if (!em) return EXA_UNITS_PER_CALLBACK;
    if (units == EXA_UNITS_SEPARATE) return eval_modes(em, false).size() > 1 ? units : EXA_UNITS_PER_CALLBACK;
    return valid_units(em, units);
}

// Modes of the evaluation launch(es) of a mask under units.
std::vector<int> modes_of(uint32_t em, int units) {
    if (!em) return {};
    if (units == EXA_UNITS_SEPARATE) return eval_modes(em, false);
    return launch_modes(em, units);
}

const std::vector<int>& main_modes(const exa_batch::Sched& S, uint32_t mask, std::vector<int>& tmp) {
    tmp = modes_of(eval_mask(mask), S.units);
    return tmp;
}

// A launch of one plain mode runs that mode's own kernel (exa_k_<mode>);
// several modes, or units of several callbacks, run a several-callback kernel.
bool single_kernel(const std::vector<int>& modes) { return modes.size() == 1 && !multi_unit_mode(modes[0]); }

// Per-instance algorithmic bytes of a mask's evaluation, the cost by which
// instances are binned over the XCDs.
std::vector<int64_t> instance_cost(const exa_batch& b, uint32_t mask, int units, bool fused) {
    std::vector<int64_t> cost(b.B, 0);
    const uint32_t em = eval_mask(mask);
    for (int i = 0; i < b.B; ++i) {
        const Model& M = b.models[i]->impl;
        int64_t rd = 0, wr = 0;
        if (em) {
            kernel_bytes(M, modes_of(em, batch_units(em, units)), fused, rd, wr, b.own_code ? &b.live : nullptr);
            cost[i] += rd + wr;
        }
        if (mask & EXA_EV_ADJ) {
            kernel_bytes(M, {M_ADJ}, fused, rd, wr, b.own_code ? &b.live : nullptr);
            cost[i] += rd + wr;
        }
    }
    return cost;
}

void make_bins(exa_batch& b, exa_batch::Sched& S, uint32_t mask) {
    S.bins.assign(8, {});
    if (!b.xcd_aware) {
        // instances in order, cut into eight contiguous runs of similar cost
        const std::vector<int64_t> cost = instance_cost(b, mask, S.units, S.fused);
        const int64_t tot = std::accumulate(cost.begin(), cost.end(), (int64_t)0);
        int64_t acc = 0;
        for (int i = 0; i < b.B; ++i) {
            const int j = tot > 0 ? (int)std::min<int64_t>(7, 8 * acc / tot) : 0;
            S.bins[j].push_back(i);
            acc += cost[i];
        }
        return;
    }
    const std::vector<int64_t> cost = instance_cost(b, mask, S.units, S.fused);
    std::vector<int> order(b.B);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] > cost[c]; });
    std::vector<int64_t> load(8, 0);
    for (int i : order) {
        const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        S.bins[j].push_back(i);
        load[j] += cost[i];
    }
    for (auto& bin : S.bins) std::sort(bin.begin(), bin.end());
}

// Tiles of instance i for one launch of `modes` (mode bits in the codes when
// the launch is a several-callback kernel).
void instance_tiles(const exa_batch& b, int i, const std::vector<int>& modes, bool tagged, uint32_t em,
                    int64_t tp, bool fused, std::vector<ExaTile>& out) {
    const Model& M = b.models[i]->impl;
    for (int mode : modes) {
        std::vector<ExaTile> t = mode == M_OBJ ? make_tiles(M, M_OBJ, i, (int64_t)kObjBlock * kObjEpl, kObjFused)
                                               : make_tiles(M, mode, i, tp, fused, true);
        if (mode == M_GRAD || (multi_unit_mode(mode) && (em & EXA_EV_GRAD))) {
            std::vector<ExaTile> z;
            add_zero_tiles(M, tp, z);
            for (ExaTile& x : z) {
                x.inst = i;
                if (tagged) x.pat |= M_GRAD << EXA_MODE_SHIFT;
            }
            if (tagged || mode == M_GRAD) t.insert(t.end(), z.begin(), z.end());
        }
        for (ExaTile& x : t) {
            x.inst = i;
            if (tagged && x.pat != ((M_GRAD << EXA_MODE_SHIFT) | EXA_ZERO_TILE)) x.pat |= mode << EXA_MODE_SHIFT;
        }
        out.insert(out.end(), t.begin(), t.end());
    }
}

// Bin j's tiles, then bin j+1's, each bin padded with no-op tiles to the
// longest, so that XCD j (workgroups w with w % 8 == j) takes exactly bin j.
ExaTile* upload_binned(exa_batch& b, const exa_batch::Sched& S, const std::vector<std::vector<ExaTile>>& per,
                       int64_t& n) {
    int64_t longest = 0;
    for (const auto& bin : S.bins) {
        int64_t c = 0;
        for (int i : bin) c += (int64_t)per[i].size();
        longest = std::max(longest, c);
    }
    n = 8 * longest;
    if (n == 0) return nullptr;
    std::vector<ExaTile> v;
    v.reserve(n);
    ExaTile pad{};
    pad.pat = EXA_PAD_TILE;
    for (int j = 0; j < 8; ++j) {
        for (int i : S.bins[j]) v.insert(v.end(), per[i].begin(), per[i].end());
        while ((int64_t)v.size() < (j + 1) * longest) v.push_back(pad);
    }
    return (ExaTile*)b.mem.upload(v.data(), v.size() * sizeof(ExaTile));
}

void set_batch_schedule(exa_batch& b, uint32_t mask, int block, int epl, bool fused, int units) {
    exa_batch::Sched& S = b.sched[mask];
    const uint32_t em = eval_mask(mask);
    S.units = batch_units(em, units);
    S.block = block;
    S.epl = epl;
    S.fused = fused;
    if (S.bins.empty()) make_bins(b, S, mask);
    const int64_t tp = (int64_t)block * epl;
    std::vector<int> tmp;
    const std::vector<int>& modes = main_modes(S, mask, tmp);
    b.mem.release(S.tiles);
    b.mem.release(S.atiles);
    for (auto& p : S.parts) b.mem.release(p.tiles);
    S.tiles = nullptr;
    S.ntiles = 0;
    S.parts.clear();
    std::vector<std::vector<ExaTile>> per(b.B), adj(b.B);
    if (S.units == EXA_UNITS_SEPARATE) {
        for (int mode : modes) {
            for (auto& v : per) v.clear();
            for (int i = 0; i < b.B; ++i) instance_tiles(b, i, {mode}, false, em, tp, fused, per[i]);
            exa_batch::Sched::Part part{mode, nullptr, 0};
            part.tiles = upload_binned(b, S, per, part.ntiles);
            S.parts.push_back(part);
        }
    } else if (!modes.empty()) {
        for (int i = 0; i < b.B; ++i) instance_tiles(b, i, modes, !single_kernel(modes), em, tp, fused, per[i]);
        S.tiles = upload_binned(b, S, per, S.ntiles);
    }
    if (mask & EXA_EV_ADJ) {
        for (int i = 0; i < b.B; ++i) instance_tiles(b, i, {M_ADJ}, false, 0, tp, fused, adj[i]);
        S.atiles = upload_binned(b, S, adj, S.antiles);
    }
}

double* need_buf(exa_batch& b, int k) {
    if (!b.buf[k]) b.buf[k] = (double*)b.mem.alloc(std::max<int64_t>(1, b.buf_len[k]) * sizeof(double));
    return b.buf[k];
}

ExaBatchJob seg_batch_job(const DevMap& m, int bufk, int64_t buf_off, int out, int64_t out_off, bool ep,
                          int64_t w_off = 0) {
    ExaBatchJob J;
    std::memset(&J, 0, sizeof J);
    J.ptr = m.ptr;
    J.idx = m.idx;
    J.lanes = m.lanes;
    J.lidx = m.lidx;
    J.longs = m.longs;
    J.lpart = m.lpart;
    J.lsum = m.lsum;
    J.nseg = m.nseg;
    J.nlanes = m.nlanes;
    J.nparts = m.nparts;
    J.nlong = m.nlong;
    J.wide = m.wide;
    J.chunked = m.chunked;
    J.buf = bufk;
    J.buf_off = buf_off;
    J.out = out;
    J.out_off = out_off;
    J.w_off = w_off;
    J.ep = ep ? 1 : 0;
    return J;
}

int64_t batch_job_blocks(const ExaBatchJob& J) {
    if (J.kind == 1) return 1;
    ExaSegJob S;
    std::memset(&S, 0, sizeof S);
    S.nseg = J.nseg;
    S.chunked = J.chunked;
    S.nlanes = J.nlanes;
    S.nparts = J.nparts;
    return exa_job_blocks(S);
}

// The reduction table of a mask: every instance's jobs, their blocks laid out
// by the mask's XCD bins (bin j's blocks are the j-th eighth of the launch).
void build_reductions(exa_batch& b, exa_batch::Sched& S, uint32_t mask) {
    std::vector<ExaBatchJob> jobs;
    std::vector<std::vector<int32_t>> per_bin(8);
    std::vector<int32_t> lbl;
    S.axpy = false;
    for (int j = 0; j < 8; ++j)
        for (int i : S.bins[j]) {
            const exa_batch::Maps& mp = b.maps[i];
            const int64_t xo = b.offsets[kNoff * i + kOffX], yo = b.offsets[kNoff * i + kOffY];
            const int64_t fo = b.base[kBufFo].empty() ? 0 : b.base[kBufFo][i];
            std::vector<ExaBatchJob> mine;
            if ((mask & EXA_EV_GRAD) && !b.grad_direct_all) mine.push_back(seg_batch_job(mp.grad, kBufFo, fo, kOutG, xo, false));
            if (mask & EXA_EV_LAG) {
                if (b.grad_direct_all) {
                    // g was written in place by the evaluation launch: the
                    // J^T y sums finish it as g = sigma g + J^T y
                    mine.push_back(seg_batch_job(mp.jt, kBufFo, fo, kOutLag, xo, true, yo));
                } else {
                    mine.push_back(seg_batch_job(mp.grad, kBufFo, fo, kOutLag, xo, false));
                    mine.push_back(seg_batch_job(mp.jt, kBufFo, fo, kOutLagTmp, xo, false, yo));
                    S.axpy = true;
                }
            }
            if (mask & EXA_EV_JTPROD) mine.push_back(seg_batch_job(mp.jt, kBufFo, fo, kOutJtw, xo, false, yo));
            if (mask & EXA_EV_HPROD) mine.push_back(seg_batch_job(mp.h, kBufHv, b.base[kBufHv][i], kOutHv, xo, false));
            if (mask & EXA_EV_ADJ)
                mine.push_back(seg_batch_job(mp.par, kBufPar, b.base[kBufPar][i], kOutThetaBar,
                                             b.offsets[kNoff * i + kOffTheta], false));
            if (mask & EXA_EV_OBJ) {
                ExaBatchJob J;
                std::memset(&J, 0, sizeof J);
                J.kind = 1;
                J.buf = kBufTile;
                J.buf_off = b.base[kBufTile][i];
                J.nseg = b.nobj[i];
                J.out = kOutF;
                J.out_off = i;
                mine.push_back(J);
            }
            for (const ExaBatchJob& J : mine) {
                const int32_t id = (int32_t)jobs.size();
                jobs.push_back(J);
                const int64_t nb = batch_job_blocks(J);
                for (int64_t k = 0; k < nb; ++k) per_bin[j].insert(per_bin[j].end(), {id, (int32_t)k});
                if (J.kind == 0 && J.nparts > 0)
                    for (int64_t l = 0; l < J.nlong; ++l) lbl.insert(lbl.end(), {id, (int32_t)l});
            }
        }
    size_t longest = 0;
    for (auto& v : per_bin) longest = std::max(longest, v.size() / 2);
    std::vector<int32_t> blocks;
    for (auto& v : per_bin) {
        blocks.insert(blocks.end(), v.begin(), v.end());
        for (size_t k = v.size() / 2; k < longest; ++k) blocks.insert(blocks.end(), {-1, 0});
    }
    b.mem.release(S.jobs);
    b.mem.release(S.blocks);
    b.mem.release(S.lblocks);
    S.jobs = jobs.empty() ? nullptr : (ExaBatchJob*)b.mem.upload(jobs.data(), jobs.size() * sizeof(ExaBatchJob));
    S.nblocks = (int64_t)blocks.size() / 2;
    S.blocks = blocks.empty() ? nullptr : (int32_t*)b.mem.upload(blocks.data(), blocks.size() * sizeof(int32_t));
    S.nlblocks = (int64_t)lbl.size() / 2;
    S.lblocks = lbl.empty() ? nullptr : (int32_t*)b.mem.upload(lbl.data(), lbl.size() * sizeof(int32_t));
    S.reduce_built = true;
}

// Call records of the selected callbacks, as exa_eval sets them up for one
// model, with the batch's buffers and instance table.
ExaMulti call_records(exa_batch& b, uint32_t mask, const exa_batch_io& io) {
    ExaMulti mc;
    std::memset(&mc, 0, sizeof mc);
    const bool lag = (mask & EXA_EV_LAG) != 0;
    const bool unstaged = b.sched.count(mask) && b.sched.at(mask).unstaged;
    for (int mode = 0; mode < M_COUNT; ++mode) {
        ExaCall& c = mc.c[mode];
        c.inst = b.inst;
        c.x = io.x;
        c.unstaged = unstaged ? 1 : 0;
        switch (mode) {
            case M_OBJ: c.out0 = b.buf[kBufTile]; break;
            case M_GRAD:
                c.direct = b.grad_direct_all ? 1 : 0;
                c.out0 = b.grad_direct_all ? (lag ? io.lag : io.g) : b.buf[kBufFo];
                break;
            case M_CONS: c.out0 = io.c; break;
            case M_JAC: c.out0 = io.jac; break;
            case M_HESS:
                c.y = io.y;
                c.sigma = io.obj_weight;
                c.out0 = io.hess;
                break;
            case M_JH:
                c.y = io.y;
                c.sigma = io.obj_weight;
                c.out0 = io.jac;
                c.out1 = io.hess;
                break;
            case M_JPROD:
                c.v = io.v;
                c.out0 = io.jv;
                break;
            case M_JTPROD:
                c.y = lag ? io.y : io.w;
                c.out0 = b.buf[kBufFo];
                break;
            case M_HPROD:
                c.y = io.y;
                c.v = io.v;
                c.sigma = io.obj_weight;
                c.out0 = b.buf[kBufHv];
                c.out1 = io.hv;
                break;
            case M_ADJ:
                c.y = io.y;
                c.v = io.wx;
                c.sigma = io.obj_weight;
                c.out0 = b.buf[kBufPar];
                break;
            default: break;
        }
    }
    return mc;
}

// The evaluation launch(es) of a mask under its current schedule.
void launch_eval(exa_batch& b, uint32_t mask, const ExaMulti& rec, hipStream_t s) {
    const exa_batch::Sched& S = b.sched.at(mask);
    const Module& K = *b.module;
    std::vector<int> tmp;
    const std::vector<int>& modes = main_modes(S, mask, tmp);
    auto launch_single = [&](int mode, ExaTile* tiles, int64_t n) {
        if (n == 0) return;
        ExaCall c = rec.c[mode];
        c.tiles = tiles;
        c.ntiles = n;
        c.per_xcd = n / 8;
        void* args[] = {&c};
        hip_check(hipModuleLaunchKernel(K.fn[mode], (unsigned)n, 1, 1, (unsigned)S.block, 1, 1, 0, s, args, nullptr),
                  "hipModuleLaunchKernel");
    };
    for (const auto& p : S.parts) launch_single(p.mode, p.tiles, p.ntiles);
    if (S.ntiles > 0) {
        if (single_kernel(modes)) {
            ExaCall c = rec.c[modes[0]];
            c.tiles = S.tiles;
            c.ntiles = S.ntiles;
            c.per_xcd = S.ntiles / 8;
            void* args[] = {&c};
            hip_check(hipModuleLaunchKernel(K.fn[modes[0]], (unsigned)S.ntiles, 1, 1, (unsigned)S.block, 1, 1, 0, s,
                                            args, nullptr),
                      "hipModuleLaunchKernel");
        } else {
            ExaMulti mc = rec;
            mc.tiles = S.tiles;
            mc.ntiles = S.ntiles;
            mc.per_xcd = S.ntiles / 8;
            hipFunction_t fn = S.units == EXA_UNITS_ONE_PASS   ? K.fn_onepass
                               : S.units == EXA_UNITS_JAC_HESS ? K.fn_multijh
                                                               : K.fn_multi;
            void* args[] = {&mc};
            hip_check(hipModuleLaunchKernel(fn, (unsigned)S.ntiles, 1, 1, (unsigned)S.block, 1, 1, 0, s, args, nullptr),
                      "hipModuleLaunchKernel");
        }
    }
    if (S.antiles > 0) {
        ExaCall c = rec.c[M_ADJ];
        c.tiles = S.atiles;
        c.ntiles = S.antiles;
        c.per_xcd = S.antiles / 8;
        void* args[] = {&c};
        hip_check(hipModuleLaunchKernel(K.fn[M_ADJ], (unsigned)S.antiles, 1, 1, (unsigned)S.block, 1, 1, 0, s, args,
                                        nullptr),
                  "hipModuleLaunchKernel");
    }
}

// The reduction launch(es) of a mask.  Returns whether anything was launched.
bool launch_reduce(exa_batch& b, uint32_t mask, const exa_batch_io& io, hipStream_t s) {
    const exa_batch::Sched& S = b.sched.at(mask);
    ExaBatchReduce R;
    std::memset(&R, 0, sizeof R);
    R.jobs = S.jobs;
    R.blocks = S.blocks;
    R.nblocks = S.nblocks;
    R.lblocks = S.lblocks;
    R.nlblocks = S.nlblocks;
    for (int k = 0; k < kWorkBufs; ++k) R.bufs[k] = b.buf[k];
    R.outs[kOutF] = io.f;
    R.outs[kOutG] = io.g;
    R.outs[kOutJtw] = io.jtw;
    R.outs[kOutHv] = io.hv;
    R.outs[kOutLag] = io.lag;
    R.outs[kOutLagTmp] = b.lag_tmp;
    R.outs[kOutThetaBar] = io.theta_bar;
    // the weights of J^T w (J^T y for the Lagrangian gradient)
    R.w = (mask & EXA_EV_LAG) ? io.y : io.w;
    R.alpha = io.obj_weight;
    hip_check(exa_launch_reduce_batch(R, s), "batched reductions");
    if (S.axpy) {
        // lag = sigma * lag + J^T y, each operation rounded on its own (as
        // exa_lag_grad finishes a reduced gradient)
        ExaReduce A;
        std::memset(&A, 0, sizeof A);
        A.ep_job = -1;
        A.ax_out = io.lag;
        A.ax_add = b.lag_tmp;
        A.ax_alpha = io.obj_weight;
        A.ax_n = b.offsets[kNoff * b.B + kOffX];
        hip_check(exa_launch_reduce(A, s), "batched Lagrangian gradient");
    }
    return S.nblocks > 0 || S.nlblocks > 0 || S.axpy;
}

void run(exa_batch& b, uint32_t mask, const exa_batch_io& io, hipStream_t s) {
    const ExaMulti rec = call_records(b, mask, io);
    exa_batch::Timing& T = b.timing;
    const bool timed = T.on && T.used < (int64_t)T.reduced.size();
    hipEvent_t* ev = timed ? &T.ev[4 * T.used] : nullptr;
    if (timed) hip_check(hipEventRecord(ev[0], s), "hipEventRecord");
    launch_eval(b, mask, rec, s);
    if (timed) {
        hip_check(hipEventRecord(ev[1], s), "hipEventRecord");
        hip_check(hipEventRecord(ev[2], s), "hipEventRecord");
    }
    const bool red = launch_reduce(b, mask, io, s);
    if (timed) {
        hip_check(hipEventRecord(ev[3], s), "hipEventRecord");
        T.reduced[T.used++] = red ? 1 : 0;
    }
}

// First call with a mask under autotune: time every candidate schedule's
// evaluation launch(es) on the caller's arguments and keep the fastest.
void tune_batch(exa_batch& b, uint32_t mask, const exa_batch_io& io, hipStream_t s) {
    const uint32_t em = eval_mask(mask);
    const int blocks[] = {64, 128, 256};
    const int epls[] = {1, 2, 4, 8};
    std::vector<int> fuses = {0};
    bool fusable = false;
    for (int mode : eval_modes(em, false))
        if (mode != M_OBJ && has_fusable_group(b.models[0]->impl, mode)) fusable = true;
    if ((mask & EXA_EV_ADJ) && has_fusable_group(b.models[0]->impl, M_ADJ)) fusable = true;
    if (fusable) fuses.push_back(1);
    std::vector<int> combos = {EXA_UNITS_PER_CALLBACK};
    if (em && has_jh(em)) combos.push_back(EXA_UNITS_JAC_HESS);
    if (em && combined_mode_of(em) >= 0) combos.push_back(EXA_UNITS_ONE_PASS);
    if (em && eval_modes(em, false).size() > 1) combos.push_back(EXA_UNITS_SEPARATE);
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    struct Cand {
        float ms;
        int block, epl, fused, units;
    };
    const ExaMulti rec = call_records(b, mask, io);
    auto time_it = [&](int reps) {
        launch_eval(b, mask, rec, s);
        hip_check(hipEventRecord(e0, s), "hipEventRecord");
        for (int r = 0; r < reps; ++r) launch_eval(b, mask, rec, s);
        hip_check(hipEventRecord(e1, s), "hipEventRecord");
        hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        return ms / reps;
    };
    std::vector<Cand> cands;
    try {
        for (int u : combos)
            for (int f : fuses)
                for (int bk : blocks)
                    for (int ep : epls) {
                        set_batch_schedule(b, mask, bk, ep, f != 0, u);
                        cands.push_back({time_it(2), bk, ep, f, u});
                    }
        // neighbouring schedules differ by less than one timing's noise: the
        // fastest few again, longer, in turns; the best of their rounds decides
        std::sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
        cands.resize(std::min<size_t>(cands.size(), 6));
        for (auto& c : cands) c.ms = 1e30f;
        for (int round = 0; round < 3; ++round)
            for (auto& c : cands) {
                set_batch_schedule(b, mask, c.block, c.epl, c.fused != 0, c.units);
                c.ms = std::min(c.ms, time_it(6));
            }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    const Cand& w = *std::min_element(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
    set_batch_schedule(b, mask, w.block, w.epl, w.fused != 0, w.units);
    b.sched[mask].tuned_ns = (int64_t)(w.ms * 1e6);
    // staged or each lane's own stores of the Jacobian and Hessian values
    if (mask & (EXA_EV_JAC | EXA_EV_HESS)) {
        float best[2] = {1e30f, 1e30f};
        for (int round = 0; round < 2; ++round)
            for (int u = 0; u < 2; ++u) {
                b.sched[mask].unstaged = u != 0;
                const ExaMulti r2 = call_records(b, mask, io);
                launch_eval(b, mask, r2, s);
                hip_check(hipEventRecord(e0, s), "hipEventRecord");
                for (int r = 0; r < 6; ++r) launch_eval(b, mask, r2, s);
                hip_check(hipEventRecord(e1, s), "hipEventRecord");
                hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
                float ms = 0;
                hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
                best[u] = std::min(best[u], ms / 6);
            }
        b.sched[mask].unstaged = best[1] < best[0];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (log_on())
        log_msg("tuned batch of " + std::to_string(b.B) + " mask " + std::to_string(mask) + ": block " +
                std::to_string(w.block) + ", points per lane " + std::to_string(w.epl) + ", fused " +
                std::to_string(w.fused) + ", units " + std::to_string(w.units) + " (" + std::to_string(w.ms * 1e3) +
                " us)");
}

void check_mask(uint32_t mask) {
    if (mask == 0 || (mask & ~(uint32_t)EXA_BATCH_ALL))
        fail(EXA_EINVAL, "mask must select callbacks with the EXA_EV_* bits");
    if ((mask & EXA_EV_LAG) && (mask & (EXA_EV_GRAD | EXA_EV_JTPROD)))
        fail(EXA_EINVAL, "EXA_EV_LAG cannot be combined with EXA_EV_GRAD or EXA_EV_JTPROD");
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
        for (int i = 0; i < B; ++i) {
            if (!models[i]) fail(EXA_EINVAL, "null model in batch");
            if (models[i]->impl.signature != models[0]->impl.signature)
                fail(EXA_EINVAL, "model " + std::to_string(i) + " does not share the pattern trees of model 0");
        }
        for (int i = 0; i < B; ++i)
            if (models[i]->impl.host_only || !models[i]->impl.dev)
                fail(EXA_ESTATE, "batched models need a device");
        std::unique_ptr<exa_batch> b(new exa_batch());
        b->B = B;
        b->models.assign(models, models + B);
        if (opt) {
            b->autotune = opt->autotune != 0;
            if (opt->block) b->block = opt->block;
            if (opt->epl) b->epl = opt->epl;
            b->fuse = opt->fuse != 0;
            b->units = opt->units;
            b->use_graph = opt->use_graph != 0;
            b->xcd_aware = opt->xcd_aware != 0;
        }
        if (b->block != 64 && b->block != 128 && b->block != 256) fail(EXA_EINVAL, "block must be 64, 128 or 256");
        if (b->epl < 1 || b->epl > 16) fail(EXA_EINVAL, "epl must be in 1..16");
        if ((b->units & ~EXA_UNSTAGED) < EXA_UNITS_PER_CALLBACK || (b->units & ~EXA_UNSTAGED) > EXA_UNITS_SEPARATE)
            fail(EXA_EINVAL, "units must be one of the EXA_UNITS_* values");
        // every instance runs the same generated code
        const Model& M0 = models[0]->impl;
        std::vector<std::vector<char>> ident;
        for (const Pattern& P : M0.pats) ident.push_back(P.ident);
        for (int i = 1; i < B; ++i)
            for (size_t p = 0; p < ident.size(); ++p)
                for (size_t c = 0; c < ident[p].size(); ++c) ident[p][c] &= models[i]->impl.pats[p].ident[c];
        // H v references stored into the output: code for any instance that
        // may (the others take the buffer path by their own bits)
        std::vector<std::vector<char>> hvd;
        for (const Group& G : M0.groups) hvd.push_back(G.hv_direct);
        for (int i = 1; i < B; ++i)
            for (size_t g = 0; g < hvd.size(); ++g)
                for (size_t r = 0; r < hvd[g].size(); ++r) hvd[g][r] |= models[i]->impl.groups[g].hv_direct[r];
        bool same = true;
        for (size_t p = 0; p < ident.size(); ++p) same = same && ident[p] == M0.pats[p].ident;
        for (size_t g = 0; g < hvd.size(); ++g) same = same && hvd[g] == M0.groups[g].hv_direct;
        if (same) {
            b->module = M0.dev->module;
        } else {
            bool hit = false;
            b->module = compile_module(generate_source(M0, &b->live, &ident, &hvd), M0.cache_dir, &hit);
            b->own_code = true;
        }

        // offsets in the concatenated arrays and bases in the work buffers
        b->offsets.assign(kNoff * (B + 1), 0);
        for (int k = 0; k < kWorkBufs; ++k) b->base[k].assign(B, 0);
        b->nobj.assign(B, 0);
        for (int i = 0; i < B; ++i) {
            const Model& M = models[i]->impl;
            const int64_t* o = &b->offsets[kNoff * i];
            int64_t* n = &b->offsets[kNoff * (i + 1)];
            n[kOffX] = o[kOffX] + M.nvar;
            n[kOffY] = o[kOffY] + M.ncon;
            n[kOffJac] = o[kOffJac] + M.nnzj;
            n[kOffHess] = o[kOffHess] + M.nnzh;
            n[kOffTheta] = o[kOffTheta] + M.ntheta;
            b->nobj[i] = M.dev->sched[M_OBJ].ntiles;
            const int64_t len[kWorkBufs] = {M.fo_obj_len + M.fo_con_len, M.hv_len, M.par_len, b->nobj[i]};
            for (int k = 0; k < kWorkBufs; ++k) {
                b->base[k][i] = b->buf_len[k];
                b->buf_len[k] += aligned(len[k]);
            }
            b->grad_direct_all = b->grad_direct_all && M.grad_direct;
            b->grad_direct_any = b->grad_direct_any || M.grad_direct;
        }
        // the batch's parameters: a copy of each model's device parameters
        const int64_t nth = b->offsets[kNoff * B + kOffTheta];
        b->theta = (double*)b->mem.alloc(std::max<int64_t>(1, nth) * sizeof(double));
        for (int i = 0; i < B; ++i) {
            const Model& M = models[i]->impl;
            if (M.ntheta)
                hip_check(hipMemcpy(b->theta + b->offsets[kNoff * i + kOffTheta], M.dev->theta,
                                    M.ntheta * sizeof(double), hipMemcpyDeviceToDevice),
                          "hipMemcpy");
        }
        // instance tables
        std::vector<ExaInstDev> inst(B);
        for (int i = 0; i < B; ++i) {
            const Model& M = models[i]->impl;
            inst[i] = M.dev->inst_host;
            std::memset(inst[i].off, 0, sizeof inst[i].off);
            inst[i].off[EXA_OFF_X] = b->offsets[kNoff * i + kOffX];
            inst[i].off[EXA_OFF_Y] = b->offsets[kNoff * i + kOffY];
            inst[i].off[EXA_OFF_ROWS] = b->offsets[kNoff * i + kOffY];
            inst[i].off[EXA_OFF_JAC] = b->offsets[kNoff * i + kOffJac];
            inst[i].off[EXA_OFF_HESS] = b->offsets[kNoff * i + kOffHess];
            inst[i].off[EXA_OFF_FO_OBJ] = b->base[kBufFo][i];
            inst[i].off[EXA_OFF_FO_CON] = b->base[kBufFo][i] + M.fo_obj_len;
            inst[i].off[EXA_OFF_HV] = b->base[kBufHv][i];
            inst[i].off[EXA_OFF_PAR] = b->base[kBufPar][i];
            inst[i].off[EXA_OFF_TILE] = b->base[kBufTile][i];
            inst[i].theta = b->theta + b->offsets[kNoff * i + kOffTheta];
        }
        b->inst = (ExaInstDev*)b->mem.upload(inst.data(), inst.size() * sizeof(ExaInstDev));
        // the models' maps, each with part sums of the batch's own
        b->maps.resize(B);
        for (int i = 0; i < B; ++i) {
            const DeviceState& D = *models[i]->impl.dev;
            exa_batch::Maps& mp = b->maps[i];
            mp.grad = D.grad_map;
            mp.jt = D.jt_map;
            mp.h = D.h_map;
            mp.par = D.par_map;
            for (DevMap* m : {&mp.grad, &mp.jt, &mp.h, &mp.par})
                if (m->nparts > 0) m->lsum = (double*)b->mem.alloc(m->nparts * sizeof(double));
        }
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

exa_status exa_batch_set_theta(exa_batch* b, const double* theta, exa_stream_t stream) {
    return guard([&] {
        if (!b) fail(EXA_EINVAL, "null batch");
        const int64_t n = b->offsets[kNoff * b->B + kOffTheta];
        if (n > 0 && !theta) fail(EXA_EINVAL, "null theta");
        if (n > 0)
            hip_check(hipMemcpyAsync(b->theta, theta, n * sizeof(double), hipMemcpyDeviceToDevice,
                                     (hipStream_t)stream),
                      "hipMemcpyAsync");
    });
}

exa_status exa_batch_schedule(const exa_batch* b, uint32_t mask, int64_t* out6) {
    return guard([&] {
        if (!b || !out6) fail(EXA_EINVAL, "null argument");
        auto it = b->sched.find(mask);
        if (it == b->sched.end()) fail(EXA_ESTATE, "no exa_batch_eval call with this mask yet");
        const exa_batch::Sched& S = it->second;
        out6[0] = S.block;
        out6[1] = S.epl;
        out6[2] = S.fused ? 1 : 0;
        out6[3] = S.units | (S.unstaged ? EXA_UNSTAGED : 0);
        int64_t nt = S.ntiles + S.antiles;
        for (const auto& p : S.parts) nt += p.ntiles;
        out6[4] = nt;
        out6[5] = S.tuned_ns;
    });
}

exa_status exa_batch_set_schedule(exa_batch* b, uint32_t mask, int32_t block, int32_t epl, int32_t fused,
                                  int32_t units) {
    return guard([&] {
        if (!b) fail(EXA_EINVAL, "null batch");
        check_mask(mask);
        if (block != 64 && block != 128 && block != 256) fail(EXA_EINVAL, "block must be 64, 128 or 256");
        if (epl < 1 || epl > 16) fail(EXA_EINVAL, "points per lane must be in 1..16");
        const bool unstaged = (units & EXA_UNSTAGED) != 0;
        units &= ~EXA_UNSTAGED;
        if (units < EXA_UNITS_PER_CALLBACK || units > EXA_UNITS_SEPARATE)
            fail(EXA_EINVAL, "units must be one of the EXA_UNITS_* values");
        set_batch_schedule(*b, mask, block, epl, fused != 0, units);
        b->sched[mask].unstaged = unstaged;
        b->sched[mask].reduce_built = false;
        b->sched[mask].tuned = true;
        b->drop_graph();
    });
}

exa_status exa_batch_bytes(const exa_batch* b, uint32_t mask, int64_t* out4) {
    return guard([&] {
        if (!b || !out4) fail(EXA_EINVAL, "null argument");
        check_mask(mask);
        int units = b->units & ~EXA_UNSTAGED;
        bool fused = b->fuse;
        auto it = b->sched.find(mask);
        if (it != b->sched.end()) {
            units = it->second.units;
            fused = it->second.fused;
        }
        const uint32_t em = eval_mask(mask);
        int64_t er = 0, ew = 0, rr = 0, rw = 0;
        for (int i = 0; i < b->B; ++i) {
            const Model& M = b->models[i]->impl;
            int64_t r = 0, w = 0;
            if (em) {
                kernel_bytes(M, modes_of(em, batch_units(em, units)), fused, r, w, b->own_code ? &b->live : nullptr);
                er += r;
                ew += w;
            }
            if (mask & EXA_EV_ADJ) {
                kernel_bytes(M, {M_ADJ}, fused, r, w, b->own_code ? &b->live : nullptr);
                er += r;
                ew += w;
            }
            reduce_bytes(M, mask, r, w);
            rr += r;
            rw += w;
            // one objective partial is copied by the reduction launch
            if ((mask & EXA_EV_OBJ) && b->nobj[i] == 1) {
                rr += 8;
                rw += 8;
            }
            // g = sigma g + J^T y reads g once; a reduced gradient is finished
            // by an elementwise launch (two reads and a write per entry)
            if (mask & EXA_EV_LAG) rr += (b->grad_direct_all ? 8 : 16) * M.nvar, rw += b->grad_direct_all ? 0 : 8 * M.nvar;
        }
        out4[0] = er;
        out4[1] = ew;
        out4[2] = rr;
        out4[3] = rw;
    });
}

exa_status exa_batch_eval(exa_batch* b, uint32_t mask, const exa_batch_io* io, exa_stream_t stream) {
    return guard([&] {
        if (!b) fail(EXA_EINVAL, "null batch");
        if (!io) fail(EXA_EINVAL, "null exa_batch_io");
        check_mask(mask);
        const int64_t* tot = &b->offsets[kNoff * b->B];
        auto need = [](const void* p, int64_t n, const char* what) {
            if (n > 0 && !p) fail(EXA_EINVAL, std::string("null pointer: ") + what);
        };
        need(io->x, tot[kOffX], "x");
        if (mask & (EXA_EV_HESS | EXA_EV_HPROD | EXA_EV_LAG | EXA_EV_ADJ)) need(io->y, tot[kOffY], "y");
        if (mask & (EXA_EV_JPROD | EXA_EV_HPROD)) need(io->v, tot[kOffX], "v");
        if (mask & EXA_EV_JTPROD) need(io->w, tot[kOffY], "w");
        if (mask & EXA_EV_ADJ) need(io->wx, tot[kOffX], "wx");
        if (mask & EXA_EV_OBJ) need(io->f, b->B, "f");
        if (mask & EXA_EV_GRAD) need(io->g, tot[kOffX], "g");
        if (mask & EXA_EV_CONS) need(io->c, tot[kOffY], "c");
        if (mask & EXA_EV_JAC) need(io->jac, tot[kOffJac], "jac");
        if (mask & EXA_EV_HESS) need(io->hess, tot[kOffHess], "hess");
        if (mask & EXA_EV_JPROD) need(io->jv, tot[kOffY], "jv");
        if (mask & EXA_EV_JTPROD) need(io->jtw, tot[kOffX], "jtw");
        if (mask & EXA_EV_HPROD) need(io->hv, tot[kOffX], "hv");
        if (mask & EXA_EV_LAG) need(io->lag, tot[kOffX], "lag");
        if (mask & EXA_EV_ADJ) need(io->theta_bar, tot[kOffTheta], "theta_bar");
        if ((mask & (EXA_EV_GRAD | EXA_EV_LAG)) && b->grad_direct_all != b->grad_direct_any)
            fail(EXA_EINVAL,
                 "the instances disagree on whether every variable has at most one objective term; their "
                 "gradients cannot be evaluated in one batch");
        hipStream_t s = (hipStream_t)stream;
        // work buffers this mask needs
        if (((mask & EXA_EV_GRAD) && !b->grad_direct_all) || (mask & (EXA_EV_LAG | EXA_EV_JTPROD)))
            need_buf(*b, kBufFo);
        if (mask & EXA_EV_HPROD) need_buf(*b, kBufHv);
        if (mask & EXA_EV_ADJ) need_buf(*b, kBufPar);
        if (mask & EXA_EV_OBJ) need_buf(*b, kBufTile);
        if ((mask & EXA_EV_LAG) && !b->grad_direct_all && !b->lag_tmp)
            b->lag_tmp = (double*)b->mem.alloc(std::max<int64_t>(1, tot[kOffX]) * sizeof(double));
        auto it = b->sched.find(mask);
        if (it == b->sched.end() || !it->second.tuned) {
            // the options' units
            set_batch_schedule(*b, mask, b->block, b->epl, b->fuse, b->units & ~EXA_UNSTAGED);
            b->sched[mask].unstaged = (b->units & EXA_UNSTAGED) != 0;
            b->sched[mask].reduce_built = false;
            if (b->autotune) tune_batch(*b, mask, *io, s);
            b->sched[mask].tuned = true;
            b->drop_graph();
        }
        exa_batch::Sched& S = b->sched[mask];
        if (!S.reduce_built) build_reductions(*b, S, mask);
        exa_batch::Key k;
        std::memset(&k, 0, sizeof k);
        k.mask = mask;
        k.io = *io;
        k.block = S.block;
        k.epl = S.epl;
        k.units = S.units;
        k.fused = S.fused;
        // a graph is recorded when a call repeats the previous one (same
        // pointers, sigma and schedule) and replayed while calls keep
        // matching it; a call with new arguments launches directly, so
        // arguments that change at every call (fresh output tensors) cost
        // no recording
        const bool replay = b->have_graph && k == b->key;
        const bool record = !replay && b->have_last && k == b->last;
        b->last = k;
        b->have_last = true;
        if (!b->use_graph || b->timing.on || (!replay && !record)) {
            run(*b, mask, *io, s);
        } else {
            if (record) {
                b->drop_graph();
                hip_check(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
                try {
                    run(*b, mask, *io, b->cap);
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
        }
        const uint32_t bits[10] = {EXA_EV_OBJ, EXA_EV_GRAD, EXA_EV_CONS, EXA_EV_JAC, EXA_EV_HESS,
                                   EXA_EV_JPROD, EXA_EV_JTPROD, EXA_EV_HPROD, EXA_EV_LAG, EXA_EV_ADJ};
        for (exa_model* m : b->models)
            for (int i = 0; i < 10; ++i)
                if (mask & bits[i]) {
                    if (i < 8) m->impl.counters[i]++;
                    else if (i == 8) m->impl.counters[1]++, m->impl.counters[6]++;
                    else m->impl.counters[8]++;
                }
    });
}

exa_status exa_batch_timing(exa_batch* b, int32_t enable) {
    return guard([&] {
        if (!b) fail(EXA_EINVAL, "null batch");
        b->timing_off();
        if (!enable) return;
        const int64_t calls = 1024;
        b->timing.ev.reserve(4 * calls);
        for (int64_t i = 0; i < 4 * calls; ++i) {
            hipEvent_t e;
            // timing only: no system-scope fence (cache writeback) per record
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
                b->timing_off();
                fail(EXA_EHIP, "hipEventCreate failed");
            }
            b->timing.ev.push_back(e);
        }
        b->timing.reduced.assign(calls, 0);
        b->timing.on = true;
    });
}

exa_status exa_batch_timing_read(exa_batch* b, double* out4) {
    return guard([&] {
        if (!b || !out4) fail(EXA_EINVAL, "null argument");
        exa_batch::Timing& T = b->timing;
        if (!T.on) fail(EXA_ESTATE, "batch timing is off");
        double se = 0.0, sr = 0.0;
        int64_t nr = 0;
        for (int64_t i = 0; i < T.used; ++i) {
            hipEvent_t* ev = &T.ev[4 * i];
            hip_check(hipEventSynchronize(ev[3]), "hipEventSynchronize");
            float ms = 0.0f;
            hip_check(hipEventElapsedTime(&ms, ev[0], ev[1]), "hipEventElapsedTime");
            se += ms;
            if (T.reduced[i]) {
                hip_check(hipEventElapsedTime(&ms, ev[2], ev[3]), "hipEventElapsedTime");
                sr += ms;
                ++nr;
            }
        }
        out4[0] = (double)T.used;
        out4[1] = T.used ? 1e3 * se / (double)T.used : 0.0;
        out4[2] = (double)nr;
        out4[3] = nr ? 1e3 * sr / (double)nr : 0.0;
        T.used = 0;
    });
}

}  // extern "C"
