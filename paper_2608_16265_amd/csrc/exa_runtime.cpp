// Device side of a model: run-time compilation of the generated kernels,
// device copies of the data, tile lists, work buffers, and the C ABI.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <unistd.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <chrono>
#include <functional>
#include <map>
#include <mutex>

#include "exa_internal.h"
#include "exa_kernels.h"
#include "exa_runtime.h"

namespace exa {

namespace {
thread_local std::string g_last_error;
}

void fail(exa_status code, const std::string& msg) { throw Error(code, msg); }
void set_last_error(const std::string& msg) { g_last_error = msg; }
const char* last_error() { return g_last_error.c_str(); }

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(EXA_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Compiled modules, shared by every model whose generated source is identical.
Module::~Module() {
    if (mod) (void)hipModuleUnload(mod);
}

namespace {
std::mutex g_mod_mu;
std::map<std::string, std::weak_ptr<Module>> g_mods;

std::string hex_hash(const std::string& s) {
    uint64_t h = 1469598103934665603ull;  // FNV-1a
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    char buf[32];
    snprintf(buf, sizeof buf, "%016llx", (unsigned long long)h);
    return buf;
}
}  // namespace

// The options every generated source is compiled with.  -ffp-contract=off:
// every multiply and add is rounded on its own, so a data point's result does
// not depend on how its code was scheduled or fused with other patterns
// (bitwise-equal batched and plain results).
const char* const kCompileOpts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
                                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};

bool log_on() {
    static const bool on = [] {
        const char* e = std::getenv("EXA_LOG");
        return e && *e && std::strcmp(e, "0") != 0;
    }();
    return on;
}

void log_msg(const std::string& msg) {
    if (log_on()) std::fprintf(stderr, "[exa] %s\n", msg.c_str());
}

std::vector<char> compile_code(const std::string& src_in) {
    // test hook: a source that cannot compile, to exercise EXA_ECOMPILE
    const char* bad = std::getenv("EXA_TEST_BAD_SOURCE");
    const std::string src =
        (bad && *bad && std::strcmp(bad, "0") != 0) ? src_in + "\nthis line does not compile;\n" : src_in;
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "exa_generated.hip", 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS)
        fail(EXA_ECOMPILE, "hiprtcCreateProgram failed");
    hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof kCompileOpts / sizeof kCompileOpts[0]), kCompileOpts);
    size_t logsz = 0;
    hiprtcGetProgramLogSize(prog, &logsz);
    std::string log(logsz, '\0');
    if (logsz) hiprtcGetProgramLog(prog, &log[0]);
    if (rc != HIPRTC_SUCCESS) {
        hiprtcDestroyProgram(&prog);
        fail(EXA_ECOMPILE, "run-time compilation failed: " + log.substr(0, 4000));
    }
    size_t csz = 0;
    hiprtcGetCodeSize(prog, &csz);
    std::vector<char> code(csz);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    return code;
}

namespace {
// ---- on-disk code-object cache --------------------------------------------
// A compiled module is stored as <dir>/exa-<key>.hsaco next to its source
// <dir>/exa-<key>.hip, where key hashes the generated source, the compile
// options and the hiprtc version.  A hit needs the stored source to equal
// the generated one byte for byte, so a hash collision cannot load the wrong
// code.  Files are written under a temporary name and renamed into place, so
// concurrent processes see whole files or none.  Cache errors are not fatal:
// the source is compiled as without a cache.
std::string cache_key(const std::string& src) {
    int maj = 0, min = 0;
    hiprtcVersion(&maj, &min);
    std::string k = src + "|hiprtc " + std::to_string(maj) + "." + std::to_string(min) + "|";
    for (const char* o : kCompileOpts) k += std::string(o) + " ";
    return hex_hash(k) + "-" + std::to_string(src.size());
}

bool read_file(const std::string& path, std::string& out) {
    FILE* f = std::fopen(path.c_str(), "rb");
    if (!f) return false;
    std::string s;
    char buf[1 << 16];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, n);
    const bool ok = !std::ferror(f);
    std::fclose(f);
    if (ok) out.swap(s);
    return ok;
}

bool write_file_atomic(const std::string& path, const char* data, size_t n) {
    const std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    const bool ok = std::fwrite(data, 1, n, f) == n;
    if (std::fclose(f) != 0 || !ok || std::rename(tmp.c_str(), path.c_str()) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}
}  // namespace

std::vector<char> cached_code(const std::string& src, const std::string& dir, bool* hit) {
    if (hit) *hit = false;
    if (dir.empty()) return compile_code(src);
    const std::string base = dir + "/exa-" + cache_key(src);
    std::string stored, code;
    if (read_file(base + ".hip", stored) && stored == src && read_file(base + ".hsaco", code) && !code.empty()) {
        if (hit) *hit = true;
        log_msg("code-object cache hit: " + base + ".hsaco");
        return std::vector<char>(code.begin(), code.end());
    }
    std::vector<char> out = compile_code(src);
    // the code object first, then the source that validates it
    if (write_file_atomic(base + ".hsaco", out.data(), out.size()) &&
        write_file_atomic(base + ".hip", src.data(), src.size()))
        log_msg("code-object cache write: " + base + ".hsaco");
    else
        log_msg("code-object cache: cannot write under " + dir + " (compiled without caching)");
    return out;
}

std::string cache_dir_of(const char* opt_dir) {
    if (opt_dir && *opt_dir) return opt_dir;
    const char* e = std::getenv("EXA_CACHE_DIR");
    return (e && *e) ? e : "";
}

std::shared_ptr<Module> compile_module(const std::string& src, const std::string& cache_dir, bool* cache_hit) {
    if (cache_hit) *cache_hit = false;
    const std::string key = hex_hash(src) + ":" + std::to_string(src.size());
    std::lock_guard<std::mutex> lk(g_mod_mu);
    auto it = g_mods.find(key);
    if (it != g_mods.end())
        if (auto m = it->second.lock())
            if (m->source == src) return m;
    auto m = std::make_shared<Module>();
    m->source = src;
    m->code = cached_code(src, cache_dir, cache_hit);
    hip_check(hipModuleLoadData(&m->mod, m->code.data()), "hipModuleLoadData");
    for (int mode = 0; mode < M_COUNT; ++mode) {
        hipFunction_t f = nullptr;
        if (hipModuleGetFunction(&f, m->mod, kernel_name(mode).c_str()) != hipSuccess)
            fail(EXA_ECOMPILE, "generated kernel missing: " + kernel_name(mode));
        m->fn[mode] = f;
    }
    if (hipModuleGetFunction(&m->fn_multi, m->mod, "exa_k_multi") != hipSuccess)
        fail(EXA_ECOMPILE, "generated kernel missing: exa_k_multi");
    if (hipModuleGetFunction(&m->fn_multijh, m->mod, "exa_k_multijh") != hipSuccess)
        fail(EXA_ECOMPILE, "generated kernel missing: exa_k_multijh");
    if (hipModuleGetFunction(&m->fn_onepass, m->mod, "exa_k_onepass") != hipSuccess)
        fail(EXA_ECOMPILE, "generated kernel missing: exa_k_onepass");
    g_mods[key] = m;
    return m;
}

// ---------------------------------------------------------------------------
DeviceState::~DeviceState() {
    timing_off();
    for (void* p : allocs) (void)hipFree(p);
    if (fhost) (void)hipHostFree(fhost);
}

void DeviceState::timing_off() {
    for (hipEvent_t e : timing.ev) (void)hipEventDestroy(e);
    timing = EvalTiming();
}

void* DeviceState::alloc(size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (budget > 0 && allocated + (int64_t)bytes > budget)
        fail(EXA_ENOMEM, "device memory budget of " + std::to_string(budget) + " bytes exceeded (" +
                             std::to_string(allocated) + " allocated, " + std::to_string(bytes) + " more asked)");
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) fail(EXA_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    allocs.push_back(p);
    sizes.push_back((int64_t)bytes);
    allocated += (int64_t)bytes;
    return p;
}

void* DeviceState::upload(const void* src, size_t bytes) {
    void* p = alloc(bytes);
    if (bytes) hip_check(hipMemcpy(p, src, bytes, hipMemcpyHostToDevice), "hipMemcpy");
    return p;
}

void DeviceState::release(void* p) {
    if (!p) return;
    auto it = std::find(allocs.begin(), allocs.end(), p);
    if (it != allocs.end()) {
        (void)hipFree(p);
        const size_t i = (size_t)(it - allocs.begin());
        allocated -= sizes[i];
        sizes.erase(sizes.begin() + i);
        allocs.erase(it);
    }
}

// Tiles of `tile_pts` consecutive data points over the units of a callback.
std::vector<ExaTile> make_tiles(const Model& M, int mode, int inst, int64_t tile_pts, bool fused, bool fills) {
    std::vector<ExaTile> tiles;
    for (const Unit& u : units_for(M, mode, fused)) {
        // a unit whose code reads nothing (constant derivatives only, such as
        // the Jacobian entries of a linear augmentation) is a plain fill: far
        // more points per tile, like the gradient's zero tiles (the
        // objective keeps its fixed tiles, which fix its summation order).
        // A launch bound by latency rather than bandwidth keeps short tiles.
        int64_t tp = tile_pts;
        const auto lv = M.live.find({mode, u.code});
        const bool many = u.ndata > (int64_t)4096 * tile_pts;
        if (mode != M_OBJ && (fills || many) && lv != M.live.end()) {
            const UnitLive& L = lv->second;
            if (L.icols.empty() && L.fcols.empty() && L.vrefs.empty() && L.vseeds.empty() && L.prefs.empty() &&
                L.weights == 0 && !L.pulls)
                tp = std::max<int64_t>(tp, kZeroTileEntries);
        }
        for (int64_t s = 0; s < u.ndata; s += tp) {
            ExaTile t{};
            t.pat = u.code;
            t.inst = inst;
            t.start = s;
            t.count = std::min(tp, u.ndata - s);
            t.slot = (int64_t)tiles.size();
            tiles.push_back(t);
        }
    }
    return tiles;
}

void fill_patdev(const Model& M, DeviceState& D, ExaInstDev& inst) {
    std::memset(&inst, 0, sizeof inst);
    for (size_t p = 0; p < M.pats.size(); ++p) {
        const Pattern& P = M.pats[p];
        ExaPatDev& d = inst.pat[p];
        const int first = M.groups[P.group].members[0];
        if (first != (int)p) {
            // same data arrays as the group's first pattern: share the copies
            for (int c = 0; c < P.n_icols; ++c) d.ic[c] = inst.pat[first].ic[c];
            for (int c = 0; c < P.n_fcols; ++c) d.fc[c] = inst.pat[first].fc[c];
        } else {
            for (int c = 0; c < P.n_icols; ++c)
                d.ic[c] = (const int*)D.upload(P.icols[c].data(), P.ndata * sizeof(int32_t));
            for (int c = 0; c < P.n_fcols; ++c)
                d.fc[c] = (const double*)D.upload(P.fcols_src[c], P.ndata * sizeof(double));
        }
        d.ndata = P.ndata;
        d.o0 = P.o0;
        d.o1 = P.o1;
        d.o2 = P.o2;
        d.op = P.op;
        d.oh = P.oh;
        d.ob = P.ob;
        d.tgt0 = P.tgt0;
        d.row_off = P.row_off;
        d.row_ic = P.row_icol;
        const Group& G = M.groups[P.group];
        for (size_t j = 0; j < G.hv_direct.size(); ++j)
            if (G.hv_direct[j]) d.hvd |= 1 << j;
        if (P.kind == EXA_AUG) {
            d.rptr = (const int*)D.upload(P.rptr.data(), P.rptr.size() * sizeof(int32_t));
            d.ridx = (const int*)D.upload(P.ridx.data(), P.ridx.size() * sizeof(int32_t));
        }
        for (int r = 0; r < P.o1step(); ++r) d.roff[r] = P.vslots[r].off;
        for (int r = 0; r < P.pstep(); ++r) d.roff[P.o1step() + r] = P.pslots[r].off;
    }
}

int64_t estimate_device_bytes(const Model& M) {
    int64_t b = 0;
    for (const Group& G : M.groups) {
        const Pattern& P = M.pats[G.members[0]];
        b += P.ndata * (4 * (int64_t)P.n_icols + 8 * (int64_t)P.n_fcols);
    }
    for (const Pattern& P : M.pats)
        if (P.kind == EXA_AUG) b += 4 * (int64_t)(P.rptr.size() + P.ridx.size());
    b += 8 * M.ntheta + (int64_t)sizeof(ExaInstDev);
    for (int mode = 0; mode < M_COUNT; ++mode) {
        const bool fixed = mode == M_OBJ;
        const int64_t tp = fixed ? (int64_t)kObjBlock * kObjEpl : (int64_t)M.block * M.epl;
        b += (int64_t)sizeof(ExaTile) * (int64_t)make_tiles(M, mode, 0, tp, fixed ? kObjFused : M.fuse).size();
    }
    const int64_t nobj = (int64_t)make_tiles(M, M_OBJ, 0, (int64_t)kObjBlock * kObjEpl, kObjFused).size();
    b += 8 * (M.fo_obj_len + M.fo_con_len + M.par_len + M.hv_len + std::max<int64_t>(1, nobj) + M.nvar + 1);
    // maps: pointers and positions, plus at most a 24-byte record per four
    // entries (chunked sums, with padding) and part sums
    for (const SegMap* S : {&M.grad_map, &M.jt_map, &M.h_map, &M.par_map}) {
        const int64_t nnz = (int64_t)S->idx.size();
        b += 8 * (S->nseg() + 1) + 8 * nnz + 8 * nnz + 24 * 256 + 8 * (nnz / kExaLongSeg + 1);
    }
    return b;
}

void build_device(Model& M) {
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    M.dev.reset(new DeviceState());
    DeviceState& D = *M.dev;
    D.device = dev;
    D.budget = M.max_device_bytes;
    auto t0 = std::chrono::steady_clock::now();
    const std::string src = generate_source(M, &M.live);
    auto t1 = std::chrono::steady_clock::now();
    {
        std::lock_guard<std::mutex> lk(g_mod_mu);
        M.module_shared = false;
        auto it = g_mods.find(hex_hash(src) + ":" + std::to_string(src.size()));
        if (it != g_mods.end())
            if (auto m = it->second.lock()) M.module_shared = m->source == src;
    }
    D.module = compile_module(src, M.cache_dir, &M.cache_hit);
    auto t2 = std::chrono::steady_clock::now();
    M.codegen_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    M.compile_ms = std::chrono::duration<double, std::milli>(t2 - t1).count();

    D.theta = (double*)D.upload(M.theta.data(), M.theta.size() * sizeof(double));
    ExaInstDev inst;
    fill_patdev(M, D, inst);
    inst.theta = D.theta;
    inst.off[EXA_OFF_FO_CON] = M.fo_obj_len;
    D.inst_host = inst;
    D.inst = (ExaInstDev*)D.upload(&inst, sizeof inst);

    for (int mode = 0; mode < M_COUNT; ++mode) {
        // the objective keeps one fixed schedule, so that its reduction order
        // (and hence its value) never depends on tuning
        const bool fixed = mode == M_OBJ;
        set_schedule(M, mode, fixed ? kObjBlock : M.block, fixed ? kObjEpl : M.epl, fixed ? kObjFused : M.fuse);
        D.sched[mode].tuned = fixed || !M.autotune;
    }
    D.fo = (double*)D.alloc((M.fo_obj_len + M.fo_con_len) * sizeof(double));
    D.par = (double*)D.alloc(M.par_len * sizeof(double));
    D.hv = (double*)D.alloc(M.hv_len * sizeof(double));
    D.tilesum = (double*)D.alloc(std::max<int64_t>(1, D.sched[M_OBJ].ntiles) * sizeof(double));
    D.lag_tmp = (double*)D.alloc(M.nvar * sizeof(double));
    D.fval = (double*)D.alloc(sizeof(double));
    if (hipHostMalloc((void**)&D.fhost, sizeof(double), hipHostMallocDefault) != hipSuccess)
        fail(EXA_ENOMEM, "hipHostMalloc of the objective's host copy failed");

    upload_map(D, M.grad_map, D.grad_map);
    upload_map(D, M.jt_map, D.jt_map);
    upload_map(D, M.h_map, D.h_map);
    upload_map(D, M.par_map, D.par_map);
    // the caller's float columns are not kept past create
    for (auto& P : M.pats) P.fcols_src.assign(P.fcols_src.size(), nullptr);
}

// Tiles that write zeros to the gradient entries no objective term touches
// (in-place gradient only).
void add_zero_tiles(const Model& M, int64_t tp, std::vector<ExaTile>& tiles) {
    if (!M.grad_direct) return;
    // a zero tile is a plain fill: far more entries than a tile of points
    // (16-byte stores, 16 entries per lane of a 256-wide workgroup), so the
    // fill takes a few workgroups instead of one per tile of points
    const int64_t tz = std::max<int64_t>(tp, kZeroTileEntries);
    for (auto& z : M.grad_zero)
        for (int64_t s = 0; s < z.second; s += tz) {
            ExaTile t{};
            t.pat = EXA_ZERO_TILE;
            t.start = z.first + s;
            t.count = std::min(tz, z.second - s);
            t.slot = (int64_t)tiles.size();
            tiles.push_back(t);
        }
}

// maps go to the device as int32 whenever every position fits
// Segments the reduction visits: skipped segments at the end of a map need
// no lane (those of the ACOPF H v map are most of its variables).
int64_t visited_segments(const SegMap& S) {
    int64_t n = S.nseg();
    while (n > 0 && !S.skip.empty() && S.skip[n - 1]) --n;
    return n;
}

void upload_map(DeviceState& D, const SegMap& S, DevMap& d) {
    d.nseg = visited_segments(S);
    int64_t top = S.idx.empty() ? 0 : *std::max_element(S.idx.begin(), S.idx.end());
    const int64_t low = S.idx.empty() ? 0 : *std::min_element(S.idx.begin(), S.idx.end());
    top = std::max<int64_t>(top, S.ptr.empty() ? 0 : S.ptr.back());
    d.wide = top >= INT32_MAX || low < INT32_MIN ? 1 : 0;
    // a segment the reduction skips has its end stored complemented (a
    // negative value; see seg_body)
    std::vector<int64_t> ptr = S.ptr;
    for (size_t s = 0; s < S.skip.size(); ++s)
        if (S.skip[s]) ptr[s + 1] = ~ptr[s + 1];
    if (d.wide) {
        d.ptr = D.upload(ptr.data(), ptr.size() * sizeof(int64_t));
        d.idx = D.upload(S.idx.data(), S.idx.size() * sizeof(int64_t));
        return;
    }
    std::vector<int32_t> p32(ptr.begin(), ptr.end()), i32(S.idx.begin(), S.idx.end());
    d.ptr = D.upload(p32.data(), p32.size() * sizeof(int32_t));
    d.idx = D.upload(i32.data(), i32.size() * sizeof(int32_t));
    const ChunkPlan P = chunk_plan(S);
    d.chunked = P.chunked ? 1 : 0;
    if (P.nlanes()) {
        d.lanes = (const int32_t*)D.upload(P.meta.data(), P.meta.size() * sizeof(int32_t));
        d.lidx = (const int32_t*)D.upload(P.lidx.data(), P.lidx.size() * sizeof(int32_t));
        d.nlanes = P.nlanes();
    }
    if (P.nparts()) {
        d.longs = (const int32_t*)D.upload(P.longs.data(), P.longs.size() * sizeof(int32_t));
        d.lpart = (const int32_t*)D.upload(P.lpart.data(), P.lpart.size() * sizeof(int32_t));  // 2 per part
        d.nparts = P.nparts();
        d.nlong = P.nlong();
        d.lsum = (double*)D.alloc(P.nparts() * sizeof(double));
    }
}

// Compressed sparse columns of a COO structure (Sec. 5.2: the compression
// across patterns and data points that the partially compressed layout
// leaves to the solver).  Positions are bucketed by column in ascending
// order, then ordered by row within each column (stable, so equal pairs keep
// ascending position); each distinct (row, col) pair is one entry.
Model::Csc& csc_form(Model& M, int which) {
    Model::Csc& C = M.csc[which];
    if (C.ready) return C;
    const int64_t nnz = which == 0 ? M.nnzj : M.nnzh;
    if (nnz >= INT32_MAX) fail(EXA_EINVAL, "compressed columns need fewer than 2^31 entries");
    std::vector<int32_t> r(nnz), c(nnz);
    if (which == 0)
        jac_structure_host(M, r.data(), c.data());
    else
        hess_structure_host(M, r.data(), c.data());
    const int64_t ncol = M.nvar;
    std::vector<int64_t> start(ncol + 1, 0);
    for (int64_t k = 0; k < nnz; ++k) start[c[k] + 1]++;
    for (int64_t j = 0; j < ncol; ++j) start[j + 1] += start[j];
    std::vector<int32_t> pos(nnz);
    {
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (int64_t k = 0; k < nnz; ++k) pos[fill[c[k]]++] = (int32_t)k;
    }
    C.colptr.assign(ncol + 1, 0);
    C.rowval.clear();
    C.map.ptr.assign(1, 0);
    C.map.idx.clear();
    C.map.idx.reserve(nnz);
    for (int64_t j = 0; j < ncol; ++j) {
        auto b = pos.begin() + start[j], e = pos.begin() + start[j + 1];
        std::stable_sort(b, e, [&](int32_t u, int32_t v) { return r[u] < r[v]; });
        for (auto it = b; it != e; ++it) {
            if (it == b || r[*it] != r[*(it - 1)]) {
                if (it != b) C.map.ptr.push_back((int64_t)C.map.idx.size());
                C.rowval.push_back(r[*it]);
            }
            C.map.idx.push_back(*it);
        }
        if (b != e) C.map.ptr.push_back((int64_t)C.map.idx.size());
        C.colptr[j + 1] = (int32_t)C.rowval.size();
    }
    C.ready = true;
    return C;
}

ChunkPlan chunk_plan(const SegMap& S) {
    ChunkPlan P;
    int64_t longest = 0, top = S.ptr.empty() ? 0 : S.ptr.back(), low = 0;
    for (int64_t s = 0; s < S.nseg(); ++s) longest = std::max(longest, S.ptr[s + 1] - S.ptr[s]);
    for (int64_t i : S.idx) top = std::max(top, i), low = std::min(low, i);
    if (longest <= 2 * kExaChunk || top >= INT32_MAX || low < INT32_MIN) return P;
    int64_t longest_short = 0, long_nnz = 0;
    for (int64_t s = 0; s < S.nseg(); ++s) {
        const int64_t len = S.ptr[s + 1] - S.ptr[s];
        if (len > kExaLongSeg)
            long_nnz += len;
        else
            longest_short = std::max(longest_short, len);
    }
    // large maps (bandwidth-bound) whose only long segments are parts
    P.chunked = !(longest_short <= kExaShortSeg && (int64_t)S.idx.size() - long_nnz >= (int64_t)1 << 22);
    // padding lanes: no segment, no entries, indices 0 (a valid position:
    // a chunked map has entries)
    auto pad_to = [&](int64_t lanes) {
        while (P.nlanes() < lanes) {
            P.meta.insert(P.meta.end(), {-1, 0});
            P.lidx.insert(P.lidx.end(), {0, 0, 0, 0});
        }
    };
    int64_t nparts = 0, most = 0;
    for (int64_t s = 0; s < S.nseg(); ++s) {
        const int64_t b = S.ptr[s], len = S.ptr[s + 1] - b;
        if (len > kExaLongSeg) {
            const int64_t parts = (len + kExaLongSeg - 1) / kExaLongSeg;
            P.longs.insert(P.longs.end(), {(int32_t)s, (int32_t)b, (int32_t)len, (int32_t)nparts, (int32_t)parts});
            nparts += parts;
            most = std::max(most, parts);
            continue;
        }
        if (!P.chunked || (!S.skip.empty() && S.skip[s])) continue;
        const int64_t nl = std::max<int64_t>(1, (len + kExaChunk - 1) / kExaChunk);
        const int64_t here = P.nlanes();
        if (here % 256 + nl > 256) pad_to((here / 256 + 1) * 256);
        for (int64_t c = 0; c < nl; ++c) {
            const int64_t cnt = std::max<int64_t>(0, std::min<int64_t>(kExaChunk, len - c * kExaChunk));
            P.meta.push_back((int32_t)s);
            P.meta.push_back((int32_t)(cnt | (c == 0 ? nl << 4 : 0)));
            // the chunk's positions, the last one repeated past its count
            for (int64_t u = 0; u < kExaChunk; ++u)
                P.lidx.push_back(cnt ? (int32_t)S.idx[b + c * kExaChunk + std::min(u, cnt - 1)] : 0);
        }
    }
    if (P.chunked) pad_to((P.nlanes() + 255) / 256 * 256);
    // part blocks: the i-th part of every long segment, then the (i+1)-th;
    // segments that share a variable over interleaved points (x_{k mod n})
    // then read the same range of the buffer in neighbouring blocks, on one
    // XCD, instead of each XCD reading every line of it
    for (int64_t i = 0; i < most; ++i)
        for (int64_t ls = 0; ls < P.nlong(); ++ls)
            if (i < P.longs[5 * ls + 4]) P.lpart.insert(P.lpart.end(), {(int32_t)ls, (int32_t)(P.longs[5 * ls + 3] + i)});
    return P;
}

// Launch order of tile lists (each list one unit's tiles over its points in
// order; a launch's workgroups go to the 8 XCDs in contiguous eighths): XCD
// j takes the j-th eighth of every unit's points, in rounds that each take
// the same fraction of every unit.  Units over related data (a grid's points
// and its interior points, the patterns of a model and its J^T w tiles) then
// read the same x lines from one L2 at about the same time, instead of each
// XCD fetching them for the units it happens to hold.  A round holds at
// least 32 tiles (one per CU of the XCD) of the largest unit, at most 16
// rounds per XCD: with fewer tiles per round, consecutive rounds would put
// a unit's tiles on the same few CUs, and a launch whose tiles all fit on
// the chip at once would wait on those CUs.  Results do not depend on the
// order (every output has one writer; objective tiles keep their slots).
std::vector<ExaTile> interleave_units(const std::vector<std::vector<ExaTile>>& units) {
    size_t most = 0;
    for (const auto& u : units) most = std::max(most, u.size());
    const int kRounds = 8 * (int)std::min<size_t>(16, std::max<size_t>(1, most / (8 * 32)));
    std::vector<ExaTile> all;
    for (int r = 0; r < kRounds; ++r)
        for (const auto& u : units)
            all.insert(all.end(), u.begin() + u.size() * r / kRounds, u.begin() + u.size() * (r + 1) / kRounds);
    return all;
}

// A tile list split at changes of unit (make_tiles lists each unit's tiles
// together).
void split_units(const std::vector<ExaTile>& t, std::vector<std::vector<ExaTile>>& out) {
    for (size_t i = 0; i < t.size(); ++i) {
        if (i == 0 || t[i].pat != t[i - 1].pat) out.emplace_back();
        out.back().push_back(t[i]);
    }
}

void set_schedule(Model& M, int mode, int block, int epl, bool fused) {
    DeviceState& D = *M.dev;
    DeviceState::Sched& S = D.sched[mode];
    const int64_t tp = (int64_t)block * epl;
    auto made = make_tiles(M, mode, 0, tp, fused);
    if (mode == M_GRAD) add_zero_tiles(M, tp, made);
    std::vector<std::vector<ExaTile>> units;
    split_units(made, units);
    const std::vector<ExaTile> tiles = interleave_units(units);
    D.release(S.tiles);
    S.tiles = (ExaTile*)D.upload(tiles.data(), tiles.size() * sizeof(ExaTile));
    S.ntiles = (int64_t)tiles.size();
    S.block = block;
    S.epl = epl;
    S.fused = fused;
}

namespace {
void raw_launch(Model& M, int mode, ExaCall call, hipStream_t s) {
    DeviceState& D = *M.dev;
    const DeviceState::Sched& S = D.sched[mode];
    if (S.ntiles == 0) return;
    call.tiles = S.tiles;
    call.ntiles = S.ntiles;
    call.per_xcd = (S.ntiles + 7) / 8;
    call.inst = D.inst;
    call.unstaged = S.unstaged ? 1 : 0;
    const int64_t grid = 8 * call.per_xcd;
    void* args[] = {&call};
    hip_check(hipModuleLaunchKernel(D.module->fn[mode], (unsigned)grid, 1, 1, (unsigned)S.block, 1, 1, 0, s,
                                    args, nullptr),
              "hipModuleLaunchKernel");
}

}  // namespace

bool has_fusable_group(const Model& M, int mode) {
    for (const Unit& u : units_for(M, mode, true))
        if (u.members.size() > 1) return true;
    return false;
}

namespace {

// First call of a callback with autotuning on: time every candidate
// schedule on the caller's own arguments and keep the fastest.  Every
// candidate evaluates each data point with the same code, so outputs are the
// same whichever wins.
void tune(Model& M, int mode, const ExaCall& call, hipStream_t s) {
    const int blocks[] = {64, 128, 256};
    const int epls[] = {1, 2, 4, 8};
    std::vector<int> fuses = {0};
    if (has_fusable_group(M, mode)) fuses.push_back(1);
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    // staged or each lane's own stores: only modes with multi-entry final outputs
    const bool stores = mode == M_JAC || mode == M_HESS || mode == M_JH;
    std::vector<int> unst = {0};
    if (stores) unst.push_back(1);
    struct Cand {
        float ms;
        int block, epl, fused, unstaged;
    };
    auto time_it = [&](int reps) {
        raw_launch(M, mode, call, s);
        hip_check(hipEventRecord(e0, s), "hipEventRecord");
        for (int r = 0; r < reps; ++r) raw_launch(M, mode, call, s);
        hip_check(hipEventRecord(e1, s), "hipEventRecord");
        hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        return ms / reps;
    };
    std::vector<Cand> cands;
    try {
        for (int u : unst)
        for (int f : fuses)
            for (int b : blocks)
                for (int ep : epls) {
                    set_schedule(M, mode, b, ep, f != 0);
                    M.dev->sched[mode].unstaged = u != 0;
                    cands.push_back({time_it(3), b, ep, f, u});
                }
        // as in tune_multi: the fastest few again, longer, in turns
        std::sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
        cands.resize(std::min<size_t>(cands.size(), 4));
        for (auto& c : cands) c.ms = 1e30f;
        for (int round = 0; round < 3; ++round)
            for (auto& c : cands) {
                set_schedule(M, mode, c.block, c.epl, c.fused != 0);
                M.dev->sched[mode].unstaged = c.unstaged != 0;
                c.ms = std::min(c.ms, time_it(12));
            }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const Cand& w = *std::min_element(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
    set_schedule(M, mode, w.block, w.epl, w.fused != 0);
    M.dev->sched[mode].unstaged = w.unstaged != 0;
    M.dev->sched[mode].tuned = true;
    if (log_on())
        log_msg("tuned " + kernel_name(mode) + ": block " + std::to_string(w.block) + ", points per lane " +
                std::to_string(w.epl) + ", fused " + std::to_string(w.fused) + ", unstaged " +
                std::to_string(w.unstaged) + " (" + std::to_string(w.ms * 1e3) + " us)");
}
}  // namespace

void launch_mode(Model& M, int mode, ExaCall call, hipStream_t s) {
    if (!M.dev->sched[mode].tuned) tune(M, mode, call, s);
    raw_launch(M, mode, call, s);
}

void launch_mode_untuned(Model& M, int mode, ExaCall call, hipStream_t s) { raw_launch(M, mode, call, s); }

// ---- several callbacks in one launch (exa_eval) ----------------------------

// Modes of an exa_eval mask; with jh, Jacobian and Hessian together run as
// JH units (both jobs of a point from one set of loads).
std::vector<int> eval_modes(uint32_t mask, bool jh) {
    std::vector<int> m;
    if (mask & EXA_EV_OBJ) m.push_back(M_OBJ);
    if (mask & EXA_EV_GRAD) m.push_back(M_GRAD);
    if (mask & EXA_EV_CONS) m.push_back(M_CONS);
    if (jh && (mask & EXA_EV_JAC) && (mask & EXA_EV_HESS))
        m.push_back(M_JH);
    else if ((mask & EXA_EV_JAC) && (mask & EXA_EV_HESS)) {
        m.push_back(M_JAC);
        m.push_back(M_HESS);
    }
    else if (mask & EXA_EV_JAC)
        m.push_back(M_JAC);
    else if (mask & EXA_EV_HESS)
        m.push_back(M_HESS);
    if (mask & EXA_EV_JPROD) m.push_back(M_JPROD);
    if (mask & EXA_EV_JTPROD) m.push_back(M_JTPROD);
    if (mask & EXA_EV_HPROD) m.push_back(M_HPROD);
    return m;
}

// Multi-unit mode that covers a mask's callbacks besides the objective in
// one pass per point, or -1.
int combined_mode_of(uint32_t mask) {
    const uint32_t full = EXA_EV_GRAD | EXA_EV_CONS | EXA_EV_JAC | EXA_EV_HESS | EXA_EV_JPROD | EXA_EV_HPROD;
    const uint32_t ipm = EXA_EV_GRAD | EXA_EV_CONS | EXA_EV_JAC | EXA_EV_HESS;
    // the objective and J^T w run as tiles of their own beside the units
    const uint32_t rest = mask & ~(uint32_t)(EXA_EV_OBJ | EXA_EV_JTPROD);
    if ((rest & full) == full) return M_SFULL;
    if (rest == ipm) return M_SIPM;
    return -1;
}

bool has_jh(uint32_t mask) { return (mask & EXA_EV_JAC) && (mask & EXA_EV_HESS); }

// The units a mask can run as asked: one-pass units need a mask that has
// them, JH units a mask with both the Jacobian and the Hessian.
int valid_units(uint32_t mask, int units) {
    if (units == EXA_UNITS_ONE_PASS && combined_mode_of(mask) < 0) units = EXA_UNITS_JAC_HESS;
    if (units == EXA_UNITS_JAC_HESS && !has_jh(mask)) units = EXA_UNITS_PER_CALLBACK;
    return units;
}

// Modes whose tiles make up a mask's launch.
std::vector<int> launch_modes(uint32_t mask, int units) {
    units = valid_units(mask, units);
    if (units != EXA_UNITS_ONE_PASS) return eval_modes(mask, units == EXA_UNITS_JAC_HESS);
    std::vector<int> m;
    if (mask & EXA_EV_OBJ) m.push_back(M_OBJ);
    m.push_back(combined_mode_of(mask));
    if (mask & EXA_EV_JTPROD) m.push_back(M_JTPROD);
    return m;
}

namespace {

// Tile list of a mask: every launch mode's tiles (the objective's under its
// fixed schedule), laid out as eight chunks that each hold an eighth of
// every mode's tiles, so that the per-XCD ranges of the launch get the same
// mix of work and contiguous point ranges.
void set_multi_schedule(Model& M, uint32_t mask, int block, int epl, bool fused, int units) {
    DeviceState& D = *M.dev;
    DeviceState::MultiSched& S = D.multi[mask];
    units = valid_units(mask, units);
    const int64_t tp = (int64_t)block * epl;
    std::vector<std::vector<ExaTile>> per;
    for (int mode : launch_modes(mask, units)) {
        std::vector<ExaTile> t = mode == M_OBJ ? make_tiles(M, M_OBJ, 0, (int64_t)kObjBlock * kObjEpl, kObjFused)
                                               : make_tiles(M, mode, 0, tp, fused);
        for (ExaTile& x : t) x.pat |= mode << EXA_MODE_SHIFT;
        if (mode == M_GRAD || (multi_unit_mode(mode) && (mask & EXA_EV_GRAD))) {
            std::vector<ExaTile> z;
            add_zero_tiles(M, tp, z);
            for (ExaTile& x : z) x.pat |= M_GRAD << EXA_MODE_SHIFT;
            t.insert(t.end(), z.begin(), z.end());
        }
        split_units(t, per);
    }
    const std::vector<ExaTile> all = interleave_units(per);
    D.release(S.tiles);
    S.tiles = all.empty() ? nullptr : (ExaTile*)D.upload(all.data(), all.size() * sizeof(ExaTile));
    S.ntiles = (int64_t)all.size();
    S.block = block;
    S.epl = epl;
    S.fused = fused;
    S.units = units;
}



void raw_launch_multi(Model& M, uint32_t mask, ExaMulti mc, hipStream_t s) {
    const DeviceState::MultiSched& S = M.dev->multi.at(mask);
    if (S.ntiles == 0) return;
    mc.tiles = S.tiles;
    mc.ntiles = S.ntiles;
    mc.per_xcd = (S.ntiles + 7) / 8;
    for (ExaCall& c : mc.c) c.unstaged = S.unstaged ? 1 : 0;
    void* args[] = {&mc};
    const Module& K = *M.dev->module;
    hipFunction_t fn = S.units == EXA_UNITS_ONE_PASS   ? K.fn_onepass
                       : S.units == EXA_UNITS_JAC_HESS ? K.fn_multijh
                                                       : K.fn_multi;
    hip_check(hipModuleLaunchKernel(fn, (unsigned)(8 * mc.per_xcd), 1, 1, (unsigned)S.block, 1,
                                    1, 0, s, args, nullptr),
              "hipModuleLaunchKernel");
}

// First exa_eval call with a mask: time the candidate schedules of the
// combined launch and keep the fastest (as tune() does for one callback).
// Objective tiles keep their fixed size and summation order under every
// candidate.
void tune_multi(Model& M, uint32_t mask, const ExaMulti& mc, hipStream_t s, const std::function<void()>& step) {
    const int blocks[] = {64, 128, 256};
    const int epls[] = {1, 2, 4, 8};
    std::vector<int> fuses = {0};
    for (int mode : eval_modes(mask, false))
        if (mode != M_OBJ && has_fusable_group(M, mode)) {
            fuses.push_back(1);
            break;
        }
    std::vector<int> combos = {EXA_UNITS_PER_CALLBACK};
    if (has_jh(mask)) combos.push_back(EXA_UNITS_JAC_HESS);
    if (combined_mode_of(mask) >= 0 && !M.eval_per_mode) combos.push_back(EXA_UNITS_ONE_PASS);
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    struct Cand {
        float ms;
        int block, epl, fused, comb;
    };
    // average of `reps` back-to-back launches of the current schedule
    auto time_it = [&](int reps) {
        raw_launch_multi(M, mask, mc, s);
        hip_check(hipEventRecord(e0, s), "hipEventRecord");
        for (int r = 0; r < reps; ++r) raw_launch_multi(M, mask, mc, s);
        hip_check(hipEventRecord(e1, s), "hipEventRecord");
        hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        return ms / reps;
    };
    std::vector<Cand> cands;
    try {
        for (int cb : combos)
        for (int f : fuses)
            for (int b : blocks)
                for (int ep : epls) {
                    set_multi_schedule(M, mask, b, ep, f != 0, cb);
                    cands.push_back({time_it(3), b, ep, f, cb});
                }
        // neighbouring schedules differ by less than one timing's noise: the
        // fastest few are timed again, longer, in turns, and the best of
        // their rounds decides
        std::sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
        cands.resize(std::min<size_t>(cands.size(), 6));
        for (auto& c : cands) c.ms = 1e30f;
        for (int round = 0; round < 3; ++round)
            for (auto& c : cands) {
                set_multi_schedule(M, mask, c.block, c.epl, c.fused != 0, c.comb);
                c.ms = std::min(c.ms, time_it(16));
            }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const Cand& w = *std::min_element(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
    set_multi_schedule(M, mask, w.block, w.epl, w.fused != 0, w.comb);
    // staged or each lane's own stores: the whole step (evaluation and
    // reductions) decides
    if (mask & (EXA_EV_JAC | EXA_EV_HESS)) {
        float best[2] = {1e30f, 1e30f};
        for (int round = 0; round < 3; ++round)
            for (int u = 0; u < 2; ++u) {
                M.dev->multi[mask].unstaged = u != 0;
                step();
                hip_check(hipEventCreate(&e0), "hipEventCreate");
                hip_check(hipEventCreate(&e1), "hipEventCreate");
                hip_check(hipEventRecord(e0, s), "hipEventRecord");
                for (int r = 0; r < 16; ++r) step();
                hip_check(hipEventRecord(e1, s), "hipEventRecord");
                hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
                float ms = 0;
                hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                best[u] = std::min(best[u], ms / 16);
            }
        M.dev->multi[mask].unstaged = best[1] < best[0];
    }
    if (log_on())
        log_msg("tuned exa_eval mask " + std::to_string(mask) + ": block " + std::to_string(w.block) +
                ", points per lane " + std::to_string(w.epl) + ", fused " + std::to_string(w.fused) + ", units " +
                std::to_string(w.comb) + " (" + std::to_string(w.ms * 1e3) + " us)");
}

}  // namespace

// Algorithmic bytes of one launch evaluating `modes` under schedule
// `fused`: per-point inputs and outputs of every unit, plus each distinct x,
// v and theta entry read, counted once over the launch.
void kernel_bytes(const Model& M, const std::vector<int>& modes, bool fused, int64_t& rd, int64_t& wr,
                  const std::map<std::pair<int, int>, UnitLive>* live) {
    const std::map<std::pair<int, int>, UnitLive>& LV = live ? *live : M.live;
    rd = wr = 0;
    std::vector<char> xs(M.nvar, 0), vs(M.nvar, 0), ts(M.ntheta, 0);
    for (int mode : modes)
    // the objective always runs its fixed schedule
    for (const Unit& u : units_for(M, mode, mode == M_OBJ ? kObjFused : fused)) {
        auto it = LV.find({mode, u.code});
        if (it == LV.end()) continue;
        const UnitLive& L = it->second;
        const Group& G = M.groups[u.group];
        const Pattern& P0 = M.pats[G.members[0]];
        rd += u.ndata * (4 * (int64_t)L.icols.size() + 8 * (int64_t)L.fcols.size() + 8 * (int64_t)L.weights);
        // the objective writes one partial sum per tile, not per data point
        if (mode != M_OBJ) wr += u.ndata * 8 * L.outputs;
        auto mark = [&](const RefKey& r, std::vector<char>& seen) {
            if (r.col < 0) {
                if (r.off >= 0 && r.off < (int64_t)seen.size()) seen[r.off] = 1;
                return;
            }
            const std::vector<int32_t>& c = P0.icols[r.col];
            for (int64_t k = 0; k < u.ndata; ++k) seen[(int64_t)c[k] + r.off] = 1;
        };
        for (int r : L.vrefs) mark(G.vrefs[r], xs);
        for (int r : L.vseeds) mark(G.vrefs[r], vs);
        for (int r : L.prefs) mark(G.prefs[r], ts);
    }
    // augmentation terms pulled by their base rows (cons, jprod)
    std::vector<int> pulled;
    for (int m : modes)
        for (int jm : job_modes(m)) pulled.push_back(jm);
    for (int mode : pulled) {
        if (mode != M_CONS && mode != M_JPROD) continue;
        for (size_t a = 0; a < M.pats.size(); ++a) {
            const Pattern& P = M.pats[a];
            auto it = LV.find({mode, 1000 + (int)a});
            if (P.kind != EXA_AUG || P.ndata == 0 || it == LV.end()) continue;
            const UnitLive& L = it->second;
            rd += P.ndata * (4 * (int64_t)L.icols.size() + 8 * (int64_t)L.fcols.size());
            rd += 4 * (int64_t)(P.rptr.size() + P.ridx.size());
            for (int s : L.vrefs) {
                const RefKey& r = P.vslots[s];
                for (int64_t k = 0; k < P.ndata; ++k) xs[r.col < 0 ? r.off : (int64_t)P.icols[r.col][k] + r.off] = 1;
            }
            for (int s : L.vseeds) {
                const RefKey& r = P.vslots[s];
                for (int64_t k = 0; k < P.ndata; ++k) vs[r.col < 0 ? r.off : (int64_t)P.icols[r.col][k] + r.off] = 1;
            }
            for (int s : L.prefs) {
                const RefKey& r = P.pslots[s];
                for (int64_t k = 0; k < P.ndata; ++k) ts[r.col < 0 ? r.off : (int64_t)P.icols[r.col][k] + r.off] = 1;
            }
        }
    }
    for (int mode : modes)
        if (mode == M_OBJ) wr += 8 * (int64_t)make_tiles(M, M_OBJ, 0, (int64_t)kObjBlock * kObjEpl, kObjFused).size();
    if (modes.size() == 1 && modes[0] == M_GRAD && M.grad_direct) wr = 8 * M.nvar;
    for (char c : xs) rd += c ? 8 : 0;
    for (char c : vs) rd += c ? 8 : 0;
    for (char c : ts) rd += c ? 8 : 0;
}

// Reduction launch of an exa_eval mask: maps (int32 when every position
// fits), buffer entries once, outputs once; objective partials when several.
void reduce_bytes(const Model& M, uint32_t mask, int64_t& rr, int64_t& rw) {
    rr = rw = 0;
    auto seg = [&](const SegMap& S) {
        const int64_t nseg = visited_segments(S), nnz = (int64_t)S.idx.size();
        const int64_t top = std::max<int64_t>(nnz, S.idx.empty() ? 0 : *std::max_element(S.idx.begin(), S.idx.end()));
        const int64_t low = S.idx.empty() ? 0 : *std::min_element(S.idx.begin(), S.idx.end());
        const int64_t w = top >= INT32_MAX || low < INT32_MIN ? 8 : 4;
        const ChunkPlan P = chunk_plan(S);
        // chunked maps read a 24-byte record per lane (segment, count,
        // four positions) instead of segment pointers and positions, and
        // positions only for the entries of long segments; maps with
        // long segments read their part tables (the long-segment table
        // once per launch), and each part sum is written once and read
        // once
        int64_t long_nnz = 0;
        for (int64_t i = 0; i < P.nlong(); ++i) long_nnz += P.longs[5 * i + 2];
        rr += (P.chunked ? 24 * P.nlanes() + 4 * long_nnz : w * (nseg + 1) + w * nnz) + 40 * P.nlong() +
              16 * P.nparts() + 8 * nnz;
        // segments written by the evaluation kernel are not written here
        const int64_t nskip = (int64_t)std::count(S.skip.begin(), S.skip.begin() + (S.skip.empty() ? 0 : nseg), 1);
        rw += 8 * (nseg - nskip) + 8 * P.nparts();
    };
    if ((mask & (EXA_EV_GRAD | EXA_EV_LAG)) && !M.grad_direct) seg(M.grad_map);
    if (mask & (EXA_EV_JTPROD | EXA_EV_LAG)) seg(M.jt_map);
    if (mask & EXA_EV_HPROD) seg(M.h_map);
    if (mask & EXA_EV_ADJ) seg(M.par_map);
    if (mask & EXA_EV_OBJ) {
        const int64_t nobj = (int64_t)make_tiles(M, M_OBJ, 0, (int64_t)kObjBlock * kObjEpl, kObjFused).size();
        if (nobj != 1) {
            rr += 8 * nobj;
            rw += 8;
        }
    }
}

ExaSegJob seg_job(const DevMap& m, const double* buf, double* out, const double* w) {
    ExaSegJob J;
    std::memset(&J, 0, sizeof J);
    J.ptr = m.ptr;
    J.idx = m.idx;
    J.wide = m.wide;
    J.nseg = m.nseg;
    J.chunked = m.chunked;
    J.lanes = m.lanes;
    J.lidx = m.lidx;
    J.nlanes = m.nlanes;
    J.longs = m.longs;
    J.lpart = m.lpart;
    J.nparts = m.nparts;
    J.nlong = m.nlong;
    J.lsum = m.lsum;
    J.buf = buf;
    J.w = w;
    J.out = out;
    return J;
}

void segsum(const DevMap& m, const double* buf, double* out, hipStream_t s, const double* w) {
    ExaReduce R;
    std::memset(&R, 0, sizeof R);
    R.ep_job = -1;
    R.job[0] = seg_job(m, buf, out, w);
    R.njobs = 1;
    hip_check(exa_launch_reduce(R, s), "segmented reduction");
}

}  // namespace exa

// ===========================================================================
// C ABI
using namespace exa;

namespace {

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

Model& live(exa_model* m) {
    if (!m) fail(EXA_EINVAL, "null model");
    if (m->impl.host_only || !m->impl.dev)
        fail(EXA_ESTATE, "model was created host-only; callbacks need a device");
    return m->impl;
}

void need(const void* p, int64_t n, const char* what) {
    if (n > 0 && !p) fail(EXA_EINVAL, std::string("null pointer: ") + what);
}

ExaCall blank_call() {
    ExaCall c;
    std::memset(&c, 0, sizeof c);
    return c;
}

}  // namespace

namespace exa {
Model::Model() {
    for (auto& c : counters) c.store(0);
}
Model::~Model() = default;
Model& live_model(exa_model* m) { return live(m); }
exa_status guard_status(const std::function<void()>& f) { return guard(f); }
}  // namespace exa

namespace {
Model::Csc& csc_checked(const exa_model* m, int32_t which) {
    if (!m) fail(EXA_EINVAL, "null model");
    if (which != EXA_CSC_JAC && which != EXA_CSC_HESS) fail(EXA_EINVAL, "which must be EXA_CSC_JAC or EXA_CSC_HESS");
    // the analysis is a cache of the structure: computing it does not change the model
    return csc_form(const_cast<exa_model*>(m)->impl, which);
}
}  // namespace

extern "C" {

const char* exa_last_error(void) { return exa::last_error(); }
const char* exa_version(void) { return "exa-mi355x 0.1 (gfx950, fp64)"; }

exa_status exa_create(const exa_pattern_desc* pats, int32_t npats, int64_t nvar, const double* xl,
                      const double* xu, int64_t ntheta, const double* theta, const exa_options* opt,
                      exa_model** out) {
    return guard([&] {
        if (!out) fail(EXA_EINVAL, "null output handle");
        *out = nullptr;
        if (nvar < 0 || ntheta < 0) fail(EXA_EINVAL, "negative size");
        if (ntheta > 0 && !theta) fail(EXA_EINVAL, "null theta");
        std::unique_ptr<exa_model> h(new exa_model());
        Model& M = h->impl;
        M.nvar = nvar;
        M.ntheta = ntheta;
        M.xl.assign(nvar, -HUGE_VAL);
        M.xu.assign(nvar, HUGE_VAL);
        if (xl) std::copy(xl, xl + nvar, M.xl.begin());
        if (xu) std::copy(xu, xu + nvar, M.xu.begin());
        M.theta.assign(theta ? theta : nullptr, theta ? theta + ntheta : nullptr);
        if (opt) {
            M.host_only = opt->host_only != 0;
            if (opt->block) M.block = opt->block;
            if (opt->epl) M.epl = opt->epl;
            M.autotune = opt->autotune != 0;
            M.fuse = opt->fuse != 0;
            M.eval_per_mode = opt->eval_per_mode != 0;
            M.max_device_bytes = opt->max_device_bytes;
        }
        M.cache_dir = cache_dir_of(opt ? opt->cache_dir : nullptr);
        if (M.max_device_bytes < 0) fail(EXA_EINVAL, "max_device_bytes must be >= 0");
        if (M.block != 64 && M.block != 128 && M.block != 256)
            fail(EXA_EINVAL, "block must be 64, 128 or 256");
        if (M.epl < 1 || M.epl > 16) fail(EXA_EINVAL, "epl must be in 1..16");
        auto t0 = std::chrono::steady_clock::now();
        build_host(M, pats, npats);
        M.host_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (M.max_device_bytes > 0) {
            const int64_t need = estimate_device_bytes(M);
            if (need > M.max_device_bytes)
                fail(EXA_ENOMEM, "the model needs about " + std::to_string(need) +
                                     " bytes of device memory, more than its budget of " +
                                     std::to_string(M.max_device_bytes));
        }
        if (!M.host_only) build_device(M);
        if (log_on()) {
            char buf[400];
            std::snprintf(buf, sizeof buf,
                          "create: %zu patterns, nvar %lld, ncon %lld, nnzj %lld, nnzh %lld; host %.1f ms, codegen "
                          "%.1f ms, compile %.1f ms (%s); device bytes %lld",
                          M.pats.size(), (long long)M.nvar, (long long)M.ncon, (long long)M.nnzj, (long long)M.nnzh,
                          M.host_ms, M.codegen_ms, M.compile_ms,
                          M.host_only ? "host only" : M.module_shared ? "shared module" : M.cache_hit ? "cache hit" : "compiled",
                          (long long)(M.dev ? M.dev->allocated : estimate_device_bytes(M)));
            log_msg(buf);
        }
        *out = h.release();
    });
}

exa_status exa_destroy(exa_model* m) {
    return guard([&] { delete m; });
}

exa_status exa_dims(const exa_model* m, int64_t* nvar, int64_t* ncon, int64_t* nnzj, int64_t* nnzh) {
    return guard([&] {
        if (!m) fail(EXA_EINVAL, "null model");
        if (nvar) *nvar = m->impl.nvar;
        if (ncon) *ncon = m->impl.ncon;
        if (nnzj) *nnzj = m->impl.nnzj;
        if (nnzh) *nnzh = m->impl.nnzh;
    });
}

exa_status exa_bounds(const exa_model* m, double* xl, double* xu, double* gl, double* gu) {
    return guard([&] {
        if (!m) fail(EXA_EINVAL, "null model");
        const Model& M = m->impl;
        if (xl) std::copy(M.xl.begin(), M.xl.end(), xl);
        if (xu) std::copy(M.xu.begin(), M.xu.end(), xu);
        for (auto& P : M.pats) {
            if (P.kind != EXA_CON) continue;
            if (gl) std::copy(P.lcon.begin(), P.lcon.end(), gl + P.o0);
            if (gu) std::copy(P.ucon.begin(), P.ucon.end(), gu + P.o0);
        }
    });
}

exa_status exa_set_theta(exa_model* m, const double* theta, exa_stream_t stream) {
    return guard([&] {
        Model& M = live(m);
        need(theta, M.ntheta, "theta");
        if (M.ntheta)
            hip_check(hipMemcpyAsync(M.dev->theta, theta, M.ntheta * sizeof(double),
                                     hipMemcpyDeviceToDevice, (hipStream_t)stream),
                      "hipMemcpyAsync");
    });
}

exa_status exa_jac_structure(const exa_model* m, int32_t* rows, int32_t* cols) {
    return guard([&] {
        if (!m) fail(EXA_EINVAL, "null model");
        need(rows, m->impl.nnzj, "rows");
        need(cols, m->impl.nnzj, "cols");
        jac_structure_host(m->impl, rows, cols);
    });
}

exa_status exa_hess_structure(const exa_model* m, int32_t* rows, int32_t* cols) {
    return guard([&] {
        if (!m) fail(EXA_EINVAL, "null model");
        need(rows, m->impl.nnzh, "rows");
        need(cols, m->impl.nnzh, "cols");
        hess_structure_host(m->impl, rows, cols);
    });
}

namespace {
void obj_body(Model& M, const double* x, double* f, hipStream_t s) {
    DeviceState& D = *M.dev;
    if (D.sched[M_OBJ].ntiles == 0) {
        hip_check(exa_launch_fill(f, 1, 0.0, s), "fill");
    } else {
        // one tile: its workgroup sum is the objective, written in place
        const bool one = D.sched[M_OBJ].ntiles == 1;
        ExaCall c = blank_call();
        c.x = x;
        c.out0 = one ? f : D.tilesum;
        launch_mode(M, M_OBJ, c, s);
        if (!one) hip_check(exa_launch_sum(D.tilesum, D.sched[M_OBJ].ntiles, f, s), "objective reduction");
    }
    M.counters[0]++;
}
}  // namespace

exa_status exa_obj(exa_model* m, const double* x, double* f, exa_stream_t stream) {
    return guard([&] {
        Model& M = live(m);
        need(x, M.nvar, "x");
        need(f, 1, "f");
        obj_body(M, x, f, (hipStream_t)stream);
    });
}

exa_status exa_obj_host(exa_model* m, const double* x, double* f, exa_stream_t stream) {
    return guard([&] {
        Model& M = live(m);
        need(x, M.nvar, "x");
        if (!f) fail(EXA_EINVAL, "null pointer: f");
        hipStream_t s = (hipStream_t)stream;
        DeviceState& D = *M.dev;
        obj_body(M, x, D.fval, s);
        hip_check(hipMemcpyAsync(D.fhost, D.fval, sizeof(double), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
        hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
        *f = *D.fhost;
    });
}

exa_status exa_grad(exa_model* m, const double* x, double* g, exa_stream_t stream) {
    return guard([&] {
        Model& M = live(m);
        need(x, M.nvar, "x");
        need(g, M.nvar, "g");
        hipStream_t s = (hipStream_t)stream;
        ExaCall c = blank_call();
        c.x = x;
        if (M.grad_direct) {
            c.out0 = g;
            c.direct = 1;
            launch_mode(M, M_GRAD, c, s);
        } else {
            c.out0 = M.dev->fo;
            launch_mode(M, M_GRAD, c, s);
            segsum(M.dev->grad_map, M.dev->fo, g, s);
        }
        M.counters[1]++;
    });
}

exa_status exa_cons(exa_model* m, const double* x, double* cv, exa_stream_t stream) {
    return guard([&] {
        Model& M = live(m);
        need(x, M.nvar, "x");
        need(cv, M.ncon, "c");
        hipStream_t s = (hipStream_t)stream;
        ExaCall c = blank_call();
        c.x = x;
        c.out0 = cv;
        launch_mode(M, M_CONS, c, s);
        M.counters[2]++;
    });
}

exa_status exa_jac_coord(exa_model* m, const double* x, double* vals, exa_stream_t stream) {
    return guard([&] {
        Model& M = live(m);
        need(x, M.nvar, "x");
        need(vals, M.nnzj, "vals");
        ExaCall c = blank_call();
        c.x = x;
        c.out0 = vals;
        launch_mode(M, M_JAC, c, (hipStream_t)stream);
        M.counters[3]++;
    });
}

exa_status exa_hess_coord(exa_model* m, const double* x, const double* y, double obj_weight,
                          double* vals, exa_stream_t stream) {
    return guard([&] {
        Model& M = live(m);
        need(x, M.nvar, "x");
        need(y, M.ncon, "y");
        need(vals, M.nnzh, "vals");
        ExaCall c = blank_call();
        c.x = x;
        c.y = y;
        c.sigma = obj_weight;
        c.out0 = vals;
        launch_mode(M, M_HESS, c, (hipStream_t)stream);
        M.counters[4]++;
    });
}

exa_status exa_jac_hess_coord(exa_model* m, const double* x, const double* y, double obj_weight,
                              double* jac_vals, double* hess_vals, exa_stream_t stream) {
    return guard([&] {
        Model& M = live(m);
        need(x, M.nvar, "x");
        need(y, M.ncon, "y");
        need(jac_vals, M.nnzj, "jac_vals");
        need(hess_vals, M.nnzh, "hess_vals");
        ExaCall c = blank_call();
        c.x = x;
        c.y = y;
        c.sigma = obj_weight;
        c.out0 = jac_vals;
        c.out1 = hess_vals;
        launch_mode(M, M_JH, c, (hipStream_t)stream);
        M.counters[3]++;
        M.counters[4]++;
    });
}

exa_status exa_jprod(exa_model* m, const double* x, const double* v, double* Jv, exa_stream_t stream) {
    return guard([&] {
        Model& M = live(m);
        need(x, M.nvar, "x");
        need(v, M.nvar, "v");
        need(Jv, M.ncon, "Jv");
        hipStream_t s = (hipStream_t)stream;
        ExaCall c = blank_call();
        c.x = x;
        c.v = v;
        c.out0 = Jv;
        launch_mode(M, M_JPROD, c, s);
        M.counters[5]++;
    });
}

exa_status exa_jtprod(exa_model* m, const double* x, const double* w, double* Jtw, exa_stream_t stream) {
    return guard([&] {
        Model& M = live(m);
        need(x, M.nvar, "x");
        need(w, M.ncon, "w");
        need(Jtw, M.nvar, "Jtw");
        hipStream_t s = (hipStream_t)stream;
        ExaCall c = blank_call();
        c.x = x;
        c.y = w;
        c.out0 = M.dev->fo;
        launch_mode(M, M_JTPROD, c, s);
        segsum(M.dev->jt_map, M.dev->fo, Jtw, s, w);
        M.counters[6]++;
    });
}

exa_status exa_hprod(exa_model* m, const double* x, const double* y, double obj_weight, const double* v,
                     double* Hv, exa_stream_t stream) {
    return guard([&] {
        Model& M = live(m);
        need(x, M.nvar, "x");
        need(y, M.ncon, "y");
        need(v, M.nvar, "v");
        need(Hv, M.nvar, "Hv");
        hipStream_t s = (hipStream_t)stream;
        ExaCall c = blank_call();
        c.x = x;
        c.y = y;
        c.v = v;
        c.sigma = obj_weight;
        c.out0 = M.dev->hv;
        c.out1 = Hv;
        launch_mode(M, M_HPROD, c, s);
        segsum(M.dev->h_map, M.dev->hv, Hv, s);
        M.counters[7]++;
    });
}

namespace {
// exa_eval's work; with lag set (the Lagrangian gradient), g then becomes
// lag_sigma * g + jtw once the reductions are done
void eval_body(Model& M, const exa_eval_args* a, hipStream_t s, bool lag = false, double lag_sigma = 0.0) {
    if (!a) fail(EXA_EINVAL, "null exa_eval_args");
    const uint32_t mask = a->mask;
    if (mask == 0 || (mask & ~(uint32_t)EXA_EV_ALL))
        fail(EXA_EINVAL, "exa_eval mask must select callbacks with the EXA_EV_* bits");
    need(a->x, M.nvar, "x");
    if (mask & (EXA_EV_HESS | EXA_EV_HPROD)) need(a->y, M.ncon, "y");
    if (mask & (EXA_EV_JPROD | EXA_EV_HPROD)) need(a->v, M.nvar, "v");
    if (mask & EXA_EV_JTPROD) need(a->w, M.ncon, "w");
    if (mask & EXA_EV_OBJ) need(a->f, 1, "f");
    if (mask & EXA_EV_GRAD) need(a->g, M.nvar, "g");
    if (mask & EXA_EV_CONS) need(a->c, M.ncon, "c");
    if (mask & EXA_EV_JAC) need(a->jac, M.nnzj, "jac");
    if (mask & EXA_EV_HESS) need(a->hess, M.nnzh, "hess");
    if (mask & EXA_EV_JPROD) need(a->jv, M.ncon, "jv");
    if (mask & EXA_EV_JTPROD) need(a->jtw, M.nvar, "jtw");
    if (mask & EXA_EV_HPROD) need(a->hv, M.nvar, "hv");
    DeviceState& D = *M.dev;
    const int64_t nobj = D.sched[M_OBJ].ntiles;

    // each mode's call, as its own entry point sets it up
    ExaMulti mc;
    std::memset(&mc, 0, sizeof mc);
    std::vector<int> rec_modes = eval_modes(mask, true);
    if (has_jh(mask)) rec_modes.insert(rec_modes.end(), {M_JAC, M_HESS});
    for (int mode : rec_modes) {
        ExaCall& c = mc.c[mode];
        c.inst = D.inst;
        c.x = a->x;
        switch (mode) {
            case M_OBJ: c.out0 = nobj == 1 ? a->f : D.tilesum; break;
            case M_GRAD:
                c.out0 = M.grad_direct ? a->g : D.fo;
                c.direct = M.grad_direct ? 1 : 0;
                break;
            case M_CONS: c.out0 = a->c; break;
            case M_JAC: c.out0 = a->jac; break;
            case M_HESS:
                c.y = a->y;
                c.sigma = a->obj_weight;
                c.out0 = a->hess;
                break;
            case M_JH:
                c.y = a->y;
                c.sigma = a->obj_weight;
                c.out0 = a->jac;
                c.out1 = a->hess;
                break;
            case M_JPROD:
                c.v = a->v;
                c.out0 = a->jv;
                break;
            case M_JTPROD:
                c.y = a->w;
                c.out0 = D.fo;
                break;
            case M_HPROD:
                c.y = a->y;
                c.v = a->v;
                c.sigma = a->obj_weight;
                c.out0 = D.hv;
                c.out1 = a->hv;
                break;
            default: break;
        }
    }
    // multi units read the Jacobian and Hessian jobs' own records
    if ((mask & EXA_EV_JAC) && (mask & EXA_EV_HESS)) {
        ExaCall& cj = mc.c[M_JAC];
        cj.inst = D.inst;
        cj.x = a->x;
        cj.out0 = a->jac;
        ExaCall& ch = mc.c[M_HESS];
        ch.inst = D.inst;
        ch.x = a->x;
        ch.y = a->y;
        ch.sigma = a->obj_weight;
        ch.out0 = a->hess;
    }
    // the reductions of every selected callback, in one launch
    auto reduce_of = [&]() {
        ExaReduce R;
        std::memset(&R, 0, sizeof R);
        R.ep_job = -1;
        auto job = [&](const DevMap& dm, const double* buf, double* out, const double* w = nullptr) {
            R.job[R.njobs++] = seg_job(dm, buf, out, w);
        };
        if ((mask & EXA_EV_GRAD) && !M.grad_direct) job(D.grad_map, D.fo, a->g);
        // the Lagrangian gradient with g written in place by the evaluation
        // launch: J^T y goes straight into g as g = sigma * g + J^T y
        const bool lag_ep = lag && M.grad_direct;
        if (lag_ep) {
            R.ep_job = R.njobs;
            R.ax_alpha = lag_sigma;
            job(D.jt_map, D.fo, a->g, a->w);
        } else if (mask & EXA_EV_JTPROD) {
            job(D.jt_map, D.fo, a->jtw, a->w);
        }
        if (mask & EXA_EV_HPROD) job(D.h_map, D.hv, a->hv);
        if ((mask & EXA_EV_OBJ) && nobj != 1) {  // no tiles: the sum of nothing, 0
            R.part = D.tilesum;
            R.npart = nobj;
            R.f = a->f;
        }
        if (lag && !lag_ep) {  // out = sigma * grad + J^T y, after the reductions
            R.ax_out = a->g;
            R.ax_add = a->jtw;
            R.ax_alpha = lag_sigma;
            R.ax_n = M.nvar;
        }
        return R;
    };
    auto it = D.multi.find(mask);
    if (it == D.multi.end() || !it->second.tuned) {
        // untuned: per-callback tiles (the kind the tuner picks on most
        // models; one-pass units hold many registers), patterns over the
        // same data in one lane
        set_multi_schedule(M, mask, M.block, M.epl, true, EXA_UNITS_PER_CALLBACK);
        if (M.autotune)
            tune_multi(M, mask, mc, s, [&]() {
                raw_launch_multi(M, mask, mc, s);
                hip_check(exa_launch_reduce(reduce_of(), s), "exa_eval reductions");
            });
        D.multi[mask].tuned = true;
    }
    const DeviceState::MultiSched& S = D.multi.at(mask);
    DeviceState::EvalTiming& Tm = D.timing;
    const bool timed = Tm.on && Tm.used < (int64_t)Tm.reduced.size();
    hipEvent_t* ev = timed ? &Tm.ev[4 * Tm.used] : nullptr;
    if (timed) hip_check(hipEventRecord(ev[0], s), "hipEventRecord");
    raw_launch_multi(M, mask, mc, s);
    if (timed) hip_check(hipEventRecord(ev[1], s), "hipEventRecord");
    const ExaReduce R = reduce_of();
    const bool reduce = R.njobs > 0 || R.part;
    if (timed && reduce) hip_check(hipEventRecord(ev[2], s), "hipEventRecord");
    hip_check(exa_launch_reduce(R, s), "exa_eval reductions");
    if (timed && reduce) hip_check(hipEventRecord(ev[3], s), "hipEventRecord");
    if (timed) Tm.reduced[Tm.used++] = reduce ? 1 : 0;

    const uint32_t bits[8] = {EXA_EV_OBJ, EXA_EV_GRAD, EXA_EV_CONS, EXA_EV_JAC,
                              EXA_EV_HESS, EXA_EV_JPROD, EXA_EV_JTPROD, EXA_EV_HPROD};
    for (int i = 0; i < 8; ++i)
        if (mask & bits[i]) M.counters[i]++;
}
}  // namespace

exa_status exa_eval(exa_model* m, const exa_eval_args* a, exa_stream_t stream) {
    return guard([&] { eval_body(live(m), a, (hipStream_t)stream); });
}

exa_status exa_lag_grad(exa_model* m, const double* x, const double* y, double obj_weight, double* out,
                        exa_stream_t stream) {
    return guard([&] {
        Model& M = live(m);
        need(x, M.nvar, "x");
        need(y, M.ncon, "y");
        need(out, M.nvar, "out");
        exa_eval_args a;
        std::memset(&a, 0, sizeof a);
        a.mask = EXA_EV_GRAD | EXA_EV_JTPROD;
        a.x = x;
        a.w = y;
        a.g = out;
        a.jtw = M.dev->lag_tmp;
        eval_body(M, &a, (hipStream_t)stream, true, obj_weight);
    });
}

exa_status exa_csc_dims(const exa_model* m, int32_t which, int64_t* nnz) {
    return guard([&] {
        if (!nnz) fail(EXA_EINVAL, "null nnz");
        *nnz = (int64_t)csc_checked(m, which).rowval.size();
    });
}

exa_status exa_csc_structure(const exa_model* m, int32_t which, int32_t* colptr, int32_t* rowval) {
    return guard([&] {
        const Model::Csc& C = csc_checked(m, which);
        need(colptr, (int64_t)C.colptr.size(), "colptr");
        need(rowval, (int64_t)C.rowval.size(), "rowval");
        std::copy(C.colptr.begin(), C.colptr.end(), colptr);
        std::copy(C.rowval.begin(), C.rowval.end(), rowval);
    });
}

exa_status exa_csc_values(exa_model* m, int32_t which, const double* coo, double* csc, exa_stream_t stream) {
    return guard([&] {
        const Model::Csc& C = csc_checked(m, which);
        Model& M = live(m);
        need(coo, which == EXA_CSC_JAC ? M.nnzj : M.nnzh, "coo");
        need(csc, (int64_t)C.rowval.size(), "csc");
        DeviceState& D = *M.dev;
        if (!D.csc_up[which]) {
            upload_map(D, C.map, D.csc_map[which]);
            D.csc_up[which] = true;
        }
        segsum(D.csc_map[which], coo, csc, (hipStream_t)stream);
    });
}

exa_status exa_device_copy(void* dst, const void* src, int64_t bytes, exa_stream_t stream) {
    return guard([&] {
        if (bytes < 0) fail(EXA_EINVAL, "negative byte count");
        if (bytes > 0 && (!dst || !src)) fail(EXA_EINVAL, "null pointer");
        hip_check(exa_launch_copy(src, dst, bytes, (hipStream_t)stream), "device copy");
    });
}

exa_status exa_eval_timing(exa_model* m, int32_t enable) {
    return guard([&] {
        Model& M = live(m);
        DeviceState& D = *M.dev;
        D.timing_off();
        if (!enable) return;
        const int64_t calls = 1024;
        D.timing.ev.reserve(4 * calls);
        for (int64_t i = 0; i < 4 * calls; ++i) {
            hipEvent_t e;
            // timing only: no system-scope fence (cache writeback) per record
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
                D.timing_off();
                fail(EXA_EHIP, "hipEventCreate failed");
            }
            D.timing.ev.push_back(e);
        }
        D.timing.reduced.assign(calls, 0);
        D.timing.on = true;
    });
}

exa_status exa_eval_timing_read(exa_model* m, double* out4) {
    return guard([&] {
        Model& M = live(m);
        if (!out4) fail(EXA_EINVAL, "null out4");
        DeviceState::EvalTiming& T = M.dev->timing;
        if (!T.on) fail(EXA_ESTATE, "exa_eval timing is off");
        double se = 0.0, sr = 0.0;
        int64_t nr = 0;
        for (int64_t i = 0; i < T.used; ++i) {
            hipEvent_t* ev = &T.ev[4 * i];
            hip_check(hipEventSynchronize(ev[1]), "hipEventSynchronize");
            float ms = 0.0f;
            hip_check(hipEventElapsedTime(&ms, ev[0], ev[1]), "hipEventElapsedTime");
            se += ms;
            if (T.reduced[i]) {
                hip_check(hipEventSynchronize(ev[3]), "hipEventSynchronize");
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

exa_status exa_eval_bytes(const exa_model* m, uint32_t mask, int64_t* out4) {
    return guard([&] {
        if (!m || !out4) fail(EXA_EINVAL, "null argument");
        if (mask == 0 || (mask & ~(uint32_t)EXA_EV_ALL))
            fail(EXA_EINVAL, "mask must select callbacks with the EXA_EV_* bits");
        const Model& M = m->impl;
        if (M.live.empty()) generate_source(M, const_cast<std::map<std::pair<int, int>, UnitLive>*>(&M.live));
        bool fused = true;  // the untuned exa_eval schedule
        int units = EXA_UNITS_PER_CALLBACK;
        if (M.dev) {
            auto it = M.dev->multi.find(mask);
            if (it != M.dev->multi.end()) {
                fused = it->second.fused;
                units = it->second.units;
            }
        }
        int64_t rd = 0, wr = 0;
        kernel_bytes(M, launch_modes(mask, valid_units(mask, units)), fused, rd, wr);
        out4[0] = rd;
        out4[1] = wr;
        int64_t rr = 0, rw = 0;
        reduce_bytes(M, mask, rr, rw);
        out4[2] = rr;
        out4[3] = rw;
    });
}

exa_status exa_eval_set_schedule(exa_model* m, uint32_t mask, int32_t block, int32_t epl, int32_t fused,
                                 int32_t units) {
    return guard([&] {
        Model& M = live(m);
        if (mask == 0 || (mask & ~(uint32_t)EXA_EV_ALL))
            fail(EXA_EINVAL, "mask must select callbacks with the EXA_EV_* bits");
        if (block != 64 && block != 128 && block != 256) fail(EXA_EINVAL, "block must be 64, 128 or 256");
        if (epl < 1 || epl > 16) fail(EXA_EINVAL, "points per lane must be in 1..16");
        if ((units & ~EXA_UNSTAGED) < EXA_UNITS_PER_CALLBACK)
            fail(EXA_EINVAL, "units must be one of the EXA_UNITS_* values");
        const bool unstaged = (units & EXA_UNSTAGED) != 0;
        units &= ~EXA_UNSTAGED;
        if (units < EXA_UNITS_PER_CALLBACK || units > EXA_UNITS_ONE_PASS)
            fail(EXA_EINVAL, "units must be one of the EXA_UNITS_* values");
        if (units == EXA_UNITS_ONE_PASS && M.eval_per_mode) units = EXA_UNITS_JAC_HESS;
        set_multi_schedule(M, mask, block, epl, fused != 0, units);
        M.dev->multi[mask].unstaged = unstaged;
        M.dev->multi[mask].tuned = true;
    });
}

exa_status exa_eval_schedule(const exa_model* m, uint32_t mask, int64_t* out4) {
    return guard([&] {
        if (!m || !out4) fail(EXA_EINVAL, "null argument");
        if (!m->impl.dev) fail(EXA_ESTATE, "host-only model has no schedule");
        auto it = m->impl.dev->multi.find(mask);
        if (it == m->impl.dev->multi.end()) fail(EXA_ESTATE, "no exa_eval call with this mask yet");
        out4[0] = it->second.block;
        out4[1] = it->second.epl;
        out4[2] = (it->second.fused ? 1 : 0) | (it->second.units == EXA_UNITS_ONE_PASS ? 2 : 0) |
                  (it->second.units == EXA_UNITS_JAC_HESS ? 4 : 0) | (it->second.unstaged ? 16 : 0);
        out4[3] = it->second.ntiles;
    });
}

exa_status exa_adjoint_theta(exa_model* m, const double* x, const double* y, double obj_weight,
                             const double* w, double* theta_bar, exa_stream_t stream) {
    return guard([&] {
        Model& M = live(m);
        need(x, M.nvar, "x");
        need(y, M.ncon, "y");
        need(w, M.nvar, "w");
        need(theta_bar, M.ntheta, "theta_bar");
        hipStream_t s = (hipStream_t)stream;
        ExaCall c = blank_call();
        c.x = x;
        c.y = y;
        c.v = w;
        c.sigma = obj_weight;
        c.out0 = M.dev->par;
        launch_mode(M, M_ADJ, c, s);
        segsum(M.dev->par_map, M.dev->par, theta_bar, s);
        M.counters[8]++;
    });
}

namespace {
// public callback ids (exa_counters order) -> internal modes
int mode_of_callback(int32_t cb) {
    static const int map[10] = {M_OBJ, M_GRAD, M_CONS, M_JAC, M_HESS, M_JPROD, M_JTPROD, M_HPROD, M_ADJ, M_JH};
    if (cb < 0 || cb > 9) fail(EXA_EINVAL, "callback id must be in 0..9");
    return map[cb];
}
}  // namespace

exa_status exa_kernel_bytes(const exa_model* m, int32_t callback, int64_t* read_bytes, int64_t* write_bytes) {
    return guard([&] {
        if (!m) fail(EXA_EINVAL, "null model");
        const int mode = mode_of_callback(callback);
        const Model& M = m->impl;
        if (M.live.empty()) generate_source(M, const_cast<std::map<std::pair<int, int>, UnitLive>*>(&M.live));
        const bool fused = M.dev ? M.dev->sched[mode].fused : false;
        int64_t rd = 0, wr = 0;
        kernel_bytes(M, {mode}, fused, rd, wr);
        if (read_bytes) *read_bytes = rd;
        if (write_bytes) *write_bytes = wr;
    });
}

exa_status exa_schedule(const exa_model* m, int32_t callback, int64_t* out4) {
    return guard([&] {
        if (!m || !out4) fail(EXA_EINVAL, "null argument");
        const int mode = mode_of_callback(callback);
        if (!m->impl.dev) fail(EXA_ESTATE, "host-only model has no schedule");
        const DeviceState::Sched& S = m->impl.dev->sched[mode];
        out4[0] = S.block;
        out4[1] = S.epl;
        out4[2] = (S.fused ? 1 : 0) | (S.unstaged ? 2 : 0);
        out4[3] = S.ntiles;
    });
}

exa_status exa_generated_source(const exa_model* m, char* buf, int64_t cap, int64_t* len) {
    return guard([&] {
        if (!m) fail(EXA_EINVAL, "null model");
        const std::string src = generate_source(m->impl);
        if (len) *len = (int64_t)src.size();
        if (buf && cap > 0) {
            const size_t n = std::min<size_t>((size_t)cap - 1, src.size());
            std::memcpy(buf, src.data(), n);
            buf[n] = '\0';
        }
    });
}

exa_status exa_compile_check(const exa_model* m) {
    return guard([&] {
        if (!m) fail(EXA_EINVAL, "null model");
        bool hit = false;
        (void)cached_code(generate_source(m->impl), m->impl.cache_dir, &hit);
    });
}

exa_status exa_device_bytes(const exa_model* m, int64_t* bytes) {
    return guard([&] {
        if (!m || !bytes) fail(EXA_EINVAL, "null argument");
        *bytes = m->impl.dev ? m->impl.dev->allocated : estimate_device_bytes(m->impl);
    });
}

exa_status exa_build_info(const exa_model* m, double* out6) {
    return guard([&] {
        if (!m || !out6) fail(EXA_EINVAL, "null argument");
        const Model& M = m->impl;
        out6[0] = M.host_ms;
        out6[1] = M.codegen_ms;
        out6[2] = M.compile_ms;
        out6[3] = M.host_only ? -1.0 : M.module_shared ? 2.0 : M.cache_hit ? 1.0 : 0.0;
        out6[4] = (double)(M.dev ? M.dev->allocated : estimate_device_bytes(M));
        out6[5] = M.cache_dir.empty() ? 0.0 : 1.0;
    });
}

exa_status exa_pattern_info(const exa_model* m, int32_t p, int64_t* out8) {
    return guard([&] {
        if (!m || !out8) fail(EXA_EINVAL, "null argument");
        if (p < 0 || p >= (int32_t)m->impl.pats.size()) fail(EXA_EINVAL, "pattern index out of range");
        const Pattern& P = m->impl.pats[p];
        const int64_t v[8] = {P.kind, P.ndata, P.o1step(), P.o2step(), P.pstep(), P.o0, P.o1, P.o2};
        std::copy(v, v + 8, out8);
    });
}

exa_status exa_counters(const exa_model* m, int64_t* out9) {
    return guard([&] {
        if (!m || !out9) fail(EXA_EINVAL, "null argument");
        for (int i = 0; i < 9; ++i) out9[i] = m->impl.counters[i].load();
    });
}

}  // extern "C"
