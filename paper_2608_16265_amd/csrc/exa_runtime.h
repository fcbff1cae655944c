// Device state of a model and the helpers shared by the runtime and batching.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "exa_internal.h"

namespace exa {

struct Module {
    hipModule_t mod = nullptr;
    hipFunction_t fn[M_COUNT] = {};
    hipFunction_t fn_multi = nullptr;    // tiles of several callbacks in one launch (Jacobian and Hessian apart)
    hipFunction_t fn_multijh = nullptr;  // the same with Jacobian + Hessian units
    hipFunction_t fn_onepass = nullptr;  // one pass per point for several callbacks
    std::string source;
    std::vector<char> code;
    ~Module();
};

struct DevMap {
    const void* ptr = nullptr;  // int32 entries unless wide
    const void* idx = nullptr;
    int64_t nseg = 0;
    int wide = 0;
    // chunked sums (see ExaSegJob) for maps with long segments
    int chunked = 0;
    const int32_t* lanes = nullptr;  // 2 per lane: segment, count | chunks << 4
    const int32_t* lidx = nullptr;   // 4 per lane: the chunk's positions
    int64_t nlanes = 0;
    const int32_t* longs = nullptr;
    const int32_t* lpart = nullptr;
    int64_t nparts = 0, nlong = 0;
    double* lsum = nullptr;
};

struct DeviceState {
    int device = 0;
    std::shared_ptr<Module> module;
    std::vector<void*> allocs;
    std::vector<int64_t> sizes;       // bytes of each allocation
    int64_t allocated = 0;            // bytes allocated now
    int64_t budget = 0;               // 0: no limit; else alloc fails past it (EXA_ENOMEM)
    double* theta = nullptr;
    ExaInstDev* inst = nullptr;       // device copy of the single-instance table
    ExaInstDev inst_host;             // host copy (device pointers), reused by batches
    // schedule of each callback's evaluation kernel
    struct Sched {
        int block = 256, epl = 4;
        bool fused = false, tuned = false;
        bool unstaged = false;  // each lane stores its own output slice (no LDS staging)
        ExaTile* tiles = nullptr;
        int64_t ntiles = 0;
    } sched[M_COUNT];
    // schedule of the several-callback launch, per exa_eval mask
    struct MultiSched {
        int block = 256, epl = 4;
        bool fused = false, tuned = false;
        bool unstaged = false;  // each lane stores its own output slices
        int units = EXA_UNITS_PER_CALLBACK;  // EXA_UNITS_*: which kernel and units run the tiles
        ExaTile* tiles = nullptr;
        int64_t ntiles = 0;
    };
    std::map<uint32_t, MultiSched> multi;
    // HIP events around exa_eval's two launches while timing is on: four per
    // recorded call (evaluation start/end, reduction start/end)
    struct EvalTiming {
        bool on = false;
        std::vector<hipEvent_t> ev;
        std::vector<char> reduced;  // per recorded call: a reduction was launched
        int64_t used = 0;
    } timing;
    void timing_off();
    double* fo = nullptr;             // first-order buffer: grad part, then jac part
    double* par = nullptr;
    double* hv = nullptr;             // H v contributions (curved slots only)
    double* tilesum = nullptr;
    double* lag_tmp = nullptr;  // J^T y of exa_lag_grad (nvar)
    double* fval = nullptr;     // objective of exa_obj_host (device)
    double* fhost = nullptr;    // its pinned host copy
    DevMap csc_map[2];          // uploaded on the first exa_csc_values call
    bool csc_up[2] = {false, false};
    DevMap grad_map, jt_map, h_map, par_map;

    void* alloc(size_t bytes);
    void* upload(const void* src, size_t bytes);
    void release(void* p);
    ~DeviceState();
};

void hip_check(hipError_t e, const char* what);
// The model's own checks of a live (device) model, for entry points in other
// source files: EXA_EINVAL / EXA_ESTATE as the callbacks raise them.
Model& live_model(exa_model* m);
// One callback's evaluation launch under its current schedule (no tuning,
// no allocation).
void launch_mode_untuned(Model& M, int mode, ExaCall call, hipStream_t s);
// The segment sums of a map from `buf` into `out` (one reduction launch,
// plus one for long segments).
void segsum(const DevMap& m, const double* buf, double* out, hipStream_t s, const double* w = nullptr);
exa_status guard_status(const std::function<void()>& f);
// Tiles that write zeros to the gradient entries no objective term touches,
// kZeroTileEntries entries each (more when a tile of points is larger).
constexpr int64_t kZeroTileEntries = 4096;
void add_zero_tiles(const Model& M, int64_t tp, std::vector<ExaTile>& tiles);
bool has_fusable_group(const Model& M, int mode);
// Modes of an exa_eval mask (with jh: Jacobian + Hessian as JH units), the
// one-pass unit mode covering a mask (or -1), whether a mask has both the
// Jacobian and the Hessian, the units a mask can run as asked, and the modes
// whose tiles make up a mask's launch under those units.
std::vector<int> eval_modes(uint32_t mask, bool jh);
int combined_mode_of(uint32_t mask);
bool has_jh(uint32_t mask);
int valid_units(uint32_t mask, int units);
std::vector<int> launch_modes(uint32_t mask, int units);
// Algorithmic bytes of the reduction launch of a mask (maps, buffer entries,
// outputs, objective partials when there are several).
void reduce_bytes(const Model& M, uint32_t mask, int64_t& rd, int64_t& wr);
std::vector<char> compile_code(const std::string& src);
// The code object of a source through the on-disk cache in `dir` (empty: no
// cache); *hit tells whether it was read from the cache.
std::vector<char> cached_code(const std::string& src, const std::string& dir, bool* hit);
// The cache directory: the option's, else $EXA_CACHE_DIR, else none.
std::string cache_dir_of(const char* opt_dir);
std::shared_ptr<Module> compile_module(const std::string& src, const std::string& cache_dir, bool* cache_hit);
// One line to stderr when the environment variable EXA_LOG is set (not "0").
bool log_on();
void log_msg(const std::string& msg);
// Tiles of tile_pts points per unit.  With fills, a unit whose code reads
// nothing (constant derivatives only) gets tiles of kZeroTileEntries points
// (the batch, which is throughput-bound); without, only when its tiles
// would far outnumber the workgroups the chip holds at once.
std::vector<ExaTile> make_tiles(const Model& M, int mode, int inst, int64_t tile_pts, bool fused,
                                bool fills = false);
std::string kernel_name(int mode);
int mode_lds_doubles(const Model& M, int mode);
void set_schedule(Model& M, int mode, int block, int epl, bool fused);
// How a map's segments are summed (see ExaSegJob): one lane per segment
// when no segment is longer than 2 * kExaChunk (or positions need 64 bits);
// otherwise parts of kExaLongSeg entries for segments longer than that, and
// for the others chunk lanes, except on large maps whose other segments are
// all short (at most kExaShortSeg entries), where one lane per segment reads
// fewer bytes than a 24-byte lane record per segment.
struct ChunkPlan {
    bool chunked = false;  // chunk lanes (else one lane per segment)
    std::vector<int32_t> meta, lidx;    // 2 and 4 per lane, a multiple of 256 lanes
    std::vector<int32_t> longs, lpart;  // 5 per long segment; 2 per part block
    int64_t nlanes() const { return (int64_t)meta.size() / 2; }
    int64_t nlong() const { return (int64_t)longs.size() / 5; }
    int64_t nparts() const { return (int64_t)lpart.size() / 2; }
};
ChunkPlan chunk_plan(const SegMap& S);
// live: the liveness records of the code that runs (default: the model's own)
void kernel_bytes(const Model& M, const std::vector<int>& modes, bool fused, int64_t& rd, int64_t& wr,
                  const std::map<std::pair<int, int>, UnitLive>* live = nullptr);
// Map and tables of a segment map on the device (int32 when positions fit,
// chunked when segments are long).
void upload_map(DeviceState& D, const SegMap& S, DevMap& d);
// CSC analysis of the Jacobian (which = 0) or Hessian (1) on first use.
Model::Csc& csc_form(Model& M, int which);
void jac_structure_host(const Model& M, int32_t* rows, int32_t* cols);
void hess_structure_host(const Model& M, int32_t* rows, int32_t* cols);
const char* last_error();

}  // namespace exa
