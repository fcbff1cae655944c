// Internal declarations of the evaluator library (not part of the C ABI).
#pragma once

#include <atomic>
#include <cstdint>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/exa.h"

namespace exa {

// ---------------------------------------------------------------------------
// Errors: thrown inside the library, turned into exa_status at the ABI.
struct Error : std::runtime_error {
    exa_status code;
    Error(exa_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};
[[noreturn]] void fail(exa_status code, const std::string& msg);
void set_last_error(const std::string& msg);

// ---------------------------------------------------------------------------
// Device-side layout.  The same text defines the structs for the host
// compiler and, stringified, for the run-time compiled kernels, so the two
// layouts cannot drift apart.
// Index into ExaInstDev::off: where an instance's slice starts in each of
// the arrays a call reads or writes.
#define EXA_OFF_ROWS 0    /* constraint rows (ncon)                          */
#define EXA_OFF_AUG 1     /* augmentation term buffer (naug)                 */
#define EXA_OFF_JAC 2     /* Jacobian values (nnzj)                          */
#define EXA_OFF_HESS 3    /* Hessian values (nnzh)                           */
#define EXA_OFF_PAR 4     /* parameter-adjoint buffer (nnzp)                 */
#define EXA_OFF_TILE 5    /* per-tile partial sums of the objective          */
#define EXA_OFF_X 6       /* x and v/w vectors (nvar)                        */
#define EXA_OFF_Y 7       /* y (ncon)                                        */
#define EXA_OFF_FO_OBJ 8  /* first-order buffer, objective part (nnzg)       */
#define EXA_OFF_FO_CON 9  /* first-order buffer, constraint part (nnzj)      */
#define EXA_OFF_HV 10     /* H v buffer (curved slots)                       */
#define EXA_NOFF 12
// Index offsets of a pattern's unique references live in ExaPatDev::roff
// (variable slots first, then parameter slots), so that every instance of a
// formulation runs the same code whatever its block offsets.
#define EXA_MAX_REFS 48
// Tile code of a zero-fill tile (entries of g no objective term touches).
#define EXA_ZERO_TILE 1023
#define EXA_PAD_TILE 4095  // a tile that matches no unit: does nothing

// ExaPatDev::hvd: bit r set when the pattern's group stores H v reference r
// straight into the output (Group::hv_direct, for this instance's data).
#define EXA_DEVICE_STRUCTS                                                       \
    struct ExaPatDev {                                                           \
        const int* ic[8];                                                        \
        const double* fc[8];                                                     \
        long long ndata;                                                         \
        long long o0;                                                            \
        long long o1;                                                            \
        long long o2;                                                            \
        long long op;                                                            \
        long long oh;                                                            \
        long long ob;                                                            \
        long long tgt0;                                                          \
        long long row_off;                                                       \
        int row_ic;                                                              \
        int hvd;                                                                 \
        const int* rptr;                                                         \
        const int* ridx;                                                         \
        long long roff[48];                                                      \
    };                                                                           \
    struct ExaInstDev {                                                          \
        long long off[12];                                                       \
        const double* theta;                                                     \
        long long pad1;                                                          \
        struct ExaPatDev pat[32];                                                \
    };                                                                           \
    struct ExaTile {                                                             \
        int pat;                                                                 \
        int inst;                                                                \
        long long start;                                                         \
        long long count;                                                         \
        long long slot;                                                          \
    };                                                                           \
    struct ExaCall {                                                             \
        const struct ExaTile* tiles;                                             \
        long long ntiles;                                                        \
        long long per_xcd;                                                       \
        const struct ExaInstDev* inst;                                           \
        const double* x;                                                         \
        const double* y;                                                         \
        const double* v;                                                         \
        double* out0;                                                            \
        double* out1;                                                            \
        double sigma;                                                            \
        int direct;                                                              \
        int unstaged;                                                            \
    };                                                                           \
    struct ExaMulti {                                                            \
        const struct ExaTile* tiles;                                             \
        long long ntiles;                                                        \
        long long per_xcd;                                                       \
        struct ExaCall c[10];                                                    \
    };

EXA_DEVICE_STRUCTS

#define EXA_STR2(...) #__VA_ARGS__
#define EXA_STR(...) EXA_STR2(__VA_ARGS__)

// ---------------------------------------------------------------------------
// Host-side model.

enum Mode : int {
    M_OBJ = 0,    // objective terms -> per-tile partial sums
    M_CONS = 1,   // constraint rows; each pulls its augmentation terms
    M_GRAD = 2,   // objective gradient: in place, or first-order buffer
    M_JAC = 3,    // Jacobian values
    M_HESS = 4,   // Lagrangian Hessian values
    M_JPROD = 5,  // J v rows; each pulls its augmentation terms
    M_JTPROD = 6, // w[row] * J -> first-order buffer (jac part)
    M_HPROD = 7,  // local (w H) v on curved slots -> H v buffer
    M_ADJ = 8,    // mixed partials -> parameter buffer
    M_JH = 9,     // Jacobian and Hessian values of each data point in one pass
    M_COUNT = 10
};
static_assert(M_COUNT == 10, "ExaMulti holds one call per mode");
// Units that run several callbacks' jobs at one point from one set of loads
// and sweeps, used by the several-callback kernel only (their jobs take
// inputs and outputs from the per-mode calls of an ExaMulti):
// M_SFULL: grad, cons, jac, hess, jprod, hprod (a J^T w of the same call is
//          summed from the Jacobian values by the reduction launch);
// M_SIPM:  grad, cons, jac, hess (an interior-point iterate).
constexpr int M_SFULL = 10, M_SIPM = 11;
inline bool multi_unit_mode(int mode) { return mode == M_SFULL || mode == M_SIPM; }
// Component modes of a unit mode (itself for plain modes, jac + hess for JH).
const std::vector<int>& job_modes(int mode);
// Tiles of the several-callback kernel carry their mode above this bit of
// the unit code (unit codes stay below 1 << EXA_MODE_SHIFT).
#define EXA_MODE_SHIFT 12

struct TNode {            // node of a simplified tree
    int op = 0;
    int a = -1, b = -1;   // children (positions in the node list)
    int col = -1;         // data column (DATA) or index column (VAR/PARAM)
    int64_t off = 0;      // index offset (VAR/PARAM)
    double val = 0.0;     // literal (CONST)
    int slot = -1;        // VAR: unique var slot; PARAM: unique param slot
};

struct RefKey {           // symbolic identity of a var/param reference
    int col;
    int64_t off;
    bool operator==(const RefKey& o) const { return col == o.col && off == o.off; }
};

struct Pattern {
    int kind = 0;
    int index = 0;                    // declaration position
    std::vector<TNode> nodes;         // simplified tree, post-order, root last
    int64_t ndata = 0;
    int n_icols = 0, n_fcols = 0;
    std::vector<std::vector<int32_t>> icols;   // host copies (index columns)
    // index column c holds 0, 1, ..., ndata - 1 (at least kIdentMin points):
    // the generated code uses the data point itself instead of loading it
    std::vector<char> ident;
    std::vector<const double*> fcols_src;      // caller's float columns (create only)
    std::vector<RefKey> vslots;       // unique var refs, first-visit order
    std::vector<RefKey> pslots;       // unique param refs
    std::vector<std::pair<int, int>> hslots;   // unique pairs of var slots
    // layout
    int64_t o0 = 0;   // CON first row; OBJ first term; AUG first aug entry
    int64_t o1 = 0;   // CON/AUG first jac entry; OBJ first grad-buffer entry
    int64_t o2 = 0;   // first hess entry
    int64_t op = 0;   // first param-buffer entry
    int64_t ob = 0;   // first entry of this pattern's block in its part of the first-order buffer
    int target = -1;
    int row_icol = -1;
    int64_t row_off = 0;
    int64_t tgt0 = 0; // AUG: first row of the target block
    std::vector<double> lcon, ucon;
    // data-set group (patterns over the same data arrays) and the group-level
    // reference each of this pattern's var / param slots maps to
    int group = -1;
    std::vector<int> vg, pg;
    // AUG: data points grouped by the target row they add to (CSR over the
    // target block's rows, points ascending): the row's lane pulls them
    std::vector<int32_t> rptr, ridx;
    // CON: augmentation patterns adding to this block, declaration order
    std::vector<int> augs;
    // var slots that occur in some Hessian pair (the only ones H v reaches)
    std::vector<int> hvs;
    // AUG whose expression is plus or minus one variable, the only J^T w
    // contribution of its data set to that reference: its contribution is
    // +-w[row], which the reduction reads from w itself (no J^T w job)
    int wread = 0;  // +1, -1, or 0
    int64_t oh = 0;   // first entry of this pattern in the H v buffer

    // work buffers (first-order, H v, parameter) hold each pattern's block
    // slot-major: slot s of data point k at block + s * bstride() + k, with
    // every slot array padded to whole 128-byte lines
    int64_t bstride() const { return (ndata + 15) & ~(int64_t)15; }
    int o1step() const { return (int)vslots.size(); }
    int o2step() const { return (int)hslots.size(); }
    int pstep() const { return (int)pslots.size(); }
    int64_t row(int64_t k) const {
        return kind == EXA_CON ? o0 + k : tgt0 + (int64_t)icols[row_icol][k] + row_off;
    }
    int64_t var_index(int s, int64_t k) const {
        const RefKey& r = vslots[s];
        return r.col < 0 ? r.off : (int64_t)icols[r.col][k] + r.off;
    }
    int64_t par_index(int s, int64_t k) const {
        const RefKey& r = pslots[s];
        return r.col < 0 ? r.off : (int64_t)icols[r.col][k] + r.off;
    }
};

// Patterns declared over the very same data arrays (same ndata, same column
// arrays in the same order).  Their evaluations can share one lane: the data
// loads, the gathers of x and common subexpressions are then done once.
struct Group {
    std::vector<int> members;          // pattern positions, declaration order
    std::vector<RefKey> vrefs, prefs;  // distinct references over all members
    std::vector<std::pair<int, int>> vsrc, psrc;  // first (member, slot) of each
    int64_t ndata = 0;
    // J^T w and H v contributions are summed over the members of a point
    // before they leave the lane: one buffer slot per group-level reference
    // that some member contributes to (ascending reference index), blocks at
    // ob (constraint part of the first-order buffer) and oh (H v buffer)
    std::vector<int> jt_refs, hv_refs;
    int64_t ob = 0, oh = 0;
    // per H v reference: every entry it stores is the only H v contribution
    // to its variable (at most 32 references).  Code generated with the flag
    // set writes the output entry itself when the instance's bit in
    // ExaPatDev::hvd is set, and the buffer entry otherwise; code generated
    // without it always writes the buffer entry (no index kept live)
    std::vector<char> hv_direct;
};

// A unit of generated code for one callback: one pattern, or the members of
// a group evaluated together.  Tile codes: pattern p -> p, group g -> 32 + g.
struct Unit {
    int code = 0;
    int group = 0;
    std::vector<int> members;
    int64_t ndata = 0;
};

// Inputs a unit's generated code really reads for one data point (after
// dead-code elimination), used to report algorithmic traffic.
struct UnitLive {
    std::vector<int> icols, fcols;     // data columns
    std::vector<int> vrefs, vseeds, prefs;  // group-level references
    int weights = 0;                   // y entries (one per member that needs it)
    int64_t outputs = 0;               // doubles written per data point
    bool pulls = false;                // base rows pull augmentation terms
};

// Sorted reduction map (CSR): segment s sums buf[idx[ptr[s] .. ptr[s+1])].
struct SegMap {
    std::vector<int64_t> ptr, idx;
    // segments the reduction leaves alone (empty: none); such a segment has
    // no entries, its output is written by the evaluation kernel
    std::vector<char> skip;
    int64_t nseg() const { return ptr.empty() ? 0 : (int64_t)ptr.size() - 1; }
};

struct DeviceState;  // defined in exa_runtime.cpp

struct Model {
    int64_t nvar = 0, ncon = 0, ntheta = 0;
    int64_t nnzj = 0, nnzh = 0, nnzg = 0, naug = 0, nnzp = 0, nobj = 0, nhv = 0;
    // work-buffer lengths (entries, slot arrays padded): first-order buffer
    // (objective part, then constraint part), H v buffer, parameter buffer
    int64_t fo_obj_len = 0, fo_con_len = 0, hv_len = 0, par_len = 0;
    // every variable gets at most one objective-gradient contribution: the
    // gradient kernel writes g directly (plus zero tiles for the rest)
    bool grad_direct = false;
    std::vector<std::pair<int64_t, int64_t>> grad_zero;  // untouched ranges of g
    std::vector<Pattern> pats;
    std::vector<Group> groups;
    std::vector<double> xl, xu, theta;
    // reduction maps (positions in the first-order buffer: grad part first)
    SegMap grad_map, jt_map, h_map, par_map;
    bool host_only = false;
    int block = 256, epl = 4;
    bool autotune = false, fuse = false;
    bool eval_per_mode = false;  // exa_eval: per-callback tiles only
    std::string signature;   // hash of the simplified trees (shared code)
    std::string cache_dir;   // code-object cache directory ("" : none)
    int64_t max_device_bytes = 0;  // device memory budget (0: none)
    // build statistics: host analysis, code generation and compilation (or
    // cache read) in milliseconds; whether the code object came from the
    // on-disk cache; whether it was shared with a live model
    double host_ms = 0, codegen_ms = 0, compile_ms = 0;
    bool cache_hit = false, module_shared = false;
    // inputs each generated unit really reads, per (mode, unit code)
    std::map<std::pair<int, int>, UnitLive> live;
    std::atomic<int64_t> counters[9];
    // compressed sparse columns of the Jacobian (0) and of the Hessian's
    // lower triangle (1), analysed on first use: colptr [nvar+1], rowval,
    // and the COO positions each entry sums (ascending)
    struct Csc {
        bool ready = false;
        std::vector<int32_t> colptr, rowval;
        SegMap map;
    };
    Csc csc[2];
    std::unique_ptr<DeviceState> dev;
    Model();
    ~Model();
};

// exa_model.cpp
void build_host(Model& M, const exa_pattern_desc* pats, int32_t npats);
std::string pattern_signature(const Model& M);
// Augmentations a and b have the same row lists (rptr / ridx): the same data
// arrays, rows from the same index column plus the same offset, and targets
// of one size.  The generated pulls of such augmentations share one walk.
bool same_walk(const Model& M, int a, int b);

// exa_codegen.cpp
#define EXA_BLOCK_MAX 256
bool pattern_in_mode(const Pattern& P, int mode);
// Modes the several-callback kernels evaluate: exa_k_multi (Jacobian and
// Hessian apart) or exa_k_multijh (with Jacobian + Hessian units).
const std::vector<int>& multi_modes(bool jh);
std::vector<Unit> units_for(const Model& M, int mode, bool fused);
// Generated source for all callbacks; fills live[(mode, unit code)].
// ident_flags: per pattern and index column, whether the code may use the
// data point itself (default: each pattern's own flags); hvd_flags: per
// group and H v reference, whether the code may store the reference into
// the output (default: each group's own Group::hv_direct)
std::string generate_source(const Model& M, std::map<std::pair<int, int>, UnitLive>* live = nullptr,
                            const std::vector<std::vector<char>>* ident_flags = nullptr,
                            const std::vector<std::vector<char>>* hvd_flags = nullptr);

// exa_runtime.cpp
// Objective tiles always hold kObjBlock * kObjEpl points (256 virtual lanes
// of 8 points), so the objective's summation order is fixed; its own launch
// uses kObjBlock-wide workgroups.
constexpr int kObjBlock = 256, kObjEpl = 8;
constexpr int64_t kIdentMin = 64;
constexpr bool kObjFused = true;
void build_device(Model& M);
// Device memory a model needs (data columns, tables, work buffers, maps),
// estimated from the host analysis before anything is allocated.
int64_t estimate_device_bytes(const Model& M);

}  // namespace exa

struct exa_model {
    exa::Model impl;
};
