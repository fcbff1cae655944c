/*
 * exa.h -- C ABI of the MI355X structured-NLP derivative evaluator.
 *
 * The library evaluates, on one AMD Instinct MI355X (gfx950) in IEEE FP64,
 * the callbacks a nonlinear-programming solver asks for at every iterate of
 *
 *     min f(x; theta)  s.t.  gl <= g(x; theta) <= gu,  xl <= x <= xu
 *
 * (paper eq. nlp, Sec. 2.1), for a model stated in the pattern-over-data
 * form of Sec. 2.2 (eq. simd): every objective group, base constraint block
 * and constraint augmentation is ONE expression tree evaluated at every
 * point of its data set.
 *
 * Conventions used by every entry point
 *   - Indices are 0-based (the paper is 1-based); sizes are int64_t, COO
 *     indices int32_t, values double.
 *   - "device" pointers are HIP device memory of the current device (e.g. a
 *     torch CUDA tensor's data_ptr()); "host" pointers are ordinary memory.
 *   - Callbacks are in place (Sec. 2.1.3): results are written into
 *     caller-owned arrays.  They are asynchronous on the given stream
 *     (exa_stream_t is a hipStream_t; NULL is the null stream) and do not
 *     synchronize, except the first call of a callback (or of an exa_eval
 *     mask) on a model with autotune on, which times candidate schedules on
 *     that stream and waits for them, and the first exa_csc_values call per
 *     matrix.  After those first calls, a callback only enqueues kernels on
 *     its stream (no allocation, no copy, no memset, no host wait), so a
 *     caller may capture it into a HIP graph and replay it.
 *   - Every call returns an exa_status; on failure nothing has been written
 *     to the outputs that the caller could mistake for a result only if the
 *     failure is reported before launch (argument checks); a failure of the
 *     HIP runtime after launch is reported as EXA_EHIP.  The text of the
 *     last error of the calling thread is returned by exa_last_error().
 *     A failed call leaves the model valid.
 *   - Environment: EXA_LOG=1 writes one line per model build, tuning
 *     decision and cache event to stderr; EXA_CACHE_DIR sets the default
 *     code-object cache (exa_options.cache_dir); EXA_TEST_BAD_SOURCE=1
 *     appends a line that does not compile to every generated source (a
 *     test hook for the EXA_ECOMPILE path).
 *   - Concurrent callbacks on ONE model from different streams race on the
 *     model's internal work buffers; serialize them (one stream per model).
 *     Calls on one model from several host threads must not overlap either
 *     (a model builds its schedules at first use); different models are
 *     independent.
 */
#ifndef EXA_H
#define EXA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t exa_status;
#define EXA_OK 0
#define EXA_EINVAL 1   /* bad argument or malformed model description        */
#define EXA_ENOMEM 2   /* device or host allocation failed                   */
#define EXA_ECOMPILE 3 /* run-time compilation of the generated kernels failed */
#define EXA_EHIP 4     /* a HIP runtime call failed                          */
#define EXA_ESTATE 5   /* call not available for this handle (host-only model) */

typedef void* exa_stream_t; /* a hipStream_t */

typedef struct exa_model exa_model;
typedef struct exa_batch exa_batch;

/* ---- Model description ---------------------------------------------------
 *
 * Expression tree of one pattern (Sec. 4), as a post-order node list: the
 * children of node i have positions < i and the root is the last node.
 * Node operators (Sec. 4.2; registered functions of Sec. 7.1.3):
 */
#define EXA_OP_CONST 0  /* literal value val[i]                               */
#define EXA_OP_DATA 1   /* float data column a[i] at the current data point   */
#define EXA_OP_VAR 2    /* x[idx],   idx = icol[a[i]][k] + off[i]  (a[i] >= 0)  */
                        /*           idx = off[i]                   (a[i] == -1) */
#define EXA_OP_PARAM 3  /* theta[idx], same index rule as EXA_OP_VAR          */
#define EXA_OP_NEG 10
#define EXA_OP_ABS2 11  /* u*u */
#define EXA_OP_INV 12   /* 1/u */
#define EXA_OP_SQRT 13
#define EXA_OP_EXP 14
#define EXA_OP_LOG 15
#define EXA_OP_SIN 16
#define EXA_OP_COS 17
#define EXA_OP_TAN 18
#define EXA_OP_ATAN 19
#define EXA_OP_SINH 20
#define EXA_OP_COSH 21
#define EXA_OP_TANH 22
#define EXA_OP_LOG1P 23
#define EXA_OP_EXPM1 24
#define EXA_OP_ADD 40
#define EXA_OP_SUB 41
#define EXA_OP_MUL 42
#define EXA_OP_DIV 43
#define EXA_OP_POW 44

/* Pattern kinds (eq. simd): objective terms, base constraint block, and an
 * augmentation adding one term per data point to a row of an earlier base
 * block (Sec. 3.3.2, ConstraintAugmentation). */
#define EXA_OBJ 0
#define EXA_CON 1
#define EXA_AUG 2

#define EXA_MAX_PATTERNS 32
#define EXA_MAX_COLS 8
#define EXA_MAX_NODES 512

typedef struct exa_pattern_desc {
    int32_t kind;          /* EXA_OBJ / EXA_CON / EXA_AUG                      */
    int32_t nnodes;        /* 1 .. EXA_MAX_NODES                               */
    const int32_t* op;     /* host [nnodes] operator codes                     */
    const int32_t* a;      /* host [nnodes] child 1 | data column | index col  */
    const int32_t* b;      /* host [nnodes] child 2 of binary nodes, else -1   */
    const int64_t* off;    /* host [nnodes] var/param index offset, else 0     */
    const double* val;     /* host [nnodes] literal of EXA_OP_CONST, else 0    */
    int64_t ndata;         /* number of data points (>= 0)                     */
    int32_t n_icols;       /* integer data columns (<= EXA_MAX_COLS)           */
    int32_t n_fcols;       /* float data columns (<= EXA_MAX_COLS)             */
    const int32_t* const* icols; /* host [n_icols][ndata]                      */
    const double* const* fcols;  /* host [n_fcols][ndata]                      */
    int32_t target;        /* AUG: position of the target EXA_CON pattern,
                              which must come earlier in the list; else -1    */
    int32_t row_icol;      /* AUG: row within target block = icols[row_icol][k] */
    int64_t row_off;       /* AUG:                          + row_off         */
    const double* lcon;    /* CON: host [ndata] lower bounds (NULL: 0)         */
    const double* ucon;    /* CON: host [ndata] upper bounds (NULL: 0)         */
} exa_pattern_desc;

typedef struct exa_options {
    int32_t host_only; /* 1: analyse only (dims, bounds, structure); no device
                          memory, no kernel compilation; callbacks then return
                          EXA_ESTATE                                           */
    int32_t block;     /* threads per workgroup: 64, 128 or 256 (0: 256)      */
    int32_t epl;       /* data points per lane per tile: 1..16 (0: 4)         */
    int32_t autotune;  /* 1: at its first call, each callback times candidate
                          schedules (workgroup size, points per lane, fused or
                          separate patterns) and keeps the fastest; results do
                          not depend on the schedule                          */
    int32_t fuse;      /* without autotune: 1 evaluates patterns declared over
                          the same data arrays in one lane (shared loads),
                          0 evaluates them separately                          */
    int32_t eval_per_mode; /* 1: exa_eval runs one tile per callback and point
                          (as the single callbacks do); 0: it may also run
                          units that evaluate all selected callbacks of a point
                          from one pass over its loads, when autotune chooses
                          them.  Without autotune exa_eval runs one tile per
                          callback, patterns over the same data in one lane,
                          with the block and epl above; results are the same  */
    int32_t reserved[2];
    const char* cache_dir; /* directory of the on-disk code-object cache (NULL
                          or "": the environment variable EXA_CACHE_DIR, else
                          no cache).  The compiled code of a pattern set is
                          stored there under a key hashing the generated
                          source, the compile options and the hiprtc version,
                          beside the source itself; a later process whose
                          generated source is byte-identical loads it instead
                          of compiling (Sec. 8.6: compilation is paid once per
                          pattern set).  Unreadable or unwritable caches only
                          cost the compilation.                              */
    int64_t max_device_bytes; /* device memory budget of the model (0: none):
                          exa_create fails with EXA_ENOMEM when the footprint
                          estimated after the host analysis (see
                          exa_device_bytes) exceeds it, or when an allocation
                          would take the model past it                     */
} exa_options;

/* ---- Library ------------------------------------------------------------ */

/* Text of the last error raised on the calling thread ("" if none). */
const char* exa_last_error(void);
/* Library version string. */
const char* exa_version(void);

/* ---- Model lifetime (Sec. 3.1 ExaCore -> Sec. 3.2 ExaModel) -------------
 *
 * exa_create validates the description, applies the build-time
 * simplification table (Sec. 7.1.2), finds each pattern's sparsity structure
 * by the probe of Sec. 5.2 (unique variable references in first-visit
 * order; unique unordered variable pairs in second-order emission order,
 * lower triangle), lays out the outputs with the offsets and strides of
 * Sec. 3.4 / Sec. 5.3.2, builds the sorted reduction maps of Sec. 7.2.3 and
 * lowers every pattern to straight-line gfx950 code compiled at run time.
 *
 *   pats, npats     host array of pattern descriptions, in declaration order;
 *                   the library copies everything it needs (the caller may
 *                   free the description afterwards).
 *   nvar            length of x; xl, xu host [nvar] bounds (NULL: -inf/+inf)
 *   ntheta, theta   parameter vector (host [ntheta]; may be NULL if 0)
 *   opt             NULL for defaults
 *   out             receives the handle (owned by the caller, freed with
 *                   exa_destroy).
 * Errors: EXA_EINVAL for a malformed description (unknown operator, child
 * index not below the node, column out of range, a variable, parameter or
 * row index outside its range at some data point, AUG target not an earlier
 * CON), EXA_ENOMEM, EXA_ECOMPILE, EXA_EHIP.
 */
exa_status exa_create(const exa_pattern_desc* pats, int32_t npats, int64_t nvar,
                      const double* xl, const double* xu, int64_t ntheta,
                      const double* theta, const exa_options* opt, exa_model** out);
exa_status exa_destroy(exa_model* m);

/* Sizes (Sec. 2.1.2 meta-information): n, m, nnzj, nnzh.  Any output may be
 * NULL.  nnzj/nnzh count the partially compressed COO entries (Sec. 5.2.2). */
exa_status exa_dims(const exa_model* m, int64_t* nvar, int64_t* ncon, int64_t* nnzj,
                    int64_t* nnzh);
/* Bounds into host arrays xl, xu [nvar] and gl, gu [ncon]; any may be NULL. */
exa_status exa_bounds(const exa_model* m, double* xl, double* xu, double* gl, double* gu);

/* Replace theta (device [ntheta]) without rebuilding the model (Sec. 2.2.3,
 * updating and resolving).  The copy is enqueued on the stream. */
exa_status exa_set_theta(exa_model* m, const double* theta, exa_stream_t stream);

/* ---- Structure callbacks (Sec. 5.3.1) -----------------------------------
 * Host arrays of nnzj (nnzh) entries.  Jacobian entry o1 + k*o1step + s of a
 * pattern is (row of data point k, global index of its s-th unique variable
 * reference).  Hessian entries are (max, min) of the two resolved indices.  */
exa_status exa_jac_structure(const exa_model* m, int32_t* rows, int32_t* cols);
exa_status exa_hess_structure(const exa_model* m, int32_t* rows, int32_t* cols);

/* ---- Callbacks (Sec. 2.1.3); x, y, v, w and all outputs are device arrays --- */

/* f(x): objective terms reduced in a fixed order (Sec. 7.2.3, buffer then
 * reduce); *f is a device scalar. */
exa_status exa_obj(exa_model* m, const double* x, double* f, exa_stream_t stream);
/* f(x) as exa_obj computes it (same bits), returned in the host scalar *f:
 * the objective reduction lands in a library-owned device scalar, is copied
 * to pinned host memory on `stream`, and the call waits for the stream (the
 * one callback that synchronizes with the host, as the objective of
 * Sec. 7.2.3 returns a number).  Not capturable into a graph.  Errors:
 * EXA_EINVAL for a NULL x (nvar > 0) or f; EXA_ESTATE for a host-only model. */
exa_status exa_obj_host(exa_model* m, const double* x, double* f, exa_stream_t stream);
/* grad f(x) into g [nvar] (dense; zero where no objective term depends on a
 * variable).  Per-term contributions are merged by a fixed-order segmented
 * reduction over a precomputed sort (Sec. 7.2.3 compress_to_dense). */
exa_status exa_grad(exa_model* m, const double* x, double* g, exa_stream_t stream);
/* g(x) into c [ncon]: base rows plus augmentation terms (eq. simd:con). */
exa_status exa_cons(exa_model* m, const double* x, double* c, exa_stream_t stream);
/* Jacobian values into vals [nnzj] (Sec. 5.3.2 jac_coord). */
exa_status exa_jac_coord(exa_model* m, const double* x, double* vals, exa_stream_t stream);
/* Lagrangian Hessian sigma*grad^2 f + sum_j y_j grad^2 g_j, lower triangle,
 * into vals [nnzh] (Sec. 5.3.2 hess_coord).  y is device [ncon].  When two
 * different references of one pattern resolve to the same variable, their
 * cross entry holds twice the mixed derivative, so that summing duplicate
 * entries gives the Hessian. */
exa_status exa_hess_coord(exa_model* m, const double* x, const double* y, double obj_weight,
                          double* vals, exa_stream_t stream);
/* Jacobian and Hessian values together (what a solver asks for at every
 * iterate): each data point's Jacobian row block and Hessian block come from
 * one pass over its loads and forward sweep, in one launch.  Outputs are
 * bit-identical to exa_jac_coord and exa_hess_coord. */
exa_status exa_jac_hess_coord(exa_model* m, const double* x, const double* y, double obj_weight,
                              double* jac_vals, double* hess_vals, exa_stream_t stream);
/* J(x) v into Jv [ncon]; v is device [nvar] (Sec. 2.1.3 jprod). */
exa_status exa_jprod(exa_model* m, const double* x, const double* v, double* Jv,
                     exa_stream_t stream);
/* J(x)^T w into Jtw [nvar]; w is device [ncon] (Sec. 2.1.3 jtprod).  The
 * patterns declared over the same data arrays add their contributions
 * (Jacobian entry times w of its row, members in declaration order) to one
 * variable reference in the lane; the reduction then sums these per
 * variable in a fixed order (Sec. 7.2.3).  An augmentation term that is
 * plus or minus one variable, and its data set's only contribution to that
 * reference, contributes plus or minus w of its row: the reduction reads
 * that weight from w itself, at the same place in the order. */
exa_status exa_jtprod(exa_model* m, const double* x, const double* w, double* Jtw,
                      exa_stream_t stream);
/* (sigma grad^2 f + sum y_j grad^2 g_j) v into Hv [nvar] (Sec. 2.1.3 hprod).
 * Contributions are summed as exa_jtprod sums them.  A variable reference
 * of a data set whose every entry is the only H v contribution to its
 * variable (ACOPF's branch flows, for instance) is written into Hv by the
 * evaluation kernel; the reduction sums the other variables. */
exa_status exa_hprod(exa_model* m, const double* x, const double* y, double obj_weight,
                     const double* v, double* Hv, exa_stream_t stream);
/* exa_hprod for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels in the same order, so Hv is bit-identical to exa_hprod's,
 * but the H v work buffer and the part sums of long segments live in a
 * fixed library array of 4,194,304 doubles (32 MiB) that each GPU the
 * library runs on holds until the process ends.  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine) and never tunes: it
 * runs hprod's schedule as it stands (the model's default, or the tuned one
 * after an autotuned exa_hprod call).  Nothing in the array needs to start
 * at zero (every entry read was written by the same call).  Every call on
 * one GPU shares that GPU's array, which keeps the last call's contents:
 * calls that overlap on one GPU (other streams, other host threads, other
 * models) race.  Arguments as exa_hprod.  Errors: EXA_EINVAL for a NULL
 * pointer a nonzero size needs, a model whose H v work space exceeds the
 * array (hv entries plus part sums; use exa_hprod), or a model on another
 * device than the current one; EXA_ESTATE for a host-only model; EXA_EHIP. */
exa_status exa_hprod_noalloc(exa_model* m, const double* x, const double* y, double obj_weight,
                             const double* v, double* Hv, exa_stream_t stream);
/* Gradient of the Lagrangian of eq. nlp, sigma grad f(x) + J(x)^T y, into
 * out [nvar]; x [nvar] and y [ncon] are device arrays, sigma = obj_weight
 * (the first-order half of what hess_coord weights, Sec. 2.1.3).  One
 * evaluation launch of the gradient and J^T y terms and their reductions,
 * which finish out = sigma * grad + J^T y with the product rounded before
 * the sum (one elementwise launch more when the gradient itself needs a
 * reduction): bit-identical to exa_grad into out, exa_jtprod into t and
 * then out = sigma * out followed by out = out + t.  Uses a library-owned
 * nvar buffer for J^T y, so overlapping calls on one model race.  Counts
 * as one grad and one jtprod evaluation.  Errors: EXA_EINVAL for a NULL
 * pointer that a nonzero size needs; EXA_ESTATE for a host-only model. */
exa_status exa_lag_grad(exa_model* m, const double* x, const double* y, double obj_weight, double* out,
                        exa_stream_t stream);

/* Compressed sparse columns (CSC) of the Jacobian (which = EXA_CSC_JAC,
 * nvar columns) or of the Hessian's lower triangle (EXA_CSC_HESS): the
 * compression across patterns and data points that the partially compressed
 * COO layout leaves to the solver (Sec. 5.2).  Each distinct (row, col)
 * pair of exa_jac_structure / exa_hess_structure is one entry; columns
 * ascend, rows ascend within a column (0-based).  The structure is analysed
 * on the host on first use (any of the three calls) and kept.
 * exa_csc_dims: number of entries into *nnz (host).
 * exa_csc_structure: host arrays colptr [nvar+1] and rowval [nnz].
 * exa_csc_values: device arrays; csc [nnz] = the sums of the COO values
 * coo [nnzj or nnzh] (as written by exa_jac_coord / exa_hess_coord) over
 * each entry's positions, added in ascending position, so the result does
 * not depend on scheduling.  One reduction launch on `stream`; the first
 * call per matrix uploads its map (allocates and synchronizes).  coo and
 * csc must not overlap.  Errors: EXA_EINVAL for a bad `which`, a NULL
 * pointer a nonzero size needs, or more than 2^31 - 1 COO entries;
 * EXA_ESTATE for exa_csc_values on a host-only model. */
#define EXA_CSC_JAC 0
#define EXA_CSC_HESS 1
exa_status exa_csc_dims(const exa_model* m, int32_t which, int64_t* nnz);
exa_status exa_csc_structure(const exa_model* m, int32_t which, int32_t* colptr, int32_t* rowval);
exa_status exa_csc_values(exa_model* m, int32_t which, const double* coo, double* csc, exa_stream_t stream);

/* Several callbacks at one point in one call (Sec. 2.1.3 callbacks,
 * evaluated together).  `mask` selects callbacks with the EXA_EV_* bits;
 * every selected callback reads the inputs it needs and writes its output
 * exactly as its own entry point would, bit for bit:
 *   EXA_EV_OBJ    f    [1]      from x             (as exa_obj)
 *   EXA_EV_GRAD   g    [nvar]   from x             (as exa_grad)
 *   EXA_EV_CONS   c    [ncon]   from x             (as exa_cons)
 *   EXA_EV_JAC    jac  [nnzj]   from x             (as exa_jac_coord)
 *   EXA_EV_HESS   hess [nnzh]   from x, y, sigma   (as exa_hess_coord)
 *   EXA_EV_JPROD  jv   [ncon]   from x, v          (as exa_jprod)
 *   EXA_EV_JTPROD jtw  [nvar]   from x, w          (as exa_jtprod)
 *   EXA_EV_HPROD  hv   [nvar]   from x, y, sigma, v (as exa_hprod)
 * All pointers are device arrays owned by the caller; inputs a selection
 * does not need may be NULL, outputs it selects may not.  Outputs must not
 * overlap each other or the inputs.  The work is one evaluation launch over
 * the tiles of every selected callback, followed by one launch of the
 * deterministic reductions when any are needed (objective partials,
 * gradient, J^T w and H v segment sums), plus one small launch that adds
 * the part sums of segments longer than 1024 entries when there are any.  The first call with a given mask times candidate
 * schedules (as with autotune) and synchronizes the stream; later calls are
 * asynchronous on `stream`.
 * Errors: EXA_EINVAL for a NULL model or args, an empty or unknown mask, or
 * a NULL pointer the mask needs; EXA_ESTATE for a host-only model. */
#define EXA_EV_OBJ (1u << 0)
#define EXA_EV_GRAD (1u << 1)
#define EXA_EV_CONS (1u << 2)
#define EXA_EV_JAC (1u << 3)
#define EXA_EV_HESS (1u << 4)
#define EXA_EV_JPROD (1u << 5)
#define EXA_EV_JTPROD (1u << 6)
#define EXA_EV_HPROD (1u << 7)
#define EXA_EV_ALL 0xffu
typedef struct exa_eval_args {
    uint32_t mask;
    uint32_t reserved; /* 0 */
    const double* x;
    const double* y;
    double obj_weight;
    const double* v;
    const double* w;
    double* f;
    double* g;
    double* c;
    double* jac;
    double* hess;
    double* jv;
    double* jtw;
    double* hv;
} exa_eval_args;
exa_status exa_eval(exa_model* m, const exa_eval_args* args, exa_stream_t stream);
/* The schedule of exa_eval for a mask: out4 = workgroup size, points per
 * lane, fused (bit 0) | one pass per point for all callbacks (bit 1) |
 * Jacobian + Hessian units (bit 2) | unstaged stores (bit 4), number of
 * tiles.  EXA_ESTATE until the mask's first exa_eval call. */
exa_status exa_eval_schedule(const exa_model* m, uint32_t mask, int64_t* out4);
/* Units of an exa_eval launch: one tile per callback and point, the
 * Jacobian and the Hessian apart (their tiles then run in a kernel with a
 * smaller register budget); the same with Jacobian + Hessian units (both of
 * a point from one set of loads; masks with both); one unit per point for
 * every selected callback (masks with every callback, or exactly obj, grad,
 * cons, jac and hess). */
#define EXA_UNITS_PER_CALLBACK 0
#define EXA_UNITS_JAC_HESS 1
#define EXA_UNITS_ONE_PASS 2
/* Flag OR'ed into `units` (exa_eval_set_schedule, exa_batch_set_schedule,
 * the batch options): Jacobian and Hessian values leave each lane as its
 * own stores instead of being staged through LDS into contiguous 16-byte
 * stores (a schedule choice the tuners time; the values are the same). */
#define EXA_UNSTAGED 0x20
/* Batched evaluation only: every callback's tiles in a launch of its own,
 * one after another (each kernel with the register budget of its own units). */
#define EXA_UNITS_SEPARATE 3
/* Fix the schedule of exa_eval for a mask instead of tuning it at the
 * mask's first call (for measurement: a profiled run can use the schedule
 * an unprofiled run chose).  block = workgroup size (64, 128 or 256), epl =
 * points per lane (1..16), fused (0/1: patterns over the same data in one
 * lane), units = EXA_UNITS_* (a choice the mask does not allow falls back
 * to the next one down, as exa_eval_schedule then reports).  Results do not
 * depend on the schedule.  Errors: EXA_EINVAL for a bad mask or value;
 * EXA_ESTATE for a host-only model. */
exa_status exa_eval_set_schedule(exa_model* m, uint32_t mask, int32_t block, int32_t epl, int32_t fused,
                                 int32_t units);
/* Algorithmic traffic of exa_eval for a mask under its current schedule
 * (the model's default before the mask's first call), host array out4:
 * out4[0], out4[1] = bytes read and written by the evaluation launch,
 * counted as exa_kernel_bytes counts one callback (x, v entries once over
 * the launch); out4[2], out4[3] = bytes read and written by the reduction
 * launch (segment maps, each buffer entry once, each output once, and the
 * objective partials when there are several).  Works on host-only models. */
exa_status exa_eval_bytes(const exa_model* m, uint32_t mask, int64_t* out4);
/* Launch timing of exa_eval, for measurement.  With enable != 0, the next
 * 1024 exa_eval calls of this model record HIP events on their stream
 * around the evaluation launch and around the reduction launch (later calls
 * are not recorded); enable == 0 frees the events.
 * exa_eval_timing_read waits for the recorded calls and stores into the host
 * array out4 {calls recorded, average evaluation launch in microseconds,
 * reduction launches recorded, their average in microseconds}, then starts a
 * new recording.  EXA_ESTATE when timing is off. */
exa_status exa_eval_timing(exa_model* m, int32_t enable);
exa_status exa_eval_timing_read(exa_model* m, double* out4);

/* Device-to-device copy of `bytes` bytes with 16-byte non-temporal loads
 * and stores (one vector per lane; a byte-wise launch for the tail or for
 * pointers not 16-byte aligned), asynchronous on `stream`.  A measurement
 * utility: the practical streaming bandwidth of the device, against which
 * the evaluation kernels' HBM rates can be read.  src and dst are device
 * arrays that must not overlap.  Errors: EXA_EINVAL for a NULL pointer with
 * bytes > 0 or bytes < 0. */
exa_status exa_device_copy(void* dst, const void* src, int64_t bytes, exa_stream_t stream);

/* Adjoint with respect to the parameters (extension of the parametric NLP of
 * eq. nlp): theta_bar = (d grad_x L / d theta)^T w with
 * grad_x L = sigma grad f + J^T y, i.e. for every pattern instance
 * weight * sum_a w[col_a] d2T/dx_a dtheta_t added into theta_bar[t].
 * w device [nvar], theta_bar device [ntheta] (overwritten). */
exa_status exa_adjoint_theta(exa_model* m, const double* x, const double* y, double obj_weight,
                             const double* w, double* theta_bar, exa_stream_t stream);

/* Introspection of the lowering (Sec. 7.2.1 compiler specialization).
 * exa_generated_source copies the generated kernel source (NUL-terminated,
 * truncated to cap bytes) into the host buffer buf and stores its full
 * length in *len; buf may be NULL to query the length.
 * exa_compile_check compiles that source for gfx950 without loading it (no
 * GPU needed) and returns EXA_ECOMPILE with the compiler log on failure.
 * Both work on host-only models. */
exa_status exa_generated_source(const exa_model* m, char* buf, int64_t cap, int64_t* len);
exa_status exa_compile_check(const exa_model* m);

/* Algorithmic traffic of one launch of a callback's evaluation kernel under
 * its current schedule: bytes every data point needs (the data columns, y
 * entries and outputs the generated code really reads or writes after dead
 * code is removed) plus each distinct entry of x, v and theta it reads, once.
 * callback: 0 obj, 1 grad, 2 cons, 3 jac, 4 hess, 5 jprod, 6 jtprod,
 * 7 hprod, 8 adjoint (the order of exa_counters), 9 jac_hess.  Host-only
 * models report the unfused schedule. */
exa_status exa_kernel_bytes(const exa_model* m, int32_t callback, int64_t* read_bytes,
                            int64_t* write_bytes);
/* The schedule a callback's kernel uses: out4 = workgroup size, points per
 * lane, fused (bit 0) | unstaged stores (bit 1), number of tiles. */
exa_status exa_schedule(const exa_model* m, int32_t callback, int64_t* out4);

/* Layout of pattern p (declaration position): out8 = kind, ndata, o1step,
 * o2step, number of unique parameter references, o0 (first row / term / aug
 * entry), o1 (first Jacobian entry, or first gradient-buffer entry for an
 * objective), o2 (first Hessian entry) -- the SIMDFunction offsets and strides
 * of Sec. 3.4, 0-based. */
exa_status exa_pattern_info(const exa_model* m, int32_t p, int64_t* out8);

/* Device memory of a model in bytes: what it holds (device models) or the
 * footprint estimated from the host analysis (host-only models: data
 * columns, tables, work buffers, reduction maps), into *bytes. */
exa_status exa_device_bytes(const exa_model* m, int64_t* bytes);
/* Build statistics of a model (Sec. 8.6 compilation study), host array
 * out6 = {host analysis ms, code generation ms, compilation ms (or cache
 * read), origin of the code object (0 compiled, 1 read from the on-disk
 * cache, 2 shared with a live model of the same pattern set, -1 host-only),
 * device bytes (as exa_device_bytes), 1 when a cache directory is in use}. */
exa_status exa_build_info(const exa_model* m, double* out6);

/* Callback counters (Sec. 3.2 NLPModels.Counters): out[0..8] = obj, grad,
 * cons, jac, hess, jprod, jtprod, hprod, adjoint. */
exa_status exa_counters(const exa_model* m, int64_t* out9);

/* ---- Batched evaluation (Sec. 7.4.3 batch models, generalised) ----------
 *
 * B models that share every pattern tree (the same description up to data
 * sizes and values: instances of one formulation, which also agree on which
 * patterns have no data points) are evaluated together: every selected
 * callback of every instance in ONE evaluation launch over a tile list of
 * (instance, unit, data range) tiles, one workgroup per tile, with the
 * instances binned over the 8 XCDs by cost (or, with EXA_UNITS_SEPARATE,
 * one such launch per callback, one after another); then ONE launch of every
 * instance's deterministic reductions (gradient, J^T w, H v, parameter
 * adjoint segment sums, objective partials), plus one small launch when a
 * segment is longer than 1024 entries.  The launches are recorded once into
 * a HIP graph and replayed (re-recorded when the call's pointers, sigma, mask
 * or schedule change).  Instance sizes may differ.  The batch keeps
 * references to the models, which must outlive it; it reads their data,
 * maps and compiled code and owns its own work buffers and parameter copy.
 *
 * Concatenated arrays: an input or output of the batch is the concatenation
 * of the per-instance arrays in instance order; exa_batch_offsets gives, for
 * i = 0..B, the start of instance i in arrays of nvar (x, v, g, jtw, hv, lag,
 * wx), ncon (y, w, c, jv), nnzj (jac), nnzh (hess) and ntheta (theta,
 * theta_bar) entries: offsets[5*i + 0..4]; row B holds the totals.  The
 * objective output f holds one value per instance.
 *
 * Every instance's outputs are bit-identical to its own single-instance
 * callbacks (exa_obj, exa_grad, exa_cons, exa_jac_coord, exa_hess_coord,
 * exa_jprod, exa_jtprod, exa_hprod, exa_lag_grad, exa_adjoint_theta) at
 * the batch's parameters: each data point is evaluated by the same code,
 * and each reduction sums the same entries in the same order.
 */
typedef struct exa_batch_options {
    int32_t autotune;  /* 1: at the first call with a mask, time the candidate
                          schedules (workgroup size, points per lane, fused or
                          separate patterns, units) and keep the fastest      */
    int32_t block;     /* schedule without autotune: workgroup size (0: 256)   */
    int32_t epl;       /*   points per lane 1..16 (0: 4)                       */
    int32_t fuse;      /*   1: patterns over the same data arrays share a lane */
    int32_t units;     /*   EXA_UNITS_* (a choice a mask does not allow falls
                            back to the next one down; EXA_UNITS_SEPARATE to
                            per-callback tiles)                                */
    int32_t use_graph; /* 1: replay the launches from a HIP graph              */
    int32_t xcd_aware; /* 1: instances are split over the 8 XCDs by cost and
                          each XCD takes its instances' tiles (an instance's x
                          stays in that XCD's L2); 0: tiles in instance order  */
    int32_t reserved;
} exa_batch_options;

/* Batched-only selection bits, beside the EXA_EV_* callbacks:
 *   EXA_EV_LAG  lag       [nvar]   sigma grad f + J^T y from x, y, sigma
 *                                  (as exa_lag_grad); not with EXA_EV_GRAD
 *                                  or EXA_EV_JTPROD in the same call
 *   EXA_EV_ADJ  theta_bar [ntheta] from x, y, sigma, wx (as
 *                                  exa_adjoint_theta with w = wx); its tiles
 *                                  run in a second evaluation launch */
#define EXA_EV_LAG (1u << 8)
#define EXA_EV_ADJ (1u << 9)
#define EXA_BATCH_ALL 0x3ffu

/* Inputs and outputs of exa_batch_eval: device arrays, concatenated over
 * the instances (see above).  Inputs a mask does not need may be NULL,
 * outputs it selects may not; outputs must not overlap each other or the
 * inputs. */
typedef struct exa_batch_io {
    const double* x;   /* [sum nvar]   the point                              */
    const double* y;   /* [sum ncon]   multipliers (hess, hprod, lag, adj)    */
    double obj_weight; /* sigma, the same for every instance                  */
    const double* v;   /* [sum nvar]   direction of jprod and hprod           */
    const double* w;   /* [sum ncon]   weights of jtprod                      */
    const double* wx;  /* [sum nvar]   cotangent of the parameter adjoint     */
    double* f;         /* [B]          objective values                       */
    double* g;         /* [sum nvar]   gradients                              */
    double* c;         /* [sum ncon]   constraint values                      */
    double* jac;       /* [sum nnzj]   Jacobian values                        */
    double* hess;      /* [sum nnzh]   Hessian values                         */
    double* jv;        /* [sum ncon]   J v                                    */
    double* jtw;       /* [sum nvar]   J^T w                                  */
    double* hv;        /* [sum nvar]   H v                                    */
    double* lag;       /* [sum nvar]   sigma grad f + J^T y                   */
    double* theta_bar; /* [sum ntheta] (d grad_x L / d theta)^T wx            */
} exa_batch_io;

/* Errors: EXA_EINVAL for B < 1, a NULL model or handle, models that do not
 * share their pattern trees, or a bad option; EXA_ESTATE for a host-only
 * model; EXA_ENOMEM, EXA_EHIP.  The batch's parameters start as a copy of
 * each model's device parameters at create. */
exa_status exa_batch_create(exa_model* const* models, int32_t B, const exa_batch_options* opt,
                            exa_batch** out);
exa_status exa_batch_destroy(exa_batch* b);
/* Host array offsets [5*(B+1)], see above. */
exa_status exa_batch_offsets(const exa_batch* b, int64_t* offsets);
/* Replace the batch's parameters: theta device [sum ntheta], copied on
 * `stream` (the models' own parameters are not changed). */
exa_status exa_batch_set_theta(exa_batch* b, const double* theta, exa_stream_t stream);
/* Evaluate the callbacks selected by `mask` (EXA_EV_* and the batched-only
 * bits above) for every instance.  The first call with a mask builds its
 * tile list and reduction table, allocates the work buffers it needs and,
 * with autotune, times candidate schedules (synchronizing the stream).  A
 * call that repeats the previous call (same mask, pointers, sigma and
 * schedule) records the launches into a HIP graph, and later calls that
 * match it are one graph launch on `stream`; a call with other arguments
 * launches directly (arguments that change at every call cost no
 * recording).
 * Errors: EXA_EINVAL for a NULL batch or io, an empty or unknown mask, LAG
 * with GRAD or JTPROD, a NULL pointer the mask needs, or GRAD or LAG over
 * instances that disagree on whether every variable has at most one
 * objective term (their gradients are written differently). */
exa_status exa_batch_eval(exa_batch* b, uint32_t mask, const exa_batch_io* io, exa_stream_t stream);
/* Algorithmic traffic of a mask under its current schedule (the batch's
 * default before the mask's first call), summed over the instances as
 * exa_eval_bytes counts one model: out4 = bytes read and written by the
 * evaluation launch(es), bytes read and written by the reduction launch. */
exa_status exa_batch_bytes(const exa_batch* b, uint32_t mask, int64_t* out4);
/* Schedule of a mask: out6 = workgroup size, points per lane, fused (0/1),
 * units (EXA_UNITS_*, | EXA_UNSTAGED), number of evaluation tiles, the autotuner's best
 * evaluation-launch time in nanoseconds (0 if not tuned).  EXA_ESTATE before
 * the mask's first call. */
exa_status exa_batch_schedule(const exa_batch* b, uint32_t mask, int64_t* out6);
/* Fix a mask's schedule instead of tuning it (for measurement: a profiled
 * run can use the schedule an unprofiled run chose).  Errors: EXA_EINVAL for
 * a bad mask or value. */
exa_status exa_batch_set_schedule(exa_batch* b, uint32_t mask, int32_t block, int32_t epl, int32_t fused,
                                  int32_t units);
/* Launch timing, for measurement: with enable != 0 the next 1024
 * exa_batch_eval calls launch directly (not from the graph) and record HIP
 * events on their stream around the evaluation launch and around the
 * reduction launch; enable == 0 frees the events and returns to graph
 * replay.  exa_batch_timing_read waits for the recorded calls and stores
 * {calls, average evaluation launch in us, reduction launches, their
 * average in us} into the host array out4, then starts a new recording.
 * EXA_ESTATE when timing is off. */
exa_status exa_batch_timing(exa_batch* b, int32_t enable);
exa_status exa_batch_timing_read(exa_batch* b, double* out4);

#ifdef __cplusplus
}
#endif
#endif /* EXA_H */
