/*
 * coot.h — C ABI of libcoot, a fused dense-expression engine for MI355X (gfx950).
 *
 * What it computes.  An Armadillo-style expression over dense matrices — the
 * element-wise node kinds eOp / eGlue and the dimension-changing Op<.., op_trans>
 * of the paper's Section 3 ("Internal Design") — is handed over as a postfix list
 * and evaluated on assignment (delayed evaluation, Section 3) as ONE fused pass
 * over device memory, or closed by a reduction: accu (sum of all elements, the
 * sum(A) of Fig. 1 and Section 5 task 1), sum along a dimension, dot, norm.
 * The axpy update y <- a*x + y of Sections 1 and 5 (task 2) is the expression
 * SCALAR LOAD(x) SCHUR LOAD(y) ADD written into y.
 *
 * Conventions that hold for every call:
 *   - Every function returns coot_status; nothing throws across the ABI.  On an
 *     error, coot_last_error() returns a message (thread-local, valid until the
 *     next coot_* call on the same thread).
 *   - Matrices are column-major (Section 2 gives the Armadillo API; Armadillo
 *     stores column-major): element (i, j) of an operand is at
 *     data + (i + j * ld) * sizeof(eT), with ld >= n_rows.  A Col is n x 1,
 *     a Row is 1 x n.
 *   - All data pointers are DEVICE pointers on the device selected by coot_init
 *     (the paper keeps all matrix data in GPU memory, Section 4).  They are owned
 *     by the caller and must stay valid until the work queued on `stream` has
 *     finished.  `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Work is queued asynchronously on `stream`; device faults surface at the
 *     caller's next synchronisation, as in HIP.
 *   - Handles (coot_expr, coot_batch) are owned by the library and freed with the
 *     matching *_release call.  Compiled code objects are cached process-wide per
 *     expression signature (in memory and in COOT_CACHE_DIR, default
 *     ~/.cache/coot), the analogue of the kernel cache of Section 4.
 *   - Scalars are passed as double and converted to the element type at launch:
 *     round-to-nearest for f32, exact for f64, truncation toward zero then
 *     reduction mod 2^32 for u32 / s32.
 *   - Floating-point semantics: IEEE binary32 / binary64, round-to-nearest-even,
 *     subnormals kept, no contraction of a*b+c into an FMA, correctly rounded
 *     division and square root.  Integer arithmetic wraps mod 2^32.
 */
#ifndef COOT_H
#define COOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
typedef enum {
  COOT_OK = 0,
  COOT_EINVAL = -1,       /* malformed argument (NULL handle, bad enum, bad slot index) */
  COOT_ESHAPE = -2,       /* element-wise operands of unequal dimensions, wrong output dims */
  COOT_ETYPE = -3,        /* mixed element types, or an operation illegal for the type */
  COOT_EALIAS = -4,       /* output overlaps an operand in a way one pass cannot honour */
  COOT_ECOMPILE = -5,     /* runtime compilation failed (the log is in coot_last_error) */
  COOT_EHIP = -6,         /* a HIP runtime call failed */
  COOT_ENOMEM = -7,       /* device workspace could not be allocated */
  COOT_EUNSUPPORTED = -8  /* valid request outside what the library implements */
} coot_status;

/* ---- element types and operand kinds (Section 2: Mat<eT>, Col, Row) ------ */
typedef enum { COOT_U32 = 0, COOT_S32 = 1, COOT_F32 = 2, COOT_F64 = 3, COOT_F16 = 4, COOT_BF16 = 5 } coot_dtype;
/* COOT_F16 (IEEE binary16) and COOT_BF16 (bfloat16: binary32's exponent range,
 * 8 significant bits) are 16-bit storage types: operands and results are stored
 * in 16 bits, every operator computes in binary32 and its result is rounded to
 * the storage type (nearest-even), which is the correctly rounded 16-bit result
 * (for bf16 while the binary32 result is normal).  Scalars are rounded to the
 * storage type.  Reductions accumulate in compensated binary32 (float-float) and
 * round the result once to the storage type.  Batches and the cost model take
 * f32 / f64 only (COOT_EUNSUPPORTED). */
typedef enum { COOT_MAT = 0, COOT_COL = 1, COOT_ROW = 2, COOT_BCAST = 3 } coot_kind;
/* COOT_BCAST: a column vector of n_rows contiguous elements read as an n_rows x
 * n_cols matrix whose every column is that vector (Armadillo's each_col()
 * broadcasting: the index map's column stride is 0); ld must be 0.  A row
 * vector broadcast down the rows is the trans() of such an operand.  Broadcast
 * operands are read through the tiled kernels, never written, and are not taken
 * by batches (COOT_EUNSUPPORTED). */

/* ---- postfix opcodes (Section 3: eOp, eGlue and Op<.., op_trans>) -------- */
typedef enum {
  COOT_OP_LOAD = 0,    /* push operand slot `arg` */
  COOT_OP_SCALAR = 1,  /* push scalar slot `arg` (broadcast) */
  COOT_OP_ADD = 2,     /* eGlue: pop b, pop a, push a + b */
  COOT_OP_SUB = 3,     /*        a - b */
  COOT_OP_SCHUR = 4,   /*        a % b (element-wise product) */
  COOT_OP_DIV = 5,     /*        a / b (floating types only) */
  COOT_OP_NEG = 6,     /* eOp:  -a */
  COOT_OP_ABS = 7,     /*        |a| (abs(INT32_MIN) = INT32_MIN) */
  COOT_OP_EXP = 8,     /*        exp(a) (floating types only) */
  COOT_OP_LOG = 9,     /*        log(a) (floating types only) */
  COOT_OP_SQRT = 10,   /*        sqrt(a) (floating types only) */
  COOT_OP_SQUARE = 11, /*        a * a */
  COOT_OP_TRANS = 12   /* Op<op_trans>: transpose (an index map, never a pass of its own) */
} coot_opcode;

typedef struct {
  int32_t code;  /* coot_opcode */
  uint32_t arg;  /* slot index for LOAD / SCALAR, 0 otherwise */
} coot_op;

typedef struct {
  int32_t dtype; /* coot_dtype: every slot of one expression has the same type */
  int32_t kind;  /* coot_kind */
} coot_slot_type;

typedef struct {
  void* data;     /* device pointer, column-major */
  int64_t n_rows;
  int64_t n_cols;
  int64_t ld;     /* leading dimension in elements, >= n_rows (0 means n_rows; COOT_BCAST: 0) */
  int32_t dtype;  /* coot_dtype */
  int32_t kind;   /* coot_kind */
} coot_operand;

/* Launch configuration.  Any field 0 = chosen by the library.
 *   vec       elements per access group: 1, 2 or 4 (8 for 16-bit types: 16 bytes)
 *   ept       vector groups per thread per loop trip: 1, 2, 4 or 8 (flat kernels)
 *   waves     64-lane wavefronts per workgroup: 1, 2, 4 or 8 (flat kernels; the tiled
 *             kernels run 4)
 *   grid_mult workgroups per compute unit for grid-stride kernels: 1..16; for a
 *             reduction along a dimension, the tiles per CU past which each
 *             workgroup folds a longer segment of tiles (default 8)
 *   tile_r, tile_c  output tile of the tiled kernels (transposed or strided leaves,
 *             dimension reductions), rows x columns: powers of two in [8, 256] with
 *             1024 <= tile_r * tile_c <= 8192, both given or both 0; the staged
 *             transposed leaves must fit 64 KiB of LDS (tile_r * (tile_c + 1) elements
 *             of the compute type each), else COOT_EINVAL.  A tall tile gives the
 *             untransposed operands longer contiguous segments, a wide one the
 *             transposed operands.  The vector width is capped at
 *             tile_r * tile_c / 256.  Default 32 x 32 below 2^22 elements and
 *             64 x 64 from there (the expression's rows x columns), 64 x 32 for a
 *             reduction along a dimension, 64 x 64 for 16-bit types (32 x 32 when
 *             its staging would not fit); with neither given and even 32 x 32
 *             staging beyond 64 KiB (8 or more transposed fp64 leaves, 16 fp32)
 *             COOT_EUNSUPPORTED.  Flat kernels ignore them. */
typedef struct {
  uint16_t vec;
  uint16_t ept;
  uint16_t waves;
  uint16_t grid_mult;
  uint16_t tile_r;
  uint16_t tile_c;
} coot_launch_cfg;

typedef enum {
  COOT_RED_ACCU = 0, /* sum of all elements -> 1 element */
  COOT_RED_SUM = 1,  /* sum along dim: 0 -> 1 x n_cols (per column), 1 -> n_rows x 1 (per row) */
  COOT_RED_DOT = 2,  /* dot(a, b): the expression's root must be a % b -> 1 element */
  COOT_RED_NORM = 3, /* 2-norm (Frobenius for a matrix) -> 1 element; floating types only */
  COOT_RED_MIN = 4,  /* smallest element -> 1 element; NaN if any element is NaN */
  COOT_RED_MAX = 5,  /* largest element -> 1 element; NaN if any element is NaN */
  COOT_RED_MEAN = 6, /* sum / number of elements -> 1 element; floating types only */
  COOT_RED_NORM1 = 7,  /* sum of |x| (1-norm of the elements as a vector); floating types only */
  COOT_RED_NORMINF = 8, /* largest |x| (infinity norm of the elements); floating; NaN if any is NaN */
  COOT_RED_MEAN_DIM = 9, /* mean along dim (shapes as SUM); floating types only */
  COOT_RED_VAR = 10,     /* variance of all elements -> 1 element; floating types only */
  COOT_RED_VAR_DIM = 11  /* variance along dim (shapes as SUM); floating types only */
} coot_red;

/* compile flags */
#define COOT_CF_UNFUSED 0x1u   /* evaluate one kernel and one temporary per operator (comparator) */
/* reduce flags */
#define COOT_RF_PLAIN 0x1u     /* uncompensated fp32/fp64 accumulation (comparator) */
#define COOT_RF_VAR_N 0x2u     /* VAR, VAR_DIM: divide by the count N instead of N - 1 */
/* prepare flag: compile into the in-memory and on-disk code-object caches only,
 * without loading the code object (no device work: usable without a GPU, e.g. from
 * helper processes that fill the on-disk cache) */
#define COOT_PF_COMPILE_ONLY 0x100u

typedef struct coot_expr coot_expr;
typedef struct coot_batch coot_batch;

/* Select the HIP device used by this thread and later calls (the coot_init of
 * Section 2, Fig. 2, reduced to the one HIP backend).  Safe to call repeatedly.
 * Errors: COOT_EHIP if the device cannot be selected. */
coot_status coot_init(int hip_device);

/* Device memory for the library's workspaces (reduction partials) and the
 * unfused comparator's temporaries comes from alloc / dealloc when given (for
 * example the caller's caching allocator), else from hipMalloc / hipFree.
 * alloc(bytes, stream, ctx) returns device memory usable in stream order on
 * `stream` (NULL: COOT_ENOMEM for the call that needed it); dealloc(ptr, stream,
 * ctx) returns it in stream order.  The call waits for the device, hands every
 * held buffer back to the allocator that provided it, then installs the new
 * one; give both functions or neither (back to hipMalloc).  Batches, models and
 * code objects keep using hipMalloc.  Errors: COOT_EINVAL (one function NULL, or
 * called while a comparator temporary is in use), COOT_EHIP. */
typedef void* (*coot_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*coot_free_fn)(void* ptr, void* stream, void* ctx);
coot_status coot_set_allocator(coot_alloc_fn alloc, coot_free_fn dealloc, void* ctx);

/* Validate and analyse a postfix expression (Section 3: the whole expression is
 * analysed before any work is issued).
 *   ops[n_ops]         postfix list
 *   slots[n_slots]     dtype and kind of each operand slot (n_slots <= 16)
 *   n_scalars          number of scalar slots (<= 32)
 *   flags              0 or COOT_CF_UNFUSED
 *   out                receives a new handle (library-owned)
 * Checks arity, one dtype for all slots, operations legal for the dtype, slot
 * indices; computes each leaf's transpose parity.  No device work and no
 * compilation happens here; code is generated and compiled on first use, or
 * ahead of time with coot_expr_prepare.
 * Errors: COOT_EINVAL, COOT_ETYPE. */
coot_status coot_expr_compile(const coot_op* ops, uint32_t n_ops, const coot_slot_type* slots,
                              uint32_t n_slots, uint32_t n_scalars, uint32_t flags, coot_expr** out);

/* Generate and compile (or fetch from the cache) the code a later call will
 * need, so that compilation stays outside timed regions (the paper's timings
 * exclude kernel compilation, Section 5).
 *   mode  -1 = element-wise eval, otherwise a coot_red value
 *   dim   for COOT_RED_SUM, MEAN_DIM and VAR_DIM: 0 or 1, else ignored
 *   rflags COOT_RF_PLAIN or 0, optionally | COOT_PF_COMPILE_ONLY
 *   cfg   launch configuration the call will use (NULL = library default)
 * Errors: COOT_EINVAL, COOT_ECOMPILE, COOT_EHIP. */
coot_status coot_expr_prepare(coot_expr* e, int32_t mode, int32_t dim, uint32_t rflags,
                              const coot_launch_cfg* cfg);

/* Output dimensions of the element-wise result for the given operands.
 * Errors: COOT_ESHAPE if element-wise operands disagree, COOT_EINVAL. */
coot_status coot_expr_out_shape(const coot_expr* e, const coot_operand* operands, int64_t* n_rows,
                                int64_t* n_cols);

/* Evaluate the expression element-wise into `out` in one fused pass.
 *   operands[n_slots]  device operands matching the compiled slot types
 *   scalars[n_scalars] host values
 *   out                caller-allocated device output with the inferred dims
 *   cfg                NULL = library default / tuned choice
 * `out` may be the same buffer as an operand that is read untransposed with the
 * same layout (y = 2.5*x + y, B += 3*A): every element is read before it is
 * written by the same thread.  Any other overlap gives COOT_EALIAS.
 * The fused evaluation takes no workspace and may be recorded into a HIP graph
 * (stream capture) once its code is loaded (a first call or coot_expr_prepare
 * outside the capture); the unfused comparator's temporaries may not.
 * Errors: COOT_EINVAL, COOT_ESHAPE, COOT_ETYPE, COOT_EALIAS, COOT_ECOMPILE,
 * COOT_EHIP, COOT_ENOMEM (unfused temporaries), COOT_EUNSUPPORTED (the unfused
 * comparator on a stream that is capturing). */
coot_status coot_expr_eval(coot_expr* e, const coot_operand* operands, const double* scalars,
                           coot_operand* out, const coot_launch_cfg* cfg, void* stream);

/* Close the expression with a reduction, fused with its evaluation.
 *   kind, dim   see coot_red; dim ignored except for SUM, MEAN_DIM and VAR_DIM
 *   flags       0 (compensated: float-float / double-double per-lane sums) or
 *               COOT_RF_PLAIN (uncompensated comparator); | COOT_RF_VAR_N for a
 *               variance normalised by N (default N - 1, Armadillo's norm_type 0)
 *   out         device output of the expression's dtype: 1 element for a full
 *               reduction; 1 x n_cols along dim 0; n_rows x 1 along dim 1
 * accu of an expression whose root is a % b is evaluated as dot (the product
 * error is carried, not rounded away).  Integer sums wrap mod 2^32.  MEAN and
 * NORM1 use the compensated sum (MEAN divides it by the element count in
 * binary64 and rounds once); MIN, MAX and NORMINF are exact (an element value).
 * Statistics (the paper lists mean and variance among the functions, Section 2):
 * MEAN_DIM divides each compensated sum by the count along dim.  VAR and VAR_DIM
 * are one pass over the expression: moments about a shift taken from the data
 * (VAR: each lane's first value, the lanes' and workgroups' (count, mean, M2)
 * merged by Chan's formula in binary64; VAR_DIM: each output's first element,
 * shared by all segments, M2 = S2 - S1^2 / N in binary64), with exact differences
 * and squares summed float-float.  M2 is divided by N - 1 (or N) in binary64 and
 * rounded once.  A count of 1 gives 0 for either normalisation.  Inf or NaN
 * elements give NaN.
 * The result is deterministic: a fixed combine order and no floating-point
 * atomics.  Workspace is taken from a per-stream cache owned by the library,
 * which a later call may free and reallocate: a stream that is capturing is
 * refused (COOT_EUNSUPPORTED), since a replayed graph would read freed memory.
 * Errors: as coot_expr_eval; COOT_EUNSUPPORTED under stream capture; COOT_ETYPE for NORM, MEAN, NORM1, NORMINF of an
 * integer expression (and for MEAN_DIM, VAR, VAR_DIM); COOT_EINVAL for DOT whose
 * root is not a Schur product, for MIN, MAX, MEAN, VAR of an empty expression and
 * for COOT_RF_VAR_N with another kind. */
coot_status coot_reduce(coot_expr* e, const coot_operand* operands, const double* scalars,
                        int32_t kind, int32_t dim, uint32_t flags, coot_operand* out,
                        const coot_launch_cfg* cfg, void* stream);

/* coot_reduce for callers that cannot allocate device memory: code recorded into a
 * HIP graph (stream capture), tight serving loops, harnesses that forbid hipMalloc.
 * Arguments, results and errors are those of coot_reduce, computed by the same
 * kernels, bit for bit.  The partial results live in a file-scope device array of
 * COOT_NOALLOC_SCRATCH_BYTES (16 MiB) that every device the library runs on holds
 * until the process ends (its address is looked up by coot_init, else by the first
 * call on a device).  The call allocates nothing, compiles nothing and loads nothing:
 *   - the reduction's kernels must be loaded already: run coot_expr_prepare (same
 *     kind, dim and flags) or one coot_reduce with the same expression, kind and
 *     operand layout first; otherwise COOT_EINVAL;
 *   - the partials must fit in half of the array each (full reductions always do;
 *     along a dimension about 2 * n_outputs * n_segments elements of the compute
 *     type): COOT_EUNSUPPORTED otherwise, with nothing launched;
 *   - the unfused comparator (COOT_CF_UNFUSED) is refused with COOT_EUNSUPPORTED.
 * A capturing stream is accepted.  Every call on one device shares that device's
 * array and each call's kernels start by writing what they later read, so calls
 * ordered on one stream are safe; calls that overlap in time on one device (other
 * streams, host threads, graph replays) race on the array and give wrong results. */
#define COOT_NOALLOC_SCRATCH_BYTES (16u << 20)
coot_status coot_reduce_noalloc(coot_expr* e, const coot_operand* operands, const double* scalars,
                                int32_t kind, int32_t dim, uint32_t flags, coot_operand* out,
                                const coot_launch_cfg* cfg, void* stream);

/* Two statements in one pass (multi-statement fusion): evaluate e into out and
 * close the expression r with a full reduction into r_out, reading every operand
 * once and writing out once (y = 2.5*x + y; d = accu(x % y) moves 12 bytes per
 * element instead of 20).  The statement pair extends the whole-expression
 * analysis of Section 3 across two assignments.
 *   operands, scalars  e's operands and scalars, as in coot_expr_eval
 *   out                e's output (it may alias an operand as in coot_expr_eval)
 *   r_src[k]           r's operand slot k: an index into `operands` (read as
 *                      loaded, before out is written) or -1 for the value of e just
 *                      computed (read as out's layout)
 *   r_scalars          r's scalars (host)
 *   kind               COOT_RED_ACCU (DOT when r's root is a % b), DOT, MIN, MAX,
 *                      MEAN, NORM1, NORMINF; r_out: one element of the dtype
 * Both statements must take the flat kernels: every leaf untransposed and
 * contiguous, out contiguous, the same shape; r may read only operands that e
 * reads.  Errors: as coot_expr_eval and coot_reduce; COOT_EUNSUPPORTED under
 * stream capture (workspace, as coot_reduce), for transposed or strided leaves, SUM / NORM, more than 32 scalars in the pair, or
 * compile-flagged comparators. */
coot_status coot_expr_eval_reduce(coot_expr* e, const coot_operand* operands, const double* scalars, coot_operand* out,
                                  coot_expr* r, const int32_t* r_src, const double* r_scalars, int32_t kind,
                                  coot_operand* r_out, const coot_launch_cfg* cfg, void* stream);

/* Release a handle from coot_expr_compile.  NULL is ignored. */
void coot_expr_release(coot_expr* e);

/* Name of the kernel (family + signature hash + variant) a call with these
 * arguments and launch configuration (NULL = library default) would launch
 * first, for attributing profiler traces.  Writes at most `cap` bytes including
 * the terminator.  Errors: COOT_EINVAL. */
coot_status coot_expr_kernel_name(coot_expr* e, int32_t mode, int32_t dim, const coot_launch_cfg* cfg, char* buf,
                                  size_t cap);

/* ---- batches: many small independent expressions in one launch ----------
 * Section 4 of the paper notes that GPUs need enough parallel work and are
 * ill-suited to small matrices; a batch fills the device with thousands of small
 * expressions at once.  Every expression is cut into TS x TS output tiles; one
 * persistent kernel walks the list of all tiles and interprets each
 * expression's register bytecode; the launch is captured into a HIP graph.
 * f32 or f64 only (one type per batch).  Transposed leaves are staged through LDS.
 *
 * coot_batch_create
 *   exprs[n]            compiled expressions (borrowed: they may be released after this call)
 *   operands[n][...]    each expression's device operands (n_slots of it)
 *   scalars[n][...]     each expression's scalars (host, copied)
 *   outs[n]             caller-allocated device outputs with the inferred dims
 *   cfg                 NULL = default (flat chunks and 2-D tiles of 32 x 32
 *                       elements, vectorised where aligned, 16 workgroups per
 *                       CU); else, for both parts: tile_r = tile_c = 16 or 32 the
 *                       tile edge and waves the wavefronts per tile (16 x 16: 1;
 *                       32 x 32: 4, 2 or 1, i.e. 4, 8 or 16 elements per thread);
 *                       without a tile, waves 1 / 2 / 4 select 16 x 16 by one wave,
 *                       32 x 32 by two, 32 x 32 by four; vec = 1 forbids 128-bit
 *                       accesses; grid_mult sets workgroups per CU.  Expressions with
 *                       untransposed contiguous leaves are cut into flat chunks of
 *                       the same element count and run in a launch of their own
 *                       (the flat part); the others in 2-D tiles (the 2-D part).
 *   stream              unused at creation (descriptors are uploaded synchronously)
 * All operand and output buffers must stay allocated, at the same addresses, for
 * the life of the batch: their addresses are baked into the descriptors.  The
 * graph runs the two parts side by side (fork / join on two captured streams).
 * The kernel addresses each operand and output as a raw buffer with 32-bit byte
 * offsets, so each must span less than 2 GiB (else COOT_EUNSUPPORTED).
 * Errors: COOT_EINVAL, COOT_ESHAPE, COOT_ETYPE, COOT_EALIAS, COOT_EUNSUPPORTED
 * (integer types, more than 12 leaves, more than 8 registers, an operand of 2 GiB
 * or more), COOT_ENOMEM, COOT_EHIP. */
coot_status coot_batch_create(uint32_t n, coot_expr* const* exprs, const coot_operand* const* operands,
                              const double* const* scalars, const coot_operand* outs,
                              const coot_launch_cfg* cfg, void* stream, coot_batch** out);

/* Replay the captured graph on `stream` (one launch for the whole batch). */
coot_status coot_batch_launch(coot_batch* b, void* stream);

/* Comparator: the same kernel launched once per expression on `stream`. */
coot_status coot_batch_launch_each(coot_batch* b, void* stream);

/* Autotune the batch launch on `stream` (synchronises it).  The flat-chunk part
 * and the 2-D-tile part of the batch are tuned separately, each on its own
 * launch: every tile shape (16 x 16 by one wavefront; 32 x 32 by four, two or
 * one wavefront(s), i.e. 4, 8 or 16 elements per thread), grid multiplier
 * (2, 4, 8, 16) and vector width (128-bit where aligned, or scalar), median of 5
 * launches each; the
 * fastest of each part is kept.  Then the whole graph is timed with the parts
 * side by side and one after the other, and the faster is captured.  best (may
 * be NULL) receives the flat part's settings (coot_batch_info reports both
 * parts); best_us (may be NULL) the median time of the captured graph. */
coot_status coot_batch_tune(coot_batch* b, void* stream, coot_launch_cfg* best, float* best_us);

/* info[0] expressions, [1] tiles, [2] algorithmic bytes (each distinct operand
 * read once + outputs written once), [3] tile edge of the flat part (chunks of
 * edge^2 elements), [4] its grid, [5] expressions on the 128-bit path,
 * [6] expressions cut into flat chunks, [7] LDS stack entries per thread,
 * [8] transposed-leaf tiles staged in LDS per workgroup, [9] tile edge of the 2-D
 * part, [10] its grid, [11] tiles of the flat part (the work-list's first),
 * [12] 1 if the graph runs the two parts side by side, [13] / [14] elements per
 * thread / 4 of the flat / 2-D part (1, 2 or 4). */
coot_status coot_batch_info(const coot_batch* b, int64_t info[15]);

void coot_batch_release(coot_batch* b);

/* ---- autotuning of the fused kernels' launch configuration ----------------
 * A configuration is (vec, ept, waves, grid_mult, tile_r, tile_c).  vec, ept and
 * the tile select compile-time variants (one tuning module per expression
 * signature holds all of them), waves and grid_mult are launch parameters.
 * Expressions that take the tiled kernels (transposed or strided leaves, and every
 * reduction along a dimension) run 256-thread workgroups: vec, grid_mult and the
 * tile vary there (ept = 1, waves = 4 in their configurations).  Along a dimension,
 * grid_mult is the number of tiles per CU past which the library lengthens the
 * segments each workgroup folds (fewer partial results).
 * Tuning covers element-wise evaluation (mode -1), accu (mode COOT_RED_ACCU; dot
 * when the root is a % b) and sum / mean / variance along dim 0 or 1 (COOT_RED_SUM,
 * COOT_RED_MEAN_DIM, COOT_RED_VAR_DIM; dim is ignored for the others; a variance is
 * timed with its N - 1 stage 2). */

/* Write the configuration space of a kernel family (0 flat, 1 tiled) into
 * cfgs[0..cap) and return its size (cfgs may be NULL to query the size).
 * Flat: vec {1,2,4} x ept {1,2,4,8} x waves {1,2,4,8} x grid_mult {2,4,8,16} = 192
 * (tile 0 x 0); tiled: tile {64x64, 128x32, 32x128, 256x16, 128x64, 32x32, 64x16,
 * 16x64, 128x8, 256x8, 128x16, 64x32} x vec {1,2,4} x grid_mult {2,4,8,16} = 144 (a
 * tile whose transposed-leaf staging
 * exceeds 64 KiB, or whose vec exceeds tile_r * tile_c / 256, cannot run).  For the 16-bit types vec 8
 * (16-byte groups) is valid too: their tuning modules hold those variants,
 * coot_tune_table accepts them (NaN for other types) and coot_tune's exhaustive
 * policy adds them to this space. */
uint32_t coot_tune_space(int32_t family, coot_launch_cfg* cfgs, uint32_t cap);

/* Compile (or fetch) the tuning module for these operands without a device and
 * report which family (0 flat, 1 tiled) the expression takes.  Safe to call from
 * several host threads at once (compilation runs outside the library's lock).
 * Errors: COOT_EINVAL, COOT_ESHAPE, COOT_ECOMPILE, COOT_EUNSUPPORTED (mode). */
coot_status coot_tune_prepare(coot_expr* e, const coot_operand* operands, int32_t mode, int32_t dim,
                              int32_t* family);

/* runnable[k] = 1 when configuration k can run on these operands (its vector
 * width fits their alignment, leading dimensions and, for the tiled family, the
 * tile), else 0; no device work.  out is needed for mode -1 (element-wise).
 * Errors: as coot_tune_prepare, COOT_EINVAL for an invalid configuration. */
coot_status coot_tune_runnable(coot_expr* e, const coot_operand* operands, const coot_operand* out, int32_t mode,
                               int32_t dim, const coot_launch_cfg* cfgs, uint32_t n_cfgs, int32_t* runnable);

/* Time each configuration: one warm-up launch each, then `reps` rounds (1..101),
 * each round timing every configuration once with HIP events on `stream` around
 * enough back-to-back launches to span 40 us (the per-launch time of a repeated
 * call, launch overhead included); flush != 0 instead times single launches, each
 * after a 512 MiB write that evicts L2 and the Infinity Cache.  times_us[k] =
 * median per launch, or NaN when the configuration cannot run on these operands
 * (e.g. vec not allowed by alignment).
 * Synchronises the stream.  out receives the result as in coot_expr_eval /
 * coot_reduce.  Errors: as coot_expr_eval, COOT_EINVAL for an invalid configuration. */
coot_status coot_tune_table(coot_expr* e, const coot_operand* operands, const double* scalars, coot_operand* out,
                            int32_t mode, int32_t dim, const coot_launch_cfg* cfgs, uint32_t n_cfgs, uint32_t reps,
                            int32_t flush, float* times_us, void* stream);

/* Evaluate with an explicit configuration through the tuning module. */
coot_status coot_tune_launch(coot_expr* e, const coot_operand* operands, const double* scalars, coot_operand* out,
                             int32_t mode, int32_t dim, const coot_launch_cfg* cfg, void* stream);

/* ---- learned tuner: MLP cost model ------------------------------------------
 * A 3-Linear-layer ReLU network in -> h1 -> h2 -> 1, binary32, trained on the
 * device with masked mean-squared error and Adam (beta 0.9 / 0.999, eps 1e-8).
 * Parameters are one array: W1[h1][in], b1[h1], W2[h2][h1], b2[h2], W3[1][h2], b3.
 * Activations are sample-major (row b holds one sample's inputs). */
typedef struct coot_mlp coot_mlp;
typedef struct coot_costmodel coot_costmodel;

/* params_host: initial parameters (host, copied).  Errors: COOT_EINVAL, COOT_ENOMEM. */
coot_status coot_mlp_create(int32_t n_in, int32_t h1, int32_t h2, const float* params_host, coot_mlp** out);
uint32_t coot_mlp_num_params(const coot_mlp* m);
/* Copy the parameters / the last gradients to host memory (synchronous). */
coot_status coot_mlp_get_params(const coot_mlp* m, float* host);
coot_status coot_mlp_get_grads(const coot_mlp* m, float* host);
/* out[b] = network(X[b]) for X: B x n_in device array; out: B device floats. */
coot_status coot_mlp_forward(coot_mlp* m, const float* X, int32_t B, float* out, void* stream);
/* Forward + backward of L = inv_count * sum_b mask_b (out_b - y_b)^2 on device
 * arrays X (B x n_in), y, mask (B); gradients are kept for coot_mlp_adam_step;
 * loss (one device float, may be NULL) receives L. */
coot_status coot_mlp_backward(coot_mlp* m, const float* X, const float* y, const float* mask, int32_t B,
                              float inv_count, float* loss, void* stream);
/* One Adam update at step t >= 1 with bias correction. */
coot_status coot_mlp_adam_step(coot_mlp* m, float lr, float beta1, float beta2, float eps, int32_t t, void* stream);
/* Minibatch Adam over `epochs` passes of the N device samples (X, y, mask; mask_host
 * is the same mask on the host, used for each batch's normaliser); batches are a
 * seeded shuffle; losses_host[epoch] = mean batch loss.  Synchronises the stream. */
coot_status coot_mlp_train(coot_mlp* m, const float* X, const float* y, const float* mask, const float* mask_host,
                           int32_t N, int32_t batch, int32_t epochs, uint32_t seed, float lr, float* losses_host,
                           void* stream);
void coot_mlp_release(coot_mlp* m);

/* Feature vectors (n x 23, host) of an expression on an n_rows x n_cols shape for
 * each configuration: n_ops, n_operands, one-hot dtype (u32 s32 f32 f64),
 * log2(1+rows), log2(1+cols), n_trans, one-hot reduction red (0 none, 1 all,
 * 2 dim0, 3 dim1), log2 vec, log2 ept, log2 waves, log2 grid_mult, then the launch
 * the configuration implies for contiguous operands on 256 CUs: log2(1+elements),
 * tiled family (transposed leaves or a dimension sum: 256 threads per tile),
 * log2(workgroups), log2(1 + elements per thread), and log2(tile_r), log2(tile_c)
 * of the tiled family (64 x 64 when the configuration gives none; 0, 0 for flat). */
coot_status coot_costmodel_features(const coot_expr* e, int64_t n_rows, int64_t n_cols, int32_t red,
                                    const coot_launch_cfg* cfgs, uint32_t n, float* out);
/* Train a cost model on N host rows: feats (N x 23), target = log(time in us)
 * (any per-signature offset may be subtracted: only the ranking within a
 * signature matters), mask (1 = use the row).  Inputs and target are z-scored with
 * the training statistics (kept in the model).  The model is an ensemble of
 * n_models (1..16) networks; network k starts from init_params[k * P .. (k+1) * P)
 * (P parameters each, layout as for coot_mlp_create with n_in 23) and draws its
 * batches with seed + k.  losses (may be NULL): the networks' mean loss per epoch. */
coot_status coot_costmodel_train(const float* feats, const float* target, const float* mask, int32_t N,
                                 const float* init_params, int32_t n_models, int32_t h1, int32_t h2, int32_t epochs,
                                 int32_t batch, uint32_t seed, float lr, float* losses, void* stream,
                                 coot_costmodel** out);
/* Predicted time of each configuration (the exponential of the networks' mean
 * output; pred_us may be NULL) and the index of the smallest (lowest index on
 * ties).  Synchronises the stream. */
coot_status coot_costmodel_predict(coot_costmodel* cm, const coot_expr* e, int64_t n_rows, int64_t n_cols,
                                   int32_t red, const coot_launch_cfg* cfgs, uint32_t n, float* pred_us,
                                   uint32_t* best, void* stream);
coot_status coot_costmodel_save(const coot_costmodel* cm, const char* path);
coot_status coot_costmodel_load(const char* path, coot_costmodel** out);
void coot_costmodel_release(coot_costmodel* cm);

/* Pick a configuration for these operands: policy 0 the library default,
 * 1 exhaustive (every configuration timed, the fastest kept), 2 the cost model's
 * argmin over the configurations these operands allow where it is predicted at least
 * 5 % faster than the library default, else the default (cm required).  Timing is
 * that of coot_tune_table with 5 rounds and no flush (the per-launch time of
 * repeated calls); under policy 1 the finalists (within 5 % of the fastest, at
 * most 4) are timed again over 21 interleaved rounds, and of those within 2 % of the
 * fastest the one fastest in a launch after a cache flush (coot_tune_table's flush;
 * the 512 MiB flush buffer is allocated on first use) is kept.  best_us (may be
 * NULL) is the chosen configuration's repeated-call median.
 * The cost model (policy 2) covers element-wise evaluation and accu only
 * (COOT_EUNSUPPORTED along a dimension).  Synchronises the stream. */
coot_status coot_tune(coot_expr* e, const coot_operand* operands, const double* scalars, coot_operand* out,
                      int32_t mode, int32_t dim, int32_t policy, coot_costmodel* cm, coot_launch_cfg* best,
                      float* best_us, void* stream);

/* Queue on `stream` a read of a 512 MiB library buffer (allocated on first use and
 * kept), larger than the L2 caches and the Infinity Cache together: every line a
 * previous kernel left in them is evicted, so that the next kernel reads its operands
 * from HBM (cache-cold timing).  Errors: COOT_ENOMEM, COOT_EHIP. */
coot_status coot_flush_caches(void* stream);

/* The in-memory code-object cache (the kernel cache of Section 4, before the disk):
 * out[0] modules it holds, out[1] its capacity (least recently used modules are
 * evicted past it; environment variable COOT_MODULE_CACHE, default 1024), out[2]
 * evictions so far, out[3] modules that no expression holds any more, still loaded
 * on the device.  An evicted module stays usable by the expressions that hold it; a
 * later request for it is served from the disk cache.  Errors: COOT_EINVAL (NULL). */
coot_status coot_cache_info(int64_t out[4]);

/* Unload every module that no expression holds any more (out[3] above), each from
 * the device it was loaded on after waiting for that device to finish its work (the
 * calling thread's current device is kept); *unloaded (may be NULL)
 * receives how many.  A HIP graph recorded with kernels of a released expression must
 * not be replayed after this call.  Call it while no stream is capturing.
 * Errors: COOT_EHIP. */
coot_status coot_cache_trim(int64_t* unloaded);

/* Counters since process start: out[0] compiles, out[1] memory-cache hits,
 * out[2] disk-cache hits, out[3] launches, out[4] total compile milliseconds. */
void coot_stats(double out[5]);

const char* coot_last_error(void);

/* Diagnostic: write the HIP source generated for one request into buf (at most
 * cap bytes including the terminator) and, if compile != 0, compile it with
 * hipRTC for gfx950 and report the code-object size.  Needs no device.
 *   mode -1 eval or a coot_red; fam 0 flat / 1 tiled; vec, ept, tile_r, tile_c the
 *   compile-time variant (ept for flat, the tile for tiled kernels; no checks: a
 *   variant the kernels cannot run fails to compile, with the reason in the log).
 * Errors: COOT_EINVAL, COOT_ECOMPILE (log in coot_last_error). */
coot_status coot_debug_codegen(coot_expr* e, int32_t mode, int32_t dim, uint32_t rflags, int32_t fam, int32_t vec,
                               int32_t ept, int32_t tile_r, int32_t tile_c, int32_t compile, char* buf, size_t cap,
                               size_t* code_size);

#ifdef __cplusplus
}
#endif
#endif /* COOT_H */
