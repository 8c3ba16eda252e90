/*
 * rd.h -- C ABI of librd, an MI355X (gfx950) parallel-reduction library.
 *
 * The operation is the reduction of Section 1.1 ("Problem Definition") of
 * Jradi, do Nascimento and Martins, "A Fast and Generic GPU-Based Parallel
 * Reduction Implementation" (arXiv 1710.07358): given X = {x0, ..., x(n-1)},
 * compute x0 (+) x1 (+) ... (+) x(n-1) for an associative combiner (+).  The
 * combiners offered are the ones Section 1.1 lists that act on numbers:
 * +, x, min, max, and, or, xor (set intersection/union on bitsets are
 * and/or on the same bits).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named x, offsets, out, y, saved, g, grad_in are DEVICE pointers
 *   owned by the caller; the library never frees them.  Element arrays must
 *   be aligned to their element size; any further alignment is optional.
 * - stream is a hipStream_t passed as void* (NULL = the null stream).  Every
 *   call only enqueues work on it: nothing synchronises, and results are
 *   valid once the stream has reached that point.
 * - Every call returns an rd_status; no exception or abort crosses the ABI.
 *   Host-detected errors return before anything is enqueued.  A failed HIP
 *   launch returns RD_ERR_HIP.  rd_last_error() then describes the failure
 *   (thread-local, valid until the next call on the same thread).
 * - n = 0 (or an empty segment) yields the neutral element of the op:
 *   + -> 0, x -> 1, min -> +inf / INT32_MAX / UINT32_MAX,
 *   max -> -inf / INT32_MIN / 0, and -> all ones, or/xor -> 0.
 * - Integer + and x wrap modulo 2^32 (2^64 for the 64-bit dtypes).  min/max on floats follow IEEE 754-2019
 *   minimum/maximum: a NaN anywhere gives NaN, and -0 < +0.  and/or/xor on a
 *   float dtype act on the stored bit patterns.
 * - Float results are deterministic: the same input, size and configuration
 *   give bitwise-identical output on every run.
 */
#ifndef RD_H
#define RD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
/* C++ sees the enums with int as their fixed underlying type, so every int a
 * C caller passes (valid or not) is a value of the enum type and the
 * library's range checks read it without undefined behaviour; the layout is
 * the C enum's (an int). */
#define RD_ENUM_INT : int
#else
#define RD_ENUM_INT
#endif

typedef enum rd_dtype RD_ENUM_INT {
    RD_I32 = 0,  /* int32 */
    RD_U32 = 1,  /* uint32 */
    RD_F32 = 2,  /* IEEE binary32 */
    RD_F64 = 3,  /* IEEE binary64 */
    RD_F16 = 4,  /* IEEE binary16 */
    RD_BF16 = 5, /* bfloat16 (upper half of a binary32) */
    RD_I64 = 6,  /* int64 */
    RD_U64 = 7   /* uint64 */
} rd_dtype;

typedef enum rd_op RD_ENUM_INT {
    RD_SUM = 0, RD_PROD = 1, RD_MIN = 2, RD_MAX = 3, RD_AND = 4, RD_OR = 5, RD_XOR = 6
} rd_op;

typedef enum rd_status RD_ENUM_INT {
    RD_OK = 0,
    RD_ERR_INVALID_ARG = -1, /* null pointer, negative size, misaligned pointer, bad enum */
    RD_ERR_UNSUPPORTED = -2, /* (dtype, op) pair the entry point does not offer */
    RD_ERR_HIP = -3,         /* a HIP runtime call or kernel launch failed */
    RD_ERR_NOMEM = -4,       /* device allocation failed */
    RD_ERR_CAPTURE = -5,     /* would allocate while the stream is being captured */
    RD_ERR_WORKSPACE = -6    /* workspace belongs to another device or is too small */
} rd_status;

/* Opaque per-stream scratch: one partial per work-group plus a completion
 * counter (the "vector of |SM| partial results" of Section 2.3, filled and
 * consumed inside one launch).  One workspace must not be used by two calls
 * that may run concurrently.  Passing ws = NULL uses a default workspace
 * owned by the library, one per (device, stream), created on first use. */
typedef struct rd_workspace rd_workspace;

/* Launch configuration (Section 3: unroll factor F; Section 2.5: persistent
 * grid of only as many work-groups as run concurrently). */
typedef struct rd_config {
    int block;          /* work-items per work-group: 64..1024, multiple of 64 */
    int unroll;         /* independent 16-byte loads per work-item per step: 1, 2, 4, 8, 16 */
    int blocks_per_cu;  /* persistent grid = blocks_per_cu x compute units (capped by the work) */
    int nontemporal;    /* 1: stream the input with non-temporal loads */
    int layout;         /* order in which work-groups visit chunks of block x unroll vectors:
                           0 grid-stride (chunk b, b+G, ...), as in Section 2.3;
                           1 grid-stride with the work-groups of one XCD on adjacent chunks;
                           2 one contiguous run of chunks per work-group */
} rd_config;

/* Kinds of launch a configuration applies to.  For the row-wise forward
 * (RD_KIND_ROWWISE) and backward (RD_KIND_ROWWISE_BWD) the work-group size is
 * fixed at 256, `unroll` is the number of 4-column stripes each work-item
 * handles per step (1, 2, 4 or 8; 16 is treated as 8), `blocks_per_cu` sizes
 * the persistent grid over rows, and `nontemporal` applies to the forward's
 * loads and the backward's stores.  For scans (RD_KIND_SCAN, and
 * RD_KIND_SEGMENTED_SCAN for rd_segmented_scan) a tile is
 * block x unroll x 16 bytes of input, with unroll 4 or 8 (8 when 8 or more
 * is given, else 4); `blocks_per_cu` sizes the persistent grid,
 * `nontemporal` applies to loads and stores, and `layout` is ignored. */
typedef enum rd_kind RD_ENUM_INT {
    RD_KIND_PLAIN = 0, RD_KIND_COMPENSATED = 1, RD_KIND_SEGMENTED = 2, RD_KIND_ROWWISE = 3,
    RD_KIND_ROWWISE_BWD = 4, RD_KIND_SCAN = 5, RD_KIND_SEGMENTED_SCAN = 6
} rd_kind;

/* ---- library and workspace management ---------------------------------- */

/* Query the current device (compute-unit count, architecture) and look up
 * the device address of its rd_reduce_noalloc array.  Called implicitly by
 * every entry point; returns RD_ERR_HIP without a device. */
rd_status rd_init(void);

/* Create a workspace on the given device (allocates device memory; must not
 * be called while a stream of that device is being captured). */
rd_status rd_workspace_create(rd_workspace** ws, int device);
rd_status rd_workspace_destroy(rd_workspace* ws);
/* Re-zero the workspace's completion counter on stream (only needed after a
 * launch that failed part-way). */
rd_status rd_workspace_reset(rd_workspace* ws, void* stream);

/* Bits of rd_workspace_status. */
typedef enum rd_wait_flags RD_ENUM_INT {
    RD_WAIT_GRID = 1, /* a grid-stage wait of rd_reduce, rd_reduce_compensated, rd_argreduce or a
                         segment-carry wait of rd_segmented_reduce ran out */
    RD_WAIT_SCAN = 2  /* a look-back wait of rd_scan / rd_segmented_scan ran out */
} rd_wait_flags;

/* Outcome of the bounded waits inside the kernels.  Stage 2 of Section 2.3
 * (the partial results of every work-group combined by one of them) and the
 * scan's tile prefixes run inside a single launch here, so a work-group waits
 * for values other work-groups publish; every such wait is bounded, and a
 * correct launch never comes close to the bound.  A wait that runs out sets a
 * status word in the workspace; the launch then ends normally but its result
 * is unspecified.
 *   ws    : one workspace, or NULL for every workspace (default and explicit)
 *           of the current device and the device's rd_reduce_noalloc array
 *   flags : out; rd_wait_flags bits of the words found set
 * Synchronises the device (so it must not be called during graph capture),
 * reads the words and clears them.  Returns RD_ERR_WORKSPACE if ws belongs to
 * another device. */
rd_status rd_workspace_status(rd_workspace* ws, unsigned* flags);

/* Test hook for the failure path of the bounded waits.  While `on` is
 * nonzero, every rd_reduce, rd_reduce_noalloc and rd_scan launch adds one wait for a slot that
 * nothing publishes: the wait runs out (after its bound; about a second for
 * rd_reduce), rd_workspace_status then reports it, and the kernel still ends
 * normally (with an unspecified result).  Not for production use. */
rd_status rd_debug_force_wait_timeout(int on);

/* Element size in bytes of a dtype (0 for an invalid value). */
size_t rd_dtype_size(rd_dtype dt);

/* Output dtype of rd_reduce / rd_segmented_reduce for (dt, op): integers and
 * float32/float64 keep their dtype; float16/bfloat16 give float32 for + and x
 * (accumulated in float32) and keep their dtype for min/max/and/or/xor. */
rd_status rd_out_dtype(rd_dtype dt, rd_op op, rd_dtype* out);

/* ---- plain reduction ------------------------------------------------------ */

/* out[0] = x[0] (+) ... (+) x[n-1]  (Section 1.1; Algorithm 1 for +).
 *   x   : device array of n elements of dtype dt (element-aligned)
 *   n   : number of elements, n >= 0
 *   out : device pointer to ONE element of rd_out_dtype(dt, op)
 *   ws  : workspace or NULL
 * One kernel launch: each work-item folds 16-byte loads of a persistent
 * grid-stride loop into private accumulators, each wavefront combines its
 * lanes with cross-lane (DPP) operations, each work-group combines its
 * wavefronts through LDS, and the last work-group to finish folds the
 * per-work-group partials in index order and writes out. */
rd_status rd_reduce(const void* x, int64_t n, rd_dtype dt, rd_op op, void* out,
                    rd_workspace* ws, void* stream);

/* rd_reduce for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same kernels, launch table and result as rd_reduce (bitwise identical for
 * the same input), but no workspace -- the grid stage's counter, status word
 * and partials live in a fixed array of 128 KiB + 256 bytes that the library
 * holds on every GPU it runs on until the process ends.  The call allocates
 * nothing and does not synchronise; it enqueues one small kernel that re-arms
 * the array (zeroes the counter and the partial slots it will use; a kernel,
 * not a memset, so it can be captured) and then the reduction.
 *   x, n, dt, op, out, stream : as for rd_reduce
 * The persistent grid is capped at the array's 4096 work-group slots; the
 * kernel loops over any n, so no input size is rejected.  The device address
 * of the array is looked up once per device (in rd_init, or on the first call
 * on that device).  Every call on one GPU shares its array: calls that may
 * overlap on one GPU (different streams, or host threads) race and give
 * unspecified results.  A bounded wait that runs out sets the array's status
 * word, which rd_workspace_status(NULL, ...) reports (RD_WAIT_GRID) and
 * clears. */
rd_status rd_reduce_noalloc(const void* x, int64_t n, rd_dtype dt, rd_op op, void* out,
                            void* stream);

/* Compensated sum (the Kahan-style remedy the footnotes of Section 1.1
 * mention): every work-item keeps error-free two-sum (value, error) pairs in
 * float32, and the pairs are merged in float64 double-double arithmetic.
 *   dt  : RD_F32, RD_F16 or RD_BF16 (else RD_ERR_UNSUPPORTED)
 *   out : device pointer to ONE double */
rd_status rd_reduce_compensated(const void* x, int64_t n, rd_dtype dt, double* out,
                                rd_workspace* ws, void* stream);

/* Minimum or maximum together with the LOWEST index attaining it, one launch:
 * the min and max combiners of Section 1.1 applied to (value, index) pairs,
 * where the pair with the smaller index wins a tie (an associative and
 * commutative combiner, so the grid of Section 2.3 and Section 2.5 applies
 * unchanged).
 *   dt        : any dtype;  op : RD_MIN or RD_MAX (else RD_ERR_UNSUPPORTED)
 *   value_out : device pointer to one element of dtype dt -- exactly the
 *               stored element at *index_out
 *   index_out : device pointer to one int64
 * Integers compare signed or unsigned by dtype; floats follow IEEE 754-2019
 * (a NaN wins and its first index is returned; -0 < +0).  n = 0 gives the
 * neutral element and index -1. */
rd_status rd_argreduce(const void* x, int64_t n, rd_dtype dt, rd_op op, void* value_out,
                       int64_t* index_out, rd_workspace* ws, void* stream);

/* The two designs the paper describes, kept as measured baselines (sum of
 * int32, wrapping, or float32; out: device pointer to one element):
 *   variant 0: the two-stage reduction of Section 2.3 -- as many work-items as
 *              the device keeps resident, one scalar load per step, a halving
 *              LDS tree with a barrier per level, a second launch for the
 *              partials (unroll must be 1);
 *   variant 1: the new approach of Section 3 -- the global loop unrolled F =
 *              `unroll` times (1..8 or 16) with the algebraic bounds guard and
 *              the barrier-free LDS tree, on one-wavefront work-groups (the
 *              only size at which that tree is race-free), then stage 2.
 * Two launches; not deterministic across unroll values for float32. */
rd_status rd_reduce_paper_design(const void* x, int64_t n, rd_dtype dt, int variant, int unroll,
                                 void* out, rd_workspace* ws, void* stream);

/* ---- segmented reduction ------------------------------------------------- */

/* out[s] = x[offsets[s]] (+) ... (+) x[offsets[s+1]-1] for s in [0, nseg):
 * the reduction of Section 1.1 applied to every segment, all segments in ONE
 * persistent launch (Section 2.5: persistent threads suit irregular work and
 * avoid returning control to the host between pieces of work; capturable in
 * a HIP graph).
 *   offsets : device int64 array of nseg+1 non-decreasing entries; only
 *             x[offsets[0] .. offsets[nseg]) is read
 *   out     : device array of nseg elements of rd_out_dtype(dt, op)
 * Work is split into equal element ranges, one per wavefront; segments that
 * straddle ranges are finished by the last work-group, folding the pieces in
 * range order (deterministic).  Offsets that decrease give unspecified values
 * for the affected segments but never reads outside
 * [offsets[0], offsets[nseg]). */
rd_status rd_segmented_reduce(const void* x, const int64_t* offsets, int64_t nseg, rd_dtype dt,
                              rd_op op, void* out, rd_workspace* ws, void* stream);

/* ---- scan ---------------------------------------------------------------- */

/* Inclusive (exclusive = 0) or exclusive (exclusive != 0) scan, the prefix
 * form of the reduction of Section 1.1 (the primitive behind the counting
 * sort, stream compaction and radix sort the Introduction names):
 *   inclusive: out[i] = x[0] (+) ... (+) x[i]
 *   exclusive: out[i] = x[0] (+) ... (+) x[i-1], out[0] = the neutral element
 *   x   : device array of n elements of dtype dt (element-aligned)
 *   out : device array of n elements of rd_out_dtype(dt, op); it may be x
 *         itself when the output dtype has x's element size, and must not
 *         otherwise overlap x
 *   n   : 0 <= n <= 2^19 tiles of block x unroll x 16 bytes of input (2^33
 *         float32 elements with the default 1024-wide work-groups); more gives
 *         RD_ERR_INVALID_ARG
 * One pass and one launch: x is read once and out written once.  Each tile
 * publishes its aggregate and folds its prefix from earlier aggregates in a
 * fixed tree (groups of 8 tiles, groups of 8 groups, ...), so float results
 * are the same on every run.  float32 sums carry prefixes across tiles in
 * float64; float products accumulate in float64 as in rd_reduce.  Capturable
 * in a HIP graph (no host synchronisation, no allocation with ws != NULL). */
rd_status rd_scan(const void* x, int64_t n, rd_dtype dt, rd_op op, int exclusive, void* out,
                  rd_workspace* ws, void* stream);

/* Scan restarted at every segment start (the prefix form of Section 1.1's
 * reduction, per segment; one persistent launch as in Section 2.5).  With the CSR offsets of nseg
 * segments (noffsets = nseg + 1 non-decreasing entries, offsets[0] = 0,
 * offsets[nseg] = n), out[i] for offsets[s] <= i < offsets[s+1] reduces
 * x[offsets[s] .. i] (inclusive) or x[offsets[s] .. i) (exclusive; the neutral
 * element at a segment's first position).  In general position 0 and every
 * offset in [0, n) start a run, so elements before offsets[0] or from
 * offsets[nseg] on are scanned as runs of their own, and empty segments
 * change nothing.  Decreasing offsets give unspecified values but no access
 * outside x, out and offsets.
 *   offsets  : device int64 array of noffsets entries, noffsets < 2^31
 * Adds one small launch that finds, per tile, its first run start. */
rd_status rd_segmented_scan(const void* x, int64_t n, const int64_t* offsets, int64_t noffsets,
                            rd_dtype dt, rd_op op, int exclusive, void* out, rd_workspace* ws,
                            void* stream);

/* ---- row-wise reduction and its gradient --------------------------------- */

/* Bytes of the `saved` buffer rd_rowreduce_fwd fills for rd_rowreduce_bwd
 * (the state the gradient of the Section 1.1 reduction of each row needs):
 * 0 for sum, 8*rows (lowest extreme index) for min/max, and per-row zero
 * bookkeeping plus per-tile products for product. */
size_t rd_saved_bytes(rd_op op, int64_t rows, int64_t cols);

/* y[r] = x[r,0] (+) ... (+) x[r,cols-1] for a row-major float32 matrix: the
 * reduction of Section 1.1 (+, max, min, x) over every row, one launch.
 *   dt    : RD_F32;  op : RD_SUM, RD_MAX, RD_MIN or RD_PROD
 *   y     : device float32[rows]
 *   saved : device buffer of rd_saved_bytes(op, rows, cols) bytes (may be
 *           NULL for RD_SUM); min/max store the LOWEST column attaining the
 *           extreme; product stores the zero count, the first zero's column,
 *           the product of the nonzero entries and per-chunk products. */
rd_status rd_rowreduce_fwd(const void* x, int64_t rows, int64_t cols, rd_dtype dt, rd_op op,
                           void* y, void* saved, void* stream);

/* grad_in[r,j] = d y[r] / d x[r,j] * g[r], the derivative of the row-wise
 * reduction of Section 1.1 (the paper defines the forward only; the
 * derivative follows from each combiner: d(sum)/dx = 1, d(max)/dx = 1 at
 * the first position attaining it, d(prod)/dx_j = the product of the
 * other entries):
 *   sum     -> g[r] everywhere;
 *   min/max -> g[r] at the saved lowest extreme index, 0 elsewhere;
 *   product -> g[r] * prod_{i != j} x[r,i], formed from prefix and suffix
 *              products (no division); rows with one zero get g*prod(nonzeros)
 *              at the zero and 0 elsewhere; rows with two or more zeros get 0.
 *   x       : the forward input (read only for product rows without zeros)
 *   g       : device float32[rows];  saved : as filled by rd_rowreduce_fwd
 *   grad_in : device float32[rows, cols]
 * The product writes its rows with zeros on a second stream that the library
 * creates once per device (default priority) and keeps until the process
 * ends: forked from `stream` by an event and joined back into it, so the
 * call's work still lies between the work enqueued on `stream` before and
 * after it (also under graph capture).  Concurrent calls on one device are
 * serialised while they enqueue. */
rd_status rd_rowreduce_bwd(const void* x, const void* g, const void* saved, int64_t rows,
                           int64_t cols, rd_dtype dt, rd_op op, void* grad_in, void* stream);

/* ---- configuration and tuning --------------------------------------------- */

/* Configuration the library would use for (kind, dt, op, n). */
rd_status rd_config_get(rd_kind kind, rd_dtype dt, rd_op op, int64_t n, rd_config* cfg);

/* Force one configuration for every later launch of `kind` (NULL clears it).
 * Used by the autotuner and by tests that sweep configurations. */
rd_status rd_config_force(rd_kind kind, const rd_config* cfg);

/* Load a tuned table written by the autotuner (NULL restores the built-in
 * defaults).  Format: one line per entry,
 *   kind dtype_size op_class log2n_lo log2n_hi block unroll blocks_per_cu nontemporal layout
 * with op_class 0 = sum/prod, 1 = min/max, 2 = and/or/xor (for the row-wise kinds,
 * which have no bitwise ops: 0 = sum, 2 = product); '#' starts a comment. */
rd_status rd_tune_load(const char* path);

/* Description of the last non-OK status returned on this thread. */
const char* rd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
