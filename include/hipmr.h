/*
 * hipmr.h -- run-time generated elementwise and map-reduce kernels for the
 * AMD Instinct MI355X (gfx950, CDNA4).  C ABI of libhipmr.so.
 *
 * Programming model (Kloeckner et al., "GPU Scripting and Code Generation
 * with PyCUDA"):
 *   - device code is given as C source text, not translated from the host
 *     language (section "Core Method");
 *   - an elementwise kernel is a C argument list plus a statement, or a
 *     semicolon-separated list of statements, run for every value of the
 *     formal index i over arrays of one common length (section "Efficient
 *     Evaluation of Element-wise Expressions");
 *   - a map-reduce kernel adds a result dtype, a map expression evaluated at
 *     every i, a reduce expression in the formal arguments a and b, and a
 *     neutral element, the identity of the reduce operation; the result stays
 *     in device memory (section "Map-Reduce");
 *   - generated sources are compiled on demand and cached, so that unchanged
 *     kernels load without recompiling (section "Core Method", compilation
 *     and caching figure); constants, types and trip counts are substituted
 *     into the source at run time (section "Code Generation", subsections
 *     "The Cost of Flexibility" and "Generating Code", textual keyword
 *     replacement);
 *   - errors surface as status codes with a message instead of requiring
 *     explicit checks (section "The Basics of GPU programming").
 *
 * General conventions
 *   - Every call returns HIPMR_OK (0) or a negative hipmr_status; the message
 *     of the last failure on the calling thread is hipmr_last_error().  No
 *     call aborts the process or throws across the ABI.
 *   - "device pointer" means memory allocated on the current HIP device (for
 *     example a torch tensor's data_ptr()).  The library never allocates,
 *     frees or retains device memory: inputs, outputs and workspaces belong
 *     to the caller and must stay valid until the work queued on the stream
 *     has finished.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).  All
 *     GPU work is enqueued asynchronously on it; kernel faults surface at the
 *     next synchronisation, as in HIP.
 *   - args: an array with one entry per declared argument, in declaration
 *     order; args[k] points to host storage holding the k-th argument's value
 *     (the device pointer value for arrays, the scalar itself for scalars),
 *     exactly like hipModuleLaunchKernel's kernelParams.  Values are copied
 *     during the call.
 *   - The library runs on the current HIP device of the calling thread; code
 *     objects are loaded once per device.
 */
#ifndef HIPMR_H_
#define HIPMR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hipmr_status;

#define HIPMR_OK               0
#define HIPMR_E_INVALID       -1  /* bad argument: NULL, n < 0, bad config, ... */
#define HIPMR_E_PARSE         -2  /* signature or expression outside the grammar */
#define HIPMR_E_COMPILE       -3  /* hipRTC rejected the generated source; log in last_error */
#define HIPMR_E_HIP           -4  /* a HIP runtime call failed */
#define HIPMR_E_MISMATCH      -5  /* argument does not match the handle (kind, map_expr, ...) */
#define HIPMR_E_UNSUPPORTED   -6  /* valid C, but not supported by this variant */
#define HIPMR_E_BUDGET        -7  /* serving: a job can never fit the memory budget */
#define HIPMR_E_WORKSPACE     -8  /* workspace missing or smaller than required */

/* Element types (dtype codes).  Spellings accepted in signatures:
 *   float | double | int8_t, char, signed char | uint8_t, unsigned char |
 *   int16_t, short | uint16_t, unsigned short | int32_t, int, signed |
 *   uint32_t, unsigned, unsigned int | int64_t, long, long long |
 *   bfloat16, __hip_bfloat16 | half, __half, float16 | fp8_e4m3 |
 *   complex64, cfloat
 * bfloat16, half and fp8_e4m3 (OCP E4M3, "fn": no infinities, max 448) are
 * storage types: a read converts exactly to float, and all arithmetic on
 * them happens in float; a store rounds to nearest even (fp8 saturates to
 * +-448).  complex64 is a complex value with float components (real,
 * imaginary; 8 bytes), the complex support of section "Complex Numbers on
 * the GPU": +, - and * with complex or real operands, unary -, conj(z),
 * real(z), imag(z) and abs(z); no division, no ordering; as a reduce
 * result only with the sum combine. */
#define HIPMR_F32   1
#define HIPMR_F64   2
#define HIPMR_I8    3
#define HIPMR_U8    4
#define HIPMR_I16   5
#define HIPMR_U16   6
#define HIPMR_I32   7
#define HIPMR_U32   8
#define HIPMR_I64   9
#define HIPMR_BF16 10
#define HIPMR_F16  11
#define HIPMR_FP8  12
#define HIPMR_C64  13

typedef struct hipmr_kernel *hipmr_handle;

/* Optional launch geometry; any field 0 means "library default".  Used by
 * the *_ex calls, the autotuner and benchmarks (section "Automated Tuning":
 * variants are kept and chosen at run time). */
typedef struct hipmr_launch_config {
    int32_t block;            /* threads per block: multiple of 64 in [64, 1024]       */
    int32_t items_per_thread; /* vector chunks per thread per grid-stride pass: 1..16  */
    int32_t grid;             /* blocks; 0: min(needed, blocks_per_cu * CU count)       */
    int32_t blocks_per_cu;    /* cap used when grid == 0                                */
    int32_t vec;              /* elements per vector chunk: 0 = 16 bytes of the narrowest
                                 array; power of two 1..16                             */
    int32_t flags;            /* HIPMR_CFG_* bits                                       */
} hipmr_launch_config;

#define HIPMR_CFG_NONTEMPORAL      1  /* streaming (non-temporal) loads and stores (default) */
#define HIPMR_CFG_FORCE_SCALAR     2  /* use the one-element-per-step kernel variant         */
#define HIPMR_CFG_TEMPORAL         4  /* ordinary (temporal) loads and stores                */
#define HIPMR_CFG_TEMPORAL_LOADS   8  /* ordinary loads, streaming stores                    */
#define HIPMR_CFG_TEMPORAL_STORES 16  /* streaming loads, ordinary stores                    */
#define HIPMR_CFG_SEG_GLOBAL      32  /* segmented: read the tile table from global memory
                                         even when it would fit in LDS                       */
#define HIPMR_CFG_TUNED           64  /* hipmr_reduce_ex / hipmr_reduce_segmented: use the
                                         geometry the autotuner stored for this handle,
                                         operation and size class, when there is one (else
                                         the other fields); never applied without the flag */
/* Streaming stores apply to chunks of at most 16 bytes per lane; a wider
 * chunk (e.g. four 64-bit results) leaves in several instructions that each
 * fill half lines, and is stored temporally so that the L2 merges them. */

/* ------------------------------------------------------------------ core */

/* Compiles (or finds in the cache) the kernels of one elementwise or map-reduce
 * operation.  Section "Efficient Evaluation of Element-wise Expressions"
 * (ElementwiseKernel(arguments, operation, name)) and section "Map-Reduce"
 * (ReductionKernel(dtype_out, arguments, map_expr, ...)).
 *   dtypes: "[result_type ':'] decl (',' decl)*", decl = "[const] type [*] name";
 *           a leading "result_type:" makes a map-reduce handle (the paper puts
 *           the result dtype first), otherwise an elementwise handle.
 *   expr:   elementwise: the statement list over the formal index i (int when
 *           n < 2^31, else 64-bit); the length is available as n.  Map-reduce:
 *           the map expression.  Writes are supported to name[i] only.
 *   name:   (compile_named) prefix of the generated kernel symbols, which are
 *           extern "C" "<name>_<kind>_<hash8>"; default "hipmr".
 *   *out:   receives a handle (reference counted; release with hipmr_release).
 * The elementwise code object is built eagerly with hipRTC for gfx950 (no GPU
 * is needed to compile); map-reduce kernels are built when the reduce
 * expression is known (hipmr_prepare_reduce or the first hipmr_reduce).
 * Errors: E_INVALID (NULL), E_PARSE (grammar; message names the position),
 * E_UNSUPPORTED (e.g. return/goto, writes in a map), E_COMPILE (hipRTC log). */
hipmr_status hipmr_compile(const char *expr, const char *dtypes, hipmr_handle *out);
hipmr_status hipmr_compile_named(const char *expr, const char *dtypes, const char *name,
                                 hipmr_handle *out);

/* Runs an elementwise handle over i in [0, n).  Section "Efficient Evaluation
 * of Element-wise Expressions" (one pass over all operands).  n == 0 enqueues
 * nothing.  Arrays accessed as name[i] or name[i +/- E] must hold at least n
 * elements (the caller checks lengths); arrays read only at fixed indices
 * (name[3]) need only hold those elements.
 * The vector kernel runs when every array access is name[i], a fixed element,
 * or a shifted read name[i + E] / name[i - E] of an array the statement does
 * not write (E built from literals, scalar arguments, n, + - * / % and
 * parentheses: the same distance for every i), and the name[i] arrays share
 * one misalignment: 16-byte chunks for name[i] (unaligned head and ragged tail
 * by scalar code), one unaligned chunk load per distinct shifted read, and,
 * for chunks within the largest distance of either end, the statement one
 * element at a time (its own guards apply there; shifted chunks are read only
 * inside [0, n)).  With shifted reads, workgroups are renumbered so that each
 * XCD (own L2) takes a contiguous run of chunks.  Otherwise the one-element
 * kernel runs.
 * Errors: E_INVALID (n < 0, NULL args or array pointer), E_MISMATCH (reduce
 * handle), E_COMPILE / E_HIP. */
hipmr_status hipmr_elementwise(hipmr_handle h, int64_t n, void *const *args, void *stream);
hipmr_status hipmr_elementwise_ex(hipmr_handle h, int64_t n, void *const *args,
                                  const hipmr_launch_config *cfg, void *stream);

/* Bytes of device workspace hipmr_reduce, hipmr_reduce_compensated and
 * hipmr_norm2 need (64 KiB of block partials, 32 KiB of the norm's first-pass
 * partials and 256 bytes for its scale; independent of n).  Returns 0 for an
 * elementwise or invalid handle. */
size_t hipmr_reduce_workspace_bytes(hipmr_handle h, int64_t n);

/* Map-reduce: *out = neutral (+) map(0) (+) ... (+) map(n-1), (+) being
 * combine_op.  Section "Map-Reduce" (reduction expression of formal arguments
 * a and b, neutral element; result left on the GPU).
 *   map_expr:   NULL or byte-equal to the handle's expression (E_MISMATCH).
 *   combine_op: C expression in a and b of the result type, assumed
 *               associative and commutative.  The spellings "a+b", "b+a",
 *               "sum", "max(a,b)", "max(b,a)", "max", "min(a,b)", "min(b,a)",
 *               "min" (blanks ignored) select specialised code; for float and
 *               double max/min mean IEEE 754-2019 maximum/minimum (NaN
 *               propagates, -0 < +0).
 *   neutral:    C expression converted to the result type.
 *   out:        device pointer to one element of the result type.
 *   workspace:  device buffer of at least hipmr_reduce_workspace_bytes(h, n)
 *               bytes (E_WORKSPACE otherwise); it is scratch for block partials.
 * Two launches on stream (block partials, then one block folding them), no
 * atomics; for a given device, n and launch configuration the result is
 * bitwise reproducible.  n == 0 writes neutral.  The map reads arrays in
 * chunks as described for hipmr_elementwise, shifted reads name[i +/- E]
 * included (every lane loads every chunk, clamped into [0, n), and chunks
 * near the ends are mapped one element at a time); the other map-reduce
 * entry points read shifted elements one at a time inside their vector
 * kernels.
 * Errors: E_INVALID, E_MISMATCH (elementwise handle or map_expr), E_PARSE,
 * E_COMPILE, E_WORKSPACE, E_HIP. */
hipmr_status hipmr_reduce(hipmr_handle h, const char *map_expr, const char *combine_op,
                          const char *neutral, int64_t n, void *const *args, void *out,
                          void *workspace, size_t workspace_bytes, void *stream);
hipmr_status hipmr_reduce_ex(hipmr_handle h, const char *map_expr, const char *combine_op,
                             const char *neutral, int64_t n, void *const *args, void *out,
                             void *workspace, size_t workspace_bytes,
                             const hipmr_launch_config *cfg, void *stream);

/* Builds the map-reduce kernels for (combine_op, neutral) ahead of the first
 * hipmr_reduce (the paper's prepared invocation, section "The Basics of GPU
 * programming", declares argument types once for later calls).  No GPU needed. */
hipmr_status hipmr_prepare_reduce(hipmr_handle h, const char *combine_op, const char *neutral);
/* Same, for one launch geometry (NULL = default). */
hipmr_status hipmr_prepare_reduce_ex(hipmr_handle h, const char *combine_op, const char *neutral,
                                     const hipmr_launch_config *cfg);

/* Message of the last failure on this thread ("" if none).  Owned by the
 * library; valid until the next call on this thread. */
const char *hipmr_last_error(void);

/* Drops one reference; the handle must not be used afterwards.  Cached code
 * objects stay in the process-wide cache. NULL is ignored. */
void hipmr_release(hipmr_handle h);

/* ------------------------------------------------------------------ precision extension */

/* Compensated sum of a float map: *out (double) = post_scale * sum_i map(i).
 * Precision extension of the map-reduce (section "Map-Reduce"): the map is
 * evaluated in float from narrow loads (bfloat16, half, fp8_e4m3 or float
 * arrays), accumulated per lane with Kahan compensation in FP32, combined
 * across lanes, waves and the block as (sum, error) pairs with error-free
 * TwoSum steps, written as FP64 block partials and folded in FP64 (Neumaier)
 * by one block, which multiplies by post_scale once (for example 1/s of a
 * per-tensor power-of-two quantisation scale s).  When the map is a single
 * FP8 load, runs of up to 64 values are summed in plain FP32, which is exact
 * (every E4M3 value is a multiple of 2^-9 of magnitude at most 448), and
 * compensated once per run.
 *   h:         map-reduce handle with result type float ("float: ...").
 *   out:       device pointer to one double.
 *   workspace: at least hipmr_reduce_workspace_bytes(h, n) bytes.
 *   cfg:       NULL or a launch geometry.
 * n == 0 writes 0.  Errors: as hipmr_reduce; E_MISMATCH for a handle whose
 * result type is not float. */
hipmr_status hipmr_reduce_compensated(hipmr_handle h, int64_t n, void *const *args,
                                      double post_scale, void *out, void *workspace,
                                      size_t workspace_bytes, const hipmr_launch_config *cfg,
                                      void *stream);

/* L2 norm of a float map: *out (double) = post_scale * sqrt(sum_i map(i)^2),
 * precision extension as above.
 *   passes == 2 (scaled): pass 1 takes the exact max |map(i)| per block;
 *     every block of pass 2 (same grid) first derives from those maxima the
 *     power of two s that puts the largest in [1, 2) (exponent clamped to
 *     [-126, 126]), then accumulates (map(i) * s)^2 with compensation; the
 *     final FP64 step returns post_scale * sqrt(sum) / s.  Reads the data
 *     twice, in three launches.
 *   passes == 1: no scaling, one read; the squares must stay inside the float
 *     range (true for every half or FP8 load: their squares are below 2^32).
 * The first pass's maxima and the scale are kept in the workspace.  Errors:
 * as hipmr_reduce_compensated; E_INVALID for passes other than 1 or 2. */
hipmr_status hipmr_norm2(hipmr_handle h, int64_t n, void *const *args, double post_scale,
                         int32_t passes, void *out, void *workspace, size_t workspace_bytes,
                         const hipmr_launch_config *cfg, void *stream);

/* ------------------------------------------------------------------ prefix scan */

/* Bytes of device workspace hipmr_scan needs (two tables of at most 65536
 * wave totals of the result type); 0 for an elementwise or invalid handle. */
size_t hipmr_scan_workspace_bytes(hipmr_handle h, int64_t n);

/* Prefix scan of a map: the parallel prefix sums of section "Further
 * Facilities", over the map, combine and neutral element of section
 * "Map-Reduce":
 *   inclusive (exclusive == 0): out[i] = neutral (+) map(0) (+) ... (+) map(i)
 *   exclusive (exclusive == 1): out[i] = neutral (+) map(0) (+) ... (+) map(i-1)
 *   h:          map-reduce handle ("T: ..."); map_expr is the handle's.
 *   combine_op, neutral: as for hipmr_reduce (associative and commutative).
 *   out:        device array of n values of the result type T; must not
 *               overlap the inputs.
 *   workspace:  at least hipmr_scan_workspace_bytes(h, n) bytes (caller-owned).
 *   cfg:        NULL or a geometry (block, items_per_thread, vec, flags).
 * Three launches on `stream`: every wave folds a contiguous range, one block
 * scans the wave totals, every wave rescans its range from its prefix.  The
 * order of combination depends only on n, alignment and geometry (bitwise
 * repeatable).  Chunked accesses when every array and out share one
 * alignment and the map reads arrays only as name[i] (by default 16 bytes of
 * the narrowest input, but at most 16 bytes of output, per lane); one
 * element at a time otherwise.  n == 0 writes nothing.  Errors: E_INVALID (NULL, exclusive not
 * 0/1), E_MISMATCH (elementwise handle), E_WORKSPACE, E_PARSE / E_COMPILE
 * (combine or neutral), E_HIP. */
hipmr_status hipmr_scan(hipmr_handle h, const char *combine_op, const char *neutral, int64_t n,
                        void *const *args, void *out, int32_t exclusive, void *workspace,
                        size_t workspace_bytes, const hipmr_launch_config *cfg, void *stream);

/* ------------------------------------------------------------------ batching extension */

/* Bytes of device workspace hipmr_reduce_segmented / hipmr_autotune_segmented
 * need for nseg segments over total_n elements (tile-start table plus one
 * partial per tile at the smallest tile size any geometry can choose); 0 for
 * an elementwise or invalid handle. */
size_t hipmr_segmented_workspace_bytes(hipmr_handle h, int32_t nseg, int64_t total_n);

/* Segmented map-reduce, many uneven segments in one launch sequence: for
 * s in [0, nseg), d_out[s] = neutral (+) map(off[s]) (+) ... (+) map(off[s+1]-1),
 * the map indexing the concatenated arrays with the global index i (and n =
 * total_n).  Batching extension of the map-reduce (section "Map-Reduce").
 *   d_offsets: device int64 array of nseg + 1 non-decreasing offsets into
 *              [0, total_n]; values outside are clamped and a decreasing pair
 *              gives an empty segment.  Offsets that are not non-decreasing
 *              (overlapping segments) may describe more tiles than the
 *              workspace holds: the planner then caps the tile table at the
 *              workspace's capacity, no kernel reads or writes past it, and
 *              the results of the segments whose tiles fall past the cap are
 *              unspecified (never an out-of-bounds access, whatever the
 *              offsets, including offsets changed between graph replays).
 *   d_out:     device array of nseg elements of the result type.
 *   workspace: at least hipmr_segmented_workspace_bytes(h, nseg, total_n).
 *   cfg:       NULL (the default geometry) or a geometry; with HIPMR_CFG_TUNED
 *              the one hipmr_autotune_segmented stored for this handle,
 *              combine_op, neutral and size class, if any.
 * Two launches on stream (three above 8191 segments): the offsets become a
 * tile table (tile 0 of a segment holds its unaligned head and up to T body
 * elements, later tiles T elements, T = 64 * vec * items_per_thread); a
 * persistent kernel whose waves each reduce one tile at a time into a tile
 * partial; one wave per segment folding its tiles in order.  Up to 8191
 * segments every block of the persistent kernel computes the table in LDS
 * itself (block 0 also writes it to the workspace); above that a one-block
 * planner launch writes it to the workspace first.  A segment's result depends
 * only on its own bounds and the geometry, so it is bitwise the same whatever
 * the other segments are.  Everything stays on the device, so the sequence
 * can be captured once and replayed with new offset values.
 * Errors: as hipmr_reduce; E_WORKSPACE for a short workspace; E_UNSUPPORTED
 * when nseg + total_n / 64 + 1 (the tile capacity) exceeds 2^31 - 1. */
hipmr_status hipmr_reduce_segmented(hipmr_handle h, const char *combine_op, const char *neutral,
                                    int32_t nseg, const int64_t *d_offsets, int64_t total_n,
                                    void *const *args, void *d_out, void *workspace,
                                    size_t workspace_bytes, const hipmr_launch_config *cfg,
                                    void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * segmented map-reduce as hipmr_reduce_segmented, with the same kernels and
 * results, but its tile table and tile partials live in a static device array
 * of the library (HIPMR_NOALLOC_SCRATCH_BYTES per device, held from the first
 * call on a device until the process ends) instead of a caller workspace.
 *   Arguments as hipmr_reduce_segmented, without the workspace.
 *   The call allocates nothing: it neither builds nor loads kernels, so run
 *   hipmr_reduce_segmented once on this device with the same handle,
 *   combine_op, neutral, geometry and argument alignment first (E_INVALID
 *   otherwise).  Its first call on a device looks up the array's device
 *   address there.
 *   Every call on one device shares that device's array: calls that overlap
 *   on one device (two streams, two threads) race and give wrong results.
 *   Nothing in the array needs to start at zero (every entry read is written
 *   first by the same call).
 * Errors: as hipmr_reduce_segmented; E_WORKSPACE when the segments need more
 * than HIPMR_NOALLOC_SCRATCH_BYTES (hipmr_segmented_workspace_bytes(h, nseg,
 * total_n) bytes: e.g. 4096 segments over about 2^27 float elements). */
#define HIPMR_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
size_t hipmr_noalloc_scratch_bytes(void);
hipmr_status hipmr_reduce_segmented_noalloc(hipmr_handle h, const char *combine_op,
                                            const char *neutral, int32_t nseg,
                                            const int64_t *d_offsets, int64_t total_n,
                                            void *const *args, void *d_out,
                                            const hipmr_launch_config *cfg, void *stream);

/* Autotuner (section "Code Generation", "Automated Tuning"; and the future-work
 * note on compiling a search's variants on all CPU cores): generates the
 * candidate geometries (block 256/512, items_per_thread 1/2/4/8, 2-16 blocks
 * per CU), compiles all their variants concurrently on host threads through
 * the same hipRTC path, times each reps times on the caller's data with HIP
 * events (median), stores the fastest for this handle, operation and size
 * class in memory and in $HIPMR_CACHE_DIR, and returns it in *best.  Runs
 * the operation (1 + reps) times per candidate, overwriting d_out / out.
 * A stored geometry is used only by calls that pass HIPMR_CFG_TUNED; a
 * stored file that does not resolve to a valid geometry is ignored. */
hipmr_status hipmr_autotune_segmented(hipmr_handle h, const char *combine_op, const char *neutral,
                                      int32_t nseg, const int64_t *d_offsets, int64_t total_n,
                                      void *const *args, void *d_out, void *workspace,
                                      size_t workspace_bytes, int32_t reps,
                                      hipmr_launch_config *best, void *stream);
hipmr_status hipmr_autotune_reduce(hipmr_handle h, const char *combine_op, const char *neutral,
                                   int64_t n, void *const *args, void *out, void *workspace,
                                   size_t workspace_bytes, int32_t reps, hipmr_launch_config *best,
                                   void *stream);

/* HIP graphs of launch sequences.  Every hipmr call between begin and end on
 * this thread and stream is captured (not executed); end instantiates the
 * graph; launch replays it with one call.  Run each operation once before
 * capturing it so that its code objects are loaded (E_INVALID otherwise).
 * The kernels write every output they own, so replays need no memory
 * clearing nodes.  The null stream cannot be captured. */
typedef struct hipmr_graph *hipmr_graph_t;
hipmr_status hipmr_graph_begin_capture(void *stream);
hipmr_status hipmr_graph_end_capture(void *stream, hipmr_graph_t *out);
hipmr_status hipmr_graph_launch(hipmr_graph_t g, void *stream);
void         hipmr_graph_destroy(hipmr_graph_t g);

/* ------------------------------------------------------------------ serving extension */

/* Map-reduce job templates of the request loop (each over float32 or
 * bfloat16 arrays of n elements; the result is one double):
 *   SUM        sum x[i]                  DOT        sum x[i]*y[i]
 *   NORM2      sqrt(sum x[i]^2)          MAX        max x[i] (IEEE maximum; -inf for n = 0)
 *   AXPBY_SUM  sum (a*x[i] + b*y[i])     COUNT_POS  #{i : x[i] > 0}
 *   SUMSQ      sum x[i]^2                WMEAN      (sum w[i]*x[i]) / (sum w[i])
 * Lanes accumulate in float, tile partials are float pairs, each job's tiles
 * are folded in FP64 in tile order. */
#define HIPMR_JOB_SUM        0
#define HIPMR_JOB_DOT        1
#define HIPMR_JOB_NORM2      2
#define HIPMR_JOB_MAX        3
#define HIPMR_JOB_AXPBY_SUM  4
#define HIPMR_JOB_COUNT_POS  5
#define HIPMR_JOB_SUMSQ      6
#define HIPMR_JOB_WMEAN      7

typedef struct hipmr_sjob {
    const void *x, *y, *w;   /* device arrays (y: DOT, AXPBY_SUM; w: WMEAN; others may be NULL) */
    int64_t n;               /* elements                                                       */
    int32_t tmpl;            /* HIPMR_JOB_*                                                     */
    int32_t dtype;           /* HIPMR_F32 or HIPMR_BF16                                         */
    int64_t arrival_ns;      /* run_schedule: arrival time relative to the call (non-decreasing) */
    double *out;             /* device pointer to one double                                    */
    float a, b;              /* AXPBY_SUM coefficients                                          */
} hipmr_sjob;

typedef struct hipmr_server_config {
    uint64_t hbm_budget_bytes;   /* bytes (inputs + output) of admitted, unfinished jobs; 0: 64 GiB */
    int32_t nstreams;            /* batches in flight, one stream each (1..16); 0: 4                */
    int32_t max_batch_jobs;      /* jobs per batch (1..4096; 1 = one launch pair per job); 0: 1024  */
    int32_t max_batch_tiles;     /* tiles per batch (a tile is 1024 float32 / 2048 bfloat16
                                    elements, P times that, P = ceil(those tiles / 4080), in
                                    jobs that would have more than 4080); 0: 2^18               */
    int32_t blocks_per_cu;       /* persistent grid of the tile kernel; 0: 8                        */
    uint64_t max_batch_bytes;    /* input bytes per batch of two or more jobs; 0: 16 MiB           */
    uint64_t solo_bytes;         /* a job of more input bytes runs in a batch of its own, and
                                    smaller jobs are packed past it, so small jobs never wait on
                                    a large one's tiles (<= max_batch_bytes); 0: 4 MiB            */
    int32_t batch_backlog;       /* jobs are packed together only while more than this many wait
                                    per free stream (a shorter queue runs one job per stream, as
                                    the one-launch-pair-per-job loop does); 0: 8                   */
    int32_t resident;            /* 0: batches launched on the streams (above); 1: one resident
                                    kernel takes the jobs from a descriptor ring in mapped host
                                    memory, no launch per job (nstreams, max_batch_jobs,
                                    max_batch_bytes, solo_bytes and batch_backlog unused;
                                    max_batch_tiles sizes its ring of tile partials, rounded up
                                    to a power of two >= 8192; blocks_per_cu: blocks of 1024
                                    threads per CU, 0: 1)                                          */
} hipmr_server_config;

typedef struct hipmr_completion {
    uint64_t ticket;         /* submit: its ticket; run_schedule: the job's index                */
    int32_t status;          /* HIPMR_OK, or the code the job was rejected with                  */
    int32_t batch_jobs;      /* jobs in the batch that carried it (resident mode: jobs on the
                                device, itself included, when it was handed over)              */
    int64_t arrival_ns;      /* run_schedule: relative to the call; submit: server clock         */
    int64_t launch_ns;       /* when its batch was launched (resident: handed to the ring)       */
    int64_t done_ns;         /* when the loop saw the batch complete (result visible on the host) */
} hipmr_completion;

typedef struct hipmr_server *hipmr_server_t;

/* Device workspace of a server (per stream: job descriptors and tile
 * partials), owned by the caller for the server's lifetime. */
size_t hipmr_server_workspace_bytes(const hipmr_server_config *cfg);

/* Serving extension of the map-reduce: starts a request loop on a host thread
 * for the current device.  The loop
 *   - releases arrivals at their time;
 *   - admits them while the bytes of admitted, unfinished jobs stay within
 *     the budget (no job is admitted while an earlier one does not fit;
 *     small jobs may pass a large one);
 *   - hands admitted jobs to the free streams, one batch per stream
 *     (continuous batching: jobs that arrive while others run join the next
 *     batch): one job per free stream while at most batch_backlog jobs per
 *     free stream wait, else ceil(waiting / free streams) jobs per batch; a
 *     job over solo_bytes runs alone and small jobs are packed past it;
 *   - launches a batch as two run-time compiled kernels: a persistent kernel
 *     whose waves take tiles of any job (wave-uniform switch over template x
 *     dtype) and one block per job folding its tiles in a fixed order.  A job
 *     of at most 16 tiles alone runs in one launch (one block computes and
 *     folds its tiles) unless max_batch_jobs is 1.
 * With cfg->resident = 1 no kernel is launched per job: admitted jobs go, in
 * arrival order, into a ring of descriptors in mapped host memory, and one
 * resident kernel (on a stream of its own) takes them as they are published:
 * a dispatcher wave copies each descriptor to the device and publishes its
 * tiles; the other blocks take tile tickets in order, and the wave completing
 * a job's last tile group folds the job and writes its flag.  Admission also
 * waits while the ring (4096 jobs) or the ring of tile partials is full.  An
 * instance runs at most 2 s (every wait in it is bounded by that deadline);
 * the loop replaces it every 250 ms and stops it after 10 ms without jobs,
 * so a device-wide synchronisation returns once the server is idle.  Jobs
 * an instance could not finish by its deadline complete with E_HIP.
 * On every path a job's tiles depend only on the job, and its tile partials
 * are folded in a fixed order (64-tile groups, then the groups), so its
 * result is bitwise the same alone, in any mix and on any path.  A job has at
 * most 4080 tiles (the resident kernel takes them in one round) and at most
 * 2^26 float32 / 2^27 bfloat16 elements (E_UNSUPPORTED beyond).
 * Completion is observed through per-job flags in mapped host memory that the
 * folding wave or block writes after the result (a stream query is the
 * watchdog for errors).  Inputs stay resident: jobs name device arrays.  The
 * server allocates pinned host memory for descriptors and flags (not device
 * memory).
 * Errors: E_INVALID (config), E_WORKSPACE, E_COMPILE, E_HIP. */
hipmr_status hipmr_server_create(const hipmr_server_config *cfg, void *workspace,
                                 size_t workspace_bytes, hipmr_server_t *out);

/* Submits one job now.  Invalid jobs are rejected here (E_INVALID,
 * E_UNSUPPORTED; E_BUDGET for a job that can never fit the budget) and never
 * packed.  *ticket identifies its completion in hipmr_server_poll. */
hipmr_status hipmr_server_submit(hipmr_server_t s, const hipmr_sjob *job, uint64_t *ticket);

/* Copies up to cap completions of submitted jobs into done, oldest first;
 * *ndone receives the count.  Reports a launch failure of the loop as its
 * status.  A job whose batch failed to launch or run completes with E_HIP;
 * if the loop's thread cannot select the device, every job completes at once
 * with E_HIP, so no wait is left without an end. */
hipmr_status hipmr_server_poll(hipmr_server_t s, hipmr_completion *done, int32_t cap,
                               int32_t *ndone);

/* Waits until every submitted job has completed. */
hipmr_status hipmr_server_wait_idle(hipmr_server_t s);

/* Open-loop replay: job k arrives at (call time + jobs[k].arrival_ns) and is
 * handled by the loop like a submission; returns when all have completed,
 * done[k] describing job k (rejected jobs carry their status and are never
 * packed).  Latency of job k = done[k].done_ns - done[k].arrival_ns. */
hipmr_status hipmr_server_run_schedule(hipmr_server_t s, const hipmr_sjob *jobs, int32_t njobs,
                                       hipmr_completion *done);

/* Stops the loop after the submitted work completes and frees its resources
 * (not the caller's workspace). */
void hipmr_server_destroy(hipmr_server_t s);

/* The server clock (monotonic nanoseconds). */
int64_t hipmr_server_now_ns(void);

/* ------------------------------------------------------------------ introspection */

typedef struct hipmr_handle_info {
    int32_t is_reduce;      /* 1: map-reduce handle                                */
    int32_t result_dtype;   /* HIPMR_* of the result (reduce), else 0              */
    int32_t nargs;          /* declared arguments                                  */
    int32_t vectorizable;   /* every array access is name[i]                       */
    int32_t vec;            /* default elements per vector chunk                   */
    uint32_t hash;          /* first 32 bits of the expression+signature hash      */
} hipmr_handle_info;

hipmr_status hipmr_get_handle_info(hipmr_handle h, hipmr_handle_info *info);

/* Declared argument k: dtype (HIPMR_*), whether it is a pointer, declared
 * const, read and/or written by the expression (as the classifier sees it). */
hipmr_status hipmr_get_arg_info(hipmr_handle h, int32_t k, int32_t *dtype, int32_t *is_pointer,
                                int32_t *is_const, int32_t *is_read, int32_t *is_written);

/* How the expression indexes declared argument k (bit flags, as the classifier
 * sees it): HIPMR_ACCESS_INDEX name[i] (read or written), HIPMR_ACCESS_SHIFTED
 * name[i +/- E] with E uniform, HIPMR_ACCESS_FIXED name[<integer literal>],
 * HIPMR_ACCESS_OTHER any other index or a bare pointer.  An array with INDEX
 * or SHIFTED access must hold at least n elements (the binding checks this);
 * one with only FIXED access needs only the elements it names.  0 for a
 * scalar argument.  Errors: E_INVALID (NULL, k out of range). */
#define HIPMR_ACCESS_INDEX   1
#define HIPMR_ACCESS_SHIFTED 2
#define HIPMR_ACCESS_FIXED   4
#define HIPMR_ACCESS_OTHER   8
hipmr_status hipmr_get_arg_access(hipmr_handle h, int32_t k, int32_t *access);

/* Generated HIP source of one kernel variant (for inspection and tests).
 *   kind: 0 elementwise (vector), 1 elementwise (scalar), 2 reduce stage 1
 *         (vector), 3 reduce stage 1 (scalar), 4 reduce stage 2.
 *   combine_op/neutral: required for kinds 2-4.
 * Copies at most cap bytes including the terminating NUL; *len gets the full
 * length (without NUL). */
hipmr_status hipmr_get_kernel_source(hipmr_handle h, int32_t kind, const char *combine_op,
                                     const char *neutral, char *buf, size_t cap, size_t *len);

/* Symbols of the kernels the most recent elementwise / reduce call on this
 * handle launched (in launch order, comma-separated), e.g. for matching
 * profiler output.  Same buffer convention as hipmr_get_kernel_source. */
hipmr_status hipmr_get_last_symbols(hipmr_handle h, char *buf, size_t cap, size_t *len);

/* Compile-cache counters (process-wide).  Section "Core Method": a source
 * already compiled is found in memory (looked up by the source text) or in
 * the on-disk cache (a file named by the SHA-256 of the source, compiler
 * options and hipRTC version, under $HIPMR_CACHE_DIR, default
 * $XDG_CACHE_HOME/hipmr or ~/.cache/hipmr) instead of recompiling. */
typedef struct hipmr_cache_stats {
    uint64_t memory_hits;
    uint64_t disk_hits;
    uint64_t compiles;
    uint64_t disk_rejects;     /* corrupt or truncated cache files rebuilt        */
    double   compile_ms;       /* wall time spent in hipRTC                       */
} hipmr_cache_stats;

hipmr_status hipmr_get_cache_stats(hipmr_cache_stats *out);

/* Forgets the in-memory cache of code objects.  Existing handles stay valid
 * and keep the kernels they have built; new handles, and kernels a handle has
 * not built yet, come from the disk cache or are recompiled.  For tests and
 * measurements of the disk cache. */
void hipmr_cache_drop_memory(void);

/* Hex SHA-256 (FIPS 180-4) of a byte string, the function behind the disk
 * cache's file names and the hash in kernel symbols.  out must hold 65 bytes. */
hipmr_status hipmr_sha256_hex(const void *data, size_t len, char *out);

/* Size in bytes of a dtype code, 0 if unknown. */
int32_t hipmr_dtype_size(int32_t dtype);

/* Compiles a representative set of kernel variants of every template with
 * hipRTC (no GPU needed); returns the number compiled in *count.  A build
 * check of the device templates. */
hipmr_status hipmr_selftest_compile(int32_t *count);

#ifdef __cplusplus
}
#endif

#endif /* HIPMR_H_ */
