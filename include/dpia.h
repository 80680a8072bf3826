/*
 * dpia.h -- C ABI of the MI355X (gfx950) strategy-preserving reduction
 * library: dot, asum and gemv computed under an explicit DPIA
 * parallelisation strategy, with the floating-point association order the
 * strategy's functional expression fixes.
 *
 * The method: Atkey, Steuwer, Lindley, Dubach, "Strategy Preserving
 * Compilation for Parallel Functional Code".  A strategy is the blocked
 * dot-product expression of Sec. 2.1, eq. (2):
 *
 *   reduceSeq (+) 0 (mapWorkgroup (lam ch. COMBINE (mapLocal
 *       (lam s. reduceSeq (lam x a. (fst x * snd x) + a) 0 s) (ROWS ch)))
 *     (split W (zip xs ys)))
 *
 * with W = L*C, ROWS ch = split C ch (contiguous: work-item l folds
 * elements l*C .. l*C+C-1 of its chunk) or the strided rows l, l+L, ...,
 * and COMBINE the in-work-group fold of the L work-item results: a binary
 * tree in local memory (Sec. 6.1 toLocal; every node (0 + left) + right,
 * leaves in work-item order) or a sequential reduceSeq.  The chunk results
 * are folded by a sequential reduceSeq from +0 in chunk order (the last
 * loop of the blocked listing of Sec. 2.2).  map and its hierarchy variants
 * mean the same (Sec. 6.1) and reduce is a left fold from its initial value
 * in increasing index order (Sec. 4.2, Stage II), so the strategy fixes
 * every rounding: results are bit-identical to a CPU evaluation of that
 * expression, independent of the physical grid, the stream, repetition and
 * the number of passes.
 *
 * Conventions for every call below:
 *  - Every array argument is a device pointer (hipMalloc'd or a torch CUDA
 *    tensor's data) owned by the caller; the library never allocates, frees
 *    or synchronises.  Calls are asynchronous on `stream` (NULL = the
 *    default stream); results stay in device memory.
 *  - Arrays are dense, unit-stride, and 16-byte aligned; gemv's A is
 *    row-major with leading dimension lda (in elements), and
 *    lda * element size must be a multiple of 16 bytes.
 *  - All validation happens before any launch.  On an error nothing is
 *    launched, no output is touched, and a description is available from
 *    dpia_last_error_detail() in the calling thread.
 *  - No floating-point atomics are used; the only atomic is an integer
 *    arrival counter of the 1-pass combine.
 */
#ifndef DPIA_H
#define DPIA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DPIA_ABI_VERSION 2u

/* Same type as hipStream_t. */
typedef struct ihipStream_t* dpia_stream_t;

typedef enum {
  DPIA_OK = 0,
  DPIA_ERR_NULL = 1,       /* a required pointer is NULL                    */
  DPIA_ERR_SHAPE = 2,      /* sizes do not fit the strategy, or misaligned   */
  DPIA_ERR_STRATEGY = 3,   /* invalid descriptor (see dpia_strategy)        */
  DPIA_ERR_DTYPE = 4,      /* unsupported element / output type combination */
  DPIA_ERR_WORKSPACE = 5,  /* workspace NULL or smaller than required       */
  DPIA_ERR_HIP = 6,        /* a HIP launch failed (detail has its text)     */
  DPIA_ERR_ABI = 7         /* descriptor abi_version != DPIA_ABI_VERSION    */
} dpia_status;

typedef enum {
  DPIA_F32 = 0,            /* IEEE binary32                                  */
  DPIA_F64 = 1,            /* IEEE binary64 (Kahan result only)              */
  DPIA_I32 = 2,            /* 32-bit integers, arithmetic modulo 2^32        */
  DPIA_BF16 = 3,           /* bfloat16 storage, decoded exactly to binary32  */
  DPIA_FP8_E4M3 = 4        /* OCP fp8 E4M3 storage (max 448, no inf)         */
} dpia_dtype;

typedef enum { DPIA_OP_DOT = 0, DPIA_OP_ASUM = 1, DPIA_OP_GEMV = 2, DPIA_OP_SCAL = 3 } dpia_op;

typedef enum {
  DPIA_ORDER_CONTIGUOUS = 0, /* ROWS ch = split C ch                          */
  DPIA_ORDER_STRIDED = 1     /* ROWS ch = transpose (split L ch): l, l+L, ... */
} dpia_order;

typedef enum {
  DPIA_COMBINE_TREE = 0,     /* pairwise tree over the L lanes, lane order     */
  DPIA_COMBINE_SEQ = 1,      /* reduceSeq (+) 0 over the L lanes              */
  DPIA_COMBINE_NONE = 2      /* no work-group combine: every lane's value is a
                                chunk value (join of the mapLocal level, as in
                                the dot expression of Sec. 6.2), so the outer
                                fold runs over G * L values; dot / asum only */
} dpia_combine;

typedef enum {
  DPIA_ACCUM_PLAIN = 0,      /* binary32 (or integer) accumulators            */
  DPIA_ACCUM_KAHAN = 1,      /* compensated (s, c) accumulators, dot only:
                                Kahan's step in the lanes (Higham, Accuracy
                                and Stability of Numerical Algorithms,
                                Alg. 4.2), Knuth's TwoSum merge in the
                                combines, value s - c                       */
  DPIA_ACCUM_SUM2 = 2        /* compensated (s, c), dot only: Sum2 of Ogita,
                                Rump and Oishi (SIAM J. Sci. Comput. 26(6),
                                2005, Alg. 4.4) over the rounded products:
                                TwoSum at every step and merge, the exact
                                errors summed in c, value s + c             */
} dpia_accum;

/*
 * Strategy descriptor.  Level assignment is implied: chunks are the
 * mapWorkgroup level, lanes the mapLocal level, the per-lane fold is
 * reduceSeq in private memory (toPrivate), a tree combine lives in local
 * memory (toLocal), chunk results in global memory.
 *
 *  seq_len      C, elements folded sequentially by one lane (>= 1)
 *  local_size   L, lanes per chunk (>= 1; a power of two for a tree)
 *  order        dpia_order
 *  wg_combine   dpia_combine (L = 1 always means 0 + lane)
 *  passes       1: the last work-group to finish folds the chunk results;
 *               2: a second kernel does.  Same expression, same bits.
 *               gemv needs no cross-work-group step and takes 1 or 2.
 *  accum        dpia_accum
 *  final_f64    compensated only: fold the chunk values (s - c for Kahan,
 *               s + c for Sum2) in binary64
 *  rows_per_wg  gemv: R rows per work-group (M must be a multiple)
 *  row_parts    gemv: 1, or 2 halves per row, each reduced with (C, L)
 *               and folded as (0 + h0) + h1
 *  max_grid     0 = automatic; else an upper bound on launched work-groups
 *               (work is distributed by a grid-stride loop; no effect on
 *               the result)
 *  vec_width    dot / asum: 0 or 1 = scalar elements; V = 2 or 4: the inputs
 *               are read as vectors of V consecutive elements (Sec. 6.1
 *               asVector V), so lanes fold vectors: a chunk is L*C vectors
 *               (V*L*C elements), every lane keeps V component accumulators
 *               (component j folds elements j, j+V, ... of its vectors), the
 *               combine acts per component, and each chunk contributes its
 *               V components (asScalar V) -- or, with DPIA_COMBINE_NONE,
 *               its L lanes' V components each, lane by lane -- to the
 *               outer fold.  Plain accumulation only.
 */
typedef struct {
  uint32_t abi_version;
  uint32_t seq_len;
  uint32_t local_size;
  uint32_t order;
  uint32_t wg_combine;
  uint32_t passes;
  uint32_t accum;
  uint32_t final_f64;
  uint32_t rows_per_wg;
  uint32_t row_parts;
  uint32_t max_grid;
  uint32_t vec_width;
} dpia_strategy;

/*
 * Validate a strategy for an operation and problem size and report the
 * workspace it needs.  Host only, no HIP call, thread-safe.
 *   op, dt   operation and input element type (for gemv: the type of A)
 *   m, n     dot/asum: m ignored, n = vector length;
 *            gemv: m rows, n = k columns
 *   ws_bytes_out (may be NULL) receives the workspace size in bytes.
 */
dpia_status dpia_strategy_check(const dpia_strategy* s, dpia_op op, dpia_dtype dt,
                                int64_t m, int64_t n, size_t* ws_bytes_out);

/*
 * out[0] = dot(x, y) under strategy s (Sec. 2.1, eq. (2)).
 *   dt       DPIA_F32 or DPIA_I32 (both x and y)
 *   n        length; a multiple of W = seq_len * local_size (n = 0 gives +0)
 *   out_dt   DPIA_F32 for F32 input, DPIA_I32 for I32, DPIA_F64 allowed only
 *            with accum = KAHAN and final_f64 = 1 (else the binary64 fold is
 *            rounded once to binary32)
 *   ws       device workspace of at least dpia_strategy_check's size.  Its
 *            arrival counters (the 256 bytes after the chunk values, and, for
 *            staged contiguous tree strategies with at most 1024 chunks, the
 *            per-chunk counts at its end) must be zero before the first call
 *            on it (allocate it zeroed); every call leaves them zero.  Calls
 *            sharing one workspace must be ordered (same stream).
 */
dpia_status dpia_dot(const dpia_strategy* s, dpia_dtype dt, int64_t n, const void* x,
                     const void* y, void* out, dpia_dtype out_dt, void* ws, size_t ws_bytes,
                     dpia_stream_t stream);

/*
 * dpia_dot without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments, results and bits as dpia_dot with
 * the same strategy; no call allocates or frees memory.  The chunk values
 * and the 1-pass arrival counter live in a 1 MiB array inside the library,
 * one per GPU, held until the process ends: strategies whose chunk values
 * need more than 1 MiB - 256 bytes (G values of 4 bytes, 8 for compensated
 * pairs) are rejected with DPIA_ERR_WORKSPACE before anything is launched.
 * The first call on a device looks the array up and launches one small
 * kernel on `stream` that clears the counter.  All calls on one GPU share
 * its array: calls that may overlap (different streams without ordering,
 * concurrent host threads on unordered streams) race and give undefined
 * results; calls ordered on one stream are safe.
 */
dpia_status dpia_dot_noalloc(const dpia_strategy* s, dpia_dtype dt, int64_t n, const void* x,
                             const void* y, void* out, dpia_dtype out_dt, dpia_stream_t stream);

/*
 * out[0] = sum |x[i]| under strategy s, with the per-lane operator
 * lam x a. abs x + a (the paper benchmarks asum, Sec. 7.1; abs is the one
 * scalar primitive added to Fig. 5a).  dt = out_dt = DPIA_F32, plain only.
 * Workspace rules as for dpia_dot.
 */
dpia_status dpia_asum(const dpia_strategy* s, dpia_dtype dt, int64_t n, const void* x,
                      void* out, dpia_dtype out_dt, void* ws, size_t ws_bytes,
                      dpia_stream_t stream);

/*
 * y = A x (BLAS gemv, alpha = 1, beta = 0; Sec. 7.1 benchmark): every row is
 * reduced like a dot product of that row with x under (C, L, order,
 * combine), R rows per work-group.
 *   a_dt       DPIA_F32, DPIA_BF16, DPIA_FP8_E4M3 (binary32 accumulation of
 *              decoded values) or DPIA_I32 (then x, y are I32 too)
 *   m, k, lda  A is m x k row-major with leading dimension lda >= k (a
 *              multiple of the strategy's vector width); m a multiple of R;
 *              1 <= k <= seq_len * local_size * row_parts, shorter rows
 *              being read as extended with zeros (which no plain fold sees)
 *   row_scale  FP8 only (else NULL): y[r] = row_scale[r] * (row r . x)
 *   x, y       k and m elements: binary32 for F32, BF16 and FP8 matrices,
 *              I32 for an I32 matrix (hence untyped pointers here;
 *              dpia_gemv_blas, which takes no I32 matrix, types them float)
 *   ws         unused (pass NULL, 0)
 */
dpia_status dpia_gemv(const dpia_strategy* s, dpia_dtype a_dt, int64_t m, int64_t k,
                      int64_t lda, const void* A, const float* row_scale, const void* x,
                      void* y, void* ws, size_t ws_bytes, dpia_stream_t stream);

/*
 * BLAS form y := alpha * (A x) + beta * y of the Sec. 7.1 gemv benchmark.
 * Row r's value v is exactly dpia_gemv's (for FP8, row_scale[r] times the
 * row reduction); then y[r] = (alpha * v) + (beta * y[r]) with each
 * operation rounded once to binary32.  When beta == 0 (either sign) the old
 * y is not read, so it need not hold numbers, and y[r] = alpha * v.
 * Arguments as for dpia_gemv; a_dt is DPIA_F32, DPIA_BF16 or DPIA_FP8_E4M3
 * (DPIA_ERR_DTYPE otherwise).  No workspace.
 */
dpia_status dpia_gemv_blas(const dpia_strategy* s, dpia_dtype a_dt, int64_t m, int64_t k,
                           int64_t lda, float alpha, const void* A, const float* row_scale,
                           const float* x, float beta, float* y, dpia_stream_t stream);

/*
 * y[i] = alpha * x[i] for i < n (the scal benchmark of Sec. 7.1; BLAS sscal
 * when y == x).  A map: each element is one binary32 product, whatever the
 * strategy, which only places elements on work-groups (chunks of W) and
 * lanes (C elements each, contiguous or strided); wg_combine, passes and
 * accum are ignored.  dt = DPIA_F32; x and y 16-byte aligned; y may equal x.
 */
dpia_status dpia_scal(const dpia_strategy* s, dpia_dtype dt, int64_t n, float alpha,
                      const void* x, void* y, dpia_stream_t stream);

/*
 * Measurement aid, not an operation of the paper: the read-bandwidth
 * ceiling that the reductions' throughput is set against (Sec. 7.1 reports
 * bandwidth).  Reads the `bytes` bytes at device address x once, with
 * 16-byte non-temporal loads from `grid` work-groups of 256 threads, and
 * stores in sink[b] (device memory, `grid` uint32_t) the XOR of the 32-bit
 * words work-group b read: the XOR of sink[0 .. grid) is that of all of x.
 * x 16-byte aligned and bytes a non-negative multiple of 16, grid in
 * [1, 65536] (DPIA_ERR_SHAPE); DPIA_ERR_NULL for a NULL sink, or a NULL x
 * with bytes > 0.  Asynchronous; nothing is launched on an error or when
 * bytes == 0 (sink is then left as it is).
 */
dpia_status dpia_read_stream(const void* x, int64_t bytes, int32_t grid, uint32_t* sink,
                             dpia_stream_t stream);

/*
 * The two stages of a dot or asum strategy as separate calls.  dpia_chunks
 * evaluates the mapWorkgroup level only: chunks[g] = value of chunk g, i.e.
 * the work-group combine of its L lane folds (the OpenCL dot kernel of
 * Sec. 6.2 likewise writes its per-work-group results and leaves the last
 * reduction to a later step).  dpia_fold then computes the outer
 * reduceSeq (+) 0 over those values in chunk order.  Together they
 * give the same bits as dpia_dot / dpia_asum with the same strategy, whatever
 * its `passes`; a caller that gathers chunk values from several devices in
 * device order can fold them the same way.
 *   op       DPIA_OP_DOT (x and y) or DPIA_OP_ASUM (x; y ignored)
 *   dt, n    as for dpia_dot / dpia_asum
 *   chunks   device buffer of chunks_bytes >= G * values per chunk * value
 *            size.  A chunk has one value, or V with vec_width V, times L
 *            with DPIA_COMBINE_NONE (in lane, then component order); a
 *            value is the accumulator: 4 bytes (binary32 or I32), or a pair
 *            of binary32 (s, c), 8 bytes, for Kahan
 *   out, out_dt  as for dpia_dot / dpia_asum
 */
dpia_status dpia_chunks(const dpia_strategy* s, dpia_op op, dpia_dtype dt, int64_t n,
                        const void* x, const void* y, void* chunks, size_t chunks_bytes,
                        dpia_stream_t stream);

dpia_status dpia_fold(const dpia_strategy* s, dpia_op op, dpia_dtype dt, int64_t n,
                      const void* chunks, void* out, dpia_dtype out_dt, dpia_stream_t stream);

/*
 * Generated kernels.  The expression generator (Secs. 4 and 6: Stage I and
 * II translation, hoisting, one kernel per top-level parallel loop) emits
 * HIP source for a DPIA expression; hipcc turns it into a gfx950 code
 * object, and these calls load it and launch its kernels.
 *   dpia_module_load    loads the code object at `path` on the current
 *                       device; *out receives an opaque handle the caller
 *                       releases with dpia_module_unload.
 *   dpia_module_launch  launches `kernel` (a name in the module) with a 1-D
 *                       grid of `grid` work-groups of `block` work-items
 *                       (1..1024) on `stream`.  Every generated kernel takes
 *                       device pointers only: args[0 .. nargs) are those
 *                       pointers in the kernel's parameter order (at most
 *                       64, none NULL).  Asynchronous, like every call here.
 */
typedef struct dpia_module dpia_module;
dpia_status dpia_module_load(const char* path, dpia_module** out);
dpia_status dpia_module_launch(dpia_module* m, const char* kernel, uint32_t grid,
                               uint32_t block, void* const* args, int32_t nargs,
                               dpia_stream_t stream);
dpia_status dpia_module_unload(dpia_module* m);

/*
 * Batched execution: many independent dot / asum / gemv instances, each with
 * its own strategy.  A tile is a group of chunks (or gemv rows) of one
 * instance; the work-groups take the tiles, largest first, by a grid-stride
 * loop (the parforWorkgroup of Sec. 6.2).  Tiles only place work on
 * work-groups, so each instance's result has exactly the bits of the single
 * call (dpia_dot / dpia_asum / dpia_gemv) with the same strategy.  This is
 * the strategy-per-size-class execution that the paper's strategy search
 * (Sec. 1, building on Steuwer et al. 2015) produces, for workloads of many
 * small problems.  Two engines run a plan:
 *  - dpia_batch_run: two launches, the tiles, then one work-group per
 *    reduction instance folding its chunk values in chunk order;
 *  - dpia_batch_run_one_launch: one persistent launch; an arrival counter
 *    per instance counts the tiles whose chunk values are complete, and the
 *    work-group that completes the count folds that instance's values.
 * Both give the same bits.
 *
 * Restrictions: F32 data, plain accumulation, strategies whose vector width
 * is 16 bytes (strided: local_size, contiguous: seq_len a multiple of 4) and
 * whose threads per chunk divide 256; 16-byte aligned operands; gemv lda a
 * multiple of 4; dot/asum n >= 1 (ragged n is zero-extended as for the
 * single calls).
 */
typedef struct {
  uint32_t op;        /* dpia_op */
  uint32_t dtype;     /* DPIA_F32 */
  uint32_t strategy;  /* index into the plan's strategy array */
  uint32_t reserved;  /* 0 */
  int64_t m;          /* gemv rows (ignored for dot / asum) */
  int64_t n;          /* dot / asum: length; gemv: k */
  int64_t lda;        /* gemv leading dimension (ignored for dot / asum) */
  const void* a;      /* dot / asum: x; gemv: A (device) */
  const void* b;      /* dot: y; gemv: x; asum: NULL (device) */
  void* out;          /* dot / asum: one float; gemv: y, m floats (device) */
} dpia_instance;

typedef struct dpia_batch_plan dpia_batch_plan;

/*
 * Validates every instance against its strategy and builds the tile tables
 * on the host (largest tiles first).  The plan copies what it needs; the
 * arrays passed in may be freed afterwards.  Destroy with
 * dpia_batch_plan_destroy.  The device pointers inside the instances must
 * stay valid for every run.
 */
dpia_status dpia_batch_plan_create(const dpia_instance* inst, int32_t count,
                                   const dpia_strategy* strategies, int32_t nstrat,
                                   dpia_batch_plan** out);

/* Device workspace bytes a run needs (tables, counters, chunk values). */
size_t dpia_batch_workspace_bytes(const dpia_batch_plan* plan);

/* Enqueues on `stream` a copy of the plan's tables, with every counter
 * zeroed, into `ws` (256-byte aligned); call once per workspace before the
 * first run.  Does not wait: the plan must not be destroyed before the copy
 * has completed (e.g. before the stream reaches a later run). */
dpia_status dpia_batch_upload(const dpia_batch_plan* plan, void* ws, size_t ws_bytes,
                              dpia_stream_t stream);

/* Runs every instance: two kernel launches on `stream`, no allocation, no
 * memset, no synchronisation (may be captured in a graph and replayed).
 * Runs sharing a workspace must be ordered (same stream). */
dpia_status dpia_batch_run(const dpia_batch_plan* plan, void* ws, size_t ws_bytes,
                           dpia_stream_t stream);

/* Runs every instance in one kernel launch on `stream`: no allocation, no
 * memset, no synchronisation.  The launch leaves every arrival counter in
 * `ws` at zero again, so it may be captured in a graph and replayed, and
 * runs of either engine may follow each other on one workspace.  Runs
 * sharing a workspace must be ordered (same stream). */
dpia_status dpia_batch_run_one_launch(const dpia_batch_plan* plan, void* ws, size_t ws_bytes,
                                      dpia_stream_t stream);

void dpia_batch_plan_destroy(dpia_batch_plan* plan);

/* Static text for a status code. */
const char* dpia_status_str(dpia_status st);

/* Description of the last error in the calling thread ("" if none). */
const char* dpia_last_error_detail(void);

/* DPIA_ABI_VERSION of the loaded library. */
uint32_t dpia_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DPIA_H */
