/*
 * comet.h -- C ABI of the MI355X (gfx950) permuted tensor-contraction library.
 *
 * The library computes the binary tensor contraction of Section 2 of the COMET
 * paper (arXiv 2102.06827): the output C over its free (external) indices is
 * the sum, over the summation indices shared by A and B, of A * B.  As in the
 * ta.tc operation of Section 5 the product is scaled by alpha; the "=", "+="
 * and "-=" forms of the operation grammar (Fig. 2) map to beta = 0, beta = 1,
 * and beta = 1 with alpha negated:
 *
 *     C[free] = alpha * sum_{summation} A[...] * B[...]  +  beta * C[free]
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * spec     "C=A*B" label strings, e.g. "abij=acik*cbkj".  One ASCII letter per
 *          tensor dimension, blanks ignored, rank <= COMET_MAX_RANK per tensor
 *          (rank 0 is allowed for C: a full contraction to a scalar).  Every
 *          label must appear in at least two of C, A, B: free labels in C and
 *          one input, summation labels in A and B, and batch labels in all
 *          three.  A batch label indexes C, A and B alike and is not summed
 *          (e.g. "bij=bik*bkj" is a batch of matrix products, "ij=ij*ij" the
 *          elementwise product); the operation grammar of Section 4 does not
 *          rule such labels out.  The native FP64 / FP32 products run all
 *          batch entries in one launch; the split modes run one contraction
 *          per entry.  The TTGT path (COMET_PATH_TTGT) has no batch labels
 *          and returns COMET_ERR_UNSUPPORTED for them.  A label
 *          in one tensor only, or repeated inside one tensor, returns
 *          COMET_ERR_INVALID_SPEC.
 * extents  one int64 per distinct label, in order of first appearance when
 *          scanning C's labels, then A's, then B's.  Negative extents and
 *          tensor sizes that overflow int64 return COMET_ERR_INVALID_SHAPE.
 *          Zero extents are allowed (empty output: nothing happens; empty
 *          summation: C = beta * C).
 * strides  element strides per tensor, in the order of that tensor's labels,
 *          or NULL for dense row-major (the storage the paper's cost model
 *          assumes, Section 6).  Negative strides return
 *          COMET_ERR_INVALID_STRIDE.  Stride 0 (broadcast) is allowed for A
 *          and B.  C must not overlap itself: stride 0 on a C dimension of
 *          extent > 1, or dimensions that interleave, return
 *          COMET_ERR_INVALID_STRIDE.
 *          A stepped index range [lo:hi:step] of a label (Section 4, index
 *          labels with a range; read here as the indices lo, lo + step, ...
 *          below hi) is a view: pass the base pointer moved to element lo,
 *          the extent ceil((hi - lo) / step) and the stride multiplied by
 *          step.
 * pointers A, B, C and workspaces are device pointers owned by the caller;
 *          the library never frees them and keeps none after the call
 *          returns (except inside a graph the caller captured).  C must not
 *          alias A or B (the same base pointer returns COMET_ERR_UNSUPPORTED).
 * stream   a hipStream_t passed as void*; NULL is the null stream.  All work
 *          is enqueued on it; calls return after the enqueue.
 * beta     beta == 0 means C is not read (NaN/Inf in C do not propagate);
 *          alpha == 0 means A and B are not read.  For FP32 storage alpha and
 *          beta are rounded to float.
 * errors   every argument is validated on the host before anything is
 *          enqueued; on error nothing is enqueued and C is untouched.
 *          comet_last_error() gives a thread-local message for the last
 *          failing call of the calling thread.  A HIP launch failure returns
 *          COMET_ERR_HIP; a device fault surfaces at the caller's next sync.
 * determinism  the same plan and inputs give bit-identical outputs: no
 *          atomics in any reduction; where the summation of an output tile
 *          is split across workgroups (stream-K, or the balanced schedule's
 *          pieces), the pieces are added in a fixed order.
 */
#ifndef COMET_H
#define COMET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define COMET_MAX_RANK 12
#define COMET_VERSION_STRING "0.1.0"

typedef enum {
  COMET_OK = 0,
  COMET_ERR_INVALID_SPEC = 1,
  COMET_ERR_INVALID_SHAPE = 2,
  COMET_ERR_INVALID_STRIDE = 3,
  COMET_ERR_NULL_POINTER = 4,
  COMET_ERR_UNSUPPORTED = 5,
  COMET_ERR_WORKSPACE = 6,
  COMET_ERR_HIP = 7,
  COMET_ERR_INTERNAL = 8
} comet_status_t;

/* Storage type of A, B and C. */
typedef enum { COMET_F64 = 0, COMET_F32 = 1 } comet_dtype_t;

/* Arithmetic used for the products.
 *   DEFAULT      the matrix-core type of the storage type (F64 -> F64, F32 -> F32).
 *   F64          FP64 MFMA, FP64 accumulation (FP32 inputs are widened exactly).
 *   F32          FP32 MFMA, FP32 accumulation (FP64 inputs are rounded to FP32).
 *   SPLIT_BF16   each row of A and column of B is scaled by a power of two to
 *                its largest magnitude over the summation labels and cut into
 *                S 8-bit integer slices held exactly in bfloat16 (error-free
 *                splitting in the manner of Ozaki et al. 2012); slice pairs
 *                with p + q < S run on BF16 MFMA with FP32 accumulation, the
 *                leading partial sums kept exact over short chunks and folded
 *                into FP64.  S comes from comet_set_split_slices (default 5).
 *   SPLIT_BF16X3 x = b0 + b1 + b2 with b_i = bf16 of the remainder (Henry,
 *                Tang and Heinecke 2019); the six products b_p*c_q with
 *                p + q <= 2 on BF16 MFMA, one FP32 accumulator.
 *   SPLIT_FP16X2 x = h0 + h1 * 2^-11, h0 = fp16(x), h1 = fp16((x - h0) * 2^11),
 *                rows scaled by a power of two into FP16 range (Ootomo and
 *                Yokota 2022); three FP16 MFMA products, FP32 accumulation.
 *   SPLIT_INT8   the same exponent-aligned splitting with 7-bit integer
 *                slices (|s| <= 127) held in int8, slice pairs with p + q < S
 *                on the INT8 matrix cores with exact int32 accumulation per
 *                diagonal p + q, combined in FP64 at the end (the error-free
 *                splitting above carried out on integer units).  S comes from
 *                comet_set_int8_slices (default 6).
 * Split modes accumulate the final result in FP64 before the alpha/beta
 * epilogue and need a workspace for the slices. */
typedef enum {
  COMET_COMPUTE_DEFAULT = 0,
  COMET_COMPUTE_F64 = 1,
  COMET_COMPUTE_F32 = 2,
  COMET_COMPUTE_SPLIT_BF16 = 3,
  COMET_COMPUTE_SPLIT_BF16X3 = 4,
  COMET_COMPUTE_SPLIT_FP16X2 = 5,
  COMET_COMPUTE_SPLIT_INT8 = 6
} comet_compute_t;

/* Which lowering a plan uses.
 *   AUTO  the planner's choice: the fused gather path, except TTGT where
 *         the autotune cache recorded it as faster for this problem class,
 *         and for native FP64 / FP32 products (no batch labels) whose
 *         operands only the gather path's element loads can read (their
 *         unit strides lie on different summation labels) where an estimate
 *         of the permutes' traffic and launches against the GEMM time they
 *         save says TTGT is faster (from about 768^3 on MI355X).
 *   GETT  operands are gathered through per-label offset tables straight into
 *         on-chip tiles; no transposed copies are made.  A native product
 *         with one output row (the vector operand has no free label) streams
 *         the matrix through a matrix-vector kernel instead, its summation
 *         cut into slabs whose partial sums are added in a fixed order
 *         (environment variable COMET_GEMV=0 keeps the tiles;
 *         COMET_GEMV_SPLIT=n asks for about n slabs).
 *   TTGT  transpose-transpose-GEMM-transpose (Section 2; Section 6 "TTGT"):
 *         A and B are permuted into matrices, multiplied, and the product is
 *         permuted into C.  The flattening (Section 6 "Optimal permutation
 *         for TTGT") is the fastest under a time model of the permute
 *         kernels and the product on MI355X; environment variable
 *         COMET_TTGT_MODEL=weights takes the cost model Section 6 publishes
 *         instead. */
typedef enum { COMET_PATH_AUTO = 0, COMET_PATH_GETT = 1, COMET_PATH_TTGT = 2 } comet_path_t;

typedef struct comet_plan_s *comet_plan_t;
typedef struct comet_batch_s *comet_batch_t;

/* One problem of a batch: the same meaning as the comet_contract arguments. */
typedef struct {
  const char *spec;
  const int64_t *extents;
  const int64_t *strides_A;   /* NULL = dense row-major */
  const int64_t *strides_B;
  const int64_t *strides_C;
  double alpha;
  double beta;
  const void *A;
  const void *B;
  void *C;
} comet_problem_t;

/*
 * comet_contract -- one contraction, C = alpha * contract(A, B) + beta * C
 * (Section 2 equations; ta.tc of Section 5).  Convenience call: plans on
 * first use (cached per spec, extents, strides, dtype, compute, device; at
 * most 1024 plans per device, past which the call waits for the device and
 * empties that device's cache) and uses a library-owned, stream-ordered
 * workspace.  Returns
 * COMET_ERR_UNSUPPORTED if the stream is being captured (use the plan API
 * there).
 */
comet_status_t comet_contract(const char *spec, const int64_t *extents,
                              comet_dtype_t dtype, comet_compute_t compute,
                              double alpha, const void *A, const int64_t *strides_A,
                              const void *B, const int64_t *strides_B,
                              double beta, void *C, const int64_t *strides_C,
                              void *stream);

/*
 * Plan API.  comet_plan_create parses and validates the problem, fuses labels
 * (consecutive indices merged as in the TTGT flattening of Section 2), builds
 * the per-label offset tables, picks the lowering and the tile shape, and
 * uploads the tables to the current device (so it allocates and is not
 * capturable).  comet_plan_execute enqueues the contraction with a caller
 * workspace of at least comet_plan_workspace_size bytes (256-byte aligned;
 * may be NULL when the size is 0) and is capturable into a HIP graph.
 * Pointer arguments of execute must satisfy the alignment the plan was
 * made for; misaligned pointers take the scalar gather, never an error.
 * The workspace holds TTGT's permuted operands, the split modes' slices, or
 * the partial sums of a stream-K or balanced schedule (output tiles whose
 * summation is split over several workgroups and summed afterwards in a
 * fixed order, so results do not depend on timing; the balanced schedule
 * cuts the tiles left after the last full round of whole tiles into one
 * more full round of equal pieces); its contents on entry do not matter and
 * executions that share one workspace must not overlap.
 */
comet_status_t comet_plan_create(comet_plan_t *plan, const char *spec, const int64_t *extents,
                                 const int64_t *strides_A, const int64_t *strides_B,
                                 const int64_t *strides_C, comet_dtype_t dtype,
                                 comet_compute_t compute);
comet_status_t comet_plan_create_ex(comet_plan_t *plan, const char *spec, const int64_t *extents,
                                    const int64_t *strides_A, const int64_t *strides_B,
                                    const int64_t *strides_C, comet_dtype_t dtype,
                                    comet_compute_t compute, comet_path_t path);
comet_status_t comet_plan_workspace_size(comet_plan_t plan, size_t *bytes);
comet_status_t comet_plan_execute(comet_plan_t plan, double alpha, const void *A, const void *B,
                                  double beta, void *C, void *workspace, size_t ws_bytes,
                                  void *stream);
comet_status_t comet_plan_destroy(comet_plan_t plan);

/*
 * comet_plan_execute_noalloc -- comet_plan_execute without a caller
 * workspace and without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The workspace is a static device
 * buffer of COMET_NOALLOC_SCRATCH_BYTES that the library holds on every GPU
 * it runs on until the process ends; the caller still passes A, B, C and the
 * stream as for comet_plan_execute, with the same meaning, layout and
 * results.  A plan whose comet_plan_workspace_size exceeds the buffer is
 * refused with COMET_ERR_WORKSPACE before anything is enqueued.  All calls on
 * one GPU share that GPU's buffer, which keeps whatever the last call left
 * (every plan writes each workspace byte before reading it, so nothing needs
 * clearing): calls that may overlap in time on one GPU (two streams, or two
 * threads) race on it and must be ordered by the caller.  The first call on a
 * device looks up that device's buffer address (hipGetSymbolAddress), which
 * is not capturable; later calls are.
 */
#define COMET_NOALLOC_SCRATCH_BYTES (128u << 20)
comet_status_t comet_plan_execute_noalloc(comet_plan_t plan, double alpha, const void *A,
                                          const void *B, double beta, void *C, void *stream);

/* Writes a JSON description of the plan into buf (host only): path, the
 * label classes after fusion ("M", "N", "K" and the batch labels "X", with
 * extents and strides), flattened sizes m, n, k and batch entries nb,
 * operand layouts and contiguous runs, tile shape, stream-K split
 * (sk_tiles, sk_blocks; with even = 1 the balanced schedule: the first
 * even_whole tiles whole, then the sk_tiles leftover tiles cut into sk_blocks
 * pieces), persistent workgroups, resident workgroups per CU, the
 * short-summation kernel's workgroups (shortk), the matrix-vector kernel
 * (gemv: 1 reads the matrix along the output, 2 along the summation; 0 not
 * used) and its summation slabs (gemv_split), the split tile and whether
 * FP32 BF16x3 runs fused, TTGT permutations with their Section 6 cost and
 * modelled time (model_us).  COMET_ERR_WORKSPACE if buf is too small (the
 * text is truncated). */
comet_status_t comet_plan_describe(comet_plan_t plan, char *buf, size_t len);

/*
 * comet_analyze -- host-only planning without a device: validates exactly as
 * comet_plan_create does and writes the same JSON as comet_plan_describe.
 * Allocates no device memory and launches nothing.
 */
comet_status_t comet_analyze(const char *spec, const int64_t *extents,
                             const int64_t *strides_A, const int64_t *strides_B,
                             const int64_t *strides_C, comet_dtype_t dtype,
                             comet_compute_t compute, comet_path_t path,
                             char *buf, size_t len);

/*
 * Batch API: n independent contractions in ONE persistent kernel launch.
 * Every problem gets a tile class (64 x 64, 128 x 64, 64 x 128 or 128 x 128
 * outputs per workgroup; element-load problems and FP64 use the classes
 * their kernels have): COMET_BATCH_CLASS=<class> forces one, the autotuner
 * (comet_autotune on) times the classes per problem class (storage dtype,
 * compute, operand layouts, power-of-two buckets of the flattened sizes) on
 * a batch of copies of a representative problem and caches the winner, and
 * otherwise a throughput model picks the class.  The work list is cut into
 * one queue per XCD; whole problems go to queues by longest processing time
 * first, heaviest first within a queue, each problem's tiles in groups of
 * tile rows.  Workgroups take (problem, tile) items from their XCD's queue
 * through a device counter and move on to the other queues once it is
 * drained, so many small, uneven problems fill the GPU together.  A problem
 * whose operands only the element-load kernel could gather (their unit
 * strides on different summation labels) gets a dense copy of one operand,
 * held by the batch and refreshed by every execute before the launch, in a
 * label order both operands can be read from in 16-byte vectors
 * (COMET_BATCH_COPY=0 keeps the element-load kernel instead).
 * All problems share dtype and compute; compute must be the storage type's
 * native MFMA (DEFAULT, or F64 / F32 matching the dtype), or SPLIT_BF16X3
 * with FP32 storage (operands split into three bfloat16 slices inside the
 * loader).  Problems with an empty summation or alpha == 0 are scaled by
 * beta before the launch.  A problem with batch labels contributes one
 * problem per batch entry to the work list (at most 2^22 problems and batch
 * entries in all, COMET_ERR_UNSUPPORTED beyond; at most 2^31 - 2^20 output
 * tiles).  The workspace holds the eight queue counters (256 bytes); its
 * contents on entry do not matter.
 * comet_batch_create plans every problem and uploads the work list and
 * offset tables (not capturable); comet_batch_execute is capturable.
 * comet_batch_describe writes JSON: output tiles, persistent grid, mode,
 * problems per tile class, items per queue, how many classes came from the
 * autotuner and how many operand copies run before the launch.
 */
comet_status_t comet_batch_create(comet_batch_t *batch, int n, const comet_problem_t *problems,
                                  comet_dtype_t dtype, comet_compute_t compute);
comet_status_t comet_batch_workspace_size(comet_batch_t batch, size_t *bytes);
comet_status_t comet_batch_execute(comet_batch_t batch, void *workspace, size_t ws_bytes,
                                   void *stream);
comet_status_t comet_batch_describe(comet_batch_t batch, char *buf, size_t len);
comet_status_t comet_batch_destroy(comet_batch_t batch);

/*
 * comet_permute -- the ta.copy operation of Section 5 (out = alpha * in with
 * the labels permuted, Section 4 "labeled tensors"), plus beta * out:
 * spec "ji=ij" (same labels on both sides).  Tiled through LDS so reads and
 * writes are both coalesced (Section 6 "Transpose optimization").
 */
comet_status_t comet_permute(const char *spec, const int64_t *extents, comet_dtype_t dtype,
                             double alpha, const void *in, const int64_t *strides_in,
                             double beta, void *out, const int64_t *strides_out,
                             void *stream);

/*
 * Multi-operand contraction chains (Section 5: ta.mult, ta.set; Section 6,
 * "Multi-Operand Expression").  spec "C=A1*A2*...*An", 2 <= n <= 8, every
 * label in at least two of the tensors (a label in more than two is a batch
 * label of the steps that meet it while another tensor still holds it);
 * extents one per distinct label, in order of first appearance scanning C
 * then A1..An.
 *
 * comet_chain_plan (host only, no device needed) chooses the grouping with
 * the fewest algorithmic operations (a search over every binary tree) and
 * writes it as JSON into buf: {"flops", "natural_flops" (left to right),
 * "steps": [{"left", "right", "spec", "flops"}]} where operands 0..n-1 are
 * the inputs and n.. the intermediates in step order.  COMET_ERR_WORKSPACE if
 * buf is too small.
 *
 * comet_contract_chain computes C = alpha * (A1 * ... * An) + beta * C in
 * that order, one binary contraction per step through the comet_contract
 * path; intermediates are dense, held in a library-owned device buffer that
 * grows as needed (so, like comet_contract, it refuses to run under stream
 * capture).  operands[i] are device pointers, strides[i] their element
 * strides (strides or any strides[i] NULL: dense row-major).
 */
comet_status_t comet_chain_plan(const char *spec, const int64_t *extents, char *buf, size_t len);
comet_status_t comet_contract_chain(const char *spec, const int64_t *extents, comet_dtype_t dtype,
                                    comet_compute_t compute, double alpha, int n, const void *const *operands,
                                    const int64_t *const *strides, double beta, void *C,
                                    const int64_t *strides_C, void *stream);

/*
 * comet_fill -- the ta.fill operation of Section 5: every element of the
 * tensor at `out` (device pointer, owned by the caller) is set to `value`
 * (rounded to FP32 for FP32 storage).  The tensor has `rank` dimensions
 * (0 <= rank <= COMET_MAX_RANK; rank 0 is one element) with the given
 * extents and element strides (NULL: dense row-major); strides must not make
 * two elements share an address.  Enqueued on `stream`, nothing is read.
 * Errors: COMET_ERR_INVALID_SHAPE (rank or a negative extent),
 * COMET_ERR_INVALID_STRIDE (negative or overlapping strides),
 * COMET_ERR_NULL_POINTER (out NULL for a non-empty tensor), COMET_ERR_HIP.
 */
comet_status_t comet_fill(int rank, const int64_t *extents, comet_dtype_t dtype, double value, void *out,
                          const int64_t *strides, void *stream);

/*
 * Autotuner (Section 6: tile sizes chosen for the memory hierarchy, here by
 * timing on the device).  mode 0: off (heuristic tiles); 1: use the cache at
 * cache_path and time candidates for problem classes it does not hold,
 * appending them; 2: re-time everything.  What is timed: for a plan, every
 * compiled gather tile (each with its stream-K split) and up to 32 TTGT
 * flattenings of the native modes; for a split mode, the slice-pair product's
 * tiles (the 128 x 64 and 192 x 192 products of the classic splits, and the
 * fused and sliced BF16x3 paths on FP32 storage); for a batch, the tile
 * classes per problem class.  Each candidate runs once to warm up, then five
 * timed runs on nonzero operands; the fastest is recorded.  A corrupt cache
 * file is ignored and rewritten.  cache_path NULL uses $COMET_TUNE_CACHE or
 * ~/.cache/comet_tune.json.  Before the first call the mode is the one the
 * environment variable COMET_AUTOTUNE names (off, on, force), off if unset.
 */
comet_status_t comet_autotune(const char *cache_path, int mode);

/* Number of slices S used by COMET_COMPUTE_SPLIT_BF16 for plans created
 * afterwards; 3 <= S <= 6 (COMET_ERR_UNSUPPORTED otherwise). */
comet_status_t comet_set_split_slices(int S);
/* Number of slices S used by COMET_COMPUTE_SPLIT_INT8 for plans created
 * afterwards; 3 <= S <= 8 (COMET_ERR_UNSUPPORTED otherwise). */
comet_status_t comet_set_int8_slices(int S);

const char *comet_last_error(void);
const char *comet_version(void);

#ifdef __cplusplus
}
#endif

#endif /* COMET_H */
