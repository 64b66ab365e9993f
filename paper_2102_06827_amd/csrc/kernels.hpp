// kernels.hpp -- launch interfaces of the HIP kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace comet {

// Offset tables of one gather product C[m,n] = sum_k A[m,k] * B[k,n]:
// addr_A(m,k) = offAm[m] + offAk[k], addr_B(k,n) = offBk[k] + offBn[n],
// addr_C(m,n) = offCm[m] + offCn[n]  (elements).
struct GettTables {
  const int64_t *offAm, *offAk, *offBk, *offBn, *offCm, *offCn;
};

// Stream-K split of the last `tiles` output tiles over `blocks` extra
// workgroups; ws holds 2 * blocks partial tiles (gett_sk_slot_bytes each).
// tiles == 0: every tile is computed whole by its own workgroup.
struct StreamK {
  int tiles = 0;
  int blocks = 0;
  void *ws = nullptr;
  // nonzero: the balanced schedule instead: the first `whole` tiles whole,
  // then one round of `blocks` workgroups that split the `tiles` leftover
  // tiles along the summation (both in one launch, gett_whole_piece_kernel),
  // tile r into
  // the pieces floor(blocks * r / tiles) .. floor(blocks * (r + 1) / tiles) - 1
  // (at least two), which gett_piece_fixup_kernel sums; ws holds one slot
  // per piece
  int even = 0;
  int whole = 0;
};

// Batch labels: entries first .. first + count - 1 of the per-entry base
// offsets (elements) of A, B and C; offA == nullptr means no batch labels.
// A launch's grid is tiles x entries (at most 65535 entries per launch);
// tiles 1 and 3.
struct GettBatch {
  const int64_t *offA = nullptr, *offB = nullptr, *offC = nullptr;
  int64_t first = 0;
  int64_t count = 1;
};

// dtype_in/out: 0 = double, 1 = float.  compute: 0 = FP64 MFMA, 1 = FP32 MFMA.
struct GettLaunch {
  const void *A;
  const void *B;
  void *C;
  GettTables t;
  int64_t M, N, K;
  double alpha, beta;
  int dtype;           // storage type of A, B, C
  int compute;         // 0: FP64 MFMA, 1: FP32 MFMA
  int layoutA;         // 0: A contiguous along K, 1: along M
  int layoutB;         // 0: B contiguous along K, 1: along N
  int vecA, vecB;      // 16-byte vector loads allowed
  int tile;            // tile variant
  int *occupancy = nullptr;   // when set: store the resident workgroups per CU, launch nothing
  int query_sk = 0;           // with occupancy: of the stream-K kernel instead (2: of the balanced one)
  StreamK sk;
  int persistent = 0;         // > 0: this many persistent workgroups walk the tiles (no stream-K)
  int shortk = 0;             // > 0: the short-summation kernel (K <= 32, tile 3) with this many workgroups
  GettBatch bt;               // batch labels: whole tiles only (no stream-K, not persistent)
};

hipError_t launch_gett(const GettLaunch &g, hipStream_t s);
// Workgroups of the kernel that launch_gett would run for g that fit on one
// CU at once (register and LDS limits), 0 if that variant does not exist.
int gett_occupancy(const GettLaunch &g);
int gett_tile_count();
// bytes of one stream-K workspace slot (one partial output tile)
size_t gett_sk_slot_bytes(int tile, int compute);
void gett_tile_shape(int tile, int *bm, int *bn, int *bk);
// whether a tile variant is compiled for this dtype/compute/vector
// combination (and with batch labels)
bool gett_tile_valid(int tile, int dtype, int compute, bool vecA, bool vecB, bool batch = false);

// GETT with FP32 operands split on the fly into three bfloat16 slices
// (the six products b_p c_q with p + q <= 2 on BF16 MFMA, FP32 accumulation);
// 64 x 64 tiles.  Requires g.dtype == 1 (FP32 storage).
hipError_t launch_fused_bf16x3(const GettLaunch &g, hipStream_t s);

// One problem of the persistent batched launch (device-resident).
struct BatchDesc {
  const void *A;
  const void *B;
  void *C;
  GettTables t;
  int64_t M, N, K;
  double alpha, beta;
  int variant;         // layoutA * 2 + layoutB, + 4 for element (non-vector) loads
  int cls;             // tile class (batch_class_shape); element loads: class 0 only
  int tilesN;          // output tiles of the class along N
};
struct BatchItem {
  int problem;
  int tile;            // tm * tilesN + tn in the problem's class
};
// The work list is cut into kBatchQueues queues, queue q holding items
// off[q] .. off[q + 1] - 1; the workgroups on XCD x (x = workgroup id mod 8)
// start with queue x and move on to the next queue once one is drained.
constexpr int kBatchQueues = 8;
struct BatchQueues {
  int64_t off[kBatchQueues + 1];
};
// Tile classes of the batched kernel (4 waves each, 2 x 2): 0: 64 x 64,
// 1: 128 x 64, 2: 64 x 128, 3: 128 x 128.
constexpr int kBatchClasses = 4;
void batch_class_shape(int cls, int *bm, int *bn);
// whether tile class `cls` is compiled for storage dtype (0 = FP64, 1 = FP32),
// mode (0: native MFMA, 1: fused BF16x3) and vector or element loads
bool batch_class_valid(int cls, int dtype, int mode, bool vec);
// mode 0: native MFMA of the storage type; 1: fused BF16x3 (FP32 storage).
// counters: kBatchQueues ints (reset inside the launch sequence).
hipError_t launch_batch(const BatchDesc *descs, const BatchItem *items, const BatchQueues &q, int *counters,
                        int dtype, int mode, int grid, hipStream_t s);
// persistent workgroups per CU for the batched kernel
int batch_blocks_per_cu(int dtype, int mode);

// C[offCb[b] + offCm[m] + offCn[n]] = beta * C over NB batch entries
// (offCb == nullptr: NB must be 1 and offCb[0] reads as 0); beta == 0 writes
// zeros without reading.
// Matrix-vector product (one free index group empty):
//   C[offC0[0] + offCj[j]] = alpha * sum_k X[offX0[0] + offXk[k]] * Y[offYj[j] + offYk[k]]
//                            + beta * C[...]   (C not read when beta == 0),
// j < J, k < K; all tables on the device.  kfast: Y is contiguous along k
// (else along j).  The summation is cut into `split` slabs of `slab` indices
// (split * slab >= K, slab <= kGemvSlab); with split > 1, ws holds split * J
// doubles of partial sums.  dtype 0: FP64 storage, 1: FP32.
constexpr int kGemvSlab = 1024;
struct GemvLaunch {
  const void *X, *Y;
  void *C;
  const int64_t *offXk, *offX0, *offYk, *offYj, *offC0, *offCj;
  int64_t J, K;
  int64_t slab;
  int split;
  int kfast;
  int dtype;
  double alpha, beta;
  void *ws;
};
hipError_t launch_gemv(const GemvLaunch &a, hipStream_t s);
// The slabs for J outputs over a summation of K on `cus` compute units.
void gemv_shape(int64_t J, int64_t K, bool kfast, int cus, int *split, int64_t *slab);

hipError_t launch_scale(void *C, int dtype, const int64_t *offCm, const int64_t *offCn, int64_t M, int64_t N,
                        double beta, hipStream_t s, const int64_t *offCb = nullptr, int64_t NB = 1);

// N-dimensional permutation out = alpha * in (+ beta * out), dims given in
// output order with both strides.
constexpr int kPermMaxDims = 12;
struct PermuteLaunch {
  const void *in;
  void *out;
  int ndim;
  int64_t ext[kPermMaxDims];
  int64_t s_in[kPermMaxDims];
  int64_t s_out[kPermMaxDims];
  double alpha, beta;
  int dtype;
  double fill = 0.0;   // with alpha == 0: out = fill + beta * out
};
hipError_t launch_permute(const PermuteLaunch &p, hipStream_t s);

}  // namespace comet
