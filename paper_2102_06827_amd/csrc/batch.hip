// batch.hip -- many independent contractions in one persistent launch, and
// the fused BF16x3 gather product.
//
// Persistent launch: the host lists every (problem, output tile) pair, each
// problem with the tile class the autotuner (or, untuned, a throughput
// model) chose for it, and starts as many workgroups as stay resident on the
// GPU.  The list is cut into one queue per XCD: the host hands whole problems
// to queues by longest-processing-time first, so that the workgroups of one
// XCD work on the same problems and find their operand panels in that XCD's
// L2, and within a queue the heaviest problems come first and each problem's
// tiles are walked in groups of tile rows.  Each workgroup takes the next
// item of its XCD's queue from a device counter, runs the gather tile routine
// for that problem's class and layout variant, and once its queue is drained
// moves on to the next queue -- every workgroup reaches the exit after at
// most one failed take per queue.  Uneven, small problems thus fill the
// machine together instead of one under-filled launch each.  The counters
// are reset by a one-workgroup kernel in the same stream, so the whole batch
// is capturable into a HIP graph.
//
// Fused BF16x3: FP32 operands are split in the loader, x = b0 + b1 + b2 with
// b0 = bf16(x) and b1, b2 the bf16 of the remainders (exact for FP32 x), and
// the six products b_p c_q with p + q <= 2 run on v_mfma_f32_16x16x32_bf16
// with FP32 accumulation -- no slice workspace and no extra pass.
#include <climits>
#include <type_traits>

#include "gather.hpp"
#include "kernels.hpp"

namespace comet {
namespace {

using namespace gather;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int TB = 64;            // the stand-alone fused kernel's 64 x 64 output tiles
constexpr int NT = 256;           // 4 waves, 2 x 2
constexpr int F3_BK = 32;         // one 16x16x32 MFMA step
constexpr int F3_LDK = F3_BK + 8;  // LDS pitch in bf16 (80 bytes: conflict-free 16-byte reads)
template <int BM, int BN>
constexpr int f3_lds() { return 3 * (BM + BN) * F3_LDK; }   // A and B, three slices (bf16 elements)

// One BM x BN output tile of the fused BF16x3 product; a WGM x WGN grid of
// waves, each (BM / WGM) x (BN / WGN) made of 16 x 16 blocks.  NBUF = 2
// double-buffers the sliced tiles in LDS: the next step's values are split
// and stored into one buffer while the products read the other, so the
// splitting (VALU and LDS writes) runs under the matrix-core work of the
// same waves and each step has one barrier; NBUF = 1 (the stand-alone
// kernel, two workgroups per CU) splits between two barriers.
template <int BM, int BN>
constexpr int f3_stage() { return 3 * (BM + BN) * F3_LDK; }

template <int BM, int BN, int WGM, int WGN, int LA, int LB, bool V, int NBUF = 1>
__device__ __forceinline__ void fused3_tile(const float *__restrict__ A, const float *__restrict__ B,
                                            float *__restrict__ C, const GettTables &t, int64_t M, int64_t N,
                                            int64_t K, double alpha, double beta, int64_t m0, int64_t n0,
                                            __bf16 *smem) {
  constexpr int NTH = 64 * WGM * WGN;
  typedef Loader<float, float, BM, F3_BK, LA, V, NTH> LoadA;
  typedef Loader<float, float, BN, F3_BK, LB, V, NTH> LoadB;
  constexpr int FM = BM / WGM / 16, FN = BN / WGN / 16;
  static_assert(FM * 16 * WGM == BM && FN * 16 * WGN == BN, "wave tile must be a multiple of 16");
  constexpr int STAGE = f3_stage<BM, BN>();
  lds_t<__bf16> *const s0 = to_lds(smem);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WGN) * (BM / WGM), wn0 = (wave % WGN) * (BN / WGN);
  f4_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f4_t{0, 0, 0, 0};
  LoadA la;
  LoadB lb;
  la.init(tid, m0, M, t.offAm);
  lb.init(tid, n0, N, t.offBn);
  const int64_t nsteps = (K + F3_BK - 1) / F3_BK;
  la.fetch_k(t.offAk, 0, K);
  lb.fetch_k(t.offBk, 0, K);
  la.load(A, 0, K);
  lb.load(B, 0, K);
  la.fetch_k(t.offAk, F3_BK, K);
  lb.fetch_k(t.offBk, F3_BK, K);
  la.template store_split3<F3_LDK>(s0);
  lb.template store_split3<F3_LDK>(s0 + 3 * BM * F3_LDK);
  __syncthreads();
  for (int64_t step = 0; step < nsteps; ++step) {
    lds_t<__bf16> *const sA = s0 + (NBUF == 2 ? int(step & 1) * STAGE : 0);
    lds_t<__bf16> *const sB = sA + 3 * BM * F3_LDK;
    la.load(A, (step + 1) * F3_BK, K);
    lb.load(B, (step + 1) * F3_BK, K);
    la.fetch_k(t.offAk, (step + 2) * F3_BK, K);
    lb.fetch_k(t.offBk, (step + 2) * F3_BK, K);
    bf16x8 bF[3][FN];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        bF[q][j] = *reinterpret_cast<const lds_t<bf16x8> *>(
            &sB[q * BN * F3_LDK + split3_pos<F3_LDK>(wn0 + j * 16 + (lane & 15), 8 * (lane >> 4))]);
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      bf16x8 aF[FM];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        aF[i] = *reinterpret_cast<const lds_t<bf16x8> *>(
            &sA[p * BM * F3_LDK + split3_pos<F3_LDK>(wm0 + i * 16 + (lane & 15), 8 * (lane >> 4))]);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        if (p + q <= 2) {
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aF[i], bF[q][j], acc[i][j], 0, 0, 0);
        }
      }
    }
    if constexpr (NBUF == 2) {
      // the other buffer was last read before the previous barrier
      lds_t<__bf16> *const nA = s0 + int((step + 1) & 1) * STAGE;
      la.template store_split3<F3_LDK>(nA);
      lb.template store_split3<F3_LDK>(nA + 3 * BM * F3_LDK);
      __syncthreads();
    } else {
      __syncthreads();
      la.template store_split3<F3_LDK>(sA);
      lb.template store_split3<F3_LDK>(sB);
      __syncthreads();
    }
  }
  // the epilogue of the gather kernels (C offsets staged in LDS, which the
  // loop above no longer reads)
  WaveTile<float, BM, BN, WGM, WGN> w;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) w.acc[i][j] = acc[i][j];
  gett_store<float, float, BM, BN, WGM, WGN>(w, C, t, M, N, alpha, beta, m0, n0, reinterpret_cast<float *>(smem));
}

template <int LA, int LB, bool V>
__global__ __launch_bounds__(NT) void fused3_kernel(const float *__restrict__ A, const float *__restrict__ B,
                                                    float *__restrict__ C, GettTables t, int64_t M, int64_t N,
                                                    int64_t K, double alpha, double beta, int tilesM, int tilesN) {
  __shared__ __attribute__((aligned(16))) __bf16 smem[f3_lds<TB, TB>()];
  int tm, tn;
  tile_coords(blockIdx.x, tilesM, tilesN, &tm, &tn);
  fused3_tile<TB, TB, 2, 2, LA, LB, V>(A, B, C, t, M, N, K, alpha, beta, int64_t(tm) * TB, int64_t(tn) * TB, smem);
}

// ---------------------------------------------------------------- batch ----

// tile classes: BM x BN, 2 x 2 waves
struct ClassShape {
  int bm, bn;
};
constexpr ClassShape kClass[kBatchClasses] = {{64, 64}, {128, 64}, {64, 128}, {128, 128}};

// which classes exist: element loads in class 0 only, and the larger
// classes for FP32 storage only.  Every class of one kernel shares its
// register allocation, which the largest class sets: the native FP32 kernel
// (4 waves) fits all four in 256 registers (two workgroups per CU) without
// spilling, the fused BF16x3 kernel does with 8 waves per workgroup (one
// workgroup per CU), while the FP64 kernel spills with any class beyond
// 64 x 64.
constexpr bool class_ok(int cls, int dtype, int mode, bool vec) {
  return cls == 0 || (vec && dtype == 1);
}

// workgroup size and wave grid of the batch kernel of each mode: 2 x 2 waves
// for the native products, 4 x 2 for the fused BF16x3 one
template <int MODE> struct BatchWaves;
template <> struct BatchWaves<0> { static constexpr int WGM = 2, WGN = 2, NT = 256, MINB = 2; };
template <> struct BatchWaves<1> { static constexpr int WGM = 4, WGN = 2, NT = 512, MINB = 1; };

template <typename T, int LA, int LB, bool V, int CLS>
constexpr int native_lds_one() {
  return int(sizeof(T)) * gett_lds_elems<T, T, kClass[CLS].bm, kClass[CLS].bn, 16, NT, LA, LB, V, V>();
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }
template <typename T, int CLS>
constexpr int native_lds_cls() {
  return cmax(cmax(native_lds_one<T, 0, 0, true, CLS>(), native_lds_one<T, 0, 1, true, CLS>()),
              cmax(native_lds_one<T, 1, 0, true, CLS>(), native_lds_one<T, 1, 1, true, CLS>()));
}
template <typename T>
constexpr int native_lds_bytes() {
  // the largest layout/vector variant of every class the dtype has
  return sizeof(T) == 4 ? cmax(cmax(native_lds_cls<T, 0>(), native_lds_cls<T, 1>()),
                               cmax(native_lds_cls<T, 2>(), native_lds_cls<T, 3>()))
                        : native_lds_cls<T, 0>();
}
constexpr int fused_lds_bytes() { return 2 * int(sizeof(__bf16)) * f3_stage<128, 128>(); }

template <typename T, int MODE, int CLS, int LA, int LB, bool V>
__device__ __forceinline__ void run_item(const BatchDesc &d, int tile, char *smem) {
  constexpr int BM = kClass[CLS].bm, BN = kClass[CLS].bn;
  const int64_t m0 = int64_t(tile / d.tilesN) * BM, n0 = int64_t(tile % d.tilesN) * BN;
  if constexpr (MODE == 0) {
    gett_tile<T, T, BM, BN, 16, 2, 2, LA, LB, V, V>(static_cast<const T *>(d.A), static_cast<const T *>(d.B),
                                                    static_cast<T *>(d.C), d.t, d.M, d.N, d.K, d.alpha, d.beta, m0,
                                                    n0, reinterpret_cast<T *>(smem));
  } else {
    fused3_tile<BM, BN, BatchWaves<1>::WGM, BatchWaves<1>::WGN, LA, LB, V, 2>(
        static_cast<const float *>(d.A), static_cast<const float *>(d.B), static_cast<float *>(d.C), d.t, d.M, d.N,
        d.K, d.alpha, d.beta, m0, n0, reinterpret_cast<__bf16 *>(smem));
  }
}

// the four layout variants of one class with vector loads
template <typename T, int MODE, int CLS>
__device__ __forceinline__ void run_vec(const BatchDesc &d, int tile, char *smem) {
  switch (d.variant) {
    case 0: run_item<T, MODE, CLS, 0, 0, true>(d, tile, smem); break;
    case 1: run_item<T, MODE, CLS, 0, 1, true>(d, tile, smem); break;
    case 2: run_item<T, MODE, CLS, 1, 0, true>(d, tile, smem); break;
    default: run_item<T, MODE, CLS, 1, 1, true>(d, tile, smem); break;
  }
}

template <typename T, int MODE>
__device__ __forceinline__ void run_any(const BatchDesc &d, int tile, char *smem) {
  constexpr int dt = sizeof(T) == 8 ? 0 : 1;
  if (d.variant >= 4) {
    switch (d.variant) {
      case 4: run_item<T, MODE, 0, 0, 0, false>(d, tile, smem); break;
      case 5: run_item<T, MODE, 0, 0, 1, false>(d, tile, smem); break;
      case 6: run_item<T, MODE, 0, 1, 0, false>(d, tile, smem); break;
      default: run_item<T, MODE, 0, 1, 1, false>(d, tile, smem); break;
    }
    return;
  }
  switch (d.cls) {
    case 1: if constexpr (class_ok(1, dt, MODE, true)) { run_vec<T, MODE, 1>(d, tile, smem); return; } break;
    case 2: if constexpr (class_ok(2, dt, MODE, true)) { run_vec<T, MODE, 2>(d, tile, smem); return; } break;
    case 3: if constexpr (class_ok(3, dt, MODE, true)) { run_vec<T, MODE, 3>(d, tile, smem); return; } break;
    default: break;
  }
  run_vec<T, MODE, 0>(d, tile, smem);
}

template <typename T, int MODE>
__global__ __launch_bounds__(BatchWaves<MODE>::NT, BatchWaves<MODE>::MINB) void batch_kernel(const BatchDesc *__restrict__ descs,
                                                   const BatchItem *__restrict__ items, BatchQueues q,
                                                   int *__restrict__ counters) {
  constexpr int LDS = MODE == 0 ? native_lds_bytes<T>() : fused_lds_bytes();
  __shared__ __attribute__((aligned(16))) char smem[LDS];
  __shared__ int s_item;
  // the XCD this workgroup runs on (workgroups are dealt to the XCDs in turn)
  int queue = int(blockIdx.x % kBatchQueues);
  for (int drained = 0; drained < kBatchQueues;) {
    const int64_t len = q.off[queue + 1] - q.off[queue];
    if (threadIdx.x == 0) s_item = len > 0 ? atomicAdd(&counters[queue], 1) : INT_MAX;
    __syncthreads();
    // the item index is the same in every lane: say so, so that the item and
    // its descriptor are read with scalar loads into scalar registers
    const int64_t item = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (item >= len) {   // this queue is drained (its counter only grows): the next one
      queue = (queue + 1) % kBatchQueues;
      ++drained;
      continue;
    }
    const BatchItem w = items[q.off[queue] + item];
    const BatchDesc d = descs[__builtin_amdgcn_readfirstlane(w.problem)];
    run_any<T, MODE>(d, w.tile, smem);
    __syncthreads();   // the next item's loads may not overwrite LDS still being read
  }
}

__global__ void reset_counters_kernel(int *counters) {
  if (threadIdx.x < kBatchQueues) counters[threadIdx.x] = 0;
}

template <int LA, int LB>
hipError_t fused_l(const GettLaunch &g, hipStream_t s, dim3 grid, int tilesM, int tilesN) {
  const float *A = static_cast<const float *>(g.A), *B = static_cast<const float *>(g.B);
  float *C = static_cast<float *>(g.C);
  if (g.vecA && g.vecB)
    hipLaunchKernelGGL((fused3_kernel<LA, LB, true>), grid, dim3(NT), 0, s, A, B, C, g.t, g.M, g.N, g.K, g.alpha,
                       g.beta, tilesM, tilesN);
  else
    hipLaunchKernelGGL((fused3_kernel<LA, LB, false>), grid, dim3(NT), 0, s, A, B, C, g.t, g.M, g.N, g.K, g.alpha,
                       g.beta, tilesM, tilesN);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fused_bf16x3(const GettLaunch &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (g.dtype != 1) return hipErrorInvalidValue;
  const int tilesM = int((g.M + TB - 1) / TB), tilesN = int((g.N + TB - 1) / TB);
  const dim3 grid(tilesM * tilesN);
  switch (g.layoutA * 2 + g.layoutB) {
    case 0: return fused_l<0, 0>(g, s, grid, tilesM, tilesN);
    case 1: return fused_l<0, 1>(g, s, grid, tilesM, tilesN);
    case 2: return fused_l<1, 0>(g, s, grid, tilesM, tilesN);
    default: return fused_l<1, 1>(g, s, grid, tilesM, tilesN);
  }
}

void batch_class_shape(int cls, int *bm, int *bn) {
  const int c = (cls >= 0 && cls < kBatchClasses) ? cls : 0;
  *bm = kClass[c].bm;
  *bn = kClass[c].bn;
}

bool batch_class_valid(int cls, int dtype, int mode, bool vec) {
  return cls >= 0 && cls < kBatchClasses && class_ok(cls, dtype, mode, vec);
}

int batch_blocks_per_cu(int dtype, int mode) {
  int n = 0;
  hipError_t e;
  if (mode == 1)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<float, 1>, BatchWaves<1>::NT, 0);
  else if (dtype == 0)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<double, 0>, NT, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<float, 0>, NT, 0);
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_batch(const BatchDesc *descs, const BatchItem *items, const BatchQueues &q, int *counters,
                        int dtype, int mode, int grid, hipStream_t s) {
  hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, s, counters);
  if (q.off[kBatchQueues] <= 0) return hipGetLastError();
  if (mode == 1) {
    if (dtype != 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((batch_kernel<float, 1>), dim3(grid), dim3(BatchWaves<1>::NT), 0, s, descs, items, q,
                       counters);
  } else if (dtype == 0) {
    hipLaunchKernelGGL((batch_kernel<double, 0>), dim3(grid), dim3(NT), 0, s, descs, items, q, counters);
  } else {
    hipLaunchKernelGGL((batch_kernel<float, 0>), dim3(grid), dim3(NT), 0, s, descs, items, q, counters);
  }
  return hipGetLastError();
}

}  // namespace comet
