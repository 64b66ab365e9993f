// batch.hip -- many independent contractions in one persistent launch, and
// the fused BF16x3 gather product.
//
// Persistent launch: the host lists every (problem, 64 x 64 output tile)
// pair, problems with the longest summation first (longest-processing-time
// order), and starts as many workgroups as stay resident on the GPU.  Each
// workgroup repeatedly takes the next item from a device counter and runs the
// gather tile routine for that problem's layout variant, until the list is
// exhausted -- every workgroup reaches that exit.  Uneven, small problems
// thus fill the machine together instead of one under-filled launch each.
// The counter is reset by a one-thread kernel in the same stream, so the
// whole batch is capturable into a HIP graph.
//
// Fused BF16x3: FP32 operands are split in the loader, x = b0 + b1 + b2 with
// b0 = bf16(x) and b1, b2 the bf16 of the remainders (exact for FP32 x), and
// the six products b_p c_q with p + q <= 2 run on v_mfma_f32_16x16x32_bf16
// with FP32 accumulation -- no slice workspace and no extra pass.
#include <type_traits>

#include "gather.hpp"
#include "kernels.hpp"

namespace comet {
namespace {

using namespace gather;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int TB = kBatchTile;    // 64 x 64 output tiles
constexpr int NT = 256;           // 4 waves, 2 x 2, each 32 x 32
constexpr int F3_BK = 32;         // one 16x16x32 MFMA step
constexpr int F3_LDK = F3_BK + 8;  // LDS pitch in bf16 (80 bytes: conflict-free 16-byte reads)
constexpr int F3_LDS = 2 * 3 * TB * F3_LDK;   // A and B, three slices (bf16 elements)

template <int LA, int LB, bool V>
__device__ __forceinline__ void fused3_tile(const float *__restrict__ A, const float *__restrict__ B,
                                            float *__restrict__ C, const GettTables &t, int64_t M, int64_t N,
                                            int64_t K, double alpha, double beta, int64_t m0, int64_t n0,
                                            __bf16 *smem) {
  typedef Loader<float, float, TB, F3_BK, LA, V, NT> LoadA;
  typedef Loader<float, float, TB, F3_BK, LB, V, NT> LoadB;
  lds_t<__bf16> *const sA = to_lds(smem);
  lds_t<__bf16> *const sB = sA + 3 * TB * F3_LDK;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * 32, wn0 = (wave & 1) * 32;
  f4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4_t{0, 0, 0, 0};
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
  la.template store_split3<F3_LDK>(sA);
  lb.template store_split3<F3_LDK>(sB);
  __syncthreads();
  for (int64_t step = 0; step < nsteps; ++step) {
    la.load(A, (step + 1) * F3_BK, K);
    lb.load(B, (step + 1) * F3_BK, K);
    la.fetch_k(t.offAk, (step + 2) * F3_BK, K);
    lb.fetch_k(t.offBk, (step + 2) * F3_BK, K);
    bf16x8 bF[3][2];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        bF[q][j] = *reinterpret_cast<const lds_t<bf16x8> *>(
            &sB[(q * TB + wn0 + j * 16 + (lane & 15)) * F3_LDK + 8 * (lane >> 4)]);
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      bf16x8 aF[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        aF[i] = *reinterpret_cast<const lds_t<bf16x8> *>(
            &sA[(p * TB + wm0 + i * 16 + (lane & 15)) * F3_LDK + 8 * (lane >> 4)]);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        if (p + q <= 2) {
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aF[i], bF[q][j], acc[i][j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
    la.template store_split3<F3_LDK>(sA);
    lb.template store_split3<F3_LDK>(sB);
    __syncthreads();
  }
  // the epilogue of the gather kernels (C offsets staged in LDS, which the
  // loop above no longer reads)
  WaveTile<float, TB, TB, 2, 2> w;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) w.acc[i][j] = acc[i][j];
  gett_store<float, float, TB, TB, 2, 2>(w, C, t, M, N, alpha, beta, m0, n0, reinterpret_cast<float *>(smem));
}

template <int LA, int LB, bool V>
__global__ __launch_bounds__(NT) void fused3_kernel(const float *__restrict__ A, const float *__restrict__ B,
                                                    float *__restrict__ C, GettTables t, int64_t M, int64_t N,
                                                    int64_t K, double alpha, double beta, int tilesM, int tilesN) {
  __shared__ __attribute__((aligned(16))) __bf16 smem[F3_LDS];
  int tm, tn;
  tile_coords(blockIdx.x, tilesM, tilesN, &tm, &tn);
  fused3_tile<LA, LB, V>(A, B, C, t, M, N, K, alpha, beta, int64_t(tm) * TB, int64_t(tn) * TB, smem);
}

// ---------------------------------------------------------------- batch ----

template <typename T>
constexpr int native_lds_bytes() {
  // the largest of the eight layout/vector variants of the 64 x 64 tile
  return int(sizeof(T)) * gett_lds_elems<T, T, TB, TB, 16, NT, 0, 0, true, true>();
}

template <typename T, int LA, int LB, bool V>
__device__ __forceinline__ void native_item(const BatchDesc &d, int64_t m0, int64_t n0, char *smem) {
  gett_tile<T, T, TB, TB, 16, 2, 2, LA, LB, V, V>(static_cast<const T *>(d.A), static_cast<const T *>(d.B),
                                                  static_cast<T *>(d.C), d.t, d.M, d.N, d.K, d.alpha, d.beta, m0,
                                                  n0, reinterpret_cast<T *>(smem));
}

template <int LA, int LB, bool V>
__device__ __forceinline__ void fused_item(const BatchDesc &d, int64_t m0, int64_t n0, char *smem) {
  fused3_tile<LA, LB, V>(static_cast<const float *>(d.A), static_cast<const float *>(d.B), static_cast<float *>(d.C),
                         d.t, d.M, d.N, d.K, d.alpha, d.beta, m0, n0, reinterpret_cast<__bf16 *>(smem));
}

template <typename T, int MODE, int LA, int LB, bool V>
__device__ __forceinline__ void run_item(const BatchDesc &d, int64_t m0, int64_t n0, char *smem) {
  if constexpr (MODE == 0)
    native_item<T, LA, LB, V>(d, m0, n0, smem);
  else
    fused_item<LA, LB, V>(d, m0, n0, smem);
}

template <typename T, int MODE>
__global__ __launch_bounds__(NT) void batch_kernel(const BatchDesc *__restrict__ descs,
                                                   const BatchItem *__restrict__ items, int64_t total,
                                                   int *__restrict__ counter) {
  constexpr int LDS = MODE == 0 ? native_lds_bytes<T>() : int(sizeof(__bf16)) * F3_LDS;
  __shared__ __attribute__((aligned(16))) char smem[LDS];
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    // the item index is the same in every lane: say so, so that the item and
    // its descriptor are read with scalar loads into scalar registers
    const int64_t item = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (item >= total) break;   // every workgroup ends here once the list is drained
    const BatchItem w = items[item];
    const BatchDesc d = descs[__builtin_amdgcn_readfirstlane(w.problem)];
    const int64_t m0 = int64_t(w.tile / d.tilesN) * TB, n0 = int64_t(w.tile % d.tilesN) * TB;
    switch (d.variant) {
      case 0: run_item<T, MODE, 0, 0, true>(d, m0, n0, smem); break;
      case 1: run_item<T, MODE, 0, 1, true>(d, m0, n0, smem); break;
      case 2: run_item<T, MODE, 1, 0, true>(d, m0, n0, smem); break;
      case 3: run_item<T, MODE, 1, 1, true>(d, m0, n0, smem); break;
      case 4: run_item<T, MODE, 0, 0, false>(d, m0, n0, smem); break;
      case 5: run_item<T, MODE, 0, 1, false>(d, m0, n0, smem); break;
      case 6: run_item<T, MODE, 1, 0, false>(d, m0, n0, smem); break;
      default: run_item<T, MODE, 1, 1, false>(d, m0, n0, smem); break;
    }
    __syncthreads();   // the next item's loads may not overwrite LDS still being read
  }
}

__global__ void reset_counter_kernel(int *counter) { *counter = 0; }

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

int batch_blocks_per_cu(int dtype, int mode) {
  int n = 0;
  hipError_t e;
  if (mode == 1)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<float, 1>, NT, 0);
  else if (dtype == 0)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<double, 0>, NT, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<float, 0>, NT, 0);
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_batch(const BatchDesc *descs, const BatchItem *items, int64_t total, int *counter, int dtype,
                        int mode, int grid, hipStream_t s) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, counter);
  if (total <= 0) return hipGetLastError();
  if (mode == 1) {
    if (dtype != 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((batch_kernel<float, 1>), dim3(grid), dim3(NT), 0, s, descs, items, total, counter);
  } else if (dtype == 0) {
    hipLaunchKernelGGL((batch_kernel<double, 0>), dim3(grid), dim3(NT), 0, s, descs, items, total, counter);
  } else {
    hipLaunchKernelGGL((batch_kernel<float, 0>), dim3(grid), dim3(NT), 0, s, descs, items, total, counter);
  }
  return hipGetLastError();
}

}  // namespace comet
