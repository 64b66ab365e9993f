// gemv.hip -- products in which one of the free index groups is empty, so
// the contraction (Section 2) is a matrix times a vector:
//   C[j] = alpha * sum_k x[k] * Y[k, j] + beta * C[j].
// They move the matrix once and do two FLOP per element, so they are bound by
// HBM.  The gather kernel's tiles would spend 63 of every 64 MFMA rows and
// write 64 x 64 partial tiles per summation piece; here each workgroup
// streams a slab of Y along its unit stride instead:
//
//   j-fast:  Y is contiguous along j.  A wave's 64 lanes take 64 consecutive
//            outputs and walk the slab's summation indices together; the
//            block's four waves take every fourth index.
//   k-fast:  Y is contiguous along k.  A wave's lanes walk the summation
//            indices, 64 apart, of four outputs at once and add up each with
//            a fixed butterfly; the four waves take sixteen outputs.
//
// The summation is cut into `split` slabs of at most kGemvSlab indices, whose
// x values and Y offsets a block stages in LDS.  With one slab the block
// writes C; otherwise it writes a partial sum per output and slab, and a
// fix-up adds the slabs in order (the result does not depend on timing).
// Sums are kept in FP64 for both storage types.
#include <algorithm>
#include <climits>

#include "kernels.hpp"

namespace comet {
namespace {

constexpr int kGemvThreads = 256;

constexpr int kJW = 4;   // outputs per wave when reading along the summation

// one output's sum over a slab: C itself with a single slab, else the slab's
// partial sum
template <typename T>
__device__ __forceinline__ void emit(const GemvLaunch &a, int64_t j, double sum) {
  if (a.split == 1) {
    T *__restrict__ C = static_cast<T *>(a.C);
    const int64_t c = a.offC0[0] + a.offCj[j];
    double v = a.alpha * sum;
    if (a.beta != 0.0) v += a.beta * double(C[c]);
    C[c] = T(v);
  } else {
    static_cast<double *>(a.ws)[int64_t(blockIdx.y) * a.J + j] = sum;
  }
}

template <typename T, bool KFAST>
__global__ __launch_bounds__(kGemvThreads) void gemv_kernel(GemvLaunch a) {
  constexpr int BJ = KFAST ? 4 * kJW : 64;   // outputs per block
  constexpr int BK = KFAST ? 64 : 4;         // threads sharing an output
  __shared__ double xs[kGemvSlab];
  __shared__ int64_t yk[kGemvSlab];
  __shared__ double red[kGemvThreads];
  const T *__restrict__ X = static_cast<const T *>(a.X);
  const T *__restrict__ Y = static_cast<const T *>(a.Y);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t k0 = int64_t(blockIdx.y) * a.slab;
  const int n = int(std::min<int64_t>(a.K - k0, a.slab));
  const int64_t x0 = a.offX0[0];
  for (int i = tid; i < n; i += kGemvThreads) {
    xs[i] = double(X[x0 + a.offXk[k0 + i]]);
    yk[i] = a.offYk[k0 + i];
  }
  __syncthreads();
  if constexpr (KFAST) {
    // each wave: kJW outputs, their loads interleaved, then one butterfly each
    const int64_t j0 = int64_t(blockIdx.x) * BJ + wave * kJW;
    const T *__restrict__ Yj[kJW];
    double acc[kJW];
#pragma unroll
    for (int u = 0; u < kJW; ++u) {
      acc[u] = 0.0;
      Yj[u] = Y + a.offYj[j0 + u < a.J ? j0 + u : a.J - 1];   // a past-the-end output re-reads the last one
    }
    int i = lane;
    for (; i + BK < n; i += 2 * BK) {
      double y[2][kJW];
#pragma unroll
      for (int u = 0; u < kJW; ++u) {
        y[0][u] = double(Yj[u][yk[i]]);
        y[1][u] = double(Yj[u][yk[i + BK]]);
      }
#pragma unroll
      for (int u = 0; u < kJW; ++u) {
        acc[u] += xs[i] * y[0][u];
        acc[u] += xs[i + BK] * y[1][u];
      }
    }
    if (i < n) {
#pragma unroll
      for (int u = 0; u < kJW; ++u) acc[u] += xs[i] * double(Yj[u][yk[i]]);
    }
    // butterfly over the wave's 64 lanes: every lane ends with the same sums
#pragma unroll
    for (int u = 0; u < kJW; ++u)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc[u] += __shfl_xor(acc[u], off, 64);
    if (lane < kJW && j0 + lane < a.J) {
      double sum = acc[0];
#pragma unroll
      for (int u = 1; u < kJW; ++u)
        if (lane == u) sum = acc[u];
      emit<T>(a, j0 + lane, sum);
    }
    return;
  }
  const int64_t j = int64_t(blockIdx.x) * BJ + lane;
  double acc = 0.0;
  if (j < a.J) {
    const T *__restrict__ Yj = Y + a.offYj[j];
    int i = wave;
    // four independent loads in flight per thread
    for (; i + 3 * BK < n; i += 4 * BK) {
      const double y0 = double(Yj[yk[i]]), y1 = double(Yj[yk[i + BK]]);
      const double y2 = double(Yj[yk[i + 2 * BK]]), y3 = double(Yj[yk[i + 3 * BK]]);
      acc += xs[i] * y0;
      acc += xs[i + BK] * y1;
      acc += xs[i + 2 * BK] * y2;
      acc += xs[i + 3 * BK] * y3;
    }
    for (; i < n; i += BK) acc += xs[i] * double(Yj[yk[i]]);
  }
  red[tid] = acc;
  __syncthreads();
  if (wave != 0 || j >= a.J) return;
  double sum = 0.0;
#pragma unroll
  for (int w = 0; w < 4; ++w) sum += red[w * 64 + lane];
  emit<T>(a, j, sum);
}

constexpr int kFixThreads = 64;

template <typename T>
__global__ __launch_bounds__(kFixThreads) void gemv_fixup_kernel(GemvLaunch a) {
  const int64_t j = int64_t(blockIdx.x) * kFixThreads + threadIdx.x;
  if (j >= a.J) return;
  const double *__restrict__ ws = static_cast<const double *>(a.ws) + j;
  // four slabs' partial sums in flight, added in slab order
  double sum = 0.0;
  int s = 0;
  for (; s + 4 <= a.split; s += 4) {
    const double p0 = ws[int64_t(s) * a.J], p1 = ws[int64_t(s + 1) * a.J];
    const double p2 = ws[int64_t(s + 2) * a.J], p3 = ws[int64_t(s + 3) * a.J];
    sum += p0;
    sum += p1;
    sum += p2;
    sum += p3;
  }
  for (; s < a.split; ++s) sum += ws[int64_t(s) * a.J];
  T *__restrict__ C = static_cast<T *>(a.C);
  const int64_t c = a.offC0[0] + a.offCj[j];
  double v = a.alpha * sum;
  if (a.beta != 0.0) v += a.beta * double(C[c]);
  C[c] = T(v);
}

template <typename T>
hipError_t launch_gemv_t(const GemvLaunch &a, hipStream_t s) {
  const int bj = a.kfast ? 4 * kJW : 64;
  const int64_t gx = (a.J + bj - 1) / bj;
  if (gx > INT32_MAX || a.split < 1 || a.split > 65535 || a.slab < 1 || a.slab > kGemvSlab ||
      int64_t(a.split) * a.slab < a.K || (a.split > 1 && !a.ws))
    return hipErrorInvalidValue;
  const dim3 grid(unsigned(gx), unsigned(a.split));
  if (a.kfast)
    hipLaunchKernelGGL((gemv_kernel<T, true>), grid, dim3(kGemvThreads), 0, s, a);
  else
    hipLaunchKernelGGL((gemv_kernel<T, false>), grid, dim3(kGemvThreads), 0, s, a);
  if (a.split > 1) {
    const int64_t fx = (a.J + kFixThreads - 1) / kFixThreads;
    if (fx > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gemv_fixup_kernel<T>), dim3(unsigned(fx)), dim3(kFixThreads), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace

void gemv_shape(int64_t J, int64_t K, bool kfast, int cus, int *split, int64_t *slab) {
  const int64_t bj = kfast ? 4 * kJW : 64;
  const int64_t gx = std::max<int64_t>(1, (J + bj - 1) / bj);
  // about sixteen blocks per CU, but slabs of at least 256 indices (the
  // fix-up reads every slab's partial sums), and at most kGemvSlab.
  // Measured on the chain's 3072 x 3072 steps (FP64, 75 MB): read along the
  // free labels, 43 slabs 14.2 us + 7.4 us fix-up, 12 slabs 13.4 us, 3 slabs
  // 29 us; along the summation, 3 slabs 20.7 us, 6 slabs 18.7 us.
  const int64_t want = std::max<int64_t>(1, (16 * int64_t(std::max(cus, 1)) + gx - 1) / gx);
  int64_t sp = std::max<int64_t>((K + kGemvSlab - 1) / kGemvSlab, std::min<int64_t>(want, (K + 255) / 256));
  sp = std::max<int64_t>(1, sp);
  int64_t sl = (K + sp - 1) / sp;
  sp = (K + sl - 1) / sl;
  *split = int(std::min<int64_t>(sp, INT32_MAX));
  *slab = sl;
}

hipError_t launch_gemv(const GemvLaunch &a, hipStream_t s) {
  if (a.J <= 0 || a.K <= 0) return hipSuccess;
  return a.dtype == 0 ? launch_gemv_t<double>(a, s) : launch_gemv_t<float>(a, s);
}

}  // namespace comet
