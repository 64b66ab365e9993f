// permute.hip -- out-of-place N-dimensional permutation with scaling,
// out = alpha * permute(in) + beta * out.
//
// This is the transpose of the TTGT lowering (Section 2) and the ta.copy
// operation (Section 5).  The paper's transpose optimization (Section 6)
// orders the loops so that the innermost indices stay innermost and then
// tiles; on the GPU the same aim -- unit-stride access on both sides, in
// runs long enough to fill whole cache lines -- is met in two ways:
//
//   stream:    both tensors have the same unit-stride dimension u.  Every
//              row along u is copied with 16-byte vectors; consecutive
//              threads take consecutive vectors of a row and then the next
//              rows, so a short u (16 FP64 values, say) still gives each
//              wave several whole rows.
//   transpose: the unit dimensions differ.  A 32 x 32 tile spanned by the
//              input-contiguous group Gi (the input's unit dimension plus the
//              dimensions that continue it contiguously, until the group
//              holds 32 elements) and the output-contiguous group Go is
//              staged through LDS: threads read along Gi and write along Go.
//              The offsets of a tile's Gi entries in the output and of its Go
//              entries in the input are computed once per tile into LDS.
//
// All remaining dimensions are enumerated by the workgroup index.  A tensor
// that is one contiguous run on both sides takes a plain vector walk.
#include <algorithm>
#include <type_traits>
#include <vector>

#include "kernels.hpp"
#include "permute_shape.hpp"

namespace comet {
namespace {

constexpr int TP = kPermTile;   // transpose tile edge
constexpr int TR = 8;    // thread rows of the transpose block
constexpr int SB = 256;  // stream block
constexpr int SU = 4;    // vectors per stream thread per pass

template <typename T> struct Vec16;
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); static constexpr int W = 2; };
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); static constexpr int W = 4; };

// A set of dimensions with both strides; index decomposition fastest first.
struct DimSet {
  int n = 0;
  int64_t ext[kPermMaxDims];
  int64_t s_in[kPermMaxDims];
  int64_t s_out[kPermMaxDims];
};

// Offsets of linear index x over the dimensions of d (fastest first).  I is
// the index type of the divisions: 32-bit when every index fits, which is
// several times cheaper than 64-bit division.
template <typename I>
__device__ __forceinline__ void decompose(const DimSet &d, int64_t x64, int64_t *oi, int64_t *oo) {
  int64_t a = 0, b = 0;
  I x = I(x64);
  for (int k = 0; k < d.n; ++k) {
    const I e = I(d.ext[k]);
    const I q = x / e;
    const I r = x - q * e;
    x = q;
    a += int64_t(r) * d.s_in[k];
    b += int64_t(r) * d.s_out[k];
  }
  *oi = a;
  *oo = b;
}

struct StreamArgs {
  DimSet rows;            // every dimension but u, fastest first (output order)
  int64_t E;              // extent of u
  int64_t su_in, su_out;  // strides of u
  int64_t vpr;            // vectors per row (E / W)
  int64_t total;          // rows * vpr
  double fill;            // value of the alpha term when alpha == 0 (nothing is read then)
};

// Each pass of a workgroup covers SB * SU consecutive vectors, that is the
// rows [r0, r1] of its range: their input and output offsets are decomposed
// once per row into LDS (not once per vector), then every thread takes its
// SU vectors (stride SB).  The next pass's loads are issued before this
// pass's stores, so that a wait for them is not also a wait for the stores
// (loads and stores share one in-order completion counter on CDNA).
constexpr int SROWS = SB * SU;   // rows a pass can touch (one vector per row)

template <typename T, int W, typename I>
__global__ __launch_bounds__(SB) void permute_stream(const T *__restrict__ in, T *__restrict__ out, StreamArgs a,
                                                     double alpha, double beta) {
  typedef typename std::conditional<sizeof(T) == 8, double, float>::type Te;
  typedef typename Vec16<T>::type vec_t;
  typedef typename std::conditional<W == 1, T, vec_t>::type val_t;
  __shared__ int64_t row_in[SROWS + 1], row_out[SROWS + 1];
  const int64_t per_pass = int64_t(SB) * SU;
  const int64_t stride = int64_t(gridDim.x) * per_pass;
  const I vpr = I(a.vpr);
  const bool reads = alpha != 0.0;
  int64_t q0 = int64_t(blockIdx.x) * per_pass;
  if (q0 >= a.total) return;   // uniform: a workgroup without vectors
  // offsets of this thread's vectors of the pass at q0 (rows from LDS)
  auto offsets = [&](int64_t qb, int64_t *ai, int64_t *ao, bool *ok) {
    const int64_t r0 = int64_t(I(qb) / vpr);
    const int64_t qe = qb + per_pass < a.total ? qb + per_pass : a.total;
    const int64_t nrows = int64_t(I(qe - 1) / vpr) - r0 + 1;
    for (int64_t t = threadIdx.x; t < nrows; t += SB) {
      int64_t bi, bo;
      decompose<I>(a.rows, r0 + t, &bi, &bo);
      row_in[t] = bi;
      row_out[t] = bo;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int64_t q = qb + threadIdx.x + int64_t(u) * SB;
      ok[u] = q < a.total;
      const I qq = ok[u] ? I(q) : I(qb);
      const I row = qq / vpr;
      const int64_t c = int64_t(qq - row * vpr) * W;
      ai[u] = row_in[int64_t(row) - r0] + c * a.su_in;
      ao[u] = row_out[int64_t(row) - r0] + c * a.su_out;
    }
    __syncthreads();   // the table is rewritten by the next pass
  };
  auto load = [&](const int64_t *ai, const bool *ok, val_t *x) {
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      if (W > 1)
        x[u] = (reads && ok[u]) ? *reinterpret_cast<const val_t *>(in + ai[u]) : val_t{};
      else
        x[u] = (reads && ok[u]) ? val_t(in[ai[u]]) : val_t{};
    }
  };
  int64_t ai[SU], ao[SU];
  bool ok[SU];
  val_t x[SU];
  offsets(q0, ai, ao, ok);
  load(ai, ok, x);
  for (; q0 < a.total; q0 += stride) {
    // the next pass's vectors, requested before this pass is stored
    int64_t ai1[SU], ao1[SU];
    bool ok1[SU];
    val_t x1[SU];
    const bool more = q0 + stride < a.total;
    if (more) {
      offsets(q0 + stride, ai1, ao1, ok1);
      load(ai1, ok1, x1);
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      if (!ok[u]) continue;
      val_t *dst = reinterpret_cast<val_t *>(out + ao[u]);
      val_t y;
      if constexpr (W > 1) {
        const vec_t old = beta != 0.0 ? *dst : vec_t{};
#pragma unroll
        for (int k = 0; k < W; ++k) {
          Te v = reads ? Te(alpha) * Te(x[u][k]) : Te(a.fill);
          if (beta != 0.0) v = v + Te(beta) * Te(old[k]);
          y[k] = T(v);
        }
      } else {
        Te v = reads ? Te(alpha) * Te(x[u]) : Te(a.fill);
        if (beta != 0.0) v = v + Te(beta) * Te(*dst);
        y = T(v);
      }
      __builtin_nontemporal_store(y, dst);   // streamed past the caches: 3% faster here
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        ai[u] = ai1[u];
        ao[u] = ao1[u];
        ok[u] = ok1[u];
        x[u] = x1[u];
      }
    }
  }
}

// One contiguous run on both sides (every dimension merged into one of unit
// stride, 16-byte aligned): a plain grid-stride walk over 16-byte vectors,
// FL per thread and pass, with no offset tables, LDS or barriers.  Plain
// stores: on MI355X a 1 GB fill ran at 6.5 TB/s this way against 5.4 TB/s
// through the table-driven stream kernel.
constexpr int FL = 4;
template <typename T>
__global__ __launch_bounds__(SB) void permute_flat(const T *__restrict__ in, T *__restrict__ out, int64_t nv,
                                                   double alpha, double beta, double fillv) {
  typedef typename std::conditional<sizeof(T) == 8, double, float>::type Te;
  typedef typename Vec16<T>::type vec_t;
  constexpr int W = Vec16<T>::W;
  const vec_t *__restrict__ vin = reinterpret_cast<const vec_t *>(in);
  vec_t *__restrict__ vout = reinterpret_cast<vec_t *>(out);
  const bool reads = alpha != 0.0;
  const int64_t step = int64_t(gridDim.x) * SB;
  for (int64_t v0 = int64_t(blockIdx.x) * SB * FL + threadIdx.x; v0 < nv; v0 += step * FL) {
    vec_t x[FL], c[FL];
#pragma unroll
    for (int u = 0; u < FL; ++u) {
      const int64_t v = v0 + int64_t(u) * SB;
      x[u] = (reads && v < nv) ? vin[v] : vec_t{};
      c[u] = (beta != 0.0 && v < nv) ? vout[v] : vec_t{};
    }
#pragma unroll
    for (int u = 0; u < FL; ++u) {
      const int64_t v = v0 + int64_t(u) * SB;
      if (v >= nv) break;
      vec_t y;
#pragma unroll
      for (int k = 0; k < W; ++k) {
        Te t = reads ? Te(alpha) * Te(x[u][k]) : Te(fillv);
        if (beta != 0.0) t = t + Te(beta) * Te(c[u][k]);
        y[k] = T(t);
      }
      vout[v] = y;
    }
  }
}

struct TileArgs {
  DimSet gi, go, batch;      // Gi, Go fastest first; batch: the rest
  int64_t EI, EO;            // element counts of Gi and Go
  int64_t gi_sin, go_sout;   // stride of a Gi step in the input, of a Go step in the output
  int64_t tiles_i, tiles_o;
};

template <typename T, typename I>
__global__ __launch_bounds__(TP *TR) void permute_tiled(const T *__restrict__ in, T *__restrict__ out, TileArgs a,
                                                         double alpha, double beta) {
  typedef typename std::conditional<sizeof(T) == 8, double, float>::type Te;
  __shared__ T tile[TP][TP + 1];
  __shared__ int64_t gi_out[TP], go_in[TP];
  int64_t bid = blockIdx.x;
  const int64_t ti = bid % a.tiles_i;
  bid /= a.tiles_i;
  const int64_t to = bid % a.tiles_o;
  bid /= a.tiles_o;
  int64_t bi, bo;
  decompose<I>(a.batch, bid, &bi, &bo);
  const int64_t i0 = ti * TP, o0 = to * TP;
  const int x = threadIdx.x, y = threadIdx.y;
  if (y == 0) {
    int64_t di, dout;
    decompose<I>(a.gi, i0 + x < a.EI ? i0 + x : 0, &di, &dout);
    gi_out[x] = dout;
  } else if (y == 1) {
    int64_t di, dout;
    decompose<I>(a.go, o0 + x < a.EO ? o0 + x : 0, &di, &dout);
    go_in[x] = di;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < TP; r += TR) {
    const int64_t i = i0 + x, o = o0 + y + r;
    if (alpha != 0.0 && i < a.EI && o < a.EO) tile[x][y + r] = in[bi + i * a.gi_sin + go_in[y + r]];
  }
  __syncthreads();
  const Te al = Te(alpha), be = Te(beta);
#pragma unroll
  for (int r = 0; r < TP; r += TR) {
    const int64_t o = o0 + x, i = i0 + y + r;
    if (i < a.EI && o < a.EO) {
      const int64_t addr = bo + o * a.go_sout + gi_out[y + r];
      Te v = alpha != 0.0 ? al * Te(tile[y + r][x]) : Te(0);
      if (beta != 0.0) v = v + be * Te(out[addr]);
      out[addr] = T(v);   // a plain store: nontemporal ones made this kernel 18% slower
    }
  }
}

void fill(DimSet &s, const std::vector<PermDim> &d, const std::vector<int> &idx) {
  s.n = (int)idx.size();
  for (int k = 0; k < s.n; ++k) {
    s.ext[k] = d[idx[k]].ext;
    s.s_in[k] = d[idx[k]].si;
    s.s_out[k] = d[idx[k]].so;
  }
}

template <typename T>
hipError_t launch_perm_t(const PermuteLaunch &p, hipStream_t s) {
  const PermShape sh = permute_shape(p.ndim, p.ext, p.s_in, p.s_out, p.alpha != 0.0);
  if (sh.kind == PERM_EMPTY) return hipSuccess;
  const std::vector<PermDim> &d = sh.d;
  const int64_t total = sh.total;
  const T *in = static_cast<const T *>(p.in);
  T *out = static_cast<T *>(p.out);
  const int n = (int)d.size();
  constexpr int WF = Vec16<T>::W;
  if (sh.kind == PERM_FLAT && d[0].ext % WF == 0 && reinterpret_cast<uintptr_t>(out) % 16 == 0 &&
      (p.alpha == 0.0 || reinterpret_cast<uintptr_t>(in) % 16 == 0)) {
    const int64_t nv = d[0].ext / WF;
    const int64_t want = (nv + int64_t(SB) * FL - 1) / (int64_t(SB) * FL);
    const unsigned grid = unsigned(std::max<int64_t>(1, std::min<int64_t>(want, 16384)));
    hipLaunchKernelGGL((permute_flat<T>), dim3(grid), dim3(SB), 0, s, static_cast<const T *>(p.in), out, nv, p.alpha,
                       p.beta, p.fill);
    return hipGetLastError();
  }
  if (sh.kind == PERM_FLAT || sh.kind == PERM_STREAM) {
    const int uo = sh.uo;
    StreamArgs a{};
    std::vector<int> rows;
    for (int k = 0; k < n; ++k)
      if (k != uo) rows.push_back(k);
    // rows fastest first in output order
    std::sort(rows.begin(), rows.end(), [&](int x, int y) { return d[x].so < d[y].so; });
    fill(a.rows, d, rows);
    a.fill = p.fill;
    a.E = n ? d[uo].ext : 1;
    a.su_in = n ? d[uo].si : 0;
    a.su_out = n ? d[uo].so : 0;
    constexpr int W = Vec16<T>::W;
    bool vec = n > 0 && a.su_out == 1 && (p.alpha == 0.0 || a.su_in == 1) && a.E % W == 0 &&
               reinterpret_cast<uintptr_t>(out) % 16 == 0 &&
               (p.alpha == 0.0 || reinterpret_cast<uintptr_t>(in) % 16 == 0);
    for (int k = 0; k < a.rows.n && vec; ++k)
      vec = a.rows.s_out[k] % W == 0 && (p.alpha == 0.0 || a.rows.s_in[k] % W == 0);
    const int w = vec ? W : 1;
    a.vpr = a.E / w;
    a.total = (total / a.E) * a.vpr;
    const int64_t want = (a.total + int64_t(SB) * SU - 1) / (int64_t(SB) * SU);
    const unsigned grid = unsigned(std::max<int64_t>(1, std::min<int64_t>(want, 8192)));
    // 32-bit index arithmetic when every linear index (plus a pass of the
    // grid) stays below 2^31
    const bool small = total < (int64_t(1) << 30);
    if (vec && small)
      hipLaunchKernelGGL((permute_stream<T, W, uint32_t>), dim3(grid), dim3(SB), 0, s, in, out, a, p.alpha, p.beta);
    else if (vec)
      hipLaunchKernelGGL((permute_stream<T, W, uint64_t>), dim3(grid), dim3(SB), 0, s, in, out, a, p.alpha, p.beta);
    else if (small)
      hipLaunchKernelGGL((permute_stream<T, 1, uint32_t>), dim3(grid), dim3(SB), 0, s, in, out, a, p.alpha, p.beta);
    else
      hipLaunchKernelGGL((permute_stream<T, 1, uint64_t>), dim3(grid), dim3(SB), 0, s, in, out, a, p.alpha, p.beta);
    return hipGetLastError();
  }
  // transpose over the groups Gi and Go
  TileArgs a{};
  fill(a.gi, d, sh.gi);
  fill(a.go, d, sh.go);
  fill(a.batch, d, sh.rest);
  a.EI = sh.EI;
  a.EO = sh.EO;
  a.gi_sin = d[sh.ui].si;
  a.go_sout = d[sh.uo].so;
  a.tiles_i = (sh.EI + TP - 1) / TP;
  a.tiles_o = (sh.EO + TP - 1) / TP;
  const int64_t blocks = a.tiles_i * a.tiles_o * (total / (sh.EI * sh.EO));
  if (total < (int64_t(1) << 30))
    hipLaunchKernelGGL((permute_tiled<T, uint32_t>), dim3(unsigned(blocks)), dim3(TP, TR), 0, s, in, out, a, p.alpha,
                       p.beta);
  else
    hipLaunchKernelGGL((permute_tiled<T, uint64_t>), dim3(unsigned(blocks)), dim3(TP, TR), 0, s, in, out, a, p.alpha,
                       p.beta);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_permute(const PermuteLaunch &p, hipStream_t s) {
  return p.dtype == 0 ? launch_perm_t<double>(p, s) : launch_perm_t<float>(p, s);
}

}  // namespace comet
