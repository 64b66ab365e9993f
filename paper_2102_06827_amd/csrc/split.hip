// split.hip -- FP64-grade contraction from low-precision matrix-core products.
//
// Each operand is viewed as a matrix (rows = its free labels, columns = the
// summation labels; the offset tables of the gather path address it), and
// every row is cut into S slices of 16-bit floats so that the sum of the
// slice products reproduces the FP64 product:
//
//   mode 0, aligned (Ozaki et al., error-free splitting): the row is scaled by
//     2^-e, e the exponent of its largest magnitude, so |x'| < 1; slice p is
//     s_p * 2^-8(p+1) with s_p = trunc(256 * remainder), |s_p| <= 255, which a
//     bfloat16 holds exactly.  Pair products with p + q < S are summed.  The
//     (0,0) and (0,1)+(1,0) pair sums are integers times a power of two below
//     2^24 over any 128 summation indices, so their FP32 accumulators are exact
//     over such chunks; the remaining pairs are 2^-16 smaller and share one
//     FP32 accumulator.  Every 128 indices the three accumulators are folded
//     into FP64.
//   mode 1, BF16x3 (Henry, Tang and Heinecke): b0 = bf16(x'), b1 = bf16(x' - b0),
//     b2 = bf16(x' - b0 - b1); the six products with p + q <= 2 in one FP32
//     accumulator.
//   mode 2, FP16x2 (Ootomo and Yokota): h0 = fp16(x'), h1 = fp16((x' - h0) 2^11);
//     h0 g0 in one FP32 accumulator, h0 g1 + h1 g0 in another scaled by 2^-11.
//   mode 3, aligned INT8: as mode 0 with 7-bit slices s_p = trunc(128 *
//     remainder), |s_p| <= 127, stored as int8 and multiplied on
//     v_mfma_i32_16x16x64_i8.  Each diagonal d = p + q has its own int32
//     accumulator, exact while S * 127^2 * (indices summed) < 2^31; a launch
//     sums at most 8192 indices and combines the diagonals in FP64 (times
//     2^-7(d+2)) in its epilogue; longer summations take several launches,
//     each adding into C.
//
// Rows are scaled by powers of two in every mode (exact), which keeps the
// 16-bit slices in range; the epilogue multiplies by 2^(eA[m] + eB[n]).
//
// Kernels, one launch each for both operands: an exponent pass (partial row
// maxima over ranges of the summation, HBM-bound) and a pack pass (reduce a
// row's partial maxima, gather through the offset tables into an LDS tile so
// reads are coalesced along the operand's unit-stride label, then write the
// slices K-contiguous in 64-byte runs, blocked along the summation -- this
// is also the transpose of TTGT); then the
// slice-pair matrix product on v_mfma_f32_16x16x32_{bf16,f16} or
// v_mfma_i32_16x16x64_i8.
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <type_traits>

#include "split.hpp"

namespace comet {
namespace {

// LDS and global pointers with their address spaces spelled out, so that
// accesses compile to ds_* and global_* instructions (a flat access waits on
// both memory counters).
template <typename T> using lds_t = __attribute__((address_space(3))) T;
template <typename T> using glb_t = __attribute__((address_space(1))) T;
template <typename T> __device__ __forceinline__ lds_t<T> *to_lds(T *p) { return (lds_t<T> *)p; }
template <typename T> __device__ __forceinline__ glb_t<T> *to_glb(T *p) { return (glb_t<T> *)p; }

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kExpNone = -(1 << 20);   // exponent of an all-zero row

template <typename ST> struct Vec8;
template <> struct Vec8<__bf16> { typedef bf16x8 type; };
template <> struct Vec8<_Float16> { typedef f16x8 type; };
typedef signed char i8x8 __attribute__((ext_vector_type(8)));
template <> struct Vec8<signed char> { typedef i8x8 type; };
typedef int i4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4_t mfma_slice(bf16x8 a, bf16x8 b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma_slice(f16x8 a, f16x8 b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- slicing --

constexpr int PR = 64;    // slicer tile rows
constexpr int PK = 64;    // slicer tile summation indices
constexpr int PT = 256;   // slicer threads
constexpr int PI = PR * PK / PT;   // elements per thread per tile

// Element e (0..PI-1) of thread tid in a PR x PK tile.  Threads walk the
// operand's unit-stride dimension: k for LAYOUT 0, rows for LAYOUT 1, V
// consecutive elements at a time (V > 1: one vector load of V elements that
// are contiguous in memory, where the offset tables allow it).
template <int LAYOUT, int V>
__device__ __forceinline__ void tile_pos(int tid, int e, int *rl, int *kl) {
  if (LAYOUT == 0) {
    *kl = (tid % (PK / V)) * V + e % V;
    *rl = tid / (PK / V) + (PT / (PK / V)) * (e / V);
  } else {
    *rl = (tid % (PR / V)) * V + e % V;
    *kl = tid / (PR / V) + (PT / (PR / V)) * (e / V);
  }
}

// The PI elements of a thread in the PR x PK tile at (r0, k0), zero outside
// the operand.  ro[e] holds the row offset of element e (hoisted by the
// caller: rows are fixed per thread).  The loads are branch-free -- clamped
// indices, zeros applied afterwards -- so that all of them are in flight at
// once instead of one wait per element.  With V > 1 the vector's first
// element is addressed and the vector is loaded whole: the offset tables then
// make V consecutive indices along the unit-stride dimension contiguous and
// V-aligned, and that dimension's extent a multiple of V, so a vector is
// either inside the operand or wholly outside (and then clamped to the last
// vector).
template <typename Tin, int LAYOUT, int V>
__device__ __forceinline__ void load_tile(double *x, const Tin *__restrict__ base, const int64_t *ro,
                                          const int64_t *__restrict__ offK, int64_t r0, int64_t k0, int64_t R,
                                          int64_t K) {
  const int tid = threadIdx.x;
  Tin v[PI];
  if constexpr (V == 1) {
#pragma unroll
    for (int e = 0; e < PI; ++e) {
      int rl, kl;
      tile_pos<LAYOUT, V>(tid, e, &rl, &kl);
      const int64_t k = k0 + kl;
      v[e] = base[ro[e] + offK[k < K ? k : K - 1]];
    }
  } else {
    typedef Tin vec_t __attribute__((ext_vector_type(V)));
    // LAYOUT 0: the vector runs along k, so its start is clamped to K - V
    const int64_t klast = LAYOUT == 0 ? K - V : K - 1;
#pragma unroll
    for (int e = 0; e < PI; e += V) {
      int rl, kl;
      tile_pos<LAYOUT, V>(tid, e, &rl, &kl);
      const int64_t k = k0 + kl;
      const vec_t w = *reinterpret_cast<const vec_t *>(base + ro[e] + offK[k <= klast ? k : klast]);
#pragma unroll
      for (int i = 0; i < V; ++i) v[e + i] = w[i];
    }
  }
#pragma unroll
  for (int e = 0; e < PI; ++e) {
    int rl, kl;
    tile_pos<LAYOUT, V>(tid, e, &rl, &kl);
    x[e] = (r0 + rl < R && k0 + kl < K) ? double(v[e]) : 0.0;
  }
}

// Gather a PR x PK tile into LDS (zeros outside the operand).
template <typename Tin, int LAYOUT, int V>
__device__ __forceinline__ void gather_tile(double (*t)[PK + 1], const Tin *__restrict__ base, const int64_t *ro,
                                            const int64_t *__restrict__ offK, int64_t r0, int64_t k0, int64_t R,
                                            int64_t K) {
  double x[PI];
  load_tile<Tin, LAYOUT, V>(x, base, ro, offK, r0, k0, R, K);
#pragma unroll
  for (int e = 0; e < PI; ++e) {
    int rl, kl;
    tile_pos<LAYOUT, V>(threadIdx.x, e, &rl, &kl);
    t[rl][kl] = x[e];
  }
}

// Row offsets of a thread's elements (fixed for every tile of the same rows).
// A vector along rows (LAYOUT 1, V > 1) takes its first row's offset, clamped
// to the last whole vector.
template <int LAYOUT, int V>
__device__ __forceinline__ void row_offsets(int64_t *ro, const int64_t *__restrict__ offR, int64_t r0, int64_t R) {
  const int64_t rlast = (LAYOUT == 1 && V > 1) ? R - V : R - 1;
#pragma unroll
  for (int e = 0; e < PI; ++e) {
    int rl, kl;
    tile_pos<LAYOUT, V>(threadIdx.x, e, &rl, &kl);
    ro[e] = offR[r0 + rl <= rlast ? r0 + rl : rlast];
  }
}

// The packed slices of both operands share one layout, blocked along the
// summation: a block holds, for 64 bytes of summation indices (32 16-bit or
// 64 8-bit values), every row of every slice of A, then of B -- RT = S (Mp +
// Np) rows of 64 bytes, block after block.  Element (slice p, row r, index k)
// of an operand sits at row (k / CK) RT + p Rp + r of that layout counted
// from the operand's first row (A's at 0, B's at S Mp), byte (k mod CK) x
// the element size, CK = 64 / the element size.  A product's stage (one
// block of the summation for a tile's rows) is then S runs of contiguous
// rows per operand, and each 1 KB load of 16 rows reads 1 KB of memory.
__host__ __device__ constexpr int64_t slice_rows(int S, int64_t Mp, int64_t Np) { return int64_t(S) * (Mp + Np); }

// The two operands of one product, as the slicer kernels see them: rows R
// (M or N) and summation K through the offset tables, tilesR slicer tiles of
// rows, `part` the partial row maxima (ky ranges of the summation, pitch Rp),
// `e` the final row exponents, `out` the operand's first slice row in the
// blocked layout (Rp rows per slice).
struct SliceOperand {
  const void *base;
  const int64_t *offR, *offK;
  int64_t R;
  int layout;
  int vec;             // vector loads along the unit-stride dimension
  int tilesR;
  int *part;
  int *e;
  void *out;
  int64_t Rp;
};
struct SliceArgs {
  SliceOperand op[2];
  int64_t K, Kp;
  int64_t RT;          // rows of one summation block of the packed slices
  int ky;
};

// Partial row exponents: part[y][r] = max over the y-th of ky equal ranges of
// summation tiles of the binary exponent of operand row r.  Block (x, y)
// takes rows [64x', 64x' + 64) of operand 0 (x < tilesR of operand 0) or
// operand 1, and summation range y; the maxima stay in registers over the
// range, then in LDS, and one plain store per row and range leaves the block
// (no initialisation and no global atomics).
template <typename Tin, int LAYOUT, int V>
__device__ __forceinline__ void exp_block(const SliceOperand &op, int rt, int64_t K, int ky, int *emax) {
  const int tid = threadIdx.x;
  if (tid < PR) emax[tid] = kExpNone;
  const Tin *__restrict__ base = static_cast<const Tin *>(op.base);
  const int64_t r0 = int64_t(rt) * PR, R = op.R;
  const int64_t tilesK = (K + PK - 1) / PK;
  const int64_t kt0 = tilesK * blockIdx.y / ky, kt1 = tilesK * (blockIdx.y + 1) / ky;
  int64_t ro[PI];
  row_offsets<LAYOUT, V>(ro, op.offR, r0, R);
  // the rows of a thread's elements: LAYOUT 0, one per element; LAYOUT 1, V
  // (element e lies in row number e mod V of them)
  constexpr int NR = LAYOUT == 0 ? PI : V;
  int mx[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) mx[q] = kExpNone;
  // the next tile's loads are issued before the current tile is reduced
  double x[PI];
  if (kt0 < kt1) load_tile<Tin, LAYOUT, V>(x, base, ro, op.offK, r0, kt0 * PK, R, K);
  for (int64_t kt = kt0; kt < kt1; ++kt) {
    double xn[PI];
    if (kt + 1 < kt1) load_tile<Tin, LAYOUT, V>(xn, base, ro, op.offK, r0, (kt + 1) * PK, R, K);
#pragma unroll
    for (int e = 0; e < PI; ++e) {
      const int q = LAYOUT == 0 ? e : e % V;
      int ex = kExpNone;
      if (x[e] != 0.0) (void)frexp(x[e], &ex);
      mx[q] = ex > mx[q] ? ex : mx[q];
    }
#pragma unroll
    for (int e = 0; e < PI; ++e) x[e] = xn[e];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    int rl, kl;
    tile_pos<LAYOUT, V>(tid, q, &rl, &kl);
    if (mx[q] != kExpNone) atomicMax(&emax[rl], mx[q]);
  }
  __syncthreads();
  if (tid < PR && r0 + tid < R) op.part[int64_t(blockIdx.y) * op.Rp + r0 + tid] = emax[tid];
}

template <typename Tin>
__global__ __launch_bounds__(PT) void split_exp_kernel(SliceArgs a) {
  constexpr int VEC = 16 / int(sizeof(Tin));
  __shared__ int emax[PR];
  const int w = int(blockIdx.x) < a.op[0].tilesR ? 0 : 1;
  const int rt = int(blockIdx.x) - (w ? a.op[0].tilesR : 0);
  const SliceOperand &op = a.op[w];
  if (op.layout == 0)
    op.vec ? exp_block<Tin, 0, VEC>(op, rt, a.K, a.ky, emax) : exp_block<Tin, 0, 1>(op, rt, a.K, a.ky, emax);
  else
    op.vec ? exp_block<Tin, 1, VEC>(op, rt, a.K, a.ky, emax) : exp_block<Tin, 1, 1>(op, rt, a.K, a.ky, emax);
}

// Cut a PR x PK tile into S slices, written in the blocked layout.  Thread t
// writes 16 consecutive k of row t/4, so a wave writes, per slice and 64-byte
// block of the summation, 16 consecutive rows: 1 KB of contiguous memory.
// The block first reduces its rows' partial exponents; blocks of the first
// summation tile also store them as the rows' final exponents, which the
// product's epilogue reads.
template <typename Tin, typename ST, int LAYOUT, int V, int MODE, int S>
__device__ __forceinline__ void pack_block(const SliceOperand &op, int64_t bid, int64_t K, int64_t RT, int ky,
                                           double (*t)[PK + 1], int *erow, int *red) {
  constexpr int CK = 64 / int(sizeof(ST));
  const Tin *__restrict__ base = static_cast<const Tin *>(op.base);
  ST *__restrict__ out = static_cast<ST *>(op.out);
  const int64_t R = op.R, Rp = op.Rp;
  const int64_t r0 = (bid % op.tilesR) * PR, k0 = (bid / op.tilesR) * PK;
  const int tid = threadIdx.x;
  {
    // the rows' partial exponents, ky per row, reduced by all threads: a
    // quarter of the ranges each, then the four quarters below
    const int rr = tid % PR, y0 = tid / PR;
    int ex = kExpNone;
    if (r0 + rr < R)
      for (int y = y0; y < ky; y += PT / PR) {
        const int v = op.part[int64_t(y) * Rp + r0 + rr];
        ex = v > ex ? v : ex;
      }
    red[tid] = ex;
  }
  {
    int64_t ro[PI];
    row_offsets<LAYOUT, V>(ro, op.offR, r0, R);
    gather_tile<Tin, LAYOUT, V>(t, base, ro, op.offK, r0, k0, R, K);
  }
  __syncthreads();
  if (tid < PR) {
    int ex = red[tid];
#pragma unroll
    for (int q = 1; q < PT / PR; ++q) ex = red[tid + q * PR] > ex ? red[tid + q * PR] : ex;
    erow[tid] = ex;
    if (k0 == 0 && r0 + tid < R) op.e[r0 + tid] = ex;
  }
  __syncthreads();
  const int rl = tid / 4;
  const int64_t r = r0 + rl;
  const int ex = erow[rl];
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int kc = (tid % 4) * 16 + half * 8;
    typename Vec8<ST>::type sl[S];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      double xs = ex == kExpNone ? 0.0 : ldexp(t[rl][kc + j], -ex);   // |xs| < 1, exact
      if (MODE == 0) {
#pragma unroll
        for (int p = 0; p < S; ++p) {
          const double tt = xs * 256.0;
          const double s = trunc(tt);                                   // |s| <= 255
          sl[p][j] = ST(float(ldexp(s, -8 * (p + 1))));                 // exact in 16 bits
          xs = tt - s;                                                  // exact remainder
        }
      } else if (MODE == 1) {
#pragma unroll
        for (int p = 0; p < S; ++p) {
          const ST b = ST(float(xs));
          sl[p][j] = b;
          xs = xs - double(float(b));
        }
      } else if (MODE == 2) {
        const ST h0 = ST(float(xs));
        sl[0][j] = h0;
        sl[1][j] = ST(float((xs - double(float(h0))) * 2048.0));
      } else {
#pragma unroll
        for (int p = 0; p < S; ++p) {
          const double tt = xs * 128.0;
          const double s = trunc(tt);                                   // |s| <= 127
          sl[p][j] = ST(int(s));
          xs = tt - s;
        }
      }
    }
#pragma unroll
    for (int p = 0; p < S; ++p)
      *reinterpret_cast<typename Vec8<ST>::type *>(
          out + (((k0 + kc) / CK) * RT + int64_t(p) * Rp + r) * CK + (k0 + kc) % CK) = sl[p];
  }
}

template <typename Tin, typename ST, int MODE, int S>
__global__ __launch_bounds__(PT) void split_pack_kernel(SliceArgs a) {
  constexpr int VEC = 16 / int(sizeof(Tin));
  __shared__ double t[PR][PK + 1];
  __shared__ int erow[PR];
  __shared__ int red[PT];
  const int64_t nA = int64_t(a.op[0].tilesR) * (a.Kp / PK);
  const int w = int64_t(blockIdx.x) < nA ? 0 : 1;
  const int64_t bid = int64_t(blockIdx.x) - (w ? nA : 0);
  const SliceOperand &op = a.op[w];
  if (op.layout == 0) {
    if (op.vec)
      pack_block<Tin, ST, 0, VEC, MODE, S>(op, bid, a.K, a.RT, a.ky, t, erow, red);
    else
      pack_block<Tin, ST, 0, 1, MODE, S>(op, bid, a.K, a.RT, a.ky, t, erow, red);
  } else {
    if (op.vec)
      pack_block<Tin, ST, 1, VEC, MODE, S>(op, bid, a.K, a.RT, a.ky, t, erow, red);
    else
      pack_block<Tin, ST, 1, 1, MODE, S>(op, bid, a.K, a.RT, a.ky, t, erow, red);
  }
}

// ------------------------------------------------------- slice-pair GEMM --

template <int MODE, int S> struct Pairs {
  // which slice pairs are multiplied, into which accumulator, with what scale
  static constexpr __host__ __device__ bool use(int p, int q) { return MODE == 2 ? p + q <= 1 : p + q <= S - 1; }
  static constexpr __host__ __device__ int acc(int p, int q) {
    return MODE == 1 ? 0 : (p + q < 2 ? p + q : 2);
  }
  static constexpr int NACC = MODE == 1 ? 1 : (MODE == 2 ? 2 : 3);
  static constexpr __host__ __device__ double scale(int a) { return (MODE == 2 && a == 1) ? 1.0 / 2048.0 : 1.0; }
  // stages between folds into FP64 (0: only at the end)
  static constexpr int FOLD = MODE == 0 ? 4 : 0;
};

constexpr int GBM = 128, GBN = 64, GBK = 32;   // block tile
constexpr int GWM = 4, GWN = 2;                // wave grid
constexpr int GNT = 64 * GWM * GWN;

// LDS position (in 16-bit elements) of the 8-element chunk c (0..3) of tile
// row r: rows are 64 bytes, unpadded, and the chunk index is XOR-swizzled by
// (r / 4) mod 4.  Sixteen lanes that store four consecutive rows, and sixteen
// lanes that read one chunk of sixteen consecutive rows (an MFMA fragment),
// then hit 64 distinct banks.
__device__ __forceinline__ int sw(int r, int c) { return r * GBK + ((c ^ ((r >> 2) & 3)) << 3); }

// One stage of the slice-pair products, moved from the packed slices into
// LDS by direct-to-LDS loads (no registers, no LDS store instructions).  The
// stage is S slices of BM rows of A, then S slices of BN rows of B, each row
// 64 bytes (32 16-bit or 64 8-bit summation indices), its four 16-byte
// chunks swizzled as sw() / sw8() place them.  It is cut into 1 KB blocks of
// 16 rows; one load of 64 lanes x 16 bytes fills a block, lane L writing
// bytes 16 L .. 16 L + 15 of it, i.e. row 16 g + L / 4 at chunk position
// L mod 4, which holds the row's chunk (L mod 4) ^ ((row / 4) mod 4).  Wave w
// of NW takes blocks w, w + NW, ...  A and B: the first row of each
// operand's packed slices (64-byte rows in the blocked layout).  The
// addresses do not depend on the stage but for its summation block's offset,
// the same for A and B, so they are worked out once (init) and a stage is NU
// loads (issue).  The loads are counted by the wave's vector-memory
// counter: wait for it to reach zero, then a barrier, before the stage is
// read.
template <int BM, int BN, int S, int NW>
struct StageDMA {
  static constexpr int BLK = 16;
  static constexpr int NBA = S * BM / BLK, NBB = S * BN / BLK;
  static constexpr int NU = (NBA + NBB + NW - 1) / NW;
  const char *src[NU];   // this lane's 16 bytes of block w + u NW, at summation byte 0
  int dst[NU];           // the block's byte offset in a stage buffer (uniform)
  int nu;                // blocks of this wave (uniform)

  __device__ __forceinline__ void init(const char *__restrict__ A, const char *__restrict__ B, int64_t Mp,
                                       int64_t Np, int64_t m0, int64_t n0, int wave, int lane) {
    const int w = __builtin_amdgcn_readfirstlane(wave);   // (the compiler cannot tell it is uniform)
    nu = 0;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int blk = w + u * NW;
      int p, g, base;
      const char *rows;
      int64_t rows_p;
      if (blk < NBA) {   // constant divisors on either side
        p = blk / (BM / BLK);
        g = blk % (BM / BLK);
        rows = A;
        rows_p = int64_t(p) * Mp + m0;
        base = p * BM * 64;
      } else {
        const int b2 = blk - NBA < NBB ? blk - NBA : NBB - 1;
        p = b2 / (BN / BLK);
        g = b2 % (BN / BLK);
        rows = B;
        rows_p = int64_t(p) * Np + n0;
        base = S * BM * 64 + p * BN * 64;
      }
      const int row = g * BLK + (lane >> 2);
      const int c = (lane & 3) ^ ((row >> 2) & 3);
      src[u] = rows + (rows_p + row) * 64 + c * 16;
      dst[u] = base + g * BLK * 64;
      nu += blk < NBA + NBB ? 1 : 0;
    }
  }

  __device__ __forceinline__ void issue(lds_t<char> *buf, int64_t kb0) const {
#pragma unroll
    for (int u = 0; u < NU; ++u)
      if ((NBA + NBB) % NW == 0 || u < nu)
        __builtin_amdgcn_global_load_lds(reinterpret_cast<const glb_t<void> *>(to_glb(src[u] + kb0)),
                                         reinterpret_cast<lds_t<void> *>(buf + dst[u]), 16, 0, 0);
  }
};

// The same stage loads with 32-bit lane offsets from one base (the A slices'
// first row; B's follows dB bytes on, and a summation block of both spans
// less than 4 GB), one per block of this wave: wave w of NW
// takes blocks w, w + NW, ..., every wave the same number (a wave short of
// blocks loads the last one again, the same bytes to the same place).  A
// block's place in the stage buffer is its index x 1 KB: A's S slices of BM
// rows, then B's S slices of BN rows, 64-byte rows.
template <int BM, int BN, int S, int NW>
struct StageDMA32 {
  static constexpr int BLK = 16;
  static constexpr int NBA = S * BM / BLK, NBB = S * BN / BLK;
  static constexpr int NU = (NBA + NBB + NW - 1) / NW;
  uint32_t voff[NU];
  int w;

  __device__ __forceinline__ void init(int64_t dB, int64_t Mp, int64_t Np, int64_t m0, int64_t n0, int wave,
                                       int lane) {
    w = __builtin_amdgcn_readfirstlane(wave);
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int b0 = w + u * NW;
      const int blk = b0 < NBA + NBB ? b0 : NBA + NBB - 1;
      int64_t row;   // row of the packed slices (all S of an operand stacked), relative to its base
      int64_t base;
      int g;
      if (blk < NBA) {   // constant divisors on either side
        g = blk % (BM / BLK);
        row = int64_t(blk / (BM / BLK)) * Mp + m0;
        base = 0;
      } else {
        g = (blk - NBA) % (BN / BLK);
        row = int64_t((blk - NBA) / (BN / BLK)) * Np + n0;
        base = dB;
      }
      const int r = g * BLK + (lane >> 2);
      const int c = (lane & 3) ^ ((r >> 2) & 3);
      voff[u] = uint32_t(base + (row + r) * 64 + c * 16);
    }
  }

  __device__ __forceinline__ void issue(const char *__restrict__ base, lds_t<char> *buf, int64_t kb0) const {
    const glb_t<const char> *b = to_glb(base + kb0);
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int b0 = w + u * NW;
      const int blk = b0 < NBA + NBB ? b0 : NBA + NBB - 1;
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const glb_t<void> *>(b + voff[u]),
                                       reinterpret_cast<lds_t<void> *>(buf + blk * 1024), 16, 0, 0);
    }
  }
};

// every direct-to-LDS load of this wave has landed (vector-memory counter at
// zero, the other counters left alone); then the barrier
__device__ __forceinline__ void stage_landed() {
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __syncthreads();
}

// Epilogue of the slice-pair products: C = alpha * 2^(eA[m] + eB[n]) * val +
// beta * C for the thread's accumulator elements (row 4 * (lane / 16) + r of
// each 16 x 16 block, the layout of the 16-bit and 8-bit MFMA outputs), val(i,
// j, r) the element's unscaled sum.  The tile's C offsets and exponents are
// first staged in LDS (`smem`: free once the main loop has passed its last
// barrier), so that no global load of the epilogue follows a store: loads and
// stores share one in-order completion counter on CDNA.  With beta != 0 the C
// values of the next group of four elements are requested before the current
// group is stored.
template <typename Tout, int BM, int BN, int FM, int FN, int NTH, typename ValF>
__device__ __forceinline__ void split_store(Tout *__restrict__ C, const int64_t *__restrict__ offCm,
                                            const int64_t *__restrict__ offCn, const int *__restrict__ eA,
                                            const int *__restrict__ eB, int64_t M, int64_t N, double alpha,
                                            double beta, int64_t m0, int64_t n0, int wm0, int wn0, void *smem,
                                            ValF val) {
  typedef typename std::conditional<sizeof(Tout) == 8, double, float>::type Te;
  lds_t<int64_t> *const toff = to_lds(static_cast<int64_t *>(smem));
  lds_t<int> *const texp = to_lds(reinterpret_cast<int *>(static_cast<int64_t *>(smem) + BM + BN));
  for (int x = threadIdx.x; x < BM + BN; x += NTH) {
    if (x < BM) {
      const int64_t m = m0 + x < M ? m0 + x : M - 1;
      toff[x] = offCm[m];
      texp[x] = eA[m];
    } else {
      const int64_t n = n0 + (x - BM) < N ? n0 + (x - BM) : N - 1;
      toff[x] = offCn[n];
      texp[x] = eB[n];
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  glb_t<Tout> *const gC = to_glb(C);
  constexpr int G = FN * FM;
  auto ml = [&](int i, int r) { return wm0 + i * 16 + 4 * (lane >> 4) + r; };
  auto nl = [&](int j) { return wn0 + j * 16 + (lane & 15); };
  auto inside = [&](int i, int r, int j) { return m0 + ml(i, r) < M && n0 + nl(j) < N; };
  auto value = [&](int i, int j, int r) {
    const int em = texp[ml(i, r)], en = texp[BM + nl(j)];
    const double prod = (em == kExpNone || en == kExpNone) ? 0.0 : ldexp(val(i, j, r), em + en);
    return Te(alpha * prod);
  };
  if (beta == 0.0) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int j = g / FM, i = g % FM;
      int64_t a[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = toff[ml(i, r)] + toff[BM + nl(j)];
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (inside(i, r, j)) __builtin_nontemporal_store(Tout(value(i, j, r)), &gC[a[r]]);
    }
    return;
  }
  Tout cv[2][4];
#pragma unroll
  for (int r = 0; r < 4; ++r) cv[0][r] = gC[toff[ml(0, r)] + toff[BM + nl(0)]];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int j = g / FM, i = g % FM;
    __builtin_amdgcn_sched_barrier(0);
    if (g + 1 < G) {
      const int j1 = (g + 1) / FM, i1 = (g + 1) % FM;
#pragma unroll
      for (int r = 0; r < 4; ++r) cv[(g + 1) & 1][r] = gC[toff[ml(i1, r)] + toff[BM + nl(j1)]];
    }
    int64_t a[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = toff[ml(i, r)] + toff[BM + nl(j)];
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (inside(i, r, j)) __builtin_nontemporal_store(Tout(value(i, j, r) + Te(beta) * Te(cv[g & 1][r])), &gC[a[r]]);
  }
}

template <typename ST, typename Tout, int MODE, int S>
__global__ __launch_bounds__(GNT) void split_gemm_kernel(const ST *__restrict__ As, const ST *__restrict__ Bs,
                                                          const int *__restrict__ eA, const int *__restrict__ eB,
                                                          Tout *__restrict__ C, const int64_t *__restrict__ offCm,
                                                          const int64_t *__restrict__ offCn, int64_t M, int64_t N,
                                                          int64_t Mp, int64_t Np, int64_t Kp, double alpha,
                                                          double beta, int tilesM, int tilesN) {
  typedef Pairs<MODE, S> PP;
  typedef typename Vec8<ST>::type v8;
  constexpr int WM = GBM / GWM, WN = GBN / GWN;      // 32 x 32
  constexpr int FM = WM / 16, FN = WN / 16;          // 2 x 2
  constexpr int NVA = S * GBM * (GBK / 8);           // 16-byte vectors per stage
  constexpr int NVB = S * GBN * (GBK / 8);
  constexpr int NV = (NVA + NVB + GNT - 1) / GNT;    // per thread
  constexpr int STAGE = S * (GBM + GBN) * GBK;       // elements per LDS buffer
  // two buffers when they fit in LDS (S <= 6 with 64-byte rows), else one;
  // two buffers are two objects, filled by direct-to-LDS loads, so that the
  // compiler can tell the loads into one from the reads of the other
  constexpr int NBUF = 2 * STAGE * int(sizeof(ST)) <= 150 * 1024 ? 2 : 1;
  __shared__ __attribute__((aligned(16))) ST smem[NBUF == 1 ? STAGE : 1];
  __shared__ __attribute__((aligned(16))) ST smem0_[NBUF == 2 ? STAGE : 1];
  __shared__ __attribute__((aligned(16))) ST smem1_[NBUF == 2 ? STAGE : 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // XCD-aware tile order, as in the gather kernel
  int tm, tn;
  {
    const int total = tilesM * tilesN, X = 8, bid = blockIdx.x;
    const int xcd = bid % X, local = bid / X, q = total / X, rem = total % X;
    const int id = xcd * q + (xcd < rem ? xcd : rem) + local;
    const int G = 8, per = G * tilesN, group = id / per, first = group * G;
    const int gsize = tilesM - first < G ? tilesM - first : G;
    const int in = id - group * per;
    tm = first + in % gsize;
    tn = in / gsize;
  }
  const int64_t m0 = int64_t(tm) * GBM, n0 = int64_t(tn) * GBN;
  const int wm0 = (wave / GWN) * WM, wn0 = (wave % GWN) * WN;

  f4_t acc[PP::NACC][FM][FN];
  d4_t acc64[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      acc64[i][j] = d4_t{0, 0, 0, 0};
#pragma unroll
      for (int a = 0; a < PP::NACC; ++a) acc[a][i][j] = f4_t{0, 0, 0, 0};
    }

  // a buffer holds A slices [S][GBM rows] then B slices [S][GBN rows]
  auto a_at = [&](ST *buf, int p, int row, int c) { return buf + (p * GBM) * GBK + sw(row, c); };
  auto b_at = [&](ST *buf, int p, int row, int c) { return buf + S * GBM * GBK + (p * GBN) * GBK + sw(row, c); };

  v8 pre[NV];
  const int64_t nst = Kp / GBK;
  const int64_t RT = slice_rows(S, Mp, Np);
  auto gload = [&](int64_t st) {
    const int64_t kr = (st < nst ? st : nst - 1) * RT;   // the stage's summation block, in rows
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int v = tid + u * GNT;
      if (v < NVA) {
        const int p = v / (GBM * 4), rem = v % (GBM * 4), row = rem / 4, kc = (rem % 4) * 8;
        pre[u] = *reinterpret_cast<const v8 *>(As + (kr + int64_t(p) * Mp + m0 + row) * GBK + kc);
      } else if (v < NVA + NVB) {
        const int w = v - NVA;
        const int p = w / (GBN * 4), rem = w % (GBN * 4), row = rem / 4, kc = (rem % 4) * 8;
        pre[u] = *reinterpret_cast<const v8 *>(Bs + (kr + int64_t(p) * Np + n0 + row) * GBK + kc);
      }
    }
  };
  auto lstore = [&](ST *buf) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int v = tid + u * GNT;
      if (v < NVA) {
        const int p = v / (GBM * 4), rem = v % (GBM * 4), row = rem / 4, c = rem % 4;
        *reinterpret_cast<v8 *>(a_at(buf, p, row, c)) = pre[u];
      } else if (v < NVA + NVB) {
        const int w = v - NVA;
        const int p = w / (GBN * 4), rem = w % (GBN * 4), row = rem / 4, c = rem % 4;
        *reinterpret_cast<v8 *>(b_at(buf, p, row, c)) = pre[u];
      }
    }
  };
  auto fold = [&]() {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int a = 0; a < PP::NACC; ++a) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[i][j][r] += double(acc[a][i][j][r]) * PP::scale(a);
          acc[a][i][j] = f4_t{0, 0, 0, 0};
        }
  };
  auto compute = [&](ST *buf) {
    v8 bF[S][FN];
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        bF[q][j] = *reinterpret_cast<const v8 *>(b_at(buf, q, wn0 + j * 16 + (lane & 15), lane >> 4));
#pragma unroll
    for (int p = 0; p < S; ++p) {
      v8 aF[FM];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        aF[i] = *reinterpret_cast<const v8 *>(a_at(buf, p, wm0 + i * 16 + (lane & 15), lane >> 4));
#pragma unroll
      for (int q = 0; q < S; ++q) {
        if (PP::use(p, q)) {
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
              acc[PP::acc(p, q)][i][j] = mfma_slice(aF[i], bF[q][j], acc[PP::acc(p, q)][i][j]);
        }
      }
    }
  };

  constexpr int FOLD = PP::FOLD > 0 ? PP::FOLD : 1;
  if constexpr (NBUF == 2) {
    // nst is even (Kp is a multiple of 64); each buffer was last read before
    // the barrier that ended the previous half step, and its loads are kept
    // ahead of the products (the scheduler would sink them, which have no
    // users, to the wait)
    StageDMA<GBM, GBN, S, GNT / 64> sd;
    sd.init(reinterpret_cast<const char *>(As), reinterpret_cast<const char *>(Bs), Mp, Np, m0, n0, wave, lane);
    auto dma = [&](ST *buf, int64_t st) {
      sd.issue(reinterpret_cast<lds_t<char> *>(to_lds(buf)), (st < nst ? st : nst - 1) * RT * 64);
    };
    dma(smem0_, 0);
    stage_landed();
    for (int64_t st = 0; st < nst; st += 2) {
      dma(smem1_, st + 1);
      __builtin_amdgcn_sched_barrier(0);
      compute(smem0_);
      if (PP::FOLD > 0 && (st + 1) % FOLD == 0) fold();
      stage_landed();
      dma(smem0_, st + 2);
      __builtin_amdgcn_sched_barrier(0);
      compute(smem1_);
      if (PP::FOLD > 0 && (st + 2) % FOLD == 0) fold();
      stage_landed();
    }
  } else {
    gload(0);
    lstore(smem);
    __syncthreads();
    for (int64_t st = 0; st < nst; ++st) {
      gload(st + 1);
      compute(smem);
      if (PP::FOLD > 0 && (st + 1) % FOLD == 0) fold();
      __syncthreads();
      lstore(smem);
      __syncthreads();
    }
  }
  fold();

  // epilogue: C = alpha * 2^(eA + eB) * acc + beta * C
  static_assert((GBM + GBN) * 12 <= STAGE * int(sizeof(ST)), "epilogue tables fit in LDS");
  split_store<Tout, GBM, GBN, FM, FN, GNT>(C, offCm, offCn, eA, eB, M, N, alpha, beta, m0, n0, wm0, wn0,
                                          NBUF == 2 ? static_cast<void *>(smem0_) : static_cast<void *>(smem),
                                          [&](int i, int j, int r) { return acc64[i][j][r]; });
}

// ------------------------------------------ large-tile slice-pair GEMM --
//
// For the classic splits (BF16x3, FP16x2: FP32 accumulation, no periodic
// fold) on large products: a 192 x 192 workgroup tile of 8 waves, each
// owning 96 x 48 outputs (6 x 3 blocks of the 16x16x32 MFMA).  Every
// fragment read from LDS then feeds 3 or 6 MFMAs (the 32 x 32 wave tile
// above: 2), which takes the kernel off the LDS read limit, and a 3072^2
// output is exactly 256 tiles, one per CU.

constexpr int XBM = 192, XBN = 192;            // block tile
constexpr int XWM = 2, XWN = 4;                // wave grid
constexpr int XNT = 64 * XWM * XWN;

template <typename ST, typename Tout, int MODE, int S>
__global__ __launch_bounds__(XNT) void split_gemm_big_kernel(const ST *__restrict__ As, const ST *__restrict__ Bs,
                                                              const int *__restrict__ eA, const int *__restrict__ eB,
                                                              Tout *__restrict__ C, const int64_t *__restrict__ offCm,
                                                              const int64_t *__restrict__ offCn, int64_t M, int64_t N,
                                                              int64_t Mp, int64_t Np, int64_t Kp, double alpha,
                                                              double beta, int tilesM, int tilesN) {
  typedef Pairs<MODE, S> PP;
  static_assert(PP::FOLD == 0, "the large tile keeps FP32 accumulators only");
  typedef typename Vec8<ST>::type v8;
  constexpr int WM = XBM / XWM, WN = XBN / XWN;      // 96 x 48
  constexpr int FM = WM / 16, FN = WN / 16;          // 6 x 3
  constexpr int STAGE = S * (XBM + XBN) * GBK;       // elements per LDS buffer
  static_assert(2 * STAGE * int(sizeof(ST)) <= 160 * 1024, "two stages must fit in LDS");
  // two buffers as two objects, so that the compiler can tell the loads
  // into one from the reads of the other and does not wait for the former
  // before the latter
  __shared__ __attribute__((aligned(16))) ST smem0_[STAGE];
  __shared__ __attribute__((aligned(16))) ST smem1_[STAGE];
  lds_t<ST> *const buf0 = to_lds(smem0_);
  lds_t<ST> *const buf1 = to_lds(smem1_);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int tm, tn;
  {
    const int total = tilesM * tilesN, X = 8, bid = blockIdx.x;
    const int xcd = bid % X, local = bid / X, q = total / X, rem = total % X;
    const int id = xcd * q + (xcd < rem ? xcd : rem) + local;
    const int G = 4, per = G * tilesN, group = id / per, first = group * G;
    const int gsize = tilesM - first < G ? tilesM - first : G;
    const int in = id - group * per;
    tm = first + in % gsize;
    tn = in / gsize;
  }
  const int64_t m0 = int64_t(tm) * XBM, n0 = int64_t(tn) * XBN;
  const int wm0 = (wave / XWN) * WM, wn0 = (wave % XWN) * WN;

  f4_t acc[PP::NACC][FM][FN];
#pragma unroll
  for (int a = 0; a < PP::NACC; ++a)
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[a][i][j] = f4_t{0, 0, 0, 0};

  // a buffer holds A slices [S][XBM rows] then B slices [S][XBN rows]
  auto a_at = [&](const lds_t<ST> *buf, int p, int row, int c) { return buf + (p * XBM) * GBK + sw(row, c); };
  auto b_at = [&](const lds_t<ST> *buf, int p, int row, int c) {
    return buf + S * XBM * GBK + (p * XBN) * GBK + sw(row, c);
  };
  const int64_t nst = Kp / GBK;   // even: Kp is a multiple of 64
  StageDMA<XBM, XBN, S, XNT / 64> sd;
  sd.init(reinterpret_cast<const char *>(As), reinterpret_cast<const char *>(Bs), Mp, Np, m0, n0, wave, lane);
  const int64_t RT = slice_rows(S, Mp, Np);
  auto dma = [&](lds_t<ST> *buf, int64_t st) {
    sd.issue(reinterpret_cast<lds_t<char> *>(buf), (st < nst ? st : nst - 1) * RT * 64);
  };
  auto compute = [&](const lds_t<ST> *buf) {
    v8 bF[S][FN];
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        bF[q][j] = *reinterpret_cast<const lds_t<v8> *>(b_at(buf, q, wn0 + j * 16 + (lane & 15), lane >> 4));
#pragma unroll
    for (int p = 0; p < S; ++p) {
      v8 aF[FM];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        aF[i] = *reinterpret_cast<const lds_t<v8> *>(a_at(buf, p, wm0 + i * 16 + (lane & 15), lane >> 4));
#pragma unroll
      for (int q = 0; q < S; ++q) {
        if (PP::use(p, q)) {
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
              acc[PP::acc(p, q)][i][j] = mfma_slice(aF[i], bF[q][j], acc[PP::acc(p, q)][i][j]);
        }
      }
    }
  };
  auto land = [&]() { stage_landed(); };

  dma(buf0, 0);
  land();
  for (int64_t st = 0; st < nst; st += 2) {
    // each buffer was last read before the barrier that ended the previous
    // half step; the loads are kept ahead of the products (the scheduler
    // would otherwise sink them, which have no users, to the wait)
    dma(buf1, st + 1);
    __builtin_amdgcn_sched_barrier(0);
    compute(buf0);
    land();
    dma(buf0, st + 2);
    __builtin_amdgcn_sched_barrier(0);
    compute(buf1);
    land();
  }

  // epilogue: C = alpha * 2^(eA + eB) * sum_a scale(a) * acc[a] + beta * C
  static_assert((XBM + XBN) * 12 <= STAGE * int(sizeof(ST)), "epilogue tables fit in LDS");
  split_store<Tout, XBM, XBN, FM, FN, XNT>(C, offCm, offCn, eA, eB, M, N, alpha, beta, m0, n0, wm0, wn0, smem0_,
                                          [&](int i, int j, int r) {
                                            double sum = 0.0;
#pragma unroll
                                            for (int a = 0; a < PP::NACC; ++a)
                                              sum += double(acc[a][i][j][r]) * PP::scale(a);
                                            return sum;
                                          });
}

// ------------------------------------- wide-tile aligned slice-pair GEMM --
//
// The aligned BF16 split (three FP32 accumulators per output block plus the
// FP64 sum they are folded into) on large products: a 128 x 96 workgroup
// tile of 8 waves, each owning 32 x 48 outputs (2 x 3 blocks of the
// 16x16x32 MFMA), one workgroup per CU (two stages of S <= 5 slices fill 140
// KB of LDS) -- a 3072^2 output is 768 tiles, three full rounds.  Against
// the 128 x 64 tile every B fragment read feeds three products instead of
// two; two waves share each SIMD, so one's LDS waits and folds run under
// the other's products (the same tile with 4 waves of 64 x 48, one per
// SIMD, measured 15% slower on the CCSD-like contraction).
//
// The folds of the accumulators into FP64 sit among the products so that
// they overlap them: the exact diagonal accumulators right after their last
// products of the stage that ends a group of FOLD stages, the third one at
// the start of the stage after (before its first product there).
constexpr int WBM = 128, WBN = 96;             // block tile
constexpr int WWM = 4, WWN = 2;                // wave grid
constexpr int WNT = 64 * WWM * WWN;

// stages of S slices (64-byte rows of 16-bit values) of a WBM x WBN tile fit
// twice in LDS
constexpr bool wide_tile_fits(int S) { return 2 * S * (WBM + WBN) * 64 <= 160 * 1024; }

template <typename ST, typename Tout, int MODE, int S>
__global__ __launch_bounds__(WNT) void split_gemm_wide_kernel(const ST *__restrict__ As, const ST *__restrict__ Bs,
                                                               const int *__restrict__ eA, const int *__restrict__ eB,
                                                               Tout *__restrict__ C, const int64_t *__restrict__ offCm,
                                                               const int64_t *__restrict__ offCn, int64_t M, int64_t N,
                                                               int64_t Mp, int64_t Np, int64_t Kp, double alpha,
                                                               double beta, int tilesM, int tilesN) {
  typedef Pairs<MODE, S> PP;
  static_assert(MODE == 0 && PP::NACC == 3 && PP::FOLD == 4, "the wide tile is for the aligned split");
  static_assert(wide_tile_fits(S), "two stages must fit in LDS");
  typedef typename Vec8<ST>::type v8;
  constexpr int WM = WBM / WWM, WN = WBN / WWN;      // 32 x 48
  constexpr int FM = WM / 16, FN = WN / 16;          // 2 x 3
  constexpr int STAGE = S * (WBM + WBN) * GBK;       // elements per LDS buffer
  __shared__ __attribute__((aligned(16))) ST smem0_[STAGE];
  __shared__ __attribute__((aligned(16))) ST smem1_[STAGE];
  lds_t<ST> *const buf0 = to_lds(smem0_);
  lds_t<ST> *const buf1 = to_lds(smem1_);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int tm, tn;
  {
    const int total = tilesM * tilesN, X = 8, bid = blockIdx.x;
    const int xcd = bid % X, local = bid / X, q = total / X, rem = total % X;
    const int id = xcd * q + (xcd < rem ? xcd : rem) + local;
    const int G = 8, per = G * tilesN, group = id / per, first = group * G;
    const int gsize = tilesM - first < G ? tilesM - first : G;
    const int in = id - group * per;
    tm = first + in % gsize;
    tn = in / gsize;
  }
  const int64_t m0 = int64_t(tm) * WBM, n0 = int64_t(tn) * WBN;
  const int wm0 = (wave / WWN) * WM, wn0 = (wave % WWN) * WN;

  f4_t acc[3][FM][FN];
  d4_t acc64[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      acc64[i][j] = d4_t{0, 0, 0, 0};
#pragma unroll
      for (int a = 0; a < 3; ++a) acc[a][i][j] = f4_t{0, 0, 0, 0};
    }

  auto a_at = [&](const lds_t<ST> *buf, int p, int row, int c) { return buf + (p * WBM) * GBK + sw(row, c); };
  auto b_at = [&](const lds_t<ST> *buf, int p, int row, int c) {
    return buf + S * WBM * GBK + (p * WBN) * GBK + sw(row, c);
  };
  const int64_t nst = Kp / GBK;   // even: Kp is a multiple of 64
  // (the launch checks that a summation block of the slices spans less
  // than 4 GB)
  const char *const base = reinterpret_cast<const char *>(As);
  StageDMA32<WBM, WBN, S, WNT / 64> sd;
  sd.init(reinterpret_cast<const char *>(Bs) - base, Mp, Np, m0, n0, wave, lane);
  const int64_t RT = slice_rows(S, Mp, Np);
  // every wave issues the same number of loads per stage, so a wait for all
  // but the newer stage's loads is one constant
  constexpr int NU = StageDMA32<WBM, WBN, S, WNT / 64>::NU;
  static_assert(NU < 64, "loads in flight per wave fit the counter");
  auto dma = [&](lds_t<ST> *buf, int64_t st) {
    sd.issue(base, reinterpret_cast<lds_t<char> *>(buf), (st < nst ? st : nst - 1) * RT * 64);
  };
  // fold the exact diagonal accumulators / the third one into FP64
  auto fold01_rows = [&](int i0, int i1) {
#pragma unroll
    for (int i = i0; i < i1; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[i][j][r] += double(acc[0][i][j][r]) + double(acc[1][i][j][r]);
        acc[0][i][j] = f4_t{0, 0, 0, 0};
        acc[1][i][j] = f4_t{0, 0, 0, 0};
      }
  };
  auto fold01 = [&]() { fold01_rows(0, FM); };
  auto fold2 = [&]() {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[i][j][r] += double(acc[2][i][j][r]);
        acc[2][i][j] = f4_t{0, 0, 0, 0};
      }
  };
  // one stage from buf: the loads of the next stage into the other buffer
  // first (it was last read before the barrier that ended the stage before),
  // then the products -- the B fragments of every slice held, the A
  // fragments of one slice at a time -- then a wait for this wave's loads
  // and the barrier.  f2 / f01: fold the third accumulator (at the start,
  // before its first product) / the exact two (after their last products,
  // slice 1's pair with B slice 0).
  // The A fragments of slice p + 1 are requested before the products of
  // slice p (scheduling barriers keep them there), so that their LDS latency
  // runs under those products.
  auto read_a = [&](v8 *aF, const lds_t<ST> *buf, int p) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
      aF[i] = *reinterpret_cast<const lds_t<v8> *>(a_at(buf, p, wm0 + i * 16 + (lane & 15), lane >> 4));
  };
  auto stage = [&](const lds_t<ST> *buf, lds_t<ST> *nxt, int64_t st, auto f2, auto f01) {
    dma(nxt, st + 1);
    __builtin_amdgcn_sched_barrier(0);
    v8 aF[2][FM], bF[S][FN];
    read_a(aF[0], buf, 0);
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        bF[q][j] = *reinterpret_cast<const lds_t<v8> *>(b_at(buf, q, wn0 + j * 16 + (lane & 15), lane >> 4));
#pragma unroll
    for (int p = 0; p < S; ++p) {
      if (p + 1 < S) read_a(aF[(p + 1) & 1], buf, p + 1);
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (decltype(f2)::value)
        if (p == 0) fold2();
#pragma unroll
      for (int q = 0; q < S - p; ++q) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[PP::acc(p, q)][i][j] = mfma_slice(aF[p & 1][i], bF[q][j], acc[PP::acc(p, q)][i][j]);
        // the exact accumulators are final after slice 1's product with B
        // slice 0; their rows are folded over the products of slices 1 to 3
        // (which add to the third accumulator only)
        if constexpr (decltype(f01)::value) {
          if (p == 1 && q == 0) fold01_rows(0, FM / 2);
          if (p == 2 && q == 0) fold01_rows(FM / 2, 3 * FM / 4);
          if (p == 3 && q == 0) fold01_rows(3 * FM / 4, FM);
        }
      }
      // spread the folds' VALU work among the products: one product, then a
      // few conversions and additions, as long as both last
      if constexpr (decltype(f2)::value)
        if (p == 0)
          for (int k = 0; k < S * FM * FN; ++k) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);
          }
      if constexpr (decltype(f01)::value)
        if (p >= 1 && p <= 3)
          for (int k = 0; k < (S - p) * FM * FN; ++k) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);
          }
    }
    stage_landed();
    __builtin_amdgcn_sched_barrier(0);
  };

  dma(buf0, 0);
  stage_landed();
  int64_t st = 0;
  for (; st + 4 <= nst; st += 4) {
    // groups of FOLD = 4 stages: the third accumulator of the group before
    // is folded in the first stage, the exact two in the last
    stage(buf0, buf1, st, std::true_type{}, std::false_type{});
    stage(buf1, buf0, st + 1, std::false_type{}, std::false_type{});
    stage(buf0, buf1, st + 2, std::false_type{}, std::false_type{});
    stage(buf1, buf0, st + 3, std::false_type{}, std::true_type{});
  }
  if (st < nst) {   // two stages left (nst is even)
    stage(buf0, buf1, st, std::true_type{}, std::false_type{});
    stage(buf1, buf0, st + 1, std::false_type{}, std::false_type{});
  }
  fold2();
  fold01();

  // (the last stage's barrier passed: both buffers are free, the clamped
  // loads past the end landed)
  static_assert((WBM + WBN) * 12 <= STAGE * int(sizeof(ST)), "epilogue tables fit in LDS");
  split_store<Tout, WBM, WBN, FM, FN, WNT>(C, offCm, offCn, eA, eB, M, N, alpha, beta, m0, n0, wm0, wn0, smem0_,
                                          [&](int i, int j, int r) { return acc64[i][j][r]; });
}

// ------------------------------------------------------ INT8 slice-pair GEMM --

constexpr int IBK = 64;          // summation indices per stage (one 16x16x64 MFMA)
constexpr int IKC = 8192;        // summation indices per launch: 8 * 127^2 * 8192 < 2^31

// byte position of the 16-byte chunk c (0..3) of tile row r (64-byte rows),
// swizzled as in sw()
__device__ __forceinline__ int sw8(int r, int c) { return r * IBK + ((c ^ ((r >> 2) & 3)) << 4); }

template <typename Tout, int S>
__global__ __launch_bounds__(GNT) void split_gemm_i8_kernel(const signed char *__restrict__ As,
                                                             const signed char *__restrict__ Bs,
                                                             const int *__restrict__ eA, const int *__restrict__ eB,
                                                             Tout *__restrict__ C, const int64_t *__restrict__ offCm,
                                                             const int64_t *__restrict__ offCn, int64_t M, int64_t N,
                                                             int64_t Mp, int64_t Np, int64_t Kp, int64_t k_begin,
                                                             int64_t k_len, double alpha, double beta, int tilesM,
                                                             int tilesN) {
  constexpr int WM = GBM / GWM, WN = GBN / GWN;      // 32 x 32
  constexpr int FM = WM / 16, FN = WN / 16;          // 2 x 2
  constexpr int NVA = S * GBM * (IBK / 16);          // 16-byte vectors per stage
  constexpr int NVB = S * GBN * (IBK / 16);
  constexpr int NV = (NVA + NVB + GNT - 1) / GNT;
  constexpr int STAGE = S * (GBM + GBN) * IBK;       // bytes per LDS buffer
  constexpr int NBUF = 2 * STAGE <= 150 * 1024 ? 2 : 1;   // two buffers as two objects, as above
  __shared__ __attribute__((aligned(16))) signed char smem[NBUF == 1 ? STAGE : 1];
  __shared__ __attribute__((aligned(16))) signed char smem0_[NBUF == 2 ? STAGE : 1];
  __shared__ __attribute__((aligned(16))) signed char smem1_[NBUF == 2 ? STAGE : 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int tm, tn;
  {
    const int total = tilesM * tilesN, X = 8, bid = blockIdx.x;
    const int xcd = bid % X, local = bid / X, q = total / X, rem = total % X;
    const int id = xcd * q + (xcd < rem ? xcd : rem) + local;
    const int G = 8, per = G * tilesN, group = id / per, first = group * G;
    const int gsize = tilesM - first < G ? tilesM - first : G;
    const int in = id - group * per;
    tm = first + in % gsize;
    tn = in / gsize;
  }
  const int64_t m0 = int64_t(tm) * GBM, n0 = int64_t(tn) * GBN;
  const int wm0 = (wave / GWN) * WM, wn0 = (wave % GWN) * WN;

  i4_t acc[S][FM][FN];       // one exact int32 accumulator per diagonal p + q
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int d = 0; d < S; ++d) acc[d][i][j] = i4_t{0, 0, 0, 0};
  auto a_at = [&](signed char *buf, int p, int row, int c) { return buf + (p * GBM) * IBK + sw8(row, c); };
  auto b_at = [&](signed char *buf, int p, int row, int c) {
    return buf + S * GBM * IBK + (p * GBN) * IBK + sw8(row, c);
  };
  i4_t pre[NV];
  const int64_t nst = k_len / IBK;
  const int64_t RT = slice_rows(S, Mp, Np);
  auto gload = [&](int64_t st) {
    const int64_t kr = (k_begin / IBK + (st < nst ? st : nst - 1)) * RT;   // the stage's summation block, in rows
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int v = tid + u * GNT;
      if (v < NVA) {
        const int p = v / (GBM * 4), rem = v % (GBM * 4), row = rem / 4, kc = (rem % 4) * 16;
        pre[u] = *reinterpret_cast<const i4_t *>(As + (kr + int64_t(p) * Mp + m0 + row) * IBK + kc);
      } else if (v < NVA + NVB) {
        const int w = v - NVA;
        const int p = w / (GBN * 4), rem = w % (GBN * 4), row = rem / 4, kc = (rem % 4) * 16;
        pre[u] = *reinterpret_cast<const i4_t *>(Bs + (kr + int64_t(p) * Np + n0 + row) * IBK + kc);
      }
    }
  };
  auto lstore = [&](signed char *buf) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int v = tid + u * GNT;
      if (v < NVA) {
        const int p = v / (GBM * 4), rem = v % (GBM * 4), row = rem / 4, c = rem % 4;
        *reinterpret_cast<i4_t *>(a_at(buf, p, row, c)) = pre[u];
      } else if (v < NVA + NVB) {
        const int w = v - NVA;
        const int p = w / (GBN * 4), rem = w % (GBN * 4), row = rem / 4, c = rem % 4;
        *reinterpret_cast<i4_t *>(b_at(buf, p, row, c)) = pre[u];
      }
    }
  };
  auto compute = [&](signed char *buf) {
    i4_t bF[S][FN];
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        bF[q][j] = *reinterpret_cast<const i4_t *>(b_at(buf, q, wn0 + j * 16 + (lane & 15), lane >> 4));
#pragma unroll
    for (int p = 0; p < S; ++p) {
      i4_t aF[FM];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        aF[i] = *reinterpret_cast<const i4_t *>(a_at(buf, p, wm0 + i * 16 + (lane & 15), lane >> 4));
#pragma unroll
      for (int q = 0; q < S; ++q) {
        if (p + q <= S - 1) {
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
              acc[p + q][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(aF[i], bF[q][j], acc[p + q][i][j], 0, 0, 0);
        }
      }
    }
  };

  if constexpr (NBUF == 2) {
    StageDMA<GBM, GBN, S, GNT / 64> sd;
    sd.init(reinterpret_cast<const char *>(As), reinterpret_cast<const char *>(Bs), Mp, Np, m0, n0, wave, lane);
    auto dma = [&](signed char *buf, int64_t st) {
      sd.issue(reinterpret_cast<lds_t<char> *>(to_lds(buf)), (k_begin / IBK + (st < nst ? st : nst - 1)) * RT * 64);
    };
    dma(smem0_, 0);
    stage_landed();
    int64_t st = 0;
    for (; st + 1 < nst; st += 2) {
      dma(smem1_, st + 1);
      __builtin_amdgcn_sched_barrier(0);
      compute(smem0_);
      stage_landed();
      dma(smem0_, st + 2);
      __builtin_amdgcn_sched_barrier(0);
      compute(smem1_);
      stage_landed();
    }
    if (st < nst) compute(smem0_);   // an odd last stage, loaded by the last half step
  } else {
    gload(0);
    lstore(smem);
    __syncthreads();
    for (int64_t st = 0; st < nst; ++st) {
      gload(st + 1);
      compute(smem);
      __syncthreads();
      lstore(smem);
      __syncthreads();
    }
  }

  static_assert((GBM + GBN) * 12 <= STAGE, "epilogue tables fit in LDS");
  // (after an odd last stage, buffer 0 is still being read: wait for every
  // wave before its first bytes take the epilogue tables)
  if constexpr (NBUF == 2) __syncthreads();
  split_store<Tout, GBM, GBN, FM, FN, GNT>(C, offCm, offCn, eA, eB, M, N, alpha, beta, m0, n0, wm0, wn0,
                                          NBUF == 2 ? static_cast<void *>(smem0_) : static_cast<void *>(smem),
                                          [&](int i, int j, int r) {
                                            double sum = 0.0;
#pragma unroll
                                            for (int d = S - 1; d >= 0; --d)
                                              sum += double(acc[d][i][j][r]) * ldexp(1.0, -7 * (d + 2));
                                            return sum;
                                          });
}

// ----------------------------------------------------------------- launch --

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

template <typename Tin, typename ST, int MODE, int S>
hipError_t run_split(const Analysis &an, const SplitPlan &sp, const GettTables &t, double alpha, const void *A,
                     const void *B, double beta, void *C, void *ws, hipStream_t s, bool vecA, bool vecB) {
  char *w = static_cast<char *>(ws);
  ST *As = reinterpret_cast<ST *>(w + sp.offA);
  ST *Bs = reinterpret_cast<ST *>(w + sp.offB);
  int *eA = reinterpret_cast<int *>(w + sp.offEA);
  int *eB = reinterpret_cast<int *>(w + sp.offEB);
  // both operands in one exponent launch and one pack launch
  SliceArgs a{};
  a.op[0] = SliceOperand{A, t.offAm, t.offAk, an.m, an.layoutA, vecA ? 1 : 0, int(sp.Mp / PR),
                         reinterpret_cast<int *>(w + sp.offPA), eA, As, sp.Mp};
  a.op[1] = SliceOperand{B, t.offBn, t.offBk, an.n, an.layoutB, vecB ? 1 : 0, int(sp.Np / PR),
                         reinterpret_cast<int *>(w + sp.offPB), eB, Bs, sp.Np};
  a.K = an.k;
  a.Kp = sp.Kp;
  a.RT = slice_rows(S, sp.Mp, sp.Np);
  a.ky = sp.ky;
  hipLaunchKernelGGL((split_exp_kernel<Tin>), dim3(unsigned(a.op[0].tilesR + a.op[1].tilesR), unsigned(sp.ky)),
                     dim3(PT), 0, s, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const int64_t packs = (int64_t(a.op[0].tilesR) + a.op[1].tilesR) * (sp.Kp / PK);
  hipLaunchKernelGGL((split_pack_kernel<Tin, ST, MODE, S>), dim3(unsigned(packs)), dim3(PT), 0, s, a);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  const int tilesM = int(sp.Mp / GBM), tilesN = int(sp.Np / GBN);
  if constexpr (MODE == 3) {
    // exact int32 diagonal sums over at most IKC indices per launch; later
    // launches add into C
    for (int64_t k0 = 0; k0 < sp.Kp; k0 += IKC) {
      const int64_t len = sp.Kp - k0 < IKC ? sp.Kp - k0 : IKC;
      hipLaunchKernelGGL((split_gemm_i8_kernel<Tin, S>), dim3(tilesM * tilesN), dim3(GNT), 0, s, As, Bs, eA, eB,
                         static_cast<Tin *>(C), t.offCm, t.offCn, an.m, an.n, sp.Mp, sp.Np, sp.Kp, k0, len, alpha,
                         k0 == 0 ? beta : 1.0, tilesM, tilesN);
    }
  } else if (sp.tile == 2) {
    if constexpr (MODE == 0 && wide_tile_fits(S)) {
      hipLaunchKernelGGL((split_gemm_wide_kernel<ST, Tin, MODE, S>), dim3(int(sp.Mp / WBM) * int(sp.Np / WBN)),
                         dim3(WNT), 0, s, As, Bs, eA, eB, static_cast<Tin *>(C), t.offCm, t.offCn, an.m, an.n, sp.Mp,
                         sp.Np, sp.Kp, alpha, beta, int(sp.Mp / WBM), int(sp.Np / WBN));
    } else {
      return hipErrorInvalidValue;
    }
  } else if (sp.tile == 1) {
    if constexpr (Pairs<MODE, S>::FOLD == 0) {
      hipLaunchKernelGGL((split_gemm_big_kernel<ST, Tin, MODE, S>), dim3(int(sp.Mp / XBM) * int(sp.Np / XBN)),
                         dim3(XNT), 0, s, As, Bs, eA, eB, static_cast<Tin *>(C), t.offCm, t.offCn, an.m, an.n, sp.Mp,
                         sp.Np, sp.Kp, alpha, beta, int(sp.Mp / XBM), int(sp.Np / XBN));
    } else {
      return hipErrorInvalidValue;
    }
  } else
    hipLaunchKernelGGL((split_gemm_kernel<ST, Tin, MODE, S>), dim3(tilesM * tilesN), dim3(GNT), 0, s, As, Bs, eA,
                       eB, static_cast<Tin *>(C), t.offCm, t.offCn, an.m, an.n, sp.Mp, sp.Np, sp.Kp, alpha, beta,
                       tilesM, tilesN);
  return hipGetLastError();
}

template <typename Tin>
hipError_t dispatch(const Analysis &an, const SplitPlan &sp, const GettTables &t, double alpha, const void *A,
                    const void *B, double beta, void *C, void *ws, hipStream_t s, bool vecA, bool vecB) {
  if (sp.mode == 1) return run_split<Tin, __bf16, 1, 3>(an, sp, t, alpha, A, B, beta, C, ws, s, vecA, vecB);
  if (sp.mode == 2) return run_split<Tin, _Float16, 2, 2>(an, sp, t, alpha, A, B, beta, C, ws, s, vecA, vecB);
  if (sp.mode == 3) {
    switch (sp.S) {
      case 3: return run_split<Tin, signed char, 3, 3>(an, sp, t, alpha, A, B, beta, C, ws, s, vecA, vecB);
      case 4: return run_split<Tin, signed char, 3, 4>(an, sp, t, alpha, A, B, beta, C, ws, s, vecA, vecB);
      case 5: return run_split<Tin, signed char, 3, 5>(an, sp, t, alpha, A, B, beta, C, ws, s, vecA, vecB);
      case 6: return run_split<Tin, signed char, 3, 6>(an, sp, t, alpha, A, B, beta, C, ws, s, vecA, vecB);
      case 7: return run_split<Tin, signed char, 3, 7>(an, sp, t, alpha, A, B, beta, C, ws, s, vecA, vecB);
      case 8: return run_split<Tin, signed char, 3, 8>(an, sp, t, alpha, A, B, beta, C, ws, s, vecA, vecB);
      default: return hipErrorInvalidValue;
    }
  }
  switch (sp.S) {
    case 3: return run_split<Tin, __bf16, 0, 3>(an, sp, t, alpha, A, B, beta, C, ws, s, vecA, vecB);
    case 4: return run_split<Tin, __bf16, 0, 4>(an, sp, t, alpha, A, B, beta, C, ws, s, vecA, vecB);
    case 5: return run_split<Tin, __bf16, 0, 5>(an, sp, t, alpha, A, B, beta, C, ws, s, vecA, vecB);
    case 6: return run_split<Tin, __bf16, 0, 6>(an, sp, t, alpha, A, B, beta, C, ws, s, vecA, vecB);
    default: return hipErrorInvalidValue;
  }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

Status split_prepare(const Analysis &an, SplitPlan &sp, int force_tile) {
  sp = SplitPlan();
  sp.mode = an.compute == COMET_COMPUTE_SPLIT_BF16     ? 0
            : an.compute == COMET_COMPUTE_SPLIT_BF16X3 ? 1
            : an.compute == COMET_COMPUTE_SPLIT_FP16X2 ? 2
                                                       : 3;
  sp.S = (sp.mode == 0 || sp.mode == 3) ? an.split_slices : sp.mode == 1 ? 3 : 2;
  if (sp.mode == 0 && (sp.S < 3 || sp.S > 6))
    return Status::error(COMET_ERR_UNSUPPORTED, "split slices must be within 3..6");
  if (sp.mode == 3 && (sp.S < 3 || sp.S > 8))
    return Status::error(COMET_ERR_UNSUPPORTED, "int8 split slices must be within 3..8");
  // the large tile for the classic splits on large products, when padding
  // to 192 wastes little (COMET_SPLIT_TILE=0/1 overrides)
  sp.tile = 0;
  const char *env = std::getenv("COMET_SPLIT_TILE");
  if (sp.mode == 1 || sp.mode == 2) {
    const double waste = double(round_up(an.m, XBM)) * double(round_up(an.n, XBN)) / (double(an.m) * double(an.n));
    sp.tile = (an.m >= 1536 && an.n >= 1536 && waste <= 1.1) ? 1 : 0;
    if (env && *env) sp.tile = std::atoi(env) == 1 ? 1 : 0;
    if (force_tile >= 0) sp.tile = force_tile == 1 ? 1 : 0;
  } else if (sp.mode == 0 && wide_tile_fits(sp.S)) {
    // the wide tile pads N to a multiple of 192 (its 96 and the slicer's 64)
    const double waste = double(round_up(an.m, WBM)) * double(round_up(an.n, 192)) / (double(an.m) * double(an.n));
    sp.tile = (an.m >= 1024 && an.n >= 1024 && waste <= 1.1) ? 2 : 0;
    if (env && *env) sp.tile = std::atoi(env) == 2 ? 2 : 0;
    if (force_tile >= 0) sp.tile = force_tile == 2 ? 2 : 0;
    // its loads address a summation block of the slices with 32-bit offsets
    if (64.0 * sp.S * (double(round_up(an.m, WBM)) + double(round_up(an.n, 192))) >= 4294967296.0) sp.tile = 0;
  }
  sp.Mp = round_up(an.m, sp.tile == 1 ? XBM : sp.tile == 2 ? WBM : GBM);
  sp.Np = round_up(an.n, sp.tile == 1 ? XBN : sp.tile == 2 ? 192 : GBN);
  sp.Kp = round_up(an.k, PK);   // whole slicer tiles (a multiple of GBK and IBK)
  const int64_t tiles = sp.tile == 1   ? (sp.Mp / XBM) * (sp.Np / XBN)
                        : sp.tile == 2 ? (sp.Mp / WBM) * (sp.Np / WBN)
                                       : (sp.Mp / GBM) * (sp.Np / GBN);
  // one pack launch covers both operands' tiles; its grid must stay below
  // 2^32 work-items
  if (tiles > INT_MAX || ((sp.Mp + sp.Np) / PR) * (sp.Kp / PK) > int64_t(INT_MAX) / PT)
    return Status::error(COMET_ERR_UNSUPPORTED, "problem too large for the split path");
  // exponent pass: about 512 blocks over both operands' row tiles and ky
  // ranges of the summation (each block walks several summation tiles with
  // the next one's loads in flight; on the CCSD-like operands 512 blocks
  // took 32.8 us, 2048 blocks 39.5 us and 256 blocks 38.5 us)
  {
    const int64_t rows = sp.Mp / PR + sp.Np / PR, tilesK = sp.Kp / PK;
    sp.ky = int(std::max<int64_t>(1, std::min<int64_t>({(512 + rows - 1) / rows, tilesK, int64_t(64)})));
  }
  const size_t es = sp.mode == 3 ? 1 : 2;
  size_t off = 0;
  // both operands' slices in the blocked layout: B's first row follows A's
  // S Mp rows of the first summation block
  sp.offA = off;
  sp.offB = off + size_t(sp.S) * sp.Mp * 64;
  off = align256(off + size_t(slice_rows(sp.S, sp.Mp, sp.Np)) * sp.Kp * es);
  sp.offEA = off;
  off = align256(off + size_t(sp.Mp) * 4);
  sp.offEB = off;
  off = align256(off + size_t(sp.Np) * 4);
  sp.offPA = off;
  off = align256(off + size_t(sp.ky) * sp.Mp * 4);
  sp.offPB = off;
  off = align256(off + size_t(sp.ky) * sp.Np * 4);
  sp.ws_bytes = off;
  return Status{};
}

hipError_t split_execute(const Analysis &an, const SplitPlan &sp, const GettTables &t, double alpha, const void *A,
                         const void *B, double beta, void *C, void *ws, hipStream_t s, bool vecA, bool vecB) {
  // the slicers read vectors only from 16-byte aligned operands
  vecA = vecA && reinterpret_cast<uintptr_t>(A) % 16 == 0;
  vecB = vecB && reinterpret_cast<uintptr_t>(B) % 16 == 0;
  if (an.dtype == COMET_F64) return dispatch<double>(an, sp, t, alpha, A, B, beta, C, ws, s, vecA, vecB);
  return dispatch<float>(an, sp, t, alpha, A, B, beta, C, ws, s, vecA, vecB);
}

}  // namespace comet
