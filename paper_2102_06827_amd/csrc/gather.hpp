// gather.hpp -- device building blocks shared by the gather kernels: the
// MFMA wrappers, XCD-aware tile ordering and the operand tile loader that
// gathers through per-label offset tables.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "kernels.hpp"

namespace comet {
namespace gather {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));

template <typename T> struct AccT;
template <> struct AccT<double> { typedef d4_t type; };
template <> struct AccT<float> { typedef f4_t type; };

__device__ __forceinline__ d4_t mfma16(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma16(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// An LDS pointer with its address space spelled out.  Every access through it
// compiles to ds_read / ds_write.  A plain pointer chosen at run time between
// the halves of a double buffer is lowered to flat instructions instead, and a
// flat load waits on every global load in flight (vmcnt), which serialises the
// software pipeline.
template <typename T> using lds_t = __attribute__((address_space(3))) T;
template <typename T> __device__ __forceinline__ lds_t<T> *to_lds(T *p) { return (lds_t<T> *)p; }

// The same for device (global) memory.  Pointers that reach a kernel through
// a descriptor in memory, rather than as kernel arguments, would otherwise be
// accessed with flat instructions, which count against the LDS wait counter
// too, so every LDS fragment read would also wait for the tile prefetch.
template <typename T> using glb_t = __attribute__((address_space(1))) T;
template <typename T> __device__ __forceinline__ glb_t<T> *to_glb(T *p) { return (glb_t<T> *)p; }

// row of the 16 x 16 output block held in accumulator element r of a lane
template <typename Tc> __device__ __forceinline__ int acc_row(int lane, int r);
template <> __device__ __forceinline__ int acc_row<double>(int lane, int r) { return (lane >> 4) + 4 * r; }
template <> __device__ __forceinline__ int acc_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }


// 16-byte vector of Tin
template <typename T> struct V16;
template <> struct V16<double> {
  static constexpr int N = 2;
  typedef double type __attribute__((ext_vector_type(2)));
};
template <> struct V16<float> {
  static constexpr int N = 4;
  typedef float type __attribute__((ext_vector_type(4)));
};

// Map a linear workgroup id in [0, total) to a tile id in [0, total) such
// that the workgroups the hardware places on one XCD (ids congruent mod 8)
// get consecutive tile ids.
__device__ __forceinline__ int xcd_remap(int bid, int total) {
  const int X = 8;
  int xcd = bid % X, local = bid / X;
  int q = total / X, rem = total % X;
  return xcd * q + (xcd < rem ? xcd : rem) + local;
}

// Tile id -> tile coordinates, walking tiles in groups of G tile-rows so that
// consecutive ids (one XCD's workgroups) share A rows and B columns in its L2.
__device__ __forceinline__ void group_coords(int id, int tilesM, int tilesN, int *tm, int *tn) {
  const int G = 8;
  int per_group = G * tilesN;
  int group = id / per_group;
  int first = group * G;
  int gsize = tilesM - first < G ? tilesM - first : G;
  int in = id - group * per_group;
  *tm = first + in % gsize;
  *tn = in / gsize;
}

__device__ __forceinline__ void tile_coords(int bid, int tilesM, int tilesN, int *tm, int *tn) {
  group_coords(xcd_remap(bid, tilesM * tilesN), tilesM, tilesN, tm, tn);
}

// One operand tile: R rows (m for A, n for B) by BK summation indices.
// LAYOUT 0: the operand is contiguous along k in memory; threads walk k and
// the LDS tile keeps k contiguous, s[r][k] with pitch BK + KPAD, so a thread's
// vector is one 16-byte LDS store.  LAYOUT 1: contiguous along r; s[k][r]
// with pitch R + PAD.  The pads make the strided 16-lane MFMA fragment reads
// of either layout hit distinct banks.
//
// Loads are branch-free: an out-of-range element is fetched from a clamped,
// valid address and replaced by zero afterwards, so no load sits under a
// divergent branch (which would force a full wait at the join).  The K-offset
// table entries a step needs are fetched one step ahead, so a data load never
// waits on the table load that addresses it.
// Position of element (row, k) in a sliced bfloat16 tile with row pitch LDK
// (32 summation indices per row): the row's four 8-element chunks are
// swizzled by (row / 16) mod 4.  Sixteen consecutive rows (one MFMA
// fragment) share the swizzle, so fragment reads stay as they were, while
// the stores of an operand contiguous along rows -- one element in each of
// 32 rows four apart, at one k -- spread over four times as many banks.
template <int LDK>
__device__ __forceinline__ int split3_pos(int row, int k) {
  return row * LDK + ((((k >> 3) ^ (row >> 4)) & 3) << 3) + (k & 7);
}

template <typename Tin, typename Tc, int R, int BK, int LAYOUT, bool VECLD, int NT>
struct Loader {
  static constexpr int VEC = V16<Tin>::N;
  static constexpr int P = R * BK / (VEC * NT);
  static_assert(P >= 1 && P * VEC * NT == R * BK, "tile does not split evenly over the workgroup");
  static constexpr int PAD = 4;
  static constexpr int LDR = R + PAD;                       // LAYOUT 1 pitch
  static constexpr int KPAD = sizeof(Tc) == 8 ? 2 : 4;       // 16 bytes
  static constexpr int LDK = BK + KPAD;                      // LAYOUT 0 pitch
  static constexpr int ELEMS = LAYOUT == 0 ? R * LDK : BK * LDR;   // per LDS buffer
  // LDS position of element (row r, summation index k)
  static __device__ __forceinline__ int idx(int r, int k) { return LAYOUT == 0 ? r * LDK + k : k * LDR + r; }
  // K-table entries held per pass: one per vector, or one per element when
  // a K-contiguous operand is read element by element
  static constexpr int NKO = (LAYOUT == 0) ? VEC : 1;

  Tin v[P][VEC];
  int64_t roff[P][VEC];     // hoisted row offsets (clamped to a valid row)
  static_assert(P * VEC <= 32, "masks hold one bit per element");
  uint32_t rmask;           // bit p * VEC + i: row of element i of pass p in range
  uint32_t vmask;           // bit p * VEC + i: element i of pass p of the last load in range
  int64_t kofs[P][NKO];     // K-table entries of the step being fetched next
  int rr[P], kk[P];

  static constexpr bool vec = VECLD;

  __device__ __forceinline__ void init(int tid, int64_t r0, int64_t Rtot, const int64_t *__restrict__ offR_) {
    init_from(tid, r0, Rtot, to_glb(offR_), 0);
  }

  // Row offsets from `rows`, where rows[g - base] holds the table entry of
  // row g (base 0: the table itself; base r0: a copy of the tile's R entries
  // staged in LDS).  Rows past Rtot are masked and read entry `base`.
  template <typename Rows>
  __device__ __forceinline__ void init_from(int tid, int64_t r0, int64_t Rtot, Rows rows, int64_t base) {
    rmask = 0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      int id = tid + p * NT;
      if (LAYOUT == 0) {
        rr[p] = id / (BK / VEC);
        kk[p] = (id % (BK / VEC)) * VEC;
      } else {
        kk[p] = id / (R / VEC);
        rr[p] = (id % (R / VEC)) * VEC;
      }
      const int64_t gr = r0 + rr[p];
#pragma unroll
      for (int i = 0; i < VEC; ++i) {
        // K-contiguous and vector reads share the vector's first row offset
        const int64_t g = (LAYOUT == 0 || vec) ? gr : gr + i;
        const bool ok = g < Rtot;
        roff[p][i] = rows[(ok ? g : base) - base];
        rmask |= (ok ? 1u : 0u) << (p * VEC + i);
      }
    }
  }

  // fetch the K-table entries for the step starting at k0.  Indices past the
  // end are clamped to the last valid start: K - 1 for single elements, and
  // K - VEC for a K-contiguous vector (K is a multiple of VEC in that mode),
  // so the clamped vector still lies inside the tensor.
  __device__ __forceinline__ void fetch_k(const int64_t *__restrict__ offK_, int64_t k0, int64_t K) {
    const glb_t<const int64_t> *offK = to_glb(offK_);
    constexpr bool kvec = LAYOUT == 0 && VECLD;
    const int64_t last = kvec ? K - VEC : K - 1;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int64_t k = k0 + kk[p];
#pragma unroll
      for (int i = 0; i < NKO; ++i) {
        int64_t ki = k + ((LAYOUT == 0 && !vec) ? i : 0);
        kofs[p][i] = offK[ki <= last ? ki : last];
      }
    }
  }

  // load the step starting at k0, addressed by the K-table entries fetched
  // for it; the raw values are kept and masked only when stored to LDS, so
  // no instruction between here and the store waits for the loads.  FULL:
  // the tile lies inside the operand and the summation is a whole number of
  // steps, so nothing is masked (a step past the end, loaded but never
  // multiplied, reads the clamped last step).
  template <bool FULL = false>
  __device__ __forceinline__ void load(const Tin *__restrict__ base_, int64_t k0, int64_t K) {
    const glb_t<const Tin> *base = to_glb(base_);
    if constexpr (FULL && VECLD) {
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const typename V16<Tin>::type x =
            *reinterpret_cast<const glb_t<typename V16<Tin>::type> *>(base + roff[p][0] + kofs[p][0]);
#pragma unroll
        for (int i = 0; i < VEC; ++i) v[p][i] = x[i];
      }
      vmask = ~0u;
      return;
    }
    uint32_t vm = 0;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int64_t k = k0 + kk[p];
      uint32_t m = 0;
      if constexpr (VECLD) {
        const typename V16<Tin>::type x =
            *reinterpret_cast<const glb_t<typename V16<Tin>::type> *>(base + roff[p][0] + kofs[p][0]);
        const bool ok = ((rmask >> (p * VEC)) & 1u) && k < K;
#pragma unroll
        for (int i = 0; i < VEC; ++i) v[p][i] = x[i];
        m = ok ? ((1u << VEC) - 1u) : 0u;
      } else {
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
          const int64_t ko = kofs[p][LAYOUT == 0 ? i : 0];
          v[p][i] = base[roff[p][LAYOUT == 0 ? 0 : i] + ko];
          const bool ok = LAYOUT == 0 ? (((rmask >> (p * VEC)) & 1u) && k + i < K)
                                      : (((rmask >> (p * VEC + i)) & 1u) && k < K);
          m |= (ok ? 1u : 0u) << i;
        }
      }
      vm |= m << (p * VEC);
    }
    vmask = vm;
  }

  // Store as three bfloat16 slices x = b0 + b1 + b2 (b0 = bf16(x), b1 = bf16 of
  // the remainder, b2 = bf16 of what is left; exact for FP32 x), in the layout
  // s[slice][row][k] with row pitch LDK (k contiguous, as the 16x16x32 MFMA
  // operands are read) and the 8-element chunks of a row swizzled by
  // split3_pos.  K-contiguous operands store each slice's four consecutive k
  // as one 8-byte write.
  template <int LDK>
  __device__ __forceinline__ void store_split3(lds_t<__bf16> *s) const {
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int p = 0; p < P; ++p) {
      __bf16 b[3][VEC];
#pragma unroll
      for (int i = 0; i < VEC; ++i) {
        const float x = ((vmask >> (p * VEC + i)) & 1u) ? float(v[p][i]) : 0.0f;
        b[0][i] = __bf16(x);
        const float r1 = x - float(b[0][i]);
        b[1][i] = __bf16(r1);
        b[2][i] = __bf16(r1 - float(b[1][i]));
      }
      if constexpr (LAYOUT == 0 && VEC == 4) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          bf16x4 w;
#pragma unroll
          for (int i = 0; i < 4; ++i) w[i] = b[q][i];
          *reinterpret_cast<lds_t<bf16x4> *>(&s[q * R * LDK + split3_pos<LDK>(rr[p], kk[p])]) = w;
        }
      } else {
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
          const int row = LAYOUT == 0 ? rr[p] : rr[p] + i;
          const int k = LAYOUT == 0 ? kk[p] + i : kk[p];
#pragma unroll
          for (int q = 0; q < 3; ++q) s[q * R * LDK + split3_pos<LDK>(row, k)] = b[q][i];
        }
      }
    }
  }

  // Direct-to-LDS load of the step whose K-table entries were fetched last
  // (unmasked: whole tiles only), for a row-contiguous operand (LAYOUT 1)
  // whose tile rows span one wave: pass p of wave w is summation index kk[p]
  // (the same in every lane), lane L the elements 2 L, 2 L + 1 -- exactly
  // the 16 bytes at L x 16 from the start of that index's row in the LDS
  // tile.  No registers hold the data; the loads are counted by the
  // vector-memory counter.
  static constexpr bool dma_ok = LAYOUT == 1 && VECLD && VEC * sizeof(Tin) == 16 && R / VEC == 64 &&
                                 sizeof(Tin) == sizeof(Tc);
  __device__ __forceinline__ void dma(const Tin *__restrict__ base_, lds_t<Tc> *s) const {
    static_assert(dma_ok, "direct-to-LDS loads need one wave per tile row");
    const glb_t<const Tin> *base = to_glb(base_);
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int kr = __builtin_amdgcn_readfirstlane(kk[p]);
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const glb_t<void> *>(base + roff[p][0] + kofs[p][0]),
                                       reinterpret_cast<lds_t<void> *>(s + idx(0, kr)), 16, 0, 0);
    }
  }

  __device__ __forceinline__ void store(lds_t<Tc> *s) const {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      Tc x[VEC];
#pragma unroll
      for (int i = 0; i < VEC; ++i) x[i] = ((vmask >> (p * VEC + i)) & 1u) ? Tc(v[p][i]) : Tc(0);
      // VEC consecutive elements along the contiguous dimension: one vector store
      // when they fill 16 bytes, element stores otherwise (FP32 arithmetic on
      // FP64 storage)
      lds_t<Tc> *dst = s + idx(rr[p], kk[p]);
      if constexpr (VEC * sizeof(Tc) == 16) {
        typedef Tc vec_t __attribute__((ext_vector_type(VEC)));
        vec_t w;
#pragma unroll
        for (int i = 0; i < VEC; ++i) w[i] = x[i];
        *reinterpret_cast<lds_t<vec_t> *>(dst) = w;
      } else {
#pragma unroll
        for (int i = 0; i < VEC; ++i) dst[i] = x[i];
      }
    }
  }
};


// Elements of LDS (of type Tc) one gett_tile call needs.
// Whether a whole-tile (FULL) accumulation moves B into LDS by direct-to-LDS
// loads, into two buffers of its own.
template <typename Tin, typename Tc, int BN, int BK, int LB, bool VB, int NT, bool FULL>
constexpr bool gett_dma_b() {
  return FULL && Loader<Tin, Tc, BN, BK, LB, VB, NT>::dma_ok;
}

// Elements of LDS (of type Tc) one gett_tile call needs (besides the B
// buffers of a direct-to-LDS accumulation, which it declares itself).
template <typename Tin, typename Tc, int BM, int BN, int BK, int NT, int LA, int LB, bool VA, bool VB,
          bool FULL = false>
constexpr int gett_lds_elems() {
  return 2 * (Loader<Tin, Tc, BM, BK, LA, VA, NT>::ELEMS +
              (gett_dma_b<Tin, Tc, BN, BK, LB, VB, NT, FULL>() ? 0 : Loader<Tin, Tc, BN, BK, LB, VB, NT>::ELEMS));
}

// The register tile of one workgroup: a WGM x WGN grid of waves, each owning
// FM x FN MFMA blocks of 16 x 16.
template <typename Tc, int BM, int BN, int WGM, int WGN>
struct WaveTile {
  typedef Tc elem_t;
  typedef typename AccT<Tc>::type acc_t;
  static constexpr int NT = 64 * WGM * WGN;
  static constexpr int WM = BM / WGM, WN = BN / WGN;
  static constexpr int FM = WM / 16, FN = WN / 16;
  static_assert(FM * 16 == WM && FN * 16 == WN, "wave tile must be a multiple of 16");
  acc_t acc[FM][FN];
};

// One BK step of the product from the LDS tiles a_s (BM x BK) and b_s
// (BN x BK): every wave multiplies its FM x FN MFMA blocks.
template <typename LoadA, typename LoadB, int BK, typename WT>
__device__ __forceinline__ void gett_mma_step(WT &w, const lds_t<typename WT::elem_t> *a_s,
                                              const lds_t<typename WT::elem_t> *b_s, int lane, int wm0,
                                              int wn0) {
  typedef typename WT::elem_t Tc;
#pragma unroll
  for (int k4 = 0; k4 < BK; k4 += 4) {
    const int kr = k4 + (lane >> 4);
    Tc af[WT::FM], bf[WT::FN];
#pragma unroll
    for (int i = 0; i < WT::FM; ++i) af[i] = a_s[LoadA::idx(wm0 + i * 16 + (lane & 15), kr)];
#pragma unroll
    for (int j = 0; j < WT::FN; ++j) bf[j] = b_s[LoadB::idx(wn0 + j * 16 + (lane & 15), kr)];
#pragma unroll
    for (int i = 0; i < WT::FM; ++i)
#pragma unroll
      for (int j = 0; j < WT::FN; ++j) w.acc[i][j] = mfma16(af[i], bf[j], w.acc[i][j]);
  }
}

// Accumulate the product of the BM x BN output tile at (m0, n0) over the
// summation steps [s_begin, s_end) of BK indices each: gather A and B through
// the offset tables into double-buffered LDS tiles and multiply on the
// 16 x 16 x 4 MFMA.  All threads of the workgroup must call it (it
// synchronizes); smem holds gett_lds_elems values.
template <typename Tin, typename Tc, int BM, int BN, int BK, int WGM, int WGN, int LA, int LB, bool VA, bool VB,
          bool FULL = false>
__device__ __forceinline__ void gett_accumulate(WaveTile<Tc, BM, BN, WGM, WGN> &w, const Tin *__restrict__ A,
                                                const Tin *__restrict__ B, const GettTables &t, int64_t M,
                                                int64_t N, int64_t K, int64_t m0, int64_t n0, int64_t s_begin,
                                                int64_t s_end, Tc *smem) {
  typedef WaveTile<Tc, BM, BN, WGM, WGN> WT;
  constexpr int NT = WT::NT, FM = WT::FM, FN = WT::FN;
  typedef Loader<Tin, Tc, BM, BK, LA, VA, NT> LoadA;
  typedef Loader<Tin, Tc, BN, BK, LB, VB, NT> LoadB;
  typedef typename WT::acc_t acc_t;
  lds_t<Tc> *const s0 = to_lds(smem);
  lds_t<Tc> *sA[2] = {s0, s0 + LoadA::ELEMS};
  lds_t<Tc> *sB[2] = {s0 + 2 * LoadA::ELEMS, s0 + 2 * LoadA::ELEMS + LoadB::ELEMS};

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WGN) * WT::WM, wn0 = (wave % WGN) * WT::WN;

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) w.acc[i][j] = acc_t{0, 0, 0, 0};

  LoadA la;
  LoadB lb;
  la.init(tid, m0, M, t.offAm);
  lb.init(tid, n0, N, t.offBn);

  if constexpr (gett_dma_b<Tin, Tc, BN, BK, LB, VB, NT, FULL>()) {
    // B by direct-to-LDS loads into two buffers that are objects of their
    // own (so that the compiler can tell the loads into one from the reads
    // of the other), the step loop unrolled by two so that each half names
    // its buffers; A as below, through registers
    __shared__ __attribute__((aligned(16))) Tc sB0_[LoadB::ELEMS];
    __shared__ __attribute__((aligned(16))) Tc sB1_[LoadB::ELEMS];
    lds_t<Tc> *const sB0 = to_lds(sB0_), *const sB1 = to_lds(sB1_);
    const lds_t<Tc> *const sA0 = s0;
    lds_t<Tc> *const sA1 = s0 + LoadA::ELEMS;
    const int64_t k_begin = s_begin * BK;
    la.fetch_k(t.offAk, k_begin, K);
    lb.fetch_k(t.offBk, k_begin, K);
    la.template load<true>(A, k_begin, K);
    lb.dma(B, sB0);
    la.fetch_k(t.offAk, k_begin + BK, K);
    lb.fetch_k(t.offBk, k_begin + BK, K);
    la.store(s0);
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vector-memory counter at zero: B landed
    __syncthreads();
    // step `step` from (sAc, sBc); step + 1 into (sAn, sBn)
    auto half = [&](int64_t step, const lds_t<Tc> *sAc, lds_t<Tc> *sAn, const lds_t<Tc> *sBc, lds_t<Tc> *sBn) {
      la.template load<true>(A, (step + 1) * BK, K);
      lb.dma(B, sBn);
      la.fetch_k(t.offAk, (step + 2) * BK, K);
      lb.fetch_k(t.offBk, (step + 2) * BK, K);
      // every load of the step issued before the products (the direct-to-LDS
      // ones have no users, and the scheduler would sink them to the wait)
      __builtin_amdgcn_sched_barrier(0);
      gett_mma_step<LoadA, LoadB, BK>(w, sAc, sBc, lane, wm0, wn0);
      la.store(sAn);
      __builtin_amdgcn_s_waitcnt(0x0F70);
      __syncthreads();
    };
    int64_t step = s_begin;
    for (; step + 1 < s_end; step += 2) {
      half(step, sA0, sA1, sB0, sB1);
      half(step + 1, sA1, const_cast<lds_t<Tc> *>(sA0), sB1, sB0);
    }
    if (step < s_end) half(step, sA0, sA1, sB0, sB1);
    return;
  }

  // Software pipeline, uniform across steps: the last step also issues a
  // (masked, clamped-address) load of the step past the end, so the loop body
  // has no branches.
  const int64_t k_begin = s_begin * BK;
  la.fetch_k(t.offAk, k_begin, K);
  lb.fetch_k(t.offBk, k_begin, K);
  la.template load<FULL>(A, k_begin, K);
  lb.template load<FULL>(B, k_begin, K);
  la.fetch_k(t.offAk, k_begin + BK, K);
  lb.fetch_k(t.offBk, k_begin + BK, K);
  la.store(sA[0]);
  lb.store(sB[0]);
  __syncthreads();
  for (int64_t step = s_begin; step < s_end; ++step) {
    const int cur = int((step - s_begin) & 1);
    la.template load<FULL>(A, (step + 1) * BK, K);
    lb.template load<FULL>(B, (step + 1) * BK, K);
    la.fetch_k(t.offAk, (step + 2) * BK, K);
    lb.fetch_k(t.offBk, (step + 2) * BK, K);
    gett_mma_step<LoadA, LoadB, BK>(w, sA[cur], sB[cur], lane, wm0, wn0);
    la.store(sA[cur ^ 1]);
    lb.store(sB[cur ^ 1]);
    __syncthreads();
  }
}

// Epilogue of one tile from its C offsets in LDS: cm[r] = offCm[m0 + r],
// cn[c] = offCn[n0 + c], entries past M or N holding the last row's or
// column's offset (their writes are masked).  C[cm + cn] = alpha * acc +
// beta * C for this thread's accumulator elements, in groups of four.  On
// CDNA loads and stores share one in-order completion counter, so a load
// placed after a store cannot be waited for without waiting for that store
// too: the offsets come from LDS (a counter of their own), and with
// beta != 0 the C values of the next group are requested before the current
// group is stored, so that every wait is for loads issued ahead of the
// stores still in flight.  C is written with nontemporal stores: the kernel
// never reads it back, and streaming it past the caches made the
// store-bound K = 32 triples contraction 10% faster on MI355X.
//
// With SINK, an element outside the output is stored to *sink (a
// dummy location) instead of being skipped, so every lane issues every
// store: the number of stores in flight is then the same on every path, and
// the compiler can wait for loads issued before them without waiting for the
// stores themselves (a skipped store makes that count unknown, and every
// later wait a full one).
template <typename Tin, typename Tc, int BM, int BN, int WGM, int WGN, bool SINK = false>
__device__ __forceinline__ void gett_store_staged(const WaveTile<Tc, BM, BN, WGM, WGN> &w, Tin *__restrict__ C,
                                                  const lds_t<int64_t> *cm, const lds_t<int64_t> *cn, int64_t M,
                                                  int64_t N, double alpha, double beta, int64_t m0, int64_t n0,
                                                  Tin *sink = nullptr) {
  typedef WaveTile<Tc, BM, BN, WGM, WGN> WT;
  typedef typename std::conditional<(sizeof(Tin) == 8 || sizeof(Tc) == 8), double, float>::type Te;
  constexpr int G = WT::FN * WT::FM;   // groups of four elements: (j, i)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm0 = (wave / WGN) * WT::WM, wn0 = (wave % WGN) * WT::WN;
  const Te al = Te(alpha), be = Te(beta);
  glb_t<Tin> *const gC = to_glb(C);
  auto ml = [&](int i, int r) { return wm0 + i * 16 + acc_row<Tc>(lane, r); };
  auto nl = [&](int j) { return wn0 + j * 16 + (lane & 15); };
  auto addr = [&](int i, int r, int j) { return int64_t(cm[ml(i, r)]) + int64_t(cn[nl(j)]); };
  auto inside = [&](int i, int r, int j) { return m0 + ml(i, r) < M && n0 + nl(j) < N; };
  if (beta == 0.0) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int j = g / WT::FM, i = g % WT::FM;
      // the group's offsets first (in-bounds reads), then the masked stores
      int64_t a[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = addr(i, r, j);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if constexpr (SINK)
          __builtin_nontemporal_store(Tin(al * Te(w.acc[i][j][r])), inside(i, r, j) ? &gC[a[r]] : to_glb(sink));
        else if (inside(i, r, j))
          __builtin_nontemporal_store(Tin(al * Te(w.acc[i][j][r])), &gC[a[r]]);
      }
    }
    return;
  }
  // the look-ahead costs registers; tiles whose accumulators already take
  // more than 64 VGPRs load and store one group at a time
  constexpr bool ahead = WT::FM * WT::FN * 4 * int(sizeof(Tc)) <= 64 * 4;
  Tin cv[2][4];
  if (ahead) {
#pragma unroll
    for (int r = 0; r < 4; ++r) cv[0][r] = gC[addr(0, r, 0)];
  }
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int j = g / WT::FM, i = g % WT::FM;
    __builtin_amdgcn_sched_barrier(0);
    if (ahead && g + 1 < G) {
      const int j1 = (g + 1) / WT::FM, i1 = (g + 1) % WT::FM;
#pragma unroll
      for (int r = 0; r < 4; ++r) cv[(g + 1) & 1][r] = gC[addr(i1, r, j1)];
    }
    if (!ahead) {
#pragma unroll
      for (int r = 0; r < 4; ++r) cv[g & 1][r] = gC[addr(i, r, j)];
    }
    int64_t a[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = addr(i, r, j);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const Tin v = Tin(al * Te(w.acc[i][j][r]) + be * Te(cv[g & 1][r]));
      if constexpr (SINK)
        __builtin_nontemporal_store(v, inside(i, r, j) ? &gC[a[r]] : to_glb(sink));
      else if (inside(i, r, j))
        __builtin_nontemporal_store(v, &gC[a[r]]);
    }
  }
}

// The same result one element at a time (offsets from LDS, each C value
// read just before its store).  The persistent kernel uses this form: there
// the grouped form above, whose code sits inside the kernel's tile loop, made
// the whole loop slower (measured on a K = 32 contraction).
template <typename Tin, typename Tc, int BM, int BN, int WGM, int WGN>
__device__ __forceinline__ void gett_store_staged_serial(const WaveTile<Tc, BM, BN, WGM, WGN> &w,
                                                         Tin *__restrict__ C, const lds_t<int64_t> *cm,
                                                         const lds_t<int64_t> *cn, int64_t M, int64_t N, double alpha,
                                                         double beta, int64_t m0, int64_t n0) {
  typedef WaveTile<Tc, BM, BN, WGM, WGN> WT;
  typedef typename std::conditional<(sizeof(Tin) == 8 || sizeof(Tc) == 8), double, float>::type Te;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm0 = (wave / WGN) * WT::WM, wn0 = (wave % WGN) * WT::WN;
  const Te al = Te(alpha), be = Te(beta);
  const bool read_c = beta != 0.0;
  glb_t<Tin> *const gC = to_glb(C);
#pragma unroll
  for (int j = 0; j < WT::FN; ++j) {
    const int nl = wn0 + j * 16 + (lane & 15);
    if (n0 + nl >= N) continue;
    const int64_t cnv = cn[nl];
#pragma unroll
    for (int i = 0; i < WT::FM; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ml = wm0 + i * 16 + acc_row<Tc>(lane, r);
        if (m0 + ml >= M) continue;
        const int64_t addr = cm[ml] + cnv;
        Te v = al * Te(w.acc[i][j][r]);
        if (read_c) v = v + be * Te(gC[addr]);
        __builtin_nontemporal_store(Tin(v), &gC[addr]);
      }
    }
  }
}

// C = alpha * acc + beta * C for the tile at (m0, n0) through the C tables,
// in double for double storage or double accumulation, in float otherwise.
// The tile's C offsets are first staged in `smem` (the tile's LDS, free once
// the main loop has passed its last barrier); the caller must pass a barrier
// before it writes smem again.
template <typename Tin, typename Tc, int BM, int BN, int WGM, int WGN>
__device__ __forceinline__ void gett_store(const WaveTile<Tc, BM, BN, WGM, WGN> &w, Tin *__restrict__ C,
                                           const GettTables &t, int64_t M, int64_t N, double alpha, double beta,
                                           int64_t m0, int64_t n0, Tc *smem) {
  constexpr int NT = 64 * WGM * WGN;
  lds_t<int64_t> *const tab = to_lds(reinterpret_cast<int64_t *>(smem));
  const glb_t<const int64_t> *const offCm = to_glb(t.offCm);
  const glb_t<const int64_t> *const offCn = to_glb(t.offCn);
  for (int x = threadIdx.x; x < BM + BN; x += NT) {
    int64_t v;
    if (x < BM)
      v = offCm[m0 + x < M ? m0 + x : M - 1];
    else
      v = offCn[n0 + (x - BM) < N ? n0 + (x - BM) : N - 1];
    tab[x] = v;
  }
  __syncthreads();
  gett_store_staged<Tin, Tc, BM, BN, WGM, WGN>(w, C, tab, tab + BM, M, N, alpha, beta, m0, n0);
}

// C = alpha * v + beta * C for accumulator element (i, j) of this thread
// only (the same outputs gett_store writes from w.acc[i][j]).
template <typename Tin, typename Tc, int BM, int BN, int WGM, int WGN>
__device__ __forceinline__ void gett_store_fragment(const typename AccT<Tc>::type &v, int i, int j,
                                                    Tin *__restrict__ C, const GettTables &t, int64_t M, int64_t N,
                                                    double alpha, double beta, int64_t m0, int64_t n0) {
  typedef WaveTile<Tc, BM, BN, WGM, WGN> WT;
  typedef typename std::conditional<(sizeof(Tin) == 8 || sizeof(Tc) == 8), double, float>::type Te;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm0 = (wave / WGN) * WT::WM, wn0 = (wave % WGN) * WT::WN;
  const int64_t n = n0 + wn0 + j * 16 + (lane & 15);
  if (n >= N) return;
  glb_t<Tin> *const gC = to_glb(C);
  const int64_t cn = to_glb(t.offCn)[n];
  const glb_t<const int64_t> *const offCm = to_glb(t.offCm);
  const Te al = Te(alpha), be = Te(beta);
  // all offsets, then all C values, then the stores (see gett_epilogue)
  int64_t addr[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t m = m0 + wm0 + i * 16 + acc_row<Tc>(lane, r);
    addr[r] = offCm[m < M ? m : M - 1] + cn;
  }
  Te x[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) x[r] = beta != 0.0 ? be * Te(gC[addr[r]]) : Te(0);
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (m0 + wm0 + i * 16 + acc_row<Tc>(lane, r) < M) __builtin_nontemporal_store(Tin(al * Te(v[r]) + x[r]), &gC[addr[r]]);
}

// A partial sum of one tile in workspace: accumulator element (i, j) of
// thread tid at ((i * FN + j) * NT + tid), one 4-vector each, so that the
// writes of a wave are contiguous.
template <typename Tc, int BM, int BN, int WGM, int WGN>
__device__ __forceinline__ void gett_store_partial(const WaveTile<Tc, BM, BN, WGM, WGN> &w,
                                                   typename AccT<Tc>::type *__restrict__ slot) {
  typedef WaveTile<Tc, BM, BN, WGM, WGN> WT;
  glb_t<typename WT::acc_t> *const g = to_glb(slot);
#pragma unroll
  for (int i = 0; i < WT::FM; ++i)
#pragma unroll
    for (int j = 0; j < WT::FN; ++j) g[(i * WT::FN + j) * WT::NT + threadIdx.x] = w.acc[i][j];
}

// One BM x BN output tile at (m0, n0) over the whole summation range.
template <typename Tin, typename Tc, int BM, int BN, int BK, int WGM, int WGN, int LA, int LB, bool VA, bool VB,
          bool FULL = false>
__device__ __forceinline__ void gett_tile(const Tin *__restrict__ A, const Tin *__restrict__ B, Tin *__restrict__ C,
                                          const GettTables &t, int64_t M, int64_t N, int64_t K, double alpha,
                                          double beta, int64_t m0, int64_t n0, Tc *smem) {
  static_assert(8 * (BM + BN) <=
                    int(sizeof(Tc)) * gett_lds_elems<Tin, Tc, BM, BN, BK, 64 * WGM * WGN, LA, LB, VA, VB, FULL>(),
                "the tile's C offsets fit in its LDS");
  WaveTile<Tc, BM, BN, WGM, WGN> w;
  gett_accumulate<Tin, Tc, BM, BN, BK, WGM, WGN, LA, LB, VA, VB, FULL>(w, A, B, t, M, N, K, m0, n0, 0,
                                                                       (K + BK - 1) / BK, smem);
  gett_store<Tin, Tc, BM, BN, WGM, WGN>(w, C, t, M, N, alpha, beta, m0, n0, smem);
}


}  // namespace gather
}  // namespace comet
