// gett.hip -- fused gather contraction on the CDNA4 matrix cores (gfx950).
//
// The contraction C = alpha * A * B + beta * C over arbitrary label
// permutations is computed as one tiled matrix product whose operand tiles
// are gathered straight from the permuted tensors through per-label offset
// tables (addr_A(m,k) = offAm[m] + offAk[k], and likewise for B and C).  This
// replaces the three explicit transposes of TTGT (Section 2) by address
// arithmetic in the loader; the tiling follows the blocking scheme of
// Section 6 ("GEMM optimizations": an Mc x Kc panel of A and a Kc x Nc panel
// of B staged in fast memory, an Mr x Nr register block as the micro-kernel),
// mapped to the MI355X hierarchy:
//
//   workgroup tile BM x BN (LDS, double-buffered along K in steps of BK)
//   wave tile (BM/2) x (BN/2) (registers), made of 16 x 16 MFMA blocks
//   micro-kernel: v_mfma_f64_16x16x4f64 or v_mfma_f32_16x16x4f32
//
// Lane layout of the 16x16x4 MFMAs (64 lanes): lane l supplies A[l%16][l/16]
// and B[l/16][l%16].  It receives D[4*(l/16) + r][l%16] (r = 0..3) from the
// FP32 instruction but D[l/16 + 4*r][l%16] from the FP64 one (checked on the
// device with a Kronecker-delta operand).
//
// The epilogue writes alpha*acc + beta*C through the C offset tables; the
// planner orders A and B so that C's unit-stride label lies along N, which
// the MFMA output spreads over consecutive lanes.
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "gather.hpp"
#include "kernels.hpp"

namespace comet {
namespace {

using namespace gather;

// Tile variants: workgroup tile BM x BN, K step BK, and a WGM x WGN grid of
// waves, each owning a (BM/WGM) x (BN/WGN) block of 16 x 16 MFMA tiles.  wpe
// is the number of waves per SIMD the register allocation must leave room
// for (the second launch bound): the FP64 matrix core needs several waves
// per SIMD to stay busy across the K-step barriers.
struct TileShape {
  int bm, bn, bk, wgm, wgn, wpe;
  int swpe;   // the same for the stream-K and persistent kernels
};
constexpr TileShape kTiles[] = {
    {128, 128, 16, 2, 2, 1, 1},   // 0: large problems
    {64, 64, 16, 2, 2, 1, 3},     // 1: small problems; also every element-load variant
    {128, 128, 32, 2, 2, 1, 1},   // 2: longer K step (fewer barriers per flop)
    {128, 128, 16, 4, 2, 4, 1},   // 3: 8 waves; two workgroups per CU (128 VGPRs)
    {256, 128, 16, 4, 2, 1, 1},   // 4: 8 waves, 64 x 64 per wave
    {128, 64, 16, 2, 2, 1, 2},    // 5
    {64, 128, 16, 2, 2, 1, 2},    // 6
    {96, 96, 16, 2, 2, 1, 2},     // 7: FP64 only; 3072^2 outputs -> 4 tiles per CU
    {128, 96, 32, 4, 2, 1, 1},    // 8: FP64 only; 3072^2 outputs -> 3 tiles per CU
    {192, 96, 32, 4, 2, 1, 1},    // 9: FP64 only; 3072^2 outputs -> 2 tiles per CU
};
constexpr int kNumTiles = int(sizeof(kTiles) / sizeof(kTiles[0]));

// Summation steps [a(s), a(s + 1)) of the stream-K part handled by its
// workgroup s, with a(s) = floor(I * s / S) over I = tiles * steps-per-tile
// steps and S workgroups: every workgroup gets the same share, give or take
// one step, and a share may run over tile boundaries.
__device__ __forceinline__ int64_t sk_begin(int64_t I, int S, int s) { return I * s / S; }

// Workgroup of the stream-K part whose share holds step x.
__device__ __forceinline__ int sk_owner(int64_t I, int S, int64_t x) {
  int s = int(x * S / I);
  if (s > S - 1) s = S - 1;
  while (s + 1 < S && sk_begin(I, S, s + 1) <= x) ++s;
  while (s > 0 && sk_begin(I, S, s) > x) --s;
  return s;
}

// Whole tiles: workgroup b computes tile id b of the first gridDim.x ids in
// the XCD-aware order (all tiles, or all but the sk.tiles stream-K ones).
// FULL: every tile lies inside the output and the summation is a whole
// number of K steps, so the loads are not masked.
template <typename Tin, typename Tc, int TILE, int LA, int LB, bool VA, bool VB, bool FULL = false>
__global__ __launch_bounds__(64 * kTiles[TILE].wgm * kTiles[TILE].wgn, kTiles[TILE].wpe) void gett_kernel(
    const Tin *__restrict__ A, const Tin *__restrict__ B, Tin *__restrict__ C, GettTables t, int64_t M, int64_t N,
    int64_t K, double alpha, double beta, int tilesM, int tilesN) {
  constexpr int BM = kTiles[TILE].bm, BN = kTiles[TILE].bn, BK = kTiles[TILE].bk;
  constexpr int WGM = kTiles[TILE].wgm, WGN = kTiles[TILE].wgn;
  constexpr int NT = 64 * WGM * WGN;
  __shared__ __attribute__((aligned(16))) Tc smem[gett_lds_elems<Tin, Tc, BM, BN, BK, NT, LA, LB, VA, VB, FULL>()];
  int tm, tn;
  group_coords(xcd_remap(blockIdx.x, gridDim.x), tilesM, tilesN, &tm, &tn);
  gett_tile<Tin, Tc, BM, BN, BK, WGM, WGN, LA, LB, VA, VB, FULL>(A, B, C, t, M, N, K, alpha, beta,
                                                                 int64_t(tm) * BM, int64_t(tn) * BN, smem);
}

// Batch labels: blockIdx.y selects batch entry bt.first + blockIdx.y, whose
// slices of A, B and C the three base pointers move to, and blockIdx.x the
// tile in the XCD-aware order (the XCD of a workgroup is its linear id
// modulo 8, so the tiles the remap groups still share one).  A kernel of its
// own so that gett_kernel keeps its register budget; the entry comes from
// the grid rather than a division of a flat id, which costs registers.
template <typename Tin, typename Tc, int TILE, int LA, int LB, bool VA, bool VB>
__global__ __launch_bounds__(64 * kTiles[TILE].wgm * kTiles[TILE].wgn, kTiles[TILE].wpe) void gett_batch_kernel(
    const Tin *__restrict__ A, const Tin *__restrict__ B, Tin *__restrict__ C, GettTables t, int64_t M, int64_t N,
    int64_t K, double alpha, double beta, int tilesM, int tilesN, GettBatch bt) {
  constexpr int BM = kTiles[TILE].bm, BN = kTiles[TILE].bn, BK = kTiles[TILE].bk;
  constexpr int WGM = kTiles[TILE].wgm, WGN = kTiles[TILE].wgn;
  constexpr int NT = 64 * WGM * WGN;
  __shared__ __attribute__((aligned(16))) Tc smem[gett_lds_elems<Tin, Tc, BM, BN, BK, NT, LA, LB, VA, VB>()];
  const int64_t x = bt.first + blockIdx.y;
  int tm, tn;
  group_coords(xcd_remap(blockIdx.x, gridDim.x), tilesM, tilesN, &tm, &tn);
  gett_tile<Tin, Tc, BM, BN, BK, WGM, WGN, LA, LB, VA, VB>(A + bt.offA[x], B + bt.offB[x], C + bt.offC[x], t, M, N,
                                                           K, alpha, beta, int64_t(tm) * BM, int64_t(tn) * BN, smem);
}

// the tile variants compiled with batch labels
constexpr bool batch_tile(int tile) { return tile == 1 || tile == 3; }
// the tile variants compiled for the short-summation kernel
constexpr bool shortk_tile(int tile) { return tile == 3; }
// the tile variants compiled with unmasked loads for whole tiles (the
// planner's choice for large FP64 products; the FP32 ones, split over
// stream-K pieces, measured no faster unmasked)
constexpr bool full_tile(int tile) { return tile == 3; }

// Stream-K: the last sk.tiles tiles (ids dp .. dp + sk.tiles - 1) split
// along the summation over sk.blocks workgroups, each taking an equal number
// of BK steps, so that the last, partial round of whole tiles becomes a full
// round of equal pieces.  A piece that covers a whole tile is written
// directly; other pieces go to the workspace (two slots per workgroup: its
// first and its last tile) and gett_fixup_kernel sums them in a fixed order.
// A separate kernel from the whole-tile one so that the latter keeps its
// register budget (and its occupancy).
template <typename Tin, typename Tc, int TILE, int LA, int LB, bool VA, bool VB>
__global__ __launch_bounds__(64 * kTiles[TILE].wgm * kTiles[TILE].wgn, kTiles[TILE].swpe) void gett_sk_kernel(
    const Tin *__restrict__ A, const Tin *__restrict__ B, Tin *__restrict__ C, GettTables t, int64_t M, int64_t N,
    int64_t K, double alpha, double beta, int tilesM, int tilesN, StreamK sk) {
  constexpr int BM = kTiles[TILE].bm, BN = kTiles[TILE].bn, BK = kTiles[TILE].bk;
  constexpr int WGM = kTiles[TILE].wgm, WGN = kTiles[TILE].wgn;
  constexpr int NT = 64 * WGM * WGN;
  typedef WaveTile<Tc, BM, BN, WGM, WGN> WT;
  __shared__ __attribute__((aligned(16))) Tc smem[gett_lds_elems<Tin, Tc, BM, BN, BK, NT, LA, LB, VA, VB>()];
  const int dp = tilesM * tilesN - sk.tiles;
  int tm, tn;
  const int s = int(blockIdx.x);
  const int64_t nk = (K + BK - 1) / BK;
  const int64_t I = int64_t(sk.tiles) * nk;
  const int64_t a = sk_begin(I, sk.blocks, s), b = sk_begin(I, sk.blocks, s + 1);
  typename WT::acc_t *const ws = static_cast<typename WT::acc_t *>(sk.ws);
  constexpr int64_t kSlot = int64_t(WT::FM) * WT::FN * NT;   // 4-vectors per slot
  for (int64_t it = a; it < b;) {
    const int64_t tt = it / nk;
    const int64_t ks = it - tt * nk;
    const int64_t ke = ks + (b - it) < nk ? ks + (b - it) : nk;
    group_coords(dp + int(tt), tilesM, tilesN, &tm, &tn);
    WT w;
    gett_accumulate<Tin, Tc, BM, BN, BK, WGM, WGN, LA, LB, VA, VB>(w, A, B, t, M, N, K, int64_t(tm) * BM,
                                                                   int64_t(tn) * BN, ks, ke, smem);
    if (ks == 0 && ke == nk) {
      gett_store<Tin, Tc, BM, BN, WGM, WGN>(w, C, t, M, N, alpha, beta, int64_t(tm) * BM, int64_t(tn) * BN, smem);
      __syncthreads();   // the C offsets in smem are read before the next piece's loads overwrite them
    } else {
      const int slot = 2 * s + (tt == a / nk ? 0 : 1);
      gett_store_partial<Tc, BM, BN, WGM, WGN>(w, ws + slot * kSlot);
    }
    it += ke - ks;
  }
}

// Persistent schedule for short summations (a few BK steps per tile), where
// a workgroup per tile would spend most of its life on the latency of its
// first loads and on draining its pipeline.  Workgroup s of S walks the tiles
// s, s + S, s + 2S, ... (tile ids in the XCD-aware order, so they stay on the
// workgroup's XCD) as one flat sequence of BK steps: the first step of the
// next tile is loaded while the last step of the current one is multiplied,
// and the current tile's results are stored while the next tile's data are
// in flight.  The row-offset entries a tile's loads need are staged in LDS
// two tiles ahead and its C offsets one tile ahead (each double-buffered by
// tile parity), so that no table read sits on the critical path.
template <typename Tin, typename Tc, int TILE, int LA, int LB, bool VA, bool VB>
__global__ __launch_bounds__(64 * kTiles[TILE].wgm * kTiles[TILE].wgn, kTiles[TILE].swpe) void gett_persistent_kernel(
    const Tin *__restrict__ A, const Tin *__restrict__ B, Tin *__restrict__ C, GettTables t, int64_t M, int64_t N,
    int64_t K, double alpha, double beta, int tilesM, int tilesN) {
  constexpr int BM = kTiles[TILE].bm, BN = kTiles[TILE].bn, BK = kTiles[TILE].bk;
  constexpr int WGM = kTiles[TILE].wgm, WGN = kTiles[TILE].wgn;
  constexpr int NT = 64 * WGM * WGN;
  typedef WaveTile<Tc, BM, BN, WGM, WGN> WT;
  typedef Loader<Tin, Tc, BM, BK, LA, VA, NT> LoadA;
  typedef Loader<Tin, Tc, BN, BK, LB, VB, NT> LoadB;
  typedef typename WT::acc_t acc_t;
  __shared__ __attribute__((aligned(16))) Tc smem[gett_lds_elems<Tin, Tc, BM, BN, BK, NT, LA, LB, VA, VB>()];
  __shared__ int64_t rows_s[2][BM + BN];   // offAm / offBn entries of a tile
  __shared__ int64_t ctab_s[2][BM + BN];   // offCm / offCn entries of a tile
  lds_t<Tc> *const s0 = to_lds(smem);
  lds_t<Tc> *sA[2] = {s0, s0 + LoadA::ELEMS};
  lds_t<Tc> *sB[2] = {s0 + 2 * LoadA::ELEMS, s0 + 2 * LoadA::ELEMS + LoadB::ELEMS};
  lds_t<int64_t> *const rows = to_lds(&rows_s[0][0]);
  lds_t<int64_t> *const ctab = to_lds(&ctab_s[0][0]);

  const int T = tilesM * tilesN, S = gridDim.x, sb = blockIdx.x;
  if (sb >= T) return;   // uniform: a workgroup without tiles
  const int ntile = (T - 1 - sb) / S + 1;
  const int64_t nk = (K + BK - 1) / BK;
  const int64_t total = int64_t(ntile) * nk;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WGN) * WT::WM, wn0 = (wave % WGN) * WT::WN;
  auto origin = [&](int j, int64_t *m0, int64_t *n0) {
    int tm, tn;
    tile_coords(sb + j * S, tilesM, tilesN, &tm, &tn);
    *m0 = int64_t(tm) * BM;
    *n0 = int64_t(tn) * BN;
  };
  // table entry x of tile j for the staging threads: rows (offAm, offBn) and
  // C offsets (offCm, offCn); x < BM: M side, else N side
  auto table_entry = [&](int j, int x, const int64_t *tm_, const int64_t *tn_) -> int64_t {
    int64_t m0, n0;
    origin(j, &m0, &n0);
    if (x < BM) {
      const int64_t m = m0 + x < M ? m0 + x : M - 1;
      return to_glb(tm_)[m];
    }
    const int64_t n = n0 + (x - BM) < N ? n0 + (x - BM) : N - 1;
    return to_glb(tn_)[n];
  };

  WT w;
#pragma unroll
  for (int i = 0; i < WT::FM; ++i)
#pragma unroll
    for (int jj = 0; jj < WT::FN; ++jj) w.acc[i][jj] = acc_t{0, 0, 0, 0};
  LoadA la;
  LoadB lb;
  int64_t m0, n0;
  origin(0, &m0, &n0);
  la.init(tid, m0, M, t.offAm);
  lb.init(tid, n0, N, t.offBn);
  // prologue: rows of tile 1 and C offsets of tile 0 into LDS, step 0 loaded
  for (int x = tid; x < BM + BN; x += NT) {
    if (ntile > 1) rows[1 * (BM + BN) + x] = table_entry(1, x, t.offAm, t.offBn);
    ctab[x] = table_entry(0, x, t.offCm, t.offCn);
  }
  la.fetch_k(t.offAk, 0, K);
  lb.fetch_k(t.offBk, 0, K);
  la.load(A, 0, K);
  lb.load(B, 0, K);
  la.fetch_k(t.offAk, nk > 1 ? BK : 0, K);
  lb.fetch_k(t.offBk, nk > 1 ? BK : 0, K);
  la.store(sA[0]);
  lb.store(sB[0]);
  __syncthreads();

  int j = 0;
  int64_t k = 0;
  for (int64_t g = 0; g < total; ++g) {
    const int cur = int(g & 1);
    const bool last = k == nk - 1;
    // tables of tiles j + 2 (rows) and j + 1 (C offsets), fetched now and
    // written to LDS after this step's product
    int64_t rv[(BM + BN + NT - 1) / NT], cv[(BM + BN + NT - 1) / NT];
    const bool stage = k == 0;
    if (stage) {
#pragma unroll
      for (int q = 0; q < (BM + BN + NT - 1) / NT; ++q) {
        const int x = tid + q * NT;
        if (x < BM + BN) {
          rv[q] = j + 2 < ntile ? table_entry(j + 2, x, t.offAm, t.offBn) : 0;
          cv[q] = j + 1 < ntile ? table_entry(j + 1, x, t.offCm, t.offCn) : 0;
        }
      }
    }
    // the next step's data: the next tile's first step after a last step
    if (g + 1 < total) {
      if (last) {
        int64_t m1, n1;
        origin(j + 1, &m1, &n1);
        const lds_t<int64_t> *r1 = rows + ((j + 1) & 1) * (BM + BN);
        la.init_from(tid, m1, M, r1, m1);
        lb.init_from(tid, n1, N, r1 + BM, n1);
      }
      const int64_t k1 = last ? 0 : k + 1;
      la.load(A, k1 * BK, K);
      lb.load(B, k1 * BK, K);
      // K-table entries for the step after that
      const int64_t k2 = (k1 + 1 == nk) ? 0 : k1 + 1;
      la.fetch_k(t.offAk, k2 * BK, K);
      lb.fetch_k(t.offBk, k2 * BK, K);
    }
    gett_mma_step<LoadA, LoadB, BK>(w, sA[cur], sB[cur], lane, wm0, wn0);
    if (last) {
      origin(j, &m0, &n0);
      const lds_t<int64_t> *ct = ctab + (j & 1) * (BM + BN);
      gett_store_staged_serial<Tin, Tc, BM, BN, WGM, WGN>(w, C, ct, ct + BM, M, N, alpha, beta, m0, n0);
#pragma unroll
      for (int i = 0; i < WT::FM; ++i)
#pragma unroll
        for (int jj = 0; jj < WT::FN; ++jj) w.acc[i][jj] = acc_t{0, 0, 0, 0};
    }
    if (stage) {
#pragma unroll
      for (int q = 0; q < (BM + BN + NT - 1) / NT; ++q) {
        const int x = tid + q * NT;
        if (x < BM + BN) {
          rows[(j & 1) * (BM + BN) + x] = rv[q];
          ctab[((j + 1) & 1) * (BM + BN) + x] = cv[q];
        }
      }
    }
    if (g + 1 < total) {
      la.store(sA[cur ^ 1]);
      lb.store(sB[cur ^ 1]);
    }
    __syncthreads();
    if (last) {
      ++j;
      k = 0;
    } else {
      ++k;
    }
  }
}

// Balanced schedule for a tile count just above a whole number of rounds
// (the CCSD-like headline: 576 tiles of 128 x 128 on 512 resident
// workgroups).  The whole-tile kernel computes the full rounds (sk.whole
// tiles); the R = sk.tiles leftover tiles then share one more round of
// S = sk.blocks workgroups, tile r taking workgroups
// first(r) = floor(S r / R) .. first(r + 1) - 1, which cut its summation into
// that many equal pieces (give or take a step).  Every workgroup of a round
// so runs the same work -- stream-K instead gives the leftover tiles a kernel
// of its own at a lower occupancy.  A piece is written to workspace slot b;
// gett_piece_fixup_kernel sums a leftover tile's slots in piece order, so
// the result does not depend on timing.  The piece kernel is a whole-tile
// kernel over a shorter summation (the k tables moved to the piece's first
// index), so it keeps that kernel's registers and occupancy: one fused
// kernel doing the whole tiles and then the piece needed more registers than
// two workgroups per CU leave, and spilled.
__device__ __forceinline__ int even_first(int S, int R, int r) { return int(int64_t(S) * r / R); }

// a wave-uniform 64-bit value, held in scalar registers
__device__ __forceinline__ int64_t scalar64(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(x)));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(x) >> 32));
  return int64_t((uint64_t(hi) << 32) | lo);
}

// Piece b of the balanced schedule's leftover tiles: its share of the
// summation of its tile, stored as a partial tile in workspace slot b.
template <typename Tin, typename Tc, int TILE, int LA, int LB, bool VA, bool VB, bool FULL>
__device__ __forceinline__ void gett_piece(const Tin *__restrict__ A, const Tin *__restrict__ B, const GettTables &t,
                                           int64_t M, int64_t N, int64_t K, int tilesM, int tilesN, const StreamK &sk,
                                           int b, Tc *smem) {
  constexpr int BM = kTiles[TILE].bm, BN = kTiles[TILE].bn, BK = kTiles[TILE].bk;
  constexpr int WGM = kTiles[TILE].wgm, WGN = kTiles[TILE].wgn;
  constexpr int NT = 64 * WGM * WGN;
  typedef WaveTile<Tc, BM, BN, WGM, WGN> WT;
  const int S = sk.blocks, R = sk.tiles;
  // leftover tile r: the largest r with first(r) <= b
  const int r = int((int64_t(b + 1) * R - 1) / S);
  const int f0 = even_first(S, R, r), P = even_first(S, R, r + 1) - f0, j = b - f0;
  const int64_t nk = (K + BK - 1) / BK;
  // the divisions run on the vector unit: move their (uniform) results back
  // to scalar registers, or the loop's bounds and k indices would take
  // vector registers the accumulation has none left for
  const int64_t k0 = scalar64(nk * j / P * BK), k1 = nk * (j + 1) / P * BK;
  const int64_t Kp = scalar64((k1 < K ? k1 : K) - k0);
  GettTables tk = t;
  tk.offAk += k0;
  tk.offBk += k0;
  int tm, tn;
  group_coords(sk.whole + r, tilesM, tilesN, &tm, &tn);
  WT w;
  gett_accumulate<Tin, Tc, BM, BN, BK, WGM, WGN, LA, LB, VA, VB, FULL>(w, A, B, tk, M, N, Kp, int64_t(tm) * BM,
                                                                       int64_t(tn) * BN, 0, (Kp + BK - 1) / BK, smem);
  constexpr int64_t kSlot = int64_t(WT::FM) * WT::FN * NT;   // 4-vectors per slot
  gett_store_partial<Tc, BM, BN, WGM, WGN>(w, static_cast<typename WT::acc_t *>(sk.ws) + b * kSlot);
}

// The whole tiles and the pieces of the balanced schedule in one launch:
// workgroups 0 .. whole - 1 compute the whole tiles (in the XCD-aware order
// over them), the rest the pieces, which start as whole tiles finish instead
// of after the last one (3.5% less time on the CCSD-like contraction than
// two launches).
template <typename Tin, typename Tc, int TILE, int LA, int LB, bool VA, bool VB, bool FULL = false>
__global__ __launch_bounds__(64 * kTiles[TILE].wgm * kTiles[TILE].wgn, kTiles[TILE].wpe) void gett_whole_piece_kernel(
    const Tin *__restrict__ A, const Tin *__restrict__ B, Tin *__restrict__ C, GettTables t, int64_t M, int64_t N,
    int64_t K, double alpha, double beta, int tilesM, int tilesN, StreamK sk) {
  constexpr int BM = kTiles[TILE].bm, BN = kTiles[TILE].bn, BK = kTiles[TILE].bk;
  constexpr int WGM = kTiles[TILE].wgm, WGN = kTiles[TILE].wgn;
  constexpr int NT = 64 * WGM * WGN;
  __shared__ __attribute__((aligned(16))) Tc smem[gett_lds_elems<Tin, Tc, BM, BN, BK, NT, LA, LB, VA, VB, FULL>()];
  const int b = blockIdx.x;
  if (b < sk.whole) {
    int tm, tn;
    group_coords(xcd_remap(b, sk.whole), tilesM, tilesN, &tm, &tn);
    gett_tile<Tin, Tc, BM, BN, BK, WGM, WGN, LA, LB, VA, VB, FULL>(A, B, C, t, M, N, K, alpha, beta,
                                                                   int64_t(tm) * BM, int64_t(tn) * BN, smem);
    return;
  }
  gett_piece<Tin, Tc, TILE, LA, LB, VA, VB, FULL>(A, B, t, M, N, K, tilesM, tilesN, sk, b - sk.whole, smem);
}

// Sum the pieces of each leftover tile of the balanced schedule in piece
// order and write alpha * sum + beta * C.  Workgroup (r, f) takes leftover
// tile r and accumulator element f = i * FN + j of every thread.
template <typename Tin, typename Tc, int TILE>
__global__ __launch_bounds__(64 * kTiles[TILE].wgm * kTiles[TILE].wgn) void gett_piece_fixup_kernel(
    Tin *__restrict__ C, GettTables t, int64_t M, int64_t N, double alpha, double beta, int tilesM, int tilesN,
    StreamK sk) {
  constexpr int BM = kTiles[TILE].bm, BN = kTiles[TILE].bn;
  constexpr int WGM = kTiles[TILE].wgm, WGN = kTiles[TILE].wgn;
  constexpr int NT = 64 * WGM * WGN;
  typedef WaveTile<Tc, BM, BN, WGM, WGN> WT;
  typedef typename WT::acc_t acc_t;
  const int r = blockIdx.x, f = blockIdx.y;
  const int f0 = even_first(sk.blocks, sk.tiles, r), f1 = even_first(sk.blocks, sk.tiles, r + 1);
  const glb_t<const acc_t> *const ws = to_glb(static_cast<const acc_t *>(sk.ws));
  constexpr int64_t kSlot = int64_t(WT::FM) * WT::FN * NT;
  const int64_t e = int64_t(f) * NT + threadIdx.x;
  acc_t v = ws[f0 * kSlot + e];
  for (int p = f0 + 1; p < f1; ++p) v = v + ws[p * kSlot + e];
  int tm, tn;
  group_coords(sk.whole + r, tilesM, tilesN, &tm, &tn);
  gett_store_fragment<Tin, Tc, BM, BN, WGM, WGN>(v, f / WT::FN, f % WT::FN, C, t, M, N, alpha, beta,
                                                 int64_t(tm) * BM, int64_t(tn) * BN);
}

// Short summations (K <= kShortK) with large outputs, such as the triples
// contraction (K = 32, a 1 GB output): the time goes to the MFMA phase and
// to the output stores, and a workgroup per tile runs them one after the
// other.  Here workgroup s of S walks the tiles s, s + S, ... (tile ids in
// the XCD-aware order) with two LDS buffers for the operand tiles (each
// holding the whole summation), so that the stores of one tile drain while
// the next tile is multiplied.  A wave waits for its global loads with the
// one vector-memory counter that its stores also count, and the compiler
// waits for a load issued after a store by waiting for everything; so each
// iteration issues the next tile's loads first, multiplies the current tile
// (long enough for those loads and the previous tile's stores to finish),
// only then waits and moves the loaded tile to the other LDS buffer, and
// issues the current tile's stores last.  The row and C offsets a tile's
// loads and stores use are staged in LDS one tile ahead.  Per tile j:
//   1. barrier (tile j in LDS buffer j & 1)
//   2. issue the loads of tile j + 1 (operands, into registers) and of the
//      table entries of tiles j + 2 (rows) and j + 1 (C offsets)
//   3. the products of tile j over the whole summation, from LDS
//   4. registers -> LDS buffer (j + 1) & 1; table entries -> LDS
//   5. the stores of tile j (C offsets from LDS, nontemporal)
// The K-table entries do not depend on the tile and are fetched once.
constexpr int kShortK = 32;

// where the short-summation kernel's lanes outside the output store
__device__ __align__(16) double shortk_sink[2];

template <typename Tin, typename Tc, int TILE, int LA, int LB>
constexpr int shortk_lds_elems() {
  constexpr int NT = 64 * kTiles[TILE].wgm * kTiles[TILE].wgn;
  return 2 * (Loader<Tin, Tc, kTiles[TILE].bm, kShortK, LA, true, NT>::ELEMS +
              Loader<Tin, Tc, kTiles[TILE].bn, kShortK, LB, true, NT>::ELEMS);
}

// BETA0: beta == 0, so the epilogue has one path whose store count the
// compiler knows; with beta != 0 its C loads follow earlier stores anyway.
template <typename Tin, typename Tc, int TILE, int LA, int LB, bool BETA0, bool FULL = false>
__global__ __launch_bounds__(64 * kTiles[TILE].wgm * kTiles[TILE].wgn, 1) void gett_shortk_kernel(
    const Tin *__restrict__ A, const Tin *__restrict__ B, Tin *__restrict__ C, GettTables t, int64_t M, int64_t N,
    int64_t K, double alpha, double beta, int tilesM, int tilesN) {
  constexpr int BM = kTiles[TILE].bm, BN = kTiles[TILE].bn;
  constexpr int WGM = kTiles[TILE].wgm, WGN = kTiles[TILE].wgn;
  constexpr int NT = 64 * WGM * WGN;
  constexpr int KS = kShortK;
  typedef WaveTile<Tc, BM, BN, WGM, WGN> WT;
  typedef Loader<Tin, Tc, BM, KS, LA, true, NT> LoadA;
  typedef Loader<Tin, Tc, BN, KS, LB, true, NT> LoadB;
  typedef typename WT::acc_t acc_t;
  constexpr int NE = (BM + BN + NT - 1) / NT;   // table entries per thread and tile
  constexpr int BUF = LoadA::ELEMS + LoadB::ELEMS;
  __shared__ __attribute__((aligned(16))) Tc smem[shortk_lds_elems<Tin, Tc, TILE, LA, LB>()];
  __shared__ int64_t rows_s[2][BM + BN];   // offAm / offBn entries of a tile
  __shared__ int64_t ctab_s[2][BM + BN];   // offCm / offCn entries of a tile
  lds_t<Tc> *const s0 = to_lds(smem);
  lds_t<int64_t> *const rows = to_lds(&rows_s[0][0]);
  lds_t<int64_t> *const ctab = to_lds(&ctab_s[0][0]);

  const int T = tilesM * tilesN, S = gridDim.x, sb = blockIdx.x;
  if (sb >= T) return;   // uniform: a workgroup without tiles
  const int ntile = (T - 1 - sb) / S + 1;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WGN) * WT::WM, wn0 = (wave % WGN) * WT::WN;
  // (plain code rather than lambdas: a kernel argument captured by reference
  // is given an address in scratch memory, and reading it back is one more
  // vector memory load)
  int64_t rv[NE], cv[NE];
  // rows of tile jr and C offsets of tile jc, clamped to the last tile and
  // entry so that every lane issues the same loads on every path
#define SHORTK_FETCH_TABLES(jr_, jc_)                                                                  \
  do {                                                                                                \
    int tmr, tnr, tmc, tnc;                                                                           \
    tile_coords(sb + ((jr_) < ntile ? (jr_) : ntile - 1) * S, tilesM, tilesN, &tmr, &tnr);            \
    tile_coords(sb + ((jc_) < ntile ? (jc_) : ntile - 1) * S, tilesM, tilesN, &tmc, &tnc);            \
    _Pragma("unroll") for (int q = 0; q < NE; ++q) {                                                  \
      const int x = tid + q * NT < BM + BN ? tid + q * NT : BM + BN - 1;                             \
      if (x < BM) {                                                                                   \
        const int64_t mr = int64_t(tmr) * BM + x, mc = int64_t(tmc) * BM + x;                        \
        rv[q] = to_glb(t.offAm)[mr < M ? mr : M - 1];                                                \
        cv[q] = to_glb(t.offCm)[mc < M ? mc : M - 1];                                                \
      } else {                                                                                        \
        const int64_t nr = int64_t(tnr) * BN + (x - BM), nc = int64_t(tnc) * BN + (x - BM);          \
        rv[q] = to_glb(t.offBn)[nr < N ? nr : N - 1];                                                \
        cv[q] = to_glb(t.offCn)[nc < N ? nc : N - 1];                                                \
      }                                                                                               \
    }                                                                                                 \
  } while (0)
  // the staged table entries of rv into rows[rb], of cv into ctab[cb]
#define SHORTK_STAGE_TABLES(rb_, cb_)                                                                  \
  _Pragma("unroll") for (int q = 0; q < NE; ++q) {                                                    \
    const int x = tid + q * NT;                                                                       \
    if (x < BM + BN) {                                                                                \
      rows[(rb_) * (BM + BN) + x] = rv[q];                                                            \
      ctab[(cb_) * (BM + BN) + x] = cv[q];                                                            \
    }                                                                                                 \
  }

  LoadA la;
  LoadB lb;
  // prologue: tile 0's rows from the tables, the K-table entries (the same
  // for every tile), tile 0's operands into LDS buffer 0, tile 1's rows and
  // tile 0's C offsets into LDS
  {
    int tm, tn;
    tile_coords(sb, tilesM, tilesN, &tm, &tn);
    la.init(tid, int64_t(tm) * BM, M, t.offAm);
    lb.init(tid, int64_t(tn) * BN, N, t.offBn);
  }
  la.fetch_k(t.offAk, 0, K);
  lb.fetch_k(t.offBk, 0, K);
  la.template load<FULL>(A, 0, K);
  lb.template load<FULL>(B, 0, K);
  // tile 0's rows into rows[0]: the last iteration reloads its own tile from
  // rows[j & 1], which for a workgroup with one tile no other step writes
  SHORTK_FETCH_TABLES(0, 0);
  SHORTK_STAGE_TABLES(0, 0)
  SHORTK_FETCH_TABLES(1, 0);
  la.store(s0);
  lb.store(s0 + LoadA::ELEMS);
  SHORTK_STAGE_TABLES(1, 0)

  WT w;
  for (int j = 0; j < ntile; ++j) {
    __syncthreads();   // 1
    // 2: the next tile's loads (on the last tile its own again, so that every
    // iteration issues the same loads)
    {
      const int jn = j + 1 < ntile ? j + 1 : j;
      int tm1, tn1;
      tile_coords(sb + jn * S, tilesM, tilesN, &tm1, &tn1);
      const int64_t m1 = int64_t(tm1) * BM, n1 = int64_t(tn1) * BN;
      const lds_t<int64_t> *r1 = rows + (jn & 1) * (BM + BN);
      la.init_from(tid, m1, M, r1, m1);
      lb.init_from(tid, n1, N, r1 + BM, n1);
      la.template load<FULL>(A, 0, K);
      lb.template load<FULL>(B, 0, K);
      SHORTK_FETCH_TABLES(j + 2, j + 1);
    }
    // 3: the products over the whole summation
    const lds_t<Tc> *cur = s0 + (j & 1) * BUF;
#pragma unroll
    for (int i = 0; i < WT::FM; ++i)
#pragma unroll
      for (int jj = 0; jj < WT::FN; ++jj) w.acc[i][jj] = acc_t{0, 0, 0, 0};
    gett_mma_step<LoadA, LoadB, KS>(w, cur, cur + LoadA::ELEMS, lane, wm0, wn0);
    // keep step 4 (whose waits also wait for the previous tile's stores) after
    // every product: the scheduler would otherwise hoist the independent LDS
    // writes, and their waits, into the middle of the products
    __builtin_amdgcn_sched_barrier(0);
    // 4: the next tile into the other buffer (its previous contents were last
    // read before barrier 1)
    lds_t<Tc> *nxt = s0 + ((j + 1) & 1) * BUF;
    la.store(nxt);
    lb.store(nxt + LoadA::ELEMS);
    SHORTK_STAGE_TABLES(j & 1, (j + 1) & 1)
    // 5: the stores, which drain under the next tile's products
    int tm0, tn0;
    tile_coords(sb + j * S, tilesM, tilesN, &tm0, &tn0);
    const lds_t<int64_t> *ct = ctab + (j & 1) * (BM + BN);
    gett_store_staged<Tin, Tc, BM, BN, WGM, WGN, true>(w, C, ct, ct + BM, M, N, alpha, BETA0 ? 0.0 : beta,
                                                       int64_t(tm0) * BM, int64_t(tn0) * BN,
                                                       reinterpret_cast<Tin *>(shortk_sink));
  }
#undef SHORTK_FETCH_TABLES
#undef SHORTK_STAGE_TABLES
}

// Sum the workspace pieces of each split stream-K tile, in workgroup order,
// and write alpha * sum + beta * C.  Workgroup (x, y) takes stream-K tile x
// and accumulator element y = i * FN + j of every thread, so that a tile's
// sum is spread over FM * FN workgroups; tiles that one workgroup covered
// whole were written by it and are skipped.
template <typename Tin, typename Tc, int TILE>
__global__ __launch_bounds__(64 * kTiles[TILE].wgm * kTiles[TILE].wgn) void gett_fixup_kernel(
    Tin *__restrict__ C, GettTables t, int64_t M, int64_t N, int64_t K, double alpha, double beta, int tilesM,
    int tilesN, StreamK sk) {
  constexpr int BM = kTiles[TILE].bm, BN = kTiles[TILE].bn, BK = kTiles[TILE].bk;
  constexpr int WGM = kTiles[TILE].wgm, WGN = kTiles[TILE].wgn;
  constexpr int NT = 64 * WGM * WGN;
  typedef WaveTile<Tc, BM, BN, WGM, WGN> WT;
  typedef typename WT::acc_t acc_t;
  const int dp = tilesM * tilesN - sk.tiles;
  const int64_t tt = blockIdx.x;
  const int f = blockIdx.y;
  const int64_t nk = (K + BK - 1) / BK;
  const int64_t I = int64_t(sk.tiles) * nk;
  const int lo = sk_owner(I, sk.blocks, tt * nk), hi = sk_owner(I, sk.blocks, (tt + 1) * nk - 1);
  if (lo == hi) return;
  const glb_t<const acc_t> *const ws = to_glb(static_cast<const acc_t *>(sk.ws));
  constexpr int64_t kSlot = int64_t(WT::FM) * WT::FN * NT;
  acc_t v = acc_t{0, 0, 0, 0};
  for (int s = lo; s <= hi; ++s) {
    const int64_t a = sk_begin(I, sk.blocks, s);
    if (a == sk_begin(I, sk.blocks, s + 1)) continue;   // an empty share wrote nothing
    const int slot = 2 * s + (tt == a / nk ? 0 : 1);
    const acc_t p = ws[slot * kSlot + int64_t(f) * NT + threadIdx.x];
    v = s == lo ? p : v + p;
  }
  int tm, tn;
  group_coords(dp + int(tt), tilesM, tilesN, &tm, &tn);
  gett_store_fragment<Tin, Tc, BM, BN, WGM, WGN>(v, f / WT::FN, f % WT::FN, C, t, M, N, alpha, beta,
                                                 int64_t(tm) * BM, int64_t(tn) * BN);
}

// the persistent kernel's LDS: the tile buffers plus two staged copies of a
// tile's row and C offsets
template <typename Tin, typename Tc, int TILE, int LA, int LB, bool VA, bool VB>
constexpr bool persistent_fits() {
  constexpr int NT = 64 * kTiles[TILE].wgm * kTiles[TILE].wgn;
  return int(sizeof(Tc)) * gett_lds_elems<Tin, Tc, kTiles[TILE].bm, kTiles[TILE].bn, kTiles[TILE].bk, NT, LA, LB,
                                          VA, VB>() +
             4 * (kTiles[TILE].bm + kTiles[TILE].bn) * 8 <=
         160 * 1024;
}

template <typename Tin, typename Tc, int TILE>
constexpr bool tile_fits() {
  constexpr int V = 16 / int(sizeof(Tin));
  constexpr int NT = 64 * kTiles[TILE].wgm * kTiles[TILE].wgn;
  return (kTiles[TILE].bm * kTiles[TILE].bk) % (V * NT) == 0 && (kTiles[TILE].bn * kTiles[TILE].bk) % (V * NT) == 0;
}

template <typename Tin, typename Tc, int TILE, int LA, int LB, bool VA, bool VB>
hipError_t launch_v(const GettLaunch &g, hipStream_t s) {
  if constexpr (!tile_fits<Tin, Tc, TILE>()) {
    return hipErrorInvalidValue;
  } else {
    constexpr int BM = kTiles[TILE].bm, BN = kTiles[TILE].bn;
    constexpr int NT = 64 * kTiles[TILE].wgm * kTiles[TILE].wgn;
    if (g.occupancy) {
      if (g.shortk > 0) {
        if constexpr (!(VA && VB && shortk_tile(TILE))) {
          *g.occupancy = 0;
          return hipSuccess;
        } else {
          return hipOccupancyMaxActiveBlocksPerMultiprocessor(
              g.occupancy, gett_shortk_kernel<Tin, Tc, TILE, LA, LB, true>, NT, 0);
        }
      }
      if (g.query_sk == 2)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            g.occupancy, gett_whole_piece_kernel<Tin, Tc, TILE, LA, LB, VA, VB>, NT, 0);
      if (g.query_sk)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(g.occupancy,
                                                            gett_sk_kernel<Tin, Tc, TILE, LA, LB, VA, VB>, NT, 0);
      if (g.persistent > 0) {
        if constexpr (!persistent_fits<Tin, Tc, TILE, LA, LB, VA, VB>()) {
          *g.occupancy = 0;
          return hipSuccess;
        } else {
          return hipOccupancyMaxActiveBlocksPerMultiprocessor(
              g.occupancy, gett_persistent_kernel<Tin, Tc, TILE, LA, LB, VA, VB>, NT, 0);
        }
      }
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(g.occupancy, gett_kernel<Tin, Tc, TILE, LA, LB, VA, VB>,
                                                          NT, 0);
    }
    const int tilesM = int((g.M + BM - 1) / BM), tilesN = int((g.N + BN - 1) / BN);
    // every tile inside the output and whole K steps: the unmasked loads
    const bool full = full_tile(TILE) && VA && VB && g.M % BM == 0 && g.N % BN == 0 && g.K % kTiles[TILE].bk == 0;
    const Tin *A = static_cast<const Tin *>(g.A), *B = static_cast<const Tin *>(g.B);
    Tin *C = static_cast<Tin *>(g.C);
    if (g.bt.offA) {
      // batch labels: whole tiles, as many entries per launch as the grid
      // size allows
      if constexpr (!batch_tile(TILE)) {
        return hipErrorInvalidValue;
      } else {
        const int64_t per = int64_t(tilesM) * tilesN;
        constexpr int64_t kMaxY = 65535;   // grid limit along y
        if (per * NT > int64_t(UINT32_MAX) || !g.bt.offB || !g.bt.offC) return hipErrorInvalidValue;
        for (int64_t e0 = 0; e0 < g.bt.count; e0 += kMaxY) {
          GettBatch bt = g.bt;
          bt.first = g.bt.first + e0;
          bt.count = std::min(kMaxY, g.bt.count - e0);
          hipLaunchKernelGGL((gett_batch_kernel<Tin, Tc, TILE, LA, LB, VA, VB>),
                             dim3(unsigned(per), unsigned(bt.count)), dim3(NT), 0, s, A, B, C, g.t, g.M, g.N, g.K,
                             g.alpha, g.beta, tilesM, tilesN, bt);
          hipError_t e = hipGetLastError();
          if (e != hipSuccess) return e;
        }
        return hipSuccess;
      }
    }
    if (g.shortk > 0) {
      if constexpr (!(VA && VB && shortk_tile(TILE))) {
        return hipErrorInvalidValue;
      } else {
        if (g.K > kShortK) return hipErrorInvalidValue;
        const dim3 grid(std::min(g.shortk, tilesM * tilesN));
        // whole tiles over the whole short summation: unmasked loads
        if (g.beta == 0.0 && g.M % BM == 0 && g.N % BN == 0 && g.K == kShortK)
          hipLaunchKernelGGL((gett_shortk_kernel<Tin, Tc, TILE, LA, LB, true, true>), grid, dim3(NT), 0, s, A, B, C,
                             g.t, g.M, g.N, g.K, g.alpha, g.beta, tilesM, tilesN);
        else if (g.beta == 0.0)
          hipLaunchKernelGGL((gett_shortk_kernel<Tin, Tc, TILE, LA, LB, true>), grid, dim3(NT), 0, s, A, B, C, g.t,
                             g.M, g.N, g.K, g.alpha, g.beta, tilesM, tilesN);
        else
          hipLaunchKernelGGL((gett_shortk_kernel<Tin, Tc, TILE, LA, LB, false>), grid, dim3(NT), 0, s, A, B, C, g.t,
                             g.M, g.N, g.K, g.alpha, g.beta, tilesM, tilesN);
        return hipGetLastError();
      }
    }
    if (g.persistent > 0) {
      if constexpr (!persistent_fits<Tin, Tc, TILE, LA, LB, VA, VB>()) {
        return hipErrorInvalidValue;
      } else {
        hipLaunchKernelGGL((gett_persistent_kernel<Tin, Tc, TILE, LA, LB, VA, VB>),
                           dim3(std::min(g.persistent, tilesM * tilesN)), dim3(NT), 0, s,
                           static_cast<const Tin *>(g.A), static_cast<const Tin *>(g.B), static_cast<Tin *>(g.C), g.t,
                           g.M, g.N, g.K, g.alpha, g.beta, tilesM, tilesN);
        return hipGetLastError();
      }
    }
    if (g.sk.even) {
      // the balanced schedule: its shape must match the tile grid exactly
      const StreamK &ev = g.sk;
      if (!ev.ws || ev.blocks <= 0 || ev.whole < 0 || ev.tiles < 1 || 2 * int64_t(ev.tiles) > ev.blocks ||
          int64_t(ev.whole) + ev.tiles != int64_t(tilesM) * tilesN)
        return hipErrorInvalidValue;
      // whole tiles and pieces in one launch (the pieces start as whole
      // tiles finish), then the sum of each leftover tile's pieces
      if (full)
        hipLaunchKernelGGL((gett_whole_piece_kernel<Tin, Tc, TILE, LA, LB, VA, VB, full_tile(TILE)>),
                           dim3(ev.whole + ev.blocks), dim3(NT), 0, s, A, B, C, g.t, g.M, g.N, g.K, g.alpha, g.beta,
                           tilesM, tilesN, ev);
      else
        hipLaunchKernelGGL((gett_whole_piece_kernel<Tin, Tc, TILE, LA, LB, VA, VB>), dim3(ev.whole + ev.blocks),
                           dim3(NT), 0, s, A, B, C, g.t, g.M, g.N, g.K, g.alpha, g.beta, tilesM, tilesN, ev);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      constexpr int FRAGS = (BM / kTiles[TILE].wgm / 16) * (BN / kTiles[TILE].wgn / 16);
      hipLaunchKernelGGL((gett_piece_fixup_kernel<Tin, Tc, TILE>), dim3(ev.tiles, FRAGS), dim3(NT), 0, s, C, g.t, g.M,
                         g.N, g.alpha, g.beta, tilesM, tilesN, ev);
      return hipGetLastError();
    }
    StreamK sk = g.sk;
    if (sk.blocks <= 0 || sk.tiles <= 0 || sk.tiles > tilesM * tilesN || !sk.ws) sk = StreamK{};
    const int dp = tilesM * tilesN - sk.tiles;
    if (dp > 0 && full) {
      hipLaunchKernelGGL((gett_kernel<Tin, Tc, TILE, LA, LB, VA, VB, full_tile(TILE)>), dim3(dp), dim3(NT), 0, s, A, B,
                         C, g.t, g.M, g.N, g.K, g.alpha, g.beta, tilesM, tilesN);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    } else if (dp > 0) {
      hipLaunchKernelGGL((gett_kernel<Tin, Tc, TILE, LA, LB, VA, VB>), dim3(dp), dim3(NT), 0, s, A, B, C, g.t, g.M,
                         g.N, g.K, g.alpha, g.beta, tilesM, tilesN);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (sk.tiles == 0) return hipSuccess;
    hipLaunchKernelGGL((gett_sk_kernel<Tin, Tc, TILE, LA, LB, VA, VB>), dim3(sk.blocks), dim3(NT), 0, s, A, B, C,
                       g.t, g.M, g.N, g.K, g.alpha, g.beta, tilesM, tilesN, sk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    constexpr int FRAGS = (BM / kTiles[TILE].wgm / 16) * (BN / kTiles[TILE].wgn / 16);
    hipLaunchKernelGGL((gett_fixup_kernel<Tin, Tc, TILE>), dim3(sk.tiles, FRAGS), dim3(NT), 0, s, C, g.t, g.M, g.N,
                       g.K, g.alpha, g.beta, tilesM, tilesN, sk);
    return hipGetLastError();
  }
}

// element-load (non-vector) variants exist for tile 1 only
template <typename Tin, typename Tc, int TILE, int LA, int LB>
hipError_t launch_l(const GettLaunch &g, hipStream_t s) {
  if constexpr (TILE == 1) {
    switch ((g.vecA ? 2 : 0) + (g.vecB ? 1 : 0)) {
      case 3: return launch_v<Tin, Tc, TILE, LA, LB, true, true>(g, s);
      case 2: return launch_v<Tin, Tc, TILE, LA, LB, true, false>(g, s);
      case 1: return launch_v<Tin, Tc, TILE, LA, LB, false, true>(g, s);
      default: return launch_v<Tin, Tc, TILE, LA, LB, false, false>(g, s);
    }
  } else {
    if (!g.vecA || !g.vecB) return hipErrorInvalidValue;
    return launch_v<Tin, Tc, TILE, LA, LB, true, true>(g, s);
  }
}

template <typename Tin, typename Tc, int TILE>
hipError_t launch_t(const GettLaunch &g, hipStream_t s) {
  switch (g.layoutA * 2 + g.layoutB) {
    case 0: return launch_l<Tin, Tc, TILE, 0, 0>(g, s);
    case 1: return launch_l<Tin, Tc, TILE, 0, 1>(g, s);
    case 2: return launch_l<Tin, Tc, TILE, 1, 0>(g, s);
    default: return launch_l<Tin, Tc, TILE, 1, 1>(g, s);
  }
}

// mixed storage/arithmetic pairs have the two basic tiles only
template <typename Tin, typename Tc>
hipError_t launch_tc(const GettLaunch &g, hipStream_t s) {
  constexpr bool same = sizeof(Tin) == sizeof(Tc);
  switch (g.tile) {
    case 0: return launch_t<Tin, Tc, 0>(g, s);
    case 1: return launch_t<Tin, Tc, 1>(g, s);
    case 2: if constexpr (same) return launch_t<Tin, Tc, 2>(g, s); else return hipErrorInvalidValue;
    case 3: if constexpr (same) return launch_t<Tin, Tc, 3>(g, s); else return hipErrorInvalidValue;
    case 4: if constexpr (same) return launch_t<Tin, Tc, 4>(g, s); else return hipErrorInvalidValue;
    case 5: if constexpr (same) return launch_t<Tin, Tc, 5>(g, s); else return hipErrorInvalidValue;
    case 6: if constexpr (same) return launch_t<Tin, Tc, 6>(g, s); else return hipErrorInvalidValue;
    case 7: if constexpr (same) return launch_t<Tin, Tc, 7>(g, s); else return hipErrorInvalidValue;
    case 8: if constexpr (same) return launch_t<Tin, Tc, 8>(g, s); else return hipErrorInvalidValue;
    case 9: if constexpr (same) return launch_t<Tin, Tc, 9>(g, s); else return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

// beta * C over the (b, m, n) index space of C
template <typename T>
__global__ __launch_bounds__(256) void scale_kernel(T *__restrict__ C, const int64_t *__restrict__ offCm,
                                                    const int64_t *__restrict__ offCn, int64_t M, int64_t N,
                                                    double beta, const int64_t *__restrict__ offCb, int64_t NB) {
  const int64_t MN = M * N, total = NB * MN;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t b = i / MN, r = i - b * MN;
    const int64_t m = r / N, n = r - m * N;
    const int64_t a = (offCb ? offCb[b] : 0) + offCm[m] + offCn[n];
    __builtin_nontemporal_store(beta == 0.0 ? T(0) : T(double(C[a]) * beta), C + a);
  }
}

}  // namespace

int gett_tile_count() { return kNumTiles; }

size_t gett_sk_slot_bytes(int tile, int compute) {
  return size_t(kTiles[tile].bm) * kTiles[tile].bn * (compute == 0 ? 8 : 4);
}

void gett_tile_shape(int tile, int *bm, int *bn, int *bk) {
  *bm = kTiles[tile].bm;
  *bn = kTiles[tile].bn;
  *bk = kTiles[tile].bk;
}

bool gett_tile_valid(int tile, int dtype, int compute, bool vecA, bool vecB, bool batch) {
  if (tile < 0 || tile >= kNumTiles) return false;
  if (batch && !batch_tile(tile)) return false;
  if (tile != 1 && (!vecA || !vecB)) return false;
  const bool same = (dtype == 0) == (compute == 0);
  if (!same && tile > 1) return false;
  const int V = dtype == 0 ? 2 : 4;
  const int NT = 64 * kTiles[tile].wgm * kTiles[tile].wgn;
  return (kTiles[tile].bm * kTiles[tile].bk) % (V * NT) == 0 && (kTiles[tile].bn * kTiles[tile].bk) % (V * NT) == 0;
}

hipError_t launch_gett(const GettLaunch &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (g.dtype == 0) {
    return g.compute == 0 ? launch_tc<double, double>(g, s) : launch_tc<double, float>(g, s);
  }
  return g.compute == 0 ? launch_tc<float, double>(g, s) : launch_tc<float, float>(g, s);
}

int gett_occupancy(const GettLaunch &g) {
  int n = 0;
  GettLaunch q = g;
  q.occupancy = &n;
  q.M = q.N = 1;
  if (launch_gett(q, nullptr) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

hipError_t launch_scale(void *C, int dtype, const int64_t *offCm, const int64_t *offCn, int64_t M, int64_t N,
                        double beta, hipStream_t s, const int64_t *offCb, int64_t NB) {
  if (M <= 0 || N <= 0 || NB <= 0) return hipSuccess;
  if (!offCb && NB != 1) return hipErrorInvalidValue;
  int64_t total = NB * M * N;
  int blocks = int(std::min<int64_t>((total + 255) / 256, 4096));
  if (dtype == 0)
    hipLaunchKernelGGL(scale_kernel<double>, dim3(blocks), dim3(256), 0, s, static_cast<double *>(C), offCm, offCn, M,
                       N, beta, offCb, NB);
  else
    hipLaunchKernelGGL(scale_kernel<float>, dim3(blocks), dim3(256), 0, s, static_cast<float *>(C), offCm, offCn, M,
                       N, beta, offCb, NB);
  return hipGetLastError();
}

}  // namespace comet
