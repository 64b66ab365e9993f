// api.cpp -- the C ABI (include/comet.h): validation, plans, workspaces and
// dispatch to the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "chain.hpp"
#include "comet.h"
#include "kernels.hpp"
#include "plan.hpp"
#include "split.hpp"
#include "tune.hpp"

using namespace comet;

namespace {

thread_local std::string g_last_error;
int g_split_slices = 5;
int g_int8_slices = 6;
std::mutex g_mu;

comet_status_t fail(comet_status_t code, const std::string &msg) {
  g_last_error = msg;
  return code;
}
comet_status_t fail(const Status &st) { return fail(st.code, st.msg); }

comet_status_t hip_fail(hipError_t e, const char *what) {
  return fail(COMET_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)              \
  do {                                   \
    hipError_t _e = (expr);              \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool tables_vec_ok(const std::vector<int64_t> &offR, const std::vector<int64_t> &offK, int layout, int runR,
                   int runK, int VEC) {
  if ((layout == 0 ? runK : runR) < VEC) return false;
  for (size_t r = 0; r < offR.size(); ++r)
    if ((layout == 0 || r % VEC == 0) && offR[r] % VEC) return false;
  for (size_t k = 0; k < offK.size(); ++k)
    if ((layout == 1 || k % VEC == 0) && offK[k] % VEC) return false;
  return true;
}

std::vector<int64_t> dense_strides(const std::vector<int64_t> &ext) {
  std::vector<int64_t> s(ext.size());
  int64_t x = 1;
  for (int p = (int)ext.size() - 1; p >= 0; --p) {
    s[p] = x;
    x *= ext[p];
  }
  return s;
}

}  // namespace

namespace comet {
// Record an error for comet_last_error (used by the other translation units
// of the C ABI).
comet_status_t api_fail(comet_status_t code, const std::string &msg) { return fail(code, msg); }
}  // namespace comet

struct comet_plan_s {
  Analysis an;
  int device = 0;
  void *dtables = nullptr;     // the six offset tables (and three batch tables), one device allocation
  GettTables t{};
  const int64_t *offAx = nullptr, *offBx = nullptr, *offCx = nullptr;   // batch tables (device), or null
  bool vecA_tables = false, vecB_tables = false;
  bool fused3 = false;         // FP32 operands split into BF16x3 inside the gather kernel
  size_t ws_bytes = 0;
  // split modes
  SplitPlan split;
  // TTGT
  std::unique_ptr<comet_plan_s> gemm;
  PermuteLaunch permA{}, permB{}, permC{};
  size_t wsA = 0, wsB = 0, wsC = 0;   // byte offsets of A_p, B_p, C_p in the workspace
  size_t wsG = 0;                     // byte offset of the GEMM stage's own workspace
  size_t sk_bytes = 0;                // stream-K partial sums (at offset 0 of a GETT plan's workspace)

  ~comet_plan_s() {
    if (dtables) (void)hipFree(dtables);
  }
};

struct comet_batch_s {
  struct ScaleJob {
    void *C;
    const int64_t *offCm, *offCn;
    int64_t m, n;
    double beta;
    const int64_t *offCb;          // batch entries of C (device), or null
    int64_t nb;
  };
  int device = 0;
  comet_dtype_t dtype = COMET_F64;
  int mode = 0;                    // 0: native MFMA, 1: fused BF16x3
  void *dbuf = nullptr;            // descriptors, work items, offset tables
  const BatchDesc *descs = nullptr;
  const BatchItem *items = nullptr;
  int64_t total = 0;
  BatchQueues queues{};            // the work list cut into one queue per XCD
  std::vector<int> classes;        // descriptors per tile class
  int tuned = 0;                   // descriptors whose class came from the autotuner
  int grid = 1;
  std::vector<ScaleJob> scales;    // empty summation or alpha == 0: C = beta * C
  // element-load problems: one operand copied, before the launch, into a
  // dense order that both operands can read in vectors (pbuf, owned here)
  void *pbuf = nullptr;
  std::vector<PermuteLaunch> perms;

  ~comet_batch_s() {
    if (dbuf) (void)hipFree(dbuf);
    if (pbuf) (void)hipFree(pbuf);
  }
};

namespace {

comet_status_t upload_tables(comet_plan_s *p) {
  const Analysis &an = p->an;
  const std::vector<int64_t> *tabs[9] = {&an.offAm, &an.offAk, &an.offBk, &an.offBn, &an.offCm,
                                         &an.offCn, &an.offAx, &an.offBx, &an.offCx};
  size_t off[9], total = 0;
  for (int i = 0; i < 9; ++i) {
    off[i] = total;
    total += align256(std::max<size_t>(tabs[i]->size(), 1) * sizeof(int64_t));
  }
  HIP_TRY(hipMalloc(&p->dtables, total), "hipMalloc(offset tables)");
  std::vector<char> host(total, 0);
  for (int i = 0; i < 9; ++i)
    if (!tabs[i]->empty()) std::memcpy(host.data() + off[i], tabs[i]->data(), tabs[i]->size() * sizeof(int64_t));
  HIP_TRY(hipMemcpy(p->dtables, host.data(), total, hipMemcpyHostToDevice), "hipMemcpy(offset tables)");
  char *b = static_cast<char *>(p->dtables);
  p->t.offAm = reinterpret_cast<const int64_t *>(b + off[0]);
  p->t.offAk = reinterpret_cast<const int64_t *>(b + off[1]);
  p->t.offBk = reinterpret_cast<const int64_t *>(b + off[2]);
  p->t.offBn = reinterpret_cast<const int64_t *>(b + off[3]);
  p->t.offCm = reinterpret_cast<const int64_t *>(b + off[4]);
  p->t.offCn = reinterpret_cast<const int64_t *>(b + off[5]);
  if (!an.offAx.empty()) {
    p->offAx = reinterpret_cast<const int64_t *>(b + off[6]);
    p->offBx = reinterpret_cast<const int64_t *>(b + off[7]);
    p->offCx = reinterpret_cast<const int64_t *>(b + off[8]);
  }
  return COMET_OK;
}

// Tile choice without timing.  For every compiled tile the time of one round
// (every CU running `resident` workgroups of the tile to the end) is
//   rt = resident * BM * BN / throughput * K / 3072,
// with `resident` from the occupancy calculator for the exact kernel and the
// per-CU output throughput measured on MI355X per tile on a matrix product
// with 6144 x 6144 outputs and K = 3072 (A contiguous along K, B along N),
// in output elements per microsecond.  T tiles over S = CUs * resident slots
// then take floor(T / S) full rounds plus a partial round, which runs at
// most twice as fast as a full one (fewer workgroups share each CU).  The
// stream-K alternative replaces the partial round by an equal split of its
// tiles' summation over all S slots, plus the partial sums it writes and
// reads back.  The autotuner replaces this model with timings.
constexpr double kThroughputF64[] = {28.7, 33.5, 30.9, 41.4, 39.5, 34.2, 33.4, 34.2, 35.0, 34.8};
constexpr double kThroughputF32[] = {76.0, 70.6, 74.2, 77.0, 80.3, 69.2, 69.5};
constexpr int kTuneTTGT = 32;           // TTGT flattenings the autotuner times against the gather tiles
constexpr int kTuneTTGTAll = 512;       // the same when TTGT is asked for: every one, up to this many,
constexpr int kTuneTTGTRetime = 8;      // and the fastest this many timed twice more
// A contraction whose operands only tile 1's element-load kernel can gather
// goes through TTGT when the time the vector-load GEMM saves exceeds what the
// permutes cost.  Rates on MI355X ("cmia=cdmn*inad" at 3072^3: element-load
// gather 2.64 ms in FP64 and 2.62 ms in FP32 when first measured, 3.3 and
// 4.0 ms on later boxes with the same kernel; the TTGT GEMM alone about 0.9
// and 0.55 ms; the element-load rate below is the fastest of those); permutes move their bytes at about 4.5 TB/s, and each of the up to
// three extra launches costs about 5 us on small problems (its launch gap
// and its ramp).  Measured crossover:
// 512^3 0.031 (gather) vs 0.034 ms (TTGT) in FP64, 768^3 0.063 vs 0.047;
// FP32 0.025 vs 0.027 and 0.054 vs 0.039.
// When an extent keeps even the TTGT matrices from vector reads (an odd
// summation length, say), their GEMM still reads dense rows: 49 TFLOP/s in
// FP64 and 50 in FP32 at 3025^3 (extents of 55), where the element-load
// gather ran at 13 and 16.
constexpr double kElemLoadFlops = 22.0e12;        // FLOP/s, FP64 and FP32
constexpr double kVecGemmFlopsF64 = 58.0e12;
constexpr double kVecGemmFlopsF32 = 100.0e12;
constexpr double kDenseElemGemmFlops = 45.0e12;
constexpr double kPermuteBytesPerS = 4.5e12;
constexpr double kPermuteLaunchS = 5.0e-6;
constexpr size_t kTTGTMaxWorkspace = size_t(4) << 30;   // no automatic TTGT needing more
constexpr size_t kGemvMaxWorkspace = size_t(256) << 20;   // partial sums of the matrix-vector kernel
constexpr double kFused3MaxMNK = 0x1p31;  // above: FP32 BF16x3 through the slicer and slice-pair product
constexpr int kSkMinSteps = 8;          // fewest BK steps a stream-K share should hold
constexpr int kSkSmallSteps = 4;        // the same for latency-bound problems (tile 1)
constexpr double kSkBytesPerUs = 4.0e6;  // partial-sum traffic rate (HBM, both directions)
constexpr double kSkLaunchUs = 4.0;      // the two extra launches

// Estimated saving (seconds, may be negative) of TTGT plan `tt` over the
// element-load gather of the same contraction `an`: the GEMM time saved
// minus the permutes' traffic and launches.
double ttgt_saving_s(const Analysis &an, const comet_plan_s &tt) {
  const double flops = 2.0 * double(an.m) * double(an.n) * double(an.k);
  const bool vec_reads = tt.gemm && tt.gemm->vecA_tables && tt.gemm->vecB_tables;
  const double vec = !vec_reads ? kDenseElemGemmFlops
                     : an.compute == COMET_COMPUTE_F64 ? kVecGemmFlopsF64 : kVecGemmFlopsF32;
  const TTGTChoice &c = tt.an.ttgt;
  const double es = double(elem_size(an.dtype));
  auto count = [&](const std::string &labels) {
    double n = 1.0;
    for (char ch : labels)
      n *= double(an.extents[std::find(an.labels.begin(), an.labels.end(), ch) - an.labels.begin()]);
    return n;
  };
  double bytes = 0.0;
  int launches = 0;
  if (c.a_copy) bytes += 2.0 * es * count(an.spec_a), ++launches;
  if (c.b_copy) bytes += 2.0 * es * count(an.spec_b), ++launches;
  if (c.c_copy) bytes += 3.0 * es * count(an.spec_c), ++launches;   // GEMM write, then read + write
  return flops / kElemLoadFlops - flops / vec - bytes / kPermuteBytesPerS - launches * kPermuteLaunchS;
}

int tile_resident(const Analysis &an, int tile, bool vecA, bool vecB) {
  GettLaunch g{};
  g.dtype = an.dtype == COMET_F64 ? 0 : 1;
  g.compute = an.compute == COMET_COMPUTE_F64 ? 0 : 1;
  g.layoutA = an.layoutA;
  g.layoutB = an.layoutB;
  g.vecA = vecA;
  g.vecB = vecB;
  g.tile = tile;
  return gett_occupancy(g);
}

struct Schedule {
  int tile = 1;
  int sk_tiles = 0, sk_blocks = 0;
  int even = 0, even_whole = 0;
  int persist = 0;
  double us = 1e300;
};

// Workgroups of the stream-K kernel of `tile` resident per CU (0: none).
int sk_resident(const Analysis &an, int tile, bool vecA, bool vecB) {
  GettLaunch g{};
  g.dtype = an.dtype == COMET_F64 ? 0 : 1;
  g.compute = an.compute == COMET_COMPUTE_F64 ? 0 : 1;
  g.layoutA = an.layoutA;
  g.layoutB = an.layoutB;
  g.vecA = vecA;
  g.vecB = vecB;
  g.tile = tile;
  g.query_sk = 1;
  return gett_occupancy(g);
}

// Workgroups of the persistent kernel of `tile` resident per CU (0: none).
int persistent_resident(const Analysis &an, int tile, bool vecA, bool vecB) {
  GettLaunch g{};
  g.dtype = an.dtype == COMET_F64 ? 0 : 1;
  g.compute = an.compute == COMET_COMPUTE_F64 ? 0 : 1;
  g.layoutA = an.layoutA;
  g.layoutB = an.layoutB;
  g.vecA = vecA;
  g.vecB = vecB;
  g.tile = tile;
  g.persistent = 1;
  return gett_occupancy(g);
}

// Short summations: the persistent kernel overlaps one tile's epilogue with
// the next tile's loads.  It beat a workgroup per tile while the epilogue
// serialized its loads behind its stores; with the staged epilogue the
// whole-tile kernel (two workgroups per CU) is as fast or faster on every
// short summation measured on MI355X (K = 16 to 128; the K = 32 triples
// contraction 0.328 -> 0.275 ms in FP64), so the persistent schedule is only
// taken when COMET_GETT_PERSIST asks for it.
constexpr int kPersistMaxSteps = 0;

void persist_choice(const Analysis &an, int cus, bool vecA, bool vecB, Schedule &sc) {
  const char *env = std::getenv("COMET_GETT_PERSIST");
  int bm, bn, bk;
  gett_tile_shape(sc.tile, &bm, &bn, &bk);
  const int64_t T = ((an.m + bm - 1) / bm) * ((an.n + bn - 1) / bn);
  const int64_t nk = (an.k + bk - 1) / bk;
  const int res = persistent_resident(an, sc.tile, vecA, vecB);
  if (env && *env) {
    const int v = std::atoi(env);
    sc.persist = (v > 0 && res > 0) ? v : 0;
  } else {
    const int64_t S = int64_t(std::max(cus, 1)) * res;
    sc.persist = (res > 0 && nk <= kPersistMaxSteps && T >= 2 * S) ? int(S) : 0;
  }
  if (sc.persist > 0) sc.sk_tiles = sc.sk_blocks = 0;
}

// Modeled time of `tile`, whole tiles only and with the stream-K split;
// returns the better of the two.  resident: workgroups of the whole-tile
// kernel per CU; sk_res: of the stream-K kernel, which runs after it and
// gets at most one round of workgroups (a second round would only queue).
Schedule model_tile(const Analysis &an, int tile, int resident, int sk_res, int cus) {
  Schedule out;
  out.tile = tile;
  const bool f64 = an.compute == COMET_COMPUTE_F64;
  const double *thr = f64 ? kThroughputF64 : kThroughputF32;
  const int nthr = f64 ? int(sizeof(kThroughputF64) / sizeof(double)) : int(sizeof(kThroughputF32) / sizeof(double));
  if (tile >= nthr || resident <= 0) return out;
  int bm, bn, bk;
  gett_tile_shape(tile, &bm, &bn, &bk);
  const int64_t T = ((an.m + bm - 1) / bm) * ((an.n + bn - 1) / bn) * std::max<int64_t>(an.nb, 1);
  const int64_t S = int64_t(std::max(cus, 1)) * resident;
  const int64_t nk = (an.k + bk - 1) / bk;
  const double rt = double(resident) * bm * bn / thr[tile] * double(nk * bk) / 3072.0;
  const int64_t full = T / S, rem = T - full * S;
  double partial = 0.0;
  if (rem > 0) {
    const int64_t per_cu = (rem + cus - 1) / std::max(cus, 1);
    partial = rt * std::max(double(per_cu) / resident, 0.5);
  }
  out.us = double(full) * rt + partial;
  if (rem > 0 && T <= INT32_MAX && sk_res > 0) {
    const int64_t blocks = std::min<int64_t>(int64_t(std::max(cus, 1)) * sk_res, rem * nk / kSkMinSteps);
    if (blocks >= 2) {
      // tiles' worth of steps per workgroup, at the speed of blocks / CUs
      // workgroups per CU (as for a partial round)
      const double share = double(rem) / double(blocks);
      const double per_cu = double((blocks + cus - 1) / std::max(cus, 1));
      const double pieces = double(std::min<int64_t>(2 * blocks, blocks + rem));
      const double bytes = pieces * bm * bn * (f64 ? 8.0 : 4.0) * 2.0;
      const double sk_us = double(full) * rt + rt * share * std::max(per_cu / resident, 0.5) +
                           bytes / kSkBytesPerUs + kSkLaunchUs;
      if (sk_us < 0.97 * out.us) {
        out.us = sk_us;
        out.sk_tiles = int(rem);
        out.sk_blocks = int(blocks);
      }
    }
  }
  return out;
}

// Apply COMET_GETT_SK: "0" turns stream-K off, "tiles,blocks" forces a split
// (clamped to the tile count; at least one block).
void sk_override(const Analysis &an, Schedule &sc) {
  const char *env = std::getenv("COMET_GETT_SK");
  if (!env || !*env) return;
  if (std::string(env) == "0") {
    sc.sk_tiles = sc.sk_blocks = 0;
    return;
  }
  int t = 0, b = 0;
  if (std::sscanf(env, "%d,%d", &t, &b) != 2) return;
  int bm, bn, bk;
  gett_tile_shape(sc.tile, &bm, &bn, &bk);
  const int64_t T = ((an.m + bm - 1) / bm) * ((an.n + bn - 1) / bn);
  sc.sk_tiles = int(std::max<int64_t>(0, std::min<int64_t>(t, T)));
  sc.sk_blocks = sc.sk_tiles > 0 ? std::max(b, 1) : 0;
}

// Latency-bound problems: fewer 64 x 64 tiles than one round of tile-1
// workgroups.  The per-step latency of a lone workgroup dominates there,
// which the throughput model does not see (the all-16 contraction on MI355X:
// the model's tile 5 took 21.5 us, tile 1 with its summation cut into 4-step
// pieces 13.2 us); take tile 1 and spread the summation over the idle CUs.
// With neither a split nor at most one tile per CU the model's larger tiles
// measured faster (2048^2 outputs, K = 256), and *sc is left alone.
void latency_schedule(const Analysis &an, int cus, bool vecA, bool vecB, Schedule *sc) {
  const int dt = an.dtype == COMET_F64 ? 0 : 1, cp = an.compute == COMET_COMPUTE_F64 ? 0 : 1;
  if (!an.X.empty() || !gett_tile_valid(1, dt, cp, vecA, vecB)) return;
  int bm, bn, bk;
  gett_tile_shape(1, &bm, &bn, &bk);
  const int64_t T1 = ((an.m + bm - 1) / bm) * ((an.n + bn - 1) / bn);
  const int64_t nk = (an.k + bk - 1) / bk;
  const int64_t C = std::max(cus, 1);
  const int res1 = tile_resident(an, 1, vecA, vecB), skres1 = sk_resident(an, 1, vecA, vecB);
  const int64_t blocks = skres1 > 0 ? std::min<int64_t>(C * skres1, T1 * nk / kSkSmallSteps) : 0;
  if (res1 <= 0 || T1 > C * res1 || !(blocks > T1 || T1 <= C)) return;
  // tile 1's element-load variant: only with at least half of the CUs idle
  // ("cmia=cdmn*inad", FP64: 64 tiles 0.039 -> 0.031 ms and 144 tiles
  // 0.069 -> 0.064 ms split, but 256 tiles 0.094 -> 0.20 ms)
  if (!(vecA && vecB) && 2 * T1 > C) return;
  Schedule out;
  out.tile = 1;
  out.us = 0.0;
  if (blocks > T1) {
    out.sk_tiles = int(T1);
    out.sk_blocks = int(blocks);
  }
  *sc = out;
}

// Tile and stream-K split of the gather kernel for an analyzed contraction.
Schedule pick_schedule(const Analysis &an, int cus, bool vecA, bool vecB, int forced_tile = -1) {
  const int dt = an.dtype == COMET_F64 ? 0 : 1, cp = an.compute == COMET_COMPUTE_F64 ? 0 : 1;
  const char *env = std::getenv("COMET_GETT_TILE");
  if (forced_tile < 0 && env && *env) {
    int t = std::atoi(env);
    if (t >= 0 && t < gett_tile_count()) forced_tile = t;
  }
  Schedule best;
  if (forced_tile >= 0) {
    best = model_tile(an, forced_tile, tile_resident(an, forced_tile, vecA, vecB),
                      sk_resident(an, forced_tile, vecA, vecB), cus);
    best.tile = forced_tile;
    // the element-load variant splits its summation only in the latency-bound
    // case (see below), forced or not
    if (!(vecA && vecB)) best.sk_tiles = best.sk_blocks = 0;
    if (forced_tile == 1) latency_schedule(an, cus, vecA, vecB, &best);
  } else {
    for (int t = 0; t < gett_tile_count(); ++t) {
      if (!gett_tile_valid(t, dt, cp, vecA, vecB, !an.X.empty())) continue;
      Schedule sc = model_tile(an, t, tile_resident(an, t, vecA, vecB), sk_resident(an, t, vecA, vecB), cus);
      if (sc.us < best.us * 0.999) best = sc;
    }
    // the throughput model describes the vector-load kernels: tile 1's
    // element-load variant splits its summation only in the latency-bound
    // case below (a ragged last round split by the model made the 3072^3
    // "cmia=cdmn*inad" 2.8 -> 3.4 ms)
    if (!(vecA && vecB)) best.sk_tiles = best.sk_blocks = 0;
    latency_schedule(an, cus, vecA, vecB, &best);
  }
  // every variant of a tile has its stream-K kernel (the element-load
  // variants are those of tile 1)
  sk_override(an, best);
  persist_choice(an, cus, vecA, vecB, best);
  return best;
}

// The balanced schedule replaces a stream-K split of the last, partial round
// when that round has at most half as many tiles as there are resident
// workgroups: the leftover tiles are cut into one full round of equal
// summation pieces, run at the whole-tile kernel's occupancy (the stream-K
// kernel, which may cross tiles, needs more registers and runs at a lower
// one).  COMET_GETT_EVEN=0 turns it off; =1 takes it wherever it fits, also
// where the model keeps whole tiles.
void even_choice(const Analysis &an, int cus, bool vecA, bool vecB, Schedule &sc) {
  const char *env = std::getenv("COMET_GETT_EVEN");
  const int mode = env && *env ? std::atoi(env) : -1;
  const bool native = an.compute == COMET_COMPUTE_F64 || an.compute == COMET_COMPUTE_F32;
  if (mode == 0 || !native || !vecA || !vecB || !an.X.empty() || an.empty_out || an.empty_sum || sc.persist > 0 ||
      std::getenv("COMET_GETT_SK"))
    return;
  if (mode < 0 && sc.sk_tiles == 0) return;
  // full rounds of the whole-tile kernel, then one round of the piece
  // kernel (at most as many workgroups per CU)
  GettLaunch g{};
  g.dtype = an.dtype == COMET_F64 ? 0 : 1;
  g.compute = an.compute == COMET_COMPUTE_F64 ? 0 : 1;
  g.layoutA = an.layoutA;
  g.layoutB = an.layoutB;
  g.vecA = g.vecB = 1;
  g.tile = sc.tile;
  g.query_sk = 2;
  const int res = tile_resident(an, sc.tile, true, true), res_p = std::min(gett_occupancy(g), res);
  if (res <= 0 || res_p <= 0) return;
  int bm, bn, bk;
  gett_tile_shape(sc.tile, &bm, &bn, &bk);
  const int64_t T = ((an.m + bm - 1) / bm) * ((an.n + bn - 1) / bn);
  const int64_t C = std::max(cus, 1);
  const int64_t S = C * res, Sp = C * res_p;
  const int64_t nk = (an.k + bk - 1) / bk;
  const int64_t q = T / S, R = T - q * S;
  if (R == 0 || 2 * R > Sp || T > INT32_MAX || nk < kSkSmallSteps * ((Sp + R - 1) / R)) return;
  sc.even = 1;
  sc.even_whole = int(q * S);
  sc.sk_tiles = int(R);
  sc.sk_blocks = int(Sp);
}

// Short summations with many output tiles take the short-summation kernel
// (tile 3, stores overlapped with the next tile's products): on MI355X the
// K = 32 triples contraction's whole-tile kernel runs its products and its
// 1 GB of stores one after the other.  Returns its workgroups, 0 if not
// taken; COMET_GETT_SHORTK=0 / 1 turns it off / on where it exists.
constexpr int kShortKMax = 32;
int shortk_choice(const Analysis &an, int cus, bool vecA, bool vecB, int forced_tile) {
  const bool native = an.compute == COMET_COMPUTE_F64 || an.compute == COMET_COMPUTE_F32;
  const int dt = an.dtype == COMET_F64 ? 0 : 1, cp = an.compute == COMET_COMPUTE_F64 ? 0 : 1;
  if (!native || !an.X.empty() || an.empty_out || an.empty_sum || an.k > kShortKMax || !vecA || !vecB ||
      !gett_tile_valid(3, dt, cp, true, true) || (forced_tile >= 0 && forced_tile != 3))
    return 0;
  GettLaunch g{};
  g.dtype = dt;
  g.compute = cp;
  g.layoutA = an.layoutA;
  g.layoutB = an.layoutB;
  g.vecA = g.vecB = 1;
  g.tile = 3;
  g.shortk = 1;
  const int res = gett_occupancy(g);
  if (res <= 0) return 0;
  const int64_t S = int64_t(std::max(cus, 1)) * res;
  const int64_t T = ((an.m + 127) / 128) * ((an.n + 127) / 128);
  const char *env = std::getenv("COMET_GETT_SHORTK");
  if (env && *env) return std::atoi(env) != 0 ? int(S) : 0;
  return T >= 4 * S ? int(S) : 0;
}

void apply_schedule(comet_plan_s *p, int cus, int forced_tile = -1) {
  Analysis &an = p->an;
  Schedule sc = pick_schedule(an, cus, p->vecA_tables, p->vecB_tables, forced_tile);
  const bool native = an.compute == COMET_COMPUTE_F64 || an.compute == COMET_COMPUTE_F32;
  if (!native || an.empty_out || an.empty_sum || !an.X.empty()) sc.sk_tiles = sc.sk_blocks = sc.persist = 0;
  int forced = forced_tile;   // the caller's tile, else COMET_GETT_TILE's
  if (const char *env = std::getenv("COMET_GETT_TILE"); forced < 0 && env && *env) {
    const int t = std::atoi(env);
    if (t >= 0 && t < gett_tile_count()) forced = t;
  }
  an.shortk = sc.persist > 0 ? 0 : shortk_choice(an, cus, p->vecA_tables, p->vecB_tables, forced);
  if (an.shortk > 0) {
    sc.tile = 3;
    sc.sk_tiles = sc.sk_blocks = 0;
  } else {
    even_choice(an, cus, p->vecA_tables, p->vecB_tables, sc);
  }
  an.tile = sc.tile;
  an.sk_tiles = sc.sk_tiles;
  an.sk_blocks = sc.sk_blocks;
  an.even = sc.even;
  an.even_whole = sc.even_whole;
  an.persist = sc.persist;
  const size_t slot = gett_sk_slot_bytes(sc.tile, an.compute == COMET_COMPUTE_F64 ? 0 : 1);
  // stream-K: two slots per workgroup (its first and last tile); balanced: one
  p->sk_bytes = sc.sk_tiles > 0 ? align256(size_t(sc.even ? 1 : 2) * size_t(sc.sk_blocks) * slot) : 0;
  // a matrix times a vector: the streaming kernel instead of the tiles,
  // unless a gather schedule is forced or COMET_GEMV=0
  an.gemv = an.gemv_split = 0;
  an.gemv_slab = 0;
  const char *genv = std::getenv("COMET_GEMV");
  const bool gather_forced = forced >= 0 || std::getenv("COMET_GETT_SK") || std::getenv("COMET_GETT_PERSIST") ||
                             std::getenv("COMET_GETT_EVEN");
  // (the vector has no free label, so C's unit stride lies in the matrix and
  // the planner's exchange makes the vector the kernel's A operand: M == 1)
  if (native && !an.empty_out && !an.empty_sum && an.X.empty() && an.m == 1 && !gather_forced &&
      !(genv && std::strcmp(genv, "0") == 0)) {
    const int64_t J = an.n;
    // read the matrix along whichever index group holds its smaller first
    // step (the fastest dimension of each group leads its table)
    auto step = [](const std::vector<int64_t> &t) {
      return t.size() > 1 ? std::llabs(t[1] - t[0]) : INT64_MAX;
    };
    const bool kfast = step(an.offBk) < step(an.offBn);
    int sp = 0;
    int64_t sl = 0;
    gemv_shape(J, an.k, kfast, cus, &sp, &sl);
    // COMET_GEMV_SPLIT=n: about n slabs (at least the summation over kGemvSlab)
    if (const char *fs = std::getenv("COMET_GEMV_SPLIT"); fs && std::atoi(fs) > 0) {
      const int64_t want = std::max<int64_t>({int64_t(std::atoi(fs)), (an.k + kGemvSlab - 1) / kGemvSlab, 1});
      sl = (an.k + std::min<int64_t>(want, an.k) - 1) / std::min<int64_t>(want, an.k);
      sp = int((an.k + sl - 1) / sl);
    }
    const size_t ws = sp > 1 ? align256(size_t(sp) * size_t(J) * sizeof(double)) : 0;
    if (sp <= 65535 && ws <= kGemvMaxWorkspace) {
      an.gemv = kfast ? 2 : 1;
      an.gemv_split = sp;
      an.gemv_slab = sl;
      an.shortk = an.sk_tiles = an.sk_blocks = an.even = an.even_whole = an.persist = 0;
      p->sk_bytes = ws;
    }
  }
}

comet_status_t build_plan(std::unique_ptr<comet_plan_s> &out, const char *spec, const int64_t *extents,
                          const int64_t *sA, const int64_t *sB, const int64_t *sC, comet_dtype_t dtype,
                          comet_compute_t compute, comet_path_t path, bool tune = true,
                          const TTGTChoice *forced_ttgt = nullptr);
comet_status_t autotune_plan(std::unique_ptr<comet_plan_s> &p, const char *spec, const int64_t *extents,
                             const int64_t *sA, const int64_t *sB, const int64_t *sC);
comet_status_t autotune_ttgt(std::unique_ptr<comet_plan_s> &p, const char *spec, const int64_t *extents,
                             const int64_t *sA, const int64_t *sB, const int64_t *sC);
hipError_t fill_value(void *p, int64_t n, int dt, double value, hipStream_t s);
comet_status_t run_gett(const comet_plan_s *p, double alpha, const void *A, const void *B, double beta, void *C,
                        hipStream_t s, void *ws);
comet_status_t execute(const comet_plan_s *p, double alpha, const void *A, const void *B, double beta, void *C,
                       void *ws, size_t ws_bytes, hipStream_t s);
comet_status_t execute_one(const comet_plan_s *p, double alpha, const void *A, const void *B, double beta, void *C,
                           void *ws, hipStream_t s);

comet_status_t build_ttgt(comet_plan_s *p) {
  Analysis &an = p->an;
  const char *forced = std::getenv("COMET_TTGT_ORDER");
  if (forced && *forced) {
    std::string s(forced);
    size_t a = s.find('|'), b = s.find('|', a == std::string::npos ? 0 : a + 1);
    if (a == std::string::npos || b == std::string::npos)
      return fail(COMET_ERR_INVALID_SPEC, "COMET_TTGT_ORDER must read Aorder|Border|Corder");
    TTGTChoice c;
    c.a_order = s.substr(0, a);
    c.b_order = s.substr(a + 1, b - a - 1);
    c.c_order = s.substr(b + 1);
    auto same_set = [](std::string x, std::string y) {
      std::sort(x.begin(), x.end());
      std::sort(y.begin(), y.end());
      return x == y;
    };
    if (!same_set(c.a_order, an.spec_a) || !same_set(c.b_order, an.spec_b) || !same_set(c.c_order, an.spec_c))
      return fail(COMET_ERR_INVALID_SPEC, "COMET_TTGT_ORDER is not a relabeling of the spec");
    c.a_copy = c.b_copy = c.c_copy = true;
    an.ttgt = c;
  }
  const TTGTChoice &tc = an.ttgt;
  const size_t es = elem_size(an.dtype);
  auto ext_of = [&](char ch) {
    return an.extents[std::find(an.labels.begin(), an.labels.end(), ch) - an.labels.begin()];
  };
  auto exts = [&](const std::string &s) {
    std::vector<int64_t> e;
    for (char ch : s) e.push_back(ext_of(ch));
    return e;
  };
  auto count = [](const std::vector<int64_t> &e) {
    int64_t n = 1;
    for (int64_t x : e) n *= x;
    return n;
  };
  std::vector<int64_t> eA = exts(tc.a_order), eB = exts(tc.b_order), eC = exts(tc.c_order);
  std::vector<int64_t> dA = dense_strides(eA), dB = dense_strides(eB), dC = dense_strides(eC);
  size_t off = 0;
  auto fill_perm = [&](PermuteLaunch &pl, const PermuteDesc &d) {
    pl = PermuteLaunch{};
    pl.ndim = (int)d.ext.size();
    for (int i = 0; i < pl.ndim; ++i) {
      pl.ext[i] = d.ext[i];
      pl.s_in[i] = d.s_in[i];
      pl.s_out[i] = d.s_out[i];
    }
    pl.dtype = an.dtype == COMET_F64 ? 0 : 1;
  };
  if (tc.a_copy) {
    p->wsA = off;
    off += align256(count(eA) * es);
    fill_perm(p->permA, make_permute(tc.a_order, dA, an.spec_a, an.strA, eA));
  }
  if (tc.b_copy) {
    p->wsB = off;
    off += align256(count(eB) * es);
    fill_perm(p->permB, make_permute(tc.b_order, dB, an.spec_b, an.strB, eB));
  }
  if (tc.c_copy) {
    p->wsC = off;
    off += align256(count(eC) * es);
    fill_perm(p->permC, make_permute(an.spec_c, an.strC, tc.c_order, dC, exts(an.spec_c)));
  }
  if (p->permA.ndim > kPermMaxDims || p->permB.ndim > kPermMaxDims || p->permC.ndim > kPermMaxDims)
    return fail(COMET_ERR_UNSUPPORTED, "too many dims for the permute kernel");
  // the GEMM stage: a contraction of the permuted operands, whose gather
  // degenerates to plain row- or column-major matrix access
  std::string gspec = tc.c_order + "=" + tc.a_order + "*" + tc.b_order;
  std::vector<int64_t> gext;
  std::string seen;
  for (const std::string *s : {&tc.c_order, &tc.a_order, &tc.b_order})
    for (char ch : *s)
      if (seen.find(ch) == std::string::npos) {
        seen += ch;
        gext.push_back(ext_of(ch));
      }
  auto reorder = [&](const std::string &to, const std::string &from, const std::vector<int64_t> &s) {
    std::vector<int64_t> r;
    for (char ch : to) r.push_back(s[from.find(ch)]);
    return r;
  };
  std::vector<int64_t> gsA = tc.a_copy ? dA : reorder(tc.a_order, an.spec_a, an.strA);
  std::vector<int64_t> gsB = tc.b_copy ? dB : reorder(tc.b_order, an.spec_b, an.strB);
  std::vector<int64_t> gsC = tc.c_copy ? dC : reorder(tc.c_order, an.spec_c, an.strC);
  comet_status_t rc = build_plan(p->gemm, gspec.c_str(), gext.data(), gsA.data(), gsB.data(), gsC.data(), an.dtype,
                                 an.compute, COMET_PATH_GETT, false);
  if (rc != COMET_OK) return rc;
  p->ws_bytes = off;
  return COMET_OK;
}

comet_status_t build_plan(std::unique_ptr<comet_plan_s> &out, const char *spec, const int64_t *extents,
                          const int64_t *sA, const int64_t *sB, const int64_t *sC, comet_dtype_t dtype,
                          comet_compute_t compute, comet_path_t path, bool tune, const TTGTChoice *forced_ttgt) {
  std::unique_ptr<comet_plan_s> p(new comet_plan_s());
  Status st = analyze(spec, extents, sA, sB, sC, dtype, compute, path, g_split_slices, p->an, g_int8_slices);
  if (!st.ok()) return fail(st);
  Analysis &an = p->an;
  if (forced_ttgt && an.path == COMET_PATH_TTGT) an.ttgt = *forced_ttgt;
  HIP_TRY(hipGetDevice(&p->device), "hipGetDevice");
  int cus = 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess) cus = 256;
  if (an.path == COMET_PATH_TTGT && !an.empty_out && !an.empty_sum) {
    comet_status_t rc = build_ttgt(p.get());
    if (rc != COMET_OK) return rc;
  }
  comet_status_t rc = upload_tables(p.get());
  if (rc != COMET_OK) return rc;
  const int VEC = an.dtype == COMET_F64 ? 2 : 4;
  // with batch labels every entry's base offset keeps the alignment too
  auto all_vec = [&](const std::vector<int64_t> &x) {
    for (int64_t v : x)
      if (v % VEC) return false;
    return true;
  };
  p->vecA_tables = tables_vec_ok(an.offAm, an.offAk, an.layoutA, an.runAm, an.runAk, VEC) && all_vec(an.offAx);
  p->vecB_tables = tables_vec_ok(an.offBn, an.offBk, an.layoutB, an.runBn, an.runBk, VEC) && all_vec(an.offBx);
  const bool native = an.compute == COMET_COMPUTE_F64 || an.compute == COMET_COMPUTE_F32;
  // Only tile 1's element-load kernel can gather these operands (their unit
  // strides lie on different summation labels, or runs are ragged): when the
  // estimate says the permutes of TTGT cost less than that kernel, take TTGT.
  // This is the untuned default only: with the autotuner on it times both
  // (or reads its cache), and a forced gather schedule keeps the gather path.
  const bool tuning = tune && tune_cache().mode() != 0;
  const bool gather_forced = std::getenv("COMET_GETT_TILE") || std::getenv("COMET_GETT_SK") ||
                             std::getenv("COMET_GETT_PERSIST") || std::getenv("COMET_GETT_EVEN");
  if (path == COMET_PATH_AUTO && native && !tuning && !gather_forced && an.path == COMET_PATH_GETT &&
      an.X.empty() && !an.empty_out && !an.empty_sum && !(p->vecA_tables && p->vecB_tables)) {
    std::unique_ptr<comet_plan_s> tt;
    if (build_plan(tt, spec, extents, sA, sB, sC, dtype, compute, COMET_PATH_TTGT, false) == COMET_OK && tt->gemm &&
        tt->ws_bytes <= kTTGTMaxWorkspace && ttgt_saving_s(an, *tt) > 0.0) {
      out = std::move(tt);
      return COMET_OK;
    }
  }
  apply_schedule(p.get(), cus);
  if (p->gemm) {
    apply_schedule(p->gemm.get(), cus);
    p->gemm->ws_bytes = p->gemm->sk_bytes;
    p->wsG = p->ws_bytes;
    p->ws_bytes += p->gemm->ws_bytes;
  } else if (an.path == COMET_PATH_GETT) {
    p->ws_bytes = p->sk_bytes;
  }
  bool split = an.compute == COMET_COMPUTE_SPLIT_BF16 || an.compute == COMET_COMPUTE_SPLIT_BF16X3 ||
               an.compute == COMET_COMPUTE_SPLIT_FP16X2 || an.compute == COMET_COMPUTE_SPLIT_INT8;
  // FP32 storage in BF16x3: split on the fly inside the gather kernel
  // (small products; large ones slice into the workspace first and run the
  // slice-pair product, whose 192 x 192 tile does more MFMA work per LDS byte:
  // on MI355X the fused kernel wins up to about 1024^3 and loses 2.4x at the
  // 3072^3 CCSD-like contraction; COMET_FUSED3=0/1 overrides)
  p->fused3 = an.compute == COMET_COMPUTE_SPLIT_BF16X3 && an.dtype == COMET_F32 &&
              double(an.m) * double(an.n) * double(an.k) * double(an.nb) < kFused3MaxMNK;
  if (an.compute == COMET_COMPUTE_SPLIT_BF16X3 && an.dtype == COMET_F32) {
    const char *env = std::getenv("COMET_FUSED3");
    if (env && *env) p->fused3 = std::atoi(env) != 0;
  }
  if (split && !p->fused3 && !an.empty_out && !an.empty_sum) {
    Status s2 = split_prepare(an, p->split);
    if (!s2.ok()) return fail(s2);
    p->ws_bytes = p->split.ws_bytes;
  }
  if (tune && path == COMET_PATH_AUTO) {
    comet_status_t rc2 = autotune_plan(p, spec, extents, sA, sB, sC);
    if (rc2 != COMET_OK) return rc2;
  }
  // TTGT asked for, tuning on, no flattening forced: time the flattenings
  if (tune && path == COMET_PATH_TTGT && an.path == COMET_PATH_TTGT && tuning && native && !forced_ttgt &&
      !std::getenv("COMET_TTGT_ORDER") && !an.empty_out && !an.empty_sum && an.X.empty()) {
    comet_status_t rc2 = autotune_ttgt(p, spec, extents, sA, sB, sC);
    if (rc2 != COMET_OK) return rc2;
  }
  out = std::move(p);
  return COMET_OK;
}

// ws: the plan's stream-K workspace (sk_bytes), unused without a split
comet_status_t run_gett(const comet_plan_s *p, double alpha, const void *A, const void *B, double beta, void *C,
                        hipStream_t s, void *ws) {
  const Analysis &an = p->an;
  if (an.gemv > 0) {
    // the kernel's A operand (B when exchanged) is the vector: M == 1
    GemvLaunch v{};
    v.X = an.swapped ? B : A;
    v.Y = an.swapped ? A : B;
    v.C = C;
    v.offXk = p->t.offAk;
    v.offX0 = p->t.offAm;
    v.offYk = p->t.offBk;
    v.offYj = p->t.offBn;
    v.offC0 = p->t.offCm;
    v.offCj = p->t.offCn;
    v.J = an.n;
    v.K = an.k;
    v.split = an.gemv_split;
    v.slab = an.gemv_slab;
    v.kfast = an.gemv == 2;
    v.dtype = an.dtype == COMET_F64 ? 0 : 1;
    v.alpha = alpha;
    v.beta = beta;
    v.ws = ws;
    HIP_TRY(launch_gemv(v, s), "matrix-vector launch");
    return COMET_OK;
  }
  GettLaunch g{};
  g.A = an.swapped ? B : A;
  g.B = an.swapped ? A : B;
  g.C = C;
  g.t = p->t;
  g.M = an.m;
  g.N = an.n;
  g.K = an.k;
  g.alpha = alpha;
  g.beta = beta;
  g.dtype = an.dtype == COMET_F64 ? 0 : 1;
  g.compute = an.compute == COMET_COMPUTE_F64 ? 0 : 1;
  g.layoutA = an.layoutA;
  g.layoutB = an.layoutB;
  g.vecA = p->vecA_tables && (reinterpret_cast<uintptr_t>(g.A) % 16 == 0);
  g.vecB = p->vecB_tables && (reinterpret_cast<uintptr_t>(g.B) % 16 == 0);
  g.tile = an.tile;
  // misaligned pointers or a tile not built for this dtype pair: the 64 x 64
  // tile has every variant
  if (!gett_tile_valid(g.tile, g.dtype, g.compute, g.vecA, g.vecB, p->offAx != nullptr)) g.tile = 1;
  if (an.sk_tiles > 0 && g.tile == an.tile && ws) {
    g.sk.tiles = an.sk_tiles;
    g.sk.blocks = an.sk_blocks;
    g.sk.ws = ws;
    // the balanced schedule reads vectors: with a misaligned operand every
    // tile is computed whole
    if (an.even && g.vecA && g.vecB) {
      g.sk.even = 1;
      g.sk.whole = an.even_whole;
    } else if (an.even) {
      g.sk = StreamK{};
    }
  }
  if (an.persist > 0 && g.tile == an.tile) g.persistent = an.persist;
  if (an.shortk > 0 && g.tile == an.tile && g.vecA && g.vecB) g.shortk = an.shortk;
  if (p->offAx) {
    g.bt.offA = p->offAx;
    g.bt.offB = p->offBx;
    g.bt.offC = p->offCx;
    g.bt.count = an.nb;
    g.sk = StreamK{};
    g.persistent = 0;
    g.shortk = 0;
  }
  HIP_TRY(launch_gett(g, s), "gett launch");
  return COMET_OK;
}

comet_status_t execute(const comet_plan_s *p, double alpha, const void *A, const void *B, double beta, void *C,
                       void *ws, size_t ws_bytes, hipStream_t s) {
  const Analysis &an = p->an;
  if (an.empty_out) return COMET_OK;
  if (!C) return fail(COMET_ERR_NULL_POINTER, "C is NULL");
  if (alpha != 0.0 && !an.empty_sum && (!A || !B)) return fail(COMET_ERR_NULL_POINTER, "A or B is NULL");
  if (alpha != 0.0 && !an.empty_sum && (C == A || C == B))
    return fail(COMET_ERR_UNSUPPORTED, "C aliases an input");
  if (an.dtype == COMET_F32) {
    alpha = double(float(alpha));
    beta = double(float(beta));
  }
  if (alpha == 0.0 || an.empty_sum) {
    HIP_TRY(launch_scale(C, an.dtype == COMET_F64 ? 0 : 1, p->t.offCm, p->t.offCn, an.m, an.n, beta, s, p->offCx,
                         an.nb),
            "scale");
    return COMET_OK;
  }
  if (p->ws_bytes > 0 && (!ws || ws_bytes < p->ws_bytes))
    return fail(COMET_ERR_WORKSPACE, "workspace smaller than comet_plan_workspace_size");
  const bool split = an.compute == COMET_COMPUTE_SPLIT_BF16 || an.compute == COMET_COMPUTE_SPLIT_BF16X3 ||
                     an.compute == COMET_COMPUTE_SPLIT_FP16X2 || an.compute == COMET_COMPUTE_SPLIT_INT8;
  if (!an.offAx.empty() && (p->fused3 || split)) {
    // batch labels on the split and fused BF16x3 paths: one contraction per
    // batch entry, in order on the stream (they share the workspace)
    const size_t es = elem_size(an.dtype);
    const int64_t *xa = an.swapped ? an.offBx.data() : an.offAx.data();
    const int64_t *xb = an.swapped ? an.offAx.data() : an.offBx.data();
    for (int64_t e = 0; e < an.nb; ++e) {
      comet_status_t rc = execute_one(p, alpha, static_cast<const char *>(A) + xa[e] * es,
                                      static_cast<const char *>(B) + xb[e] * es, beta,
                                      static_cast<char *>(C) + an.offCx[e] * es, ws, s);
      if (rc != COMET_OK) return rc;
    }
    return COMET_OK;
  }
  return execute_one(p, alpha, A, B, beta, C, ws, s);
}

// One batch entry (the whole contraction without batch labels) after the
// checks of execute().
comet_status_t execute_one(const comet_plan_s *p, double alpha, const void *A, const void *B, double beta, void *C,
                           void *ws, hipStream_t s) {
  const Analysis &an = p->an;
  if (p->fused3) {
    GettLaunch g{};
    g.A = an.swapped ? B : A;
    g.B = an.swapped ? A : B;
    g.C = C;
    g.t = p->t;
    g.M = an.m;
    g.N = an.n;
    g.K = an.k;
    g.alpha = alpha;
    g.beta = beta;
    g.dtype = 1;
    g.layoutA = an.layoutA;
    g.layoutB = an.layoutB;
    g.vecA = g.vecB = p->vecA_tables && p->vecB_tables && reinterpret_cast<uintptr_t>(g.A) % 16 == 0 &&
                      reinterpret_cast<uintptr_t>(g.B) % 16 == 0;
    HIP_TRY(launch_fused_bf16x3(g, s), "fused BF16x3 launch");
    return COMET_OK;
  }
  if (an.compute == COMET_COMPUTE_SPLIT_BF16 || an.compute == COMET_COMPUTE_SPLIT_BF16X3 ||
      an.compute == COMET_COMPUTE_SPLIT_FP16X2 || an.compute == COMET_COMPUTE_SPLIT_INT8) {
    const void *Ak = an.swapped ? B : A, *Bk = an.swapped ? A : B;
    HIP_TRY(split_execute(an, p->split, p->t, alpha, Ak, Bk, beta, C, ws, s, p->vecA_tables, p->vecB_tables),
            "split launch");
    return COMET_OK;
  }
  if (an.path == COMET_PATH_TTGT) {
    const TTGTChoice &tc = an.ttgt;
    char *w = static_cast<char *>(ws);
    const void *Ap = A, *Bp = B;
    if (tc.a_copy) {
      PermuteLaunch pl = p->permA;
      pl.in = A;
      pl.out = w + p->wsA;
      pl.alpha = 1.0;
      pl.beta = 0.0;
      HIP_TRY(launch_permute(pl, s), "permute A");
      Ap = pl.out;
    }
    if (tc.b_copy) {
      PermuteLaunch pl = p->permB;
      pl.in = B;
      pl.out = w + p->wsB;
      pl.alpha = 1.0;
      pl.beta = 0.0;
      HIP_TRY(launch_permute(pl, s), "permute B");
      Bp = pl.out;
    }
    if (tc.c_copy) {
      comet_status_t rc = run_gett(p->gemm.get(), alpha, Ap, Bp, 0.0, w + p->wsC, s, w + p->wsG);
      if (rc != COMET_OK) return rc;
      PermuteLaunch pl = p->permC;
      pl.in = w + p->wsC;
      pl.out = C;
      pl.alpha = 1.0;
      pl.beta = beta;
      HIP_TRY(launch_permute(pl, s), "permute C");
      return COMET_OK;
    }
    return run_gett(p->gemm.get(), alpha, Ap, Bp, beta, C, s, w + p->wsG);
  }
  return run_gett(p, alpha, A, B, beta, C, s, ws);
}

// ---- autotuning -------------------------------------------------------------

std::string arch_id(int device) {
  hipDeviceProp_t prop;
  int rt = 0;
  std::string a = "dev";
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) a = prop.gcnArchName;
  if (hipRuntimeGetVersion(&rt) == hipSuccess) a += "/hip" + std::to_string(rt);
  for (char &c : a)
    if (c == '"' || c == '\\') c = '_';
  return a;
}

// Time fn on stream s: one warm-up, then the best of kTimedReps runs
// (microseconds).
constexpr int kTimedReps = 5;

template <typename F>
double time_us(F fn, hipStream_t s, bool *ok) {
  hipEvent_t e0, e1;
  *ok = false;
  if (hipEventCreate(&e0) != hipSuccess) return 0;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return 0;
  }
  double best = 1e30;
  bool good = fn() == COMET_OK;
  for (int r = 0; good && r < kTimedReps; ++r) {
    (void)hipEventRecord(e0, s);
    good = fn() == COMET_OK;
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) good = false;
    float ms = 0;
    if (good && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) best = std::min(best, double(ms) * 1e3);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ok = good && best < 1e30;
  return best;
}

// The split products: time the slice-pair product's tiles -- 128 x 64 and
// 192 x 192 for the classic splits (BF16x3, FP16x2) and, for FP32 storage in
// BF16x3, the fused kernel; 128 x 64 and 128 x 96 for the aligned BF16
// slices -- and record the fastest (entry tile 0, 1, or 2 for the fused
// kernel or the 128 x 96 tile) per problem class and apply it.  Called with
// the cache lock held.
comet_status_t autotune_split(comet_plan_s *p, TuneCache &tc) {
  Analysis &an = p->an;
  const std::string key = tune_key(an, arch_id(p->device));
  const bool can_fuse = an.compute == COMET_COMPUTE_SPLIT_BF16X3 && an.dtype == COMET_F32;
  const bool aligned = an.compute == COMET_COMPUTE_SPLIT_BF16;
  auto apply = [&](int choice) -> comet_status_t {
    p->fused3 = choice == 2 && can_fuse;
    if (p->fused3) {
      p->split = SplitPlan();
      p->ws_bytes = 0;
      return COMET_OK;
    }
    Status st = split_prepare(an, p->split, choice < 0 ? -1 : aligned ? choice : choice == 1 ? 1 : 0);
    if (!st.ok()) return fail(st);
    p->ws_bytes = p->split.ws_bytes;
    return COMET_OK;
  };
  TuneEntry best;
  if (tc.mode() == 1 && tc.lookup(key, &best) && best.tile >= 0 && best.tile <= 2) return apply(best.tile);
  const size_t es = elem_size(an.dtype);
  const int dt = an.dtype == COMET_F64 ? 0 : 1;
  void *bufA = nullptr, *bufB = nullptr, *bufC = nullptr, *ws = nullptr;
  size_t wsb = 0;
  hipStream_t s = nullptr;
  bool ok = hipStreamCreate(&s) == hipSuccess && hipMalloc(&bufA, std::max<int64_t>(an.sizeA, 1) * es) == hipSuccess &&
            hipMalloc(&bufB, std::max<int64_t>(an.sizeB, 1) * es) == hipSuccess &&
            hipMalloc(&bufC, std::max<int64_t>(an.sizeC, 1) * es) == hipSuccess;
  best = TuneEntry{-1, COMET_PATH_GETT, 1e30};
  if (ok) {
    (void)fill_value(bufA, std::max<int64_t>(an.sizeA, 1), dt, 0.5, s);
    (void)fill_value(bufB, std::max<int64_t>(an.sizeB, 1), dt, -0.25, s);
    for (int choice = 0; choice <= (can_fuse || aligned ? 2 : 1); ++choice) {
      if (aligned && choice == 1) continue;
      if (apply(choice) != COMET_OK) continue;
      // (a tile the problem cannot take falls back to 128 x 64: time it once)
      if (aligned && choice == 2 && p->split.tile != 2) continue;
      if (p->ws_bytes > wsb) {
        if (ws) (void)hipFree(ws);
        ws = nullptr;
        wsb = 0;
        if (hipMalloc(&ws, p->ws_bytes) != hipSuccess) continue;
        wsb = p->ws_bytes;
      }
      bool good;
      const comet_plan_s *pp = p;
      const double us = time_us([&]() { return execute(pp, 1.0, bufA, bufB, 0.0, bufC, ws, wsb, s); }, s, &good);
      if (good && us < best.us) best = TuneEntry{choice, COMET_PATH_GETT, us};
    }
    (void)hipStreamSynchronize(s);
  }
  if (bufA) (void)hipFree(bufA);
  if (bufB) (void)hipFree(bufB);
  if (bufC) (void)hipFree(bufC);
  if (ws) (void)hipFree(ws);
  if (s) (void)hipStreamDestroy(s);
  if (best.tile < 0) {
    // tuning not possible: the size rule's choice
    p->fused3 = can_fuse && double(an.m) * double(an.n) * double(an.k) * double(an.nb) < kFused3MaxMNK;
    return apply(p->fused3 ? 2 : -1);
  }
  tc.store(key, best);
  return apply(best.tile);
}

// A plan that asks for TTGT, with the autotuner on: time every flattening
// with beta = 0 and with beta = 1 (up to kTuneTTGTAll; the fastest few
// twice more), record the fastest per
// problem class (the tuning key with "/ttgt") and rebuild the plan with it.
// On MI355X the Section 6
// cost model does not order the flattenings of the CCSD-like contractions
// (its pick is among the slowest), so the flattening is measured, as the
// gather tiles are.  Keeps the model's flattening when timing is not
// possible.
comet_status_t autotune_ttgt(std::unique_ptr<comet_plan_s> &p, const char *spec, const int64_t *extents,
                             const int64_t *sA, const int64_t *sB, const int64_t *sC) {
  Analysis &an = p->an;
  TuneCache &tc = tune_cache();
  std::lock_guard<std::mutex> lk(tc.mutex());
  const std::string key = tune_key(an, arch_id(p->device)) + "/ttgt";
  std::vector<TTGTChoice> cands = ttgt_candidates(an);
  TuneEntry best;
  if (!(tc.mode() == 1 && tc.lookup(key, &best) && best.path == COMET_PATH_TTGT)) {
    if (cands.size() > size_t(kTuneTTGTAll)) cands.resize(kTuneTTGTAll);
    const size_t es = elem_size(an.dtype);
    void *bufA = nullptr, *bufB = nullptr, *bufC = nullptr, *ws = nullptr;
    size_t wsb = 0;
    hipStream_t s = nullptr;
    bool ok = hipStreamCreate(&s) == hipSuccess && hipMalloc(&bufA, std::max<int64_t>(an.sizeA, 1) * es) == hipSuccess &&
              hipMalloc(&bufB, std::max<int64_t>(an.sizeB, 1) * es) == hipSuccess &&
              hipMalloc(&bufC, std::max<int64_t>(an.sizeC, 1) * es) == hipSuccess;
    best = TuneEntry{-1, COMET_PATH_TTGT, 1e30};
    if (ok) {
      const int dt = an.dtype == COMET_F64 ? 0 : 1;
      (void)fill_value(bufA, std::max<int64_t>(an.sizeA, 1), dt, 0.5, s);
      (void)fill_value(bufB, std::max<int64_t>(an.sizeB, 1), dt, -0.25, s);
      (void)fill_value(bufC, std::max<int64_t>(an.sizeC, 1), dt, 0.125, s);
      // every flattening once, then the fastest few again (their times lie
      // within a few percent of each other)
      std::vector<std::pair<double, size_t>> timed;
      auto time_choice = [&](size_t i, bool *good) -> double {
        std::unique_ptr<comet_plan_s> cp;
        *good = false;
        if (build_plan(cp, spec, extents, sA, sB, sC, an.dtype, an.compute, COMET_PATH_TTGT, false, &cands[i]) !=
            COMET_OK)
          return 0.0;
        if (cp->ws_bytes > wsb) {
          if (ws) (void)hipFree(ws);
          ws = nullptr;
          wsb = 0;
          if (hipMalloc(&ws, cp->ws_bytes) != hipSuccess) return 0.0;
          wsb = cp->ws_bytes;
        }
        // a plan serves any beta, and whether C is read changes which
        // flattening is fastest: the score is the sum over beta = 0 and 1
        const comet_plan_s *pt = cp.get();
        bool g1;
        const double t0 = time_us([&]() { return execute(pt, 1.0, bufA, bufB, 0.0, bufC, ws, wsb, s); }, s, good);
        const double t1 = time_us([&]() { return execute(pt, 1.0, bufA, bufB, 1.0, bufC, ws, wsb, s); }, s, &g1);
        *good = *good && g1;
        return t0 + t1;
      };
      for (size_t i = 0; i < cands.size(); ++i) {
        bool good;
        const double us = time_choice(i, &good);
        if (good) timed.emplace_back(us, i);
      }
      std::sort(timed.begin(), timed.end());
      if (timed.size() > size_t(kTuneTTGTRetime)) timed.resize(kTuneTTGTRetime);
      for (auto &tm : timed) {
        for (int r = 0; r < 2; ++r) {
          bool good;
          const double us = time_choice(tm.second, &good);
          if (good) tm.first = std::min(tm.first, us);
        }
        const TTGTChoice &ch = cands[tm.second];
        if (tm.first < best.us)
          best = TuneEntry{0, COMET_PATH_TTGT, tm.first, ch.a_order + "|" + ch.b_order + "|" + ch.c_order};
      }
      (void)hipStreamSynchronize(s);
    }
    if (bufA) (void)hipFree(bufA);
    if (bufB) (void)hipFree(bufB);
    if (bufC) (void)hipFree(bufC);
    if (ws) (void)hipFree(ws);
    if (s) (void)hipStreamDestroy(s);
    if (!ok || best.us >= 1e30) return COMET_OK;
    tc.store(key, best);
    cands = ttgt_candidates(an);
  }
  for (const TTGTChoice &ch : cands) {
    if (ch.a_order + "|" + ch.b_order + "|" + ch.c_order != best.ttgt) continue;
    std::unique_ptr<comet_plan_s> tt;
    if (build_plan(tt, spec, extents, sA, sB, sC, an.dtype, an.compute, COMET_PATH_TTGT, false, &ch) == COMET_OK)
      p = std::move(tt);
    break;
  }
  return COMET_OK;
}

comet_status_t autotune_plan(std::unique_ptr<comet_plan_s> &p, const char *spec, const int64_t *extents,
                             const int64_t *sA, const int64_t *sB, const int64_t *sC) {
  Analysis &an = p->an;
  TuneCache &tc = tune_cache();
  std::lock_guard<std::mutex> lk(tc.mutex());
  int cus = 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess) cus = 256;
  const bool native = an.compute == COMET_COMPUTE_F64 || an.compute == COMET_COMPUTE_F32;
  const bool classic = an.compute == COMET_COMPUTE_SPLIT_BF16X3 || an.compute == COMET_COMPUTE_SPLIT_FP16X2 ||
                       an.compute == COMET_COMPUTE_SPLIT_BF16;
  if (tc.mode() != 0 && classic && !an.empty_out && !an.empty_sum && an.X.empty() && !std::getenv("COMET_SPLIT_TILE") &&
      !std::getenv("COMET_FUSED3"))
    return autotune_split(p.get(), tc);
  if (tc.mode() == 0 || !native || an.empty_out || an.empty_sum) return COMET_OK;
  // a matrix times a vector streams the matrix once: nothing to time
  if (an.gemv > 0) return COMET_OK;
  if (std::getenv("COMET_GETT_TILE") || std::getenv("COMET_FORCE_PATH") || std::getenv("COMET_GETT_SK") ||
      std::getenv("COMET_GETT_PERSIST") || std::getenv("COMET_GETT_EVEN"))
    return COMET_OK;
  const std::string key = tune_key(an, arch_id(p->device));
  TuneEntry best;
  if (!(tc.mode() == 1 && tc.lookup(key, &best))) {
    // time every compiled tile variant of the gather path, and the TTGT lowering
    const size_t es = elem_size(an.dtype);
    void *bufA = nullptr, *bufB = nullptr, *bufC = nullptr, *ws = nullptr;
    hipStream_t s = nullptr;
    std::unique_ptr<comet_plan_s> tt;
    if (an.X.empty()) {   // the TTGT lowering has no batch labels
      comet_status_t rc = build_plan(tt, spec, extents, sA, sB, sC, an.dtype, an.compute, COMET_PATH_TTGT, false);
      if (rc != COMET_OK) tt.reset();
    }
    size_t wsb = tt ? tt->ws_bytes : 0;
    bool ok = hipStreamCreate(&s) == hipSuccess && hipMalloc(&bufA, std::max<int64_t>(an.sizeA, 1) * es) == hipSuccess &&
              hipMalloc(&bufB, std::max<int64_t>(an.sizeB, 1) * es) == hipSuccess &&
              hipMalloc(&bufC, std::max<int64_t>(an.sizeC, 1) * es) == hipSuccess &&
              (wsb == 0 || hipMalloc(&ws, wsb) == hipSuccess);
    if (ok) {
      // nonzero operands (the time of a product does not depend on the values,
      // but zeros could take shortcuts in future kernels)
      (void)fill_value(bufA, std::max<int64_t>(an.sizeA, 1), an.dtype == COMET_F64 ? 0 : 1, 0.5, s);
      (void)fill_value(bufB, std::max<int64_t>(an.sizeB, 1), an.dtype == COMET_F64 ? 0 : 1, -0.25, s);
      best.us = 1e30;
      void *skws = nullptr;
      size_t skws_bytes = 0;
      for (int tile = 0; tile < gett_tile_count(); ++tile) {
        if (!gett_tile_valid(tile, an.dtype == COMET_F64 ? 0 : 1, an.compute == COMET_COMPUTE_F64 ? 0 : 1,
                             p->vecA_tables, p->vecB_tables, !an.X.empty()))
          continue;
        // each tile with its own stream-K split
        apply_schedule(p.get(), cus, tile);
        if (p->sk_bytes > skws_bytes) {
          if (skws) (void)hipFree(skws);
          skws = nullptr;
          skws_bytes = 0;
          if (hipMalloc(&skws, p->sk_bytes) != hipSuccess) {
            skws = nullptr;
            continue;
          }
          skws_bytes = p->sk_bytes;
        }
        bool good;
        const comet_plan_s *pp = p.get();
        double us = time_us([&]() { return run_gett(pp, 1.0, bufA, bufB, 0.0, bufC, s, skws); }, s, &good);
        if (good && us < best.us) best = TuneEntry{tile, COMET_PATH_GETT, us};
      }
      if (tt) {
        // every TTGT flattening, cheapest by the cost model first, up to
        // kTuneTTGT of them (the model ranks them poorly on MI355X, so it only
        // orders the search)
        std::vector<TTGTChoice> cands = ttgt_candidates(tt->an);
        if (cands.size() > size_t(kTuneTTGT)) cands.resize(kTuneTTGT);
        for (const TTGTChoice &ch : cands) {
          std::unique_ptr<comet_plan_s> cp;
          if (build_plan(cp, spec, extents, sA, sB, sC, an.dtype, an.compute, COMET_PATH_TTGT, false, &ch) !=
              COMET_OK)
            continue;
          if (cp->ws_bytes > wsb) {
            if (ws) (void)hipFree(ws);
            ws = nullptr;
            wsb = 0;
            if (hipMalloc(&ws, cp->ws_bytes) != hipSuccess) {
              ws = nullptr;
              continue;
            }
            wsb = cp->ws_bytes;
          }
          bool good;
          const comet_plan_s *pt = cp.get();
          double us = time_us([&]() { return execute(pt, 1.0, bufA, bufB, 0.0, bufC, ws, wsb, s); }, s, &good);
          if (good && us < best.us) {
            best = TuneEntry{cp->gemm ? cp->gemm->an.tile : 0, COMET_PATH_TTGT, us,
                             ch.a_order + "|" + ch.b_order + "|" + ch.c_order};
          }
        }
      }
      (void)hipStreamSynchronize(s);
      if (skws) (void)hipFree(skws);
      apply_schedule(p.get(), cus);
    }
    if (bufA) (void)hipFree(bufA);
    if (bufB) (void)hipFree(bufB);
    if (bufC) (void)hipFree(bufC);
    if (ws) (void)hipFree(ws);
    if (s) (void)hipStreamDestroy(s);
    if (!ok || best.us >= 1e30) return COMET_OK;   // tuning not possible: keep the heuristic
    tc.store(key, best);
  }
  if (best.path == COMET_PATH_TTGT) {
    // the recorded flattening, if it is still one of this problem's
    const TTGTChoice *forced = nullptr;
    std::vector<TTGTChoice> cands = ttgt_candidates(an);
    for (const TTGTChoice &ch : cands)
      if (ch.a_order + "|" + ch.b_order + "|" + ch.c_order == best.ttgt) forced = &ch;
    std::unique_ptr<comet_plan_s> tt;
    comet_status_t rc =
        build_plan(tt, spec, extents, sA, sB, sC, an.dtype, an.compute, COMET_PATH_TTGT, false, forced);
    if (rc == COMET_OK) {
      p = std::move(tt);
      return COMET_OK;
    }
  }
  if (best.tile >= 0 && best.tile < gett_tile_count()) {
    apply_schedule(p.get(), cus, best.tile);
    p->ws_bytes = p->sk_bytes;
  }
  return COMET_OK;
}

// ---- batch: dense copies for element-load problems --------------------------

// A problem whose operands only the element-load kernel can gather (their
// unit strides lie on different summation labels, or runs are ragged) gets a
// dense copy of one operand X (the smaller first) in a label order that makes
// both operands readable in vectors: X's free labels in their order, then
// the summation labels in the order of the other operand's strides (so both
// share the unit-stride summation label), or the summation labels first.
// The copy's analysis replaces the problem's; `which` is 0 for A, 1 for B.
struct BatchCopy {
  int which = -1;
  std::string order;            // labels of the copy, outermost first
  std::vector<int64_t> ext;     // their extents
  int64_t count = 0;            // elements
};

bool batch_copy_choice(const comet_problem_t &pr, const Analysis &a, comet_dtype_t dtype, comet_compute_t compute,
                       int VEC, Analysis &out, BatchCopy &cp) {
  if (!a.X.empty() || a.empty_out || a.empty_sum) return false;
  const std::string &la = a.spec_a, &lb = a.spec_b, &lc = a.spec_c;
  auto ext_of = [&](char ch) {
    return a.extents[std::find(a.labels.begin(), a.labels.end(), ch) - a.labels.begin()];
  };
  auto strides_of = [&](const std::string &l, const int64_t *given) {
    std::vector<int64_t> e;
    for (char ch : l) e.push_back(ext_of(ch));
    return given ? std::vector<int64_t>(given, given + l.size()) : dense_strides(e);
  };
  const std::vector<int64_t> sa = strides_of(la, pr.strides_A), sb = strides_of(lb, pr.strides_B);
  const std::vector<int64_t> sc = strides_of(lc, pr.strides_C);
  auto count = [&](const std::string &l) {
    int64_t n = 1;
    for (char ch : l) n *= ext_of(ch);
    return n;
  };
  const int first = count(la) <= count(lb) ? 0 : 1;
  for (int t = 0; t < 2; ++t) {
    const int which = t == 0 ? first : 1 - first;
    const std::string &lx = which == 0 ? la : lb, &ly = which == 0 ? lb : la;
    const std::vector<int64_t> &sx = which == 0 ? sa : sb, &sy = which == 0 ? sb : sa;
    // X's free labels by X's strides, summation labels by Y's, outermost first
    std::vector<std::pair<int64_t, char>> fx, ky;
    for (size_t q = 0; q < lx.size(); ++q)
      if (lc.find(lx[q]) != std::string::npos) fx.push_back({-sx[q], lx[q]});
    for (size_t q = 0; q < ly.size(); ++q)
      if (lx.find(ly[q]) != std::string::npos && lc.find(ly[q]) == std::string::npos) ky.push_back({-sy[q], ly[q]});
    std::stable_sort(fx.begin(), fx.end());
    std::stable_sort(ky.begin(), ky.end());
    std::string f, k;
    for (auto &v : fx) f += v.second;
    for (auto &v : ky) k += v.second;
    for (const std::string &order : {f + k, k + f}) {
      std::vector<int64_t> e;
      for (char ch : order) e.push_back(ext_of(ch));
      const std::vector<int64_t> d = dense_strides(e);
      std::vector<int64_t> sxn(lx.size());
      for (size_t q = 0; q < lx.size(); ++q) sxn[q] = d[order.find(lx[q])];
      Analysis na;
      const Status st = analyze(pr.spec, pr.extents, which == 0 ? sxn.data() : sa.data(),
                                which == 1 ? sxn.data() : sb.data(), sc.data(), dtype, compute, COMET_PATH_GETT,
                                g_split_slices, na, g_int8_slices);
      if (!st.ok()) continue;
      if (tables_vec_ok(na.offAm, na.offAk, na.layoutA, na.runAm, na.runAk, VEC) &&
          tables_vec_ok(na.offBn, na.offBk, na.layoutB, na.runBn, na.runBk, VEC)) {
        out = na;
        cp.which = which;
        cp.order = order;
        cp.ext = e;
        cp.count = count(lx);
        return true;
      }
    }
  }
  return false;
}

// ---- batch tile classes -------------------------------------------------------

// Output elements per unit time of each batch tile class relative to the
// 64 x 64 class, for the native and the fused BF16x3 kernels (the untuned
// choice; the autotuner replaces it with timings).
constexpr double kBatchRateNative[kBatchClasses] = {1.0, 1.12, 1.12, 1.25};
constexpr double kBatchRateFused[kBatchClasses] = {1.0, 1.3, 1.3, 1.7};

// Modeled time of a descriptor in class `cls`: its padded output area times
// its summation length over the class's rate.
double batch_class_cost(const BatchDesc &d, int cls, int mode) {
  int bm, bn;
  batch_class_shape(cls, &bm, &bn);
  const double area = double((d.M + bm - 1) / bm) * bm * double((d.N + bn - 1) / bn) * bn;
  return area * double(d.K) / (mode == 1 ? kBatchRateFused[cls] : kBatchRateNative[cls]);
}

int batch_model_class(const BatchDesc &d, int dt, int mode) {
  const bool vec = d.variant < 4;
  int best = 0;
  double bc = batch_class_cost(d, 0, mode);
  for (int c = 1; c < kBatchClasses; ++c) {
    if (!batch_class_valid(c, dt, mode, vec)) continue;
    const double x = batch_class_cost(d, c, mode);
    if (x < bc * 0.999) {
      best = c;
      bc = x;
    }
  }
  return best;
}

comet_status_t batch_tune_classes(const std::vector<Analysis> &an, const std::vector<int64_t> &first,
                                  const std::vector<char> &live, std::vector<BatchDesc> &descs, int dt, int mode);

// The tile class of every live descriptor: COMET_BATCH_CLASS forces one
// (where it exists for the descriptor), else the autotuner's timings when it
// is on, else the model.
comet_status_t batch_choose_classes(const std::vector<Analysis> &an, const std::vector<int64_t> &first,
                                    const std::vector<char> &live, std::vector<BatchDesc> &descs, int dt,
                                    int mode) {
  const char *env = std::getenv("COMET_BATCH_CLASS");
  const int forced = (env && *env) ? std::atoi(env) : -1;
  for (size_t j = 0; j < descs.size(); ++j) {
    BatchDesc &d = descs[j];
    if (!live[j]) continue;
    if (forced >= 0)
      d.cls = batch_class_valid(forced, dt, mode, d.variant < 4) ? forced : 0;
    else
      d.cls = batch_model_class(d, dt, mode);
  }
  if (forced < 0 && tune_cache().mode() != 0) return batch_tune_classes(an, first, live, descs, dt, mode);
  return COMET_OK;
}

// Fill n elements of dtype dt at p with `value` (the fill form of the
// permute kernel), so that timed runs see nonzero operands.
hipError_t fill_value(void *p, int64_t n, int dt, double value, hipStream_t s) {
  PermuteLaunch pl{};
  pl.ndim = 1;
  pl.ext[0] = n;
  pl.s_in[0] = pl.s_out[0] = 1;
  pl.in = pl.out = p;
  pl.alpha = pl.beta = 0.0;
  pl.dtype = dt;
  pl.fill = value;
  return launch_permute(pl, s);
}

// Time every tile class that exists for the live descriptors' problem
// classes the cache does not hold (or all, in mode 2) and record the fastest.
// A class is timed on a batch of R copies of the problem's first live
// descriptor (operands filled with nonzero values, alpha 1, beta 0, every
// copy writing the same output), R chosen so that the copies' tiles fill
// several rounds of the persistent grid: the per-problem time then measures
// the class's throughput inside a full GPU, as in the batch, not the latency
// of one problem alone.  One warm-up, then the best of kTuneReps runs.
comet_status_t batch_tune_classes(const std::vector<Analysis> &an, const std::vector<int64_t> &first,
                                  const std::vector<char> &live, std::vector<BatchDesc> &descs, int dt, int mode) {
  TuneCache &tc = tune_cache();
  std::lock_guard<std::mutex> lk(tc.mutex());
  int device = 0;
  HIP_TRY(hipGetDevice(&device), "hipGetDevice");
  const std::string arch = arch_id(device);
  int cus = 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) cus = 256;
  const int64_t slots = int64_t(cus) * batch_blocks_per_cu(dt, mode);
  std::map<std::string, int> decided;
  // the problem each descriptor belongs to
  std::vector<int> owner(descs.size(), 0);
  for (size_t i = 0; i + 1 < first.size(); ++i)
    for (int64_t j = first[i]; j < first[i + 1]; ++j) owner[size_t(j)] = int(i);
  const size_t es = dt == 0 ? 8 : 4;
  for (size_t j = 0; j < descs.size(); ++j) {
    if (!live[j]) continue;
    BatchDesc &d = descs[j];
    const std::string key = batch_tune_key(dt, mode, d.variant, d.M, d.N, d.K, arch);
    auto hit = decided.find(key);
    if (hit != decided.end()) {
      d.cls = hit->second;
      continue;
    }
    TuneEntry e;
    if (tc.mode() == 1 && tc.lookup(key, &e) && batch_class_valid(e.tile, dt, mode, d.variant < 4)) {
      decided[key] = d.cls = e.tile;
      continue;
    }
    // time the classes on copies of this descriptor's problem
    const Analysis &a = an[size_t(owner[j])];
    void *buf = nullptr;
    hipStream_t s = nullptr;
    size_t offs[6], tb = 0;
    const std::vector<int64_t> *tabs[6] = {&a.offAm, &a.offAk, &a.offBk, &a.offBn, &a.offCm, &a.offCn};
    for (int t = 0; t < 6; ++t) {
      offs[t] = tb;
      tb += align256(std::max<size_t>(tabs[t]->size(), 1) * sizeof(int64_t));
    }
    const int64_t nA = std::max<int64_t>(a.swapped ? a.sizeB : a.sizeA, 1);
    const int64_t nB = std::max<int64_t>(a.swapped ? a.sizeA : a.sizeB, 1);
    const int64_t nC = std::max<int64_t>(a.sizeC, 1);
    const size_t oA = tb, oB = oA + align256(nA * es), oC = oB + align256(nB * es), oD = oC + align256(nC * es);
    const size_t oI = oD + align256(sizeof(BatchDesc));
    // items: at most enough copies for 4 rounds of the grid, at most 2^22 items
    int64_t max_items = 0;
    for (int c = 0; c < kBatchClasses; ++c) {
      if (!batch_class_valid(c, dt, mode, d.variant < 4)) continue;
      int bm, bn;
      batch_class_shape(c, &bm, &bn);
      const int64_t tiles = ((d.M + bm - 1) / bm) * ((d.N + bn - 1) / bn);
      const int64_t R = std::max<int64_t>(1, (4 * slots + tiles - 1) / tiles);
      max_items = std::max(max_items, std::min<int64_t>(R * tiles, std::max<int64_t>(tiles, int64_t(1) << 22)));
    }
    const size_t total_bytes = oI + align256(sizeof(BatchItem) * size_t(max_items)) + 256;
    bool ok = hipStreamCreate(&s) == hipSuccess && hipMalloc(&buf, total_bytes) == hipSuccess;
    int best = d.cls;
    double best_us = 1e30;
    if (ok) {
      char *b = static_cast<char *>(buf);
      std::vector<char> host(oA, 0);
      for (int t = 0; t < 6; ++t)
        if (!tabs[t]->empty()) std::memcpy(host.data() + offs[t], tabs[t]->data(), tabs[t]->size() * sizeof(int64_t));
      ok = hipMemcpy(b, host.data(), oA, hipMemcpyHostToDevice) == hipSuccess &&
           fill_value(b + oA, nA, dt, 0.5, s) == hipSuccess && fill_value(b + oB, nB, dt, -0.25, s) == hipSuccess;
      BatchDesc td = d;
      td.A = b + oA;
      td.B = b + oB;
      td.C = b + oC;
      td.alpha = 1.0;
      td.beta = 0.0;
      auto T = [&](int t) { return reinterpret_cast<const int64_t *>(b + offs[t]); };
      td.t = GettTables{T(0), T(1), T(2), T(3), T(4), T(5)};
      for (int c = 0; ok && c < kBatchClasses; ++c) {
        if (!batch_class_valid(c, dt, mode, d.variant < 4)) continue;
        int bm, bn;
        batch_class_shape(c, &bm, &bn);
        td.cls = c;
        td.tilesN = int((d.N + bn - 1) / bn);
        const int64_t tiles = ((d.M + bm - 1) / bm) * td.tilesN;
        const int64_t R = std::max<int64_t>(1, std::min<int64_t>((4 * slots + tiles - 1) / tiles,
                                                                 max_items / std::max<int64_t>(tiles, 1)));
        std::vector<BatchItem> items(size_t(R * tiles));
        BatchQueues q{};
        for (int qi = 0; qi <= kBatchQueues; ++qi) q.off[qi] = (R * tiles) * qi / kBatchQueues;
        for (int64_t r = 0; r < R; ++r)
          for (int64_t t = 0; t < tiles; ++t) items[size_t(r * tiles + t)] = BatchItem{0, int(t)};
        if (hipMemcpy(b + oD, &td, sizeof(td), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(b + oI, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice) != hipSuccess) {
          ok = false;
          break;
        }
        const int grid = int(std::max<int64_t>(1, std::min<int64_t>(R * tiles, slots)));
        int *cnt = reinterpret_cast<int *>(b + total_bytes - 256);
        bool good;
        const double us = time_us(
            [&]() {
              return launch_batch(reinterpret_cast<const BatchDesc *>(b + oD), reinterpret_cast<const BatchItem *>(b + oI),
                                  q, cnt, dt, mode, grid, s) == hipSuccess
                         ? COMET_OK
                         : COMET_ERR_HIP;
            },
            s, &good);
        if (good && us / double(R) < best_us) {
          best_us = us / double(R);
          best = c;
        }
      }
    }
    if (s) (void)hipStreamSynchronize(s);
    if (buf) (void)hipFree(buf);
    if (s) (void)hipStreamDestroy(s);
    if (ok && best_us < 1e30) tc.store(key, TuneEntry{best, COMET_PATH_GETT, best_us});
    decided[key] = d.cls = best;
  }
  return COMET_OK;
}

// ---- convenience-call state: plan cache and per-device workspace ----------

// A library-owned workspace of the convenience calls, one per (device,
// stream): calls on one stream are ordered by the stream, so they may share
// it; calls on two streams get two buffers.  `done` is recorded on the stream
// after the last enqueued use, and a later user waits for it (on the device)
// before touching the buffer, so a buffer whose stream handle is reused by a
// new stream, or which is grown, is never overwritten or freed under kernels
// still in flight.
struct DeviceWorkspace {
  void *ptr = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
};
typedef std::pair<int, hipStream_t> WsKey;

// Make `w` at least `bytes` large and usable by stream s; call with the
// lock that guards w held, and call ws_release after enqueuing the work.
comet_status_t ws_acquire(DeviceWorkspace &w, size_t bytes, hipStream_t s) {
  if (!w.done) HIP_TRY(hipEventCreateWithFlags(&w.done, hipEventDisableTiming), "hipEventCreate(workspace)");
  if (bytes > w.bytes) {
    // grow: the old buffer is freed only after its last use has completed
    HIP_TRY(hipEventSynchronize(w.done), "hipEventSynchronize(workspace)");
    if (w.ptr) HIP_TRY(hipFree(w.ptr), "hipFree(workspace)");
    w.ptr = nullptr;
    w.bytes = 0;
    HIP_TRY(hipMalloc(&w.ptr, bytes), "hipMalloc(workspace)");
    w.bytes = bytes;
  } else {
    HIP_TRY(hipStreamWaitEvent(s, w.done, 0), "hipStreamWaitEvent(workspace)");
  }
  return COMET_OK;
}

comet_status_t ws_release(DeviceWorkspace &w, hipStream_t s) {
  HIP_TRY(hipEventRecord(w.done, s), "hipEventRecord(workspace)");
  return COMET_OK;
}
// Plans of comet_contract, per device.  Each holds device tables, so the
// cache is bounded: past kMaxCachedPlans distinct problems on one device it
// waits for the device and starts over.
constexpr size_t kMaxCachedPlans = 1024;
std::map<int, std::map<std::string, std::unique_ptr<comet_plan_s>>> g_cache;
std::map<WsKey, DeviceWorkspace> g_ws;

std::string cache_key(const char *spec, const int64_t *ext, size_t nlab, const int64_t *sA, size_t ra,
                      const int64_t *sB, size_t rb, const int64_t *sC, size_t rc, int dtype, int compute, int dev) {
  std::string k(spec);
  auto add = [&](const int64_t *v, size_t n) {
    k += "|";
    if (!v) {
      k += "-";
      return;
    }
    for (size_t i = 0; i < n; ++i) k += std::to_string(v[i]) + ",";
  };
  add(ext, nlab);
  add(sA, ra);
  add(sB, rb);
  add(sC, rc);
  k += "|" + std::to_string(dtype) + "|" + std::to_string(compute) + "|" + std::to_string(dev) + "|" +
       std::to_string(g_split_slices) + "|" + std::to_string(g_int8_slices);
  // every planner override in the environment
  for (const char *name : {"COMET_FORCE_PATH", "COMET_TTGT_ORDER", "COMET_GETT_TILE", "COMET_GETT_SK",
                           "COMET_GETT_PERSIST", "COMET_GETT_SHORTK", "COMET_GETT_EVEN", "COMET_SPLIT_TILE", "COMET_FUSED3"}) {
    const char *v = std::getenv(name);
    k += "|";
    if (v) k += v;
  }
  k += "|t" + std::to_string(tune_cache().mode());
  return k;
}

}  // namespace

extern "C" {

const char *comet_version(void) { return COMET_VERSION_STRING; }

const char *comet_last_error(void) { return g_last_error.c_str(); }

comet_status_t comet_set_split_slices(int S) {
  if (S < 3 || S > 6) return fail(COMET_ERR_UNSUPPORTED, "split slices must be within 3..6");
  std::lock_guard<std::mutex> lk(g_mu);
  g_split_slices = S;
  return COMET_OK;
}

comet_status_t comet_set_int8_slices(int S) {
  if (S < 3 || S > 8) return fail(COMET_ERR_UNSUPPORTED, "int8 split slices must be within 3..8");
  std::lock_guard<std::mutex> lk(g_mu);
  g_int8_slices = S;
  return COMET_OK;
}

comet_status_t comet_analyze(const char *spec, const int64_t *extents, const int64_t *strides_A,
                             const int64_t *strides_B, const int64_t *strides_C, comet_dtype_t dtype,
                             comet_compute_t compute, comet_path_t path, char *buf, size_t len) {
  Analysis an;
  Status st = analyze(spec, extents, strides_A, strides_B, strides_C, dtype, compute, path, g_split_slices, an, g_int8_slices);
  if (!st.ok()) return fail(st);
  std::string js = describe_json(an);
  if (buf && len) {
    std::strncpy(buf, js.c_str(), len - 1);
    buf[len - 1] = 0;
    if (js.size() + 1 > len) return fail(COMET_ERR_WORKSPACE, "describe buffer too small");
  }
  return COMET_OK;
}

comet_status_t comet_plan_create_ex(comet_plan_t *plan, const char *spec, const int64_t *extents,
                                    const int64_t *strides_A, const int64_t *strides_B, const int64_t *strides_C,
                                    comet_dtype_t dtype, comet_compute_t compute, comet_path_t path) {
  if (!plan) return fail(COMET_ERR_NULL_POINTER, "plan is NULL");
  std::unique_ptr<comet_plan_s> p;
  comet_status_t rc = build_plan(p, spec, extents, strides_A, strides_B, strides_C, dtype, compute, path);
  if (rc != COMET_OK) return rc;
  *plan = p.release();
  return COMET_OK;
}

comet_status_t comet_plan_create(comet_plan_t *plan, const char *spec, const int64_t *extents,
                                 const int64_t *strides_A, const int64_t *strides_B, const int64_t *strides_C,
                                 comet_dtype_t dtype, comet_compute_t compute) {
  return comet_plan_create_ex(plan, spec, extents, strides_A, strides_B, strides_C, dtype, compute,
                              COMET_PATH_AUTO);
}

comet_status_t comet_plan_workspace_size(comet_plan_t plan, size_t *bytes) {
  if (!plan || !bytes) return fail(COMET_ERR_NULL_POINTER, "NULL argument");
  *bytes = plan->ws_bytes;
  return COMET_OK;
}

comet_status_t comet_plan_execute(comet_plan_t plan, double alpha, const void *A, const void *B, double beta,
                                  void *C, void *workspace, size_t ws_bytes, void *stream) {
  if (!plan) return fail(COMET_ERR_NULL_POINTER, "plan is NULL");
  return execute(plan, alpha, A, B, beta, C, workspace, ws_bytes, static_cast<hipStream_t>(stream));
}

comet_status_t comet_plan_destroy(comet_plan_t plan) {
  delete plan;
  return COMET_OK;
}

comet_status_t comet_plan_describe(comet_plan_t plan, char *buf, size_t len) {
  if (!plan || !buf || !len) return fail(COMET_ERR_NULL_POINTER, "NULL argument");
  std::string js = describe_json(plan->an);
  if (!js.empty() && js.back() == '}') {
    // resident workgroups per CU of the gather kernel this plan launches
    int res = 0;
    if (plan->an.path == COMET_PATH_GETT)
      res = tile_resident(plan->an, plan->an.tile, plan->vecA_tables, plan->vecB_tables);
    js.pop_back();
    js += ",\"resident\":" + std::to_string(res);
    if (plan->split.ws_bytes > 0) js += ",\"split_tile\":" + std::to_string(plan->split.tile);
    js += std::string(",\"fused3\":") + (plan->fused3 ? "true" : "false");
    js += "}";
  }
  std::strncpy(buf, js.c_str(), len - 1);
  buf[len - 1] = 0;
  if (js.size() + 1 > len) return fail(COMET_ERR_WORKSPACE, "describe buffer too small");
  return COMET_OK;
}

comet_status_t comet_contract(const char *spec, const int64_t *extents, comet_dtype_t dtype, comet_compute_t compute,
                              double alpha, const void *A, const int64_t *strides_A, const void *B,
                              const int64_t *strides_B, double beta, void *C, const int64_t *strides_C,
                              void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  // validate first (host only), so errors come back before any HIP call
  Analysis pre;
  Status st = parse_spec(spec, pre);
  if (!st.ok()) return fail(st);
  if (!pre.labels.empty() && !extents) return fail(COMET_ERR_NULL_POINTER, "extents is NULL");
  int dev = 0;
  hipError_t de = hipGetDevice(&dev);
  if (de != hipSuccess) {
    // no usable device: still report argument errors first
    Analysis an;
    Status vs = analyze(spec, extents, strides_A, strides_B, strides_C, dtype, compute, COMET_PATH_AUTO,
                        g_split_slices, an, g_int8_slices);
    if (!vs.ok()) return fail(vs);
    return hip_fail(de, "hipGetDevice");
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(s, &cs), "hipStreamIsCapturing");
  if (cs != hipStreamCaptureStatusNone)
    return fail(COMET_ERR_UNSUPPORTED, "comet_contract cannot run under stream capture; use the plan API");
  std::string key = cache_key(spec, extents, pre.labels.size(), strides_A, pre.spec_a.size(), strides_B,
                              pre.spec_b.size(), strides_C, pre.spec_c.size(), dtype, compute, dev);
  std::lock_guard<std::mutex> lk(g_mu);
  auto &cache = g_cache[dev];
  auto it = cache.find(key);
  comet_plan_s *p;
  if (it == cache.end()) {
    std::unique_ptr<comet_plan_s> np;
    comet_status_t rc = build_plan(np, spec, extents, strides_A, strides_B, strides_C, dtype, compute,
                                   COMET_PATH_AUTO);
    if (rc != COMET_OK) return rc;
    if (cache.size() >= kMaxCachedPlans) {
      // kernels still in flight may read the tables of the cached plans
      HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
      cache.clear();
    }
    p = np.get();
    cache[key] = std::move(np);
  } else {
    p = it->second.get();
  }
  if (p->ws_bytes == 0) return execute(p, alpha, A, B, beta, C, nullptr, 0, s);
  DeviceWorkspace &w = g_ws[WsKey(dev, s)];
  comet_status_t rc = ws_acquire(w, p->ws_bytes, s);
  if (rc != COMET_OK) return rc;
  rc = execute(p, alpha, A, B, beta, C, w.ptr, w.bytes, s);
  comet_status_t rr = ws_release(w, s);
  return rc != COMET_OK ? rc : rr;
}

comet_status_t comet_permute(const char *spec, const int64_t *extents, comet_dtype_t dtype, double alpha,
                             const void *in, const int64_t *strides_in, double beta, void *out,
                             const int64_t *strides_out, void *stream) {
  if (!spec) return fail(COMET_ERR_NULL_POINTER, "spec is NULL");
  std::string s(spec), lo, li;
  s.erase(std::remove_if(s.begin(), s.end(), [](char c) { return c == ' ' || c == '\t'; }), s.end());
  size_t eq = s.find('=');
  if (eq == std::string::npos || s.find('=', eq + 1) != std::string::npos)
    return fail(COMET_ERR_INVALID_SPEC, "permute spec must read OUT=IN");
  lo = s.substr(0, eq);
  li = s.substr(eq + 1);
  std::string a = lo, b = li;
  std::sort(a.begin(), a.end());
  std::sort(b.begin(), b.end());
  if (a != b || std::adjacent_find(a.begin(), a.end()) != a.end() || (int)lo.size() > COMET_MAX_RANK)
    return fail(COMET_ERR_INVALID_SPEC, "permute spec needs the same distinct labels on both sides");
  for (char ch : lo)
    if (!((ch >= 'a' && ch <= 'z') || (ch >= 'A' && ch <= 'Z'))) return fail(COMET_ERR_INVALID_SPEC, "bad label");
  if (dtype != COMET_F64 && dtype != COMET_F32) return fail(COMET_ERR_UNSUPPORTED, "unknown dtype");
  if (!lo.empty() && !extents) return fail(COMET_ERR_NULL_POINTER, "extents is NULL");
  std::vector<int64_t> eo(lo.size());
  int64_t total = 1;
  for (size_t p = 0; p < lo.size(); ++p) {
    eo[p] = extents[p];
    if (eo[p] < 0) return fail(COMET_ERR_INVALID_SHAPE, "negative extent");
    if (__builtin_mul_overflow(total, eo[p], &total)) return fail(COMET_ERR_INVALID_SHAPE, "size overflows int64");
  }
  std::vector<int64_t> so = strides_out ? std::vector<int64_t>(strides_out, strides_out + lo.size())
                                        : dense_strides(eo);
  std::vector<int64_t> ei(li.size());
  for (size_t q = 0; q < li.size(); ++q) ei[q] = eo[lo.find(li[q])];
  std::vector<int64_t> si = strides_in ? std::vector<int64_t>(strides_in, strides_in + li.size()) : dense_strides(ei);
  for (int64_t x : so)
    if (x < 0) return fail(COMET_ERR_INVALID_STRIDE, "negative stride");
  for (int64_t x : si)
    if (x < 0) return fail(COMET_ERR_INVALID_STRIDE, "negative stride");
  {
    std::vector<std::pair<int64_t, int64_t>> sd;
    for (size_t p = 0; p < lo.size(); ++p) {
      if (eo[p] <= 1) continue;
      if (so[p] == 0) return fail(COMET_ERR_INVALID_STRIDE, "output stride 0 on a dimension of extent > 1");
      sd.push_back({so[p], eo[p]});
    }
    std::sort(sd.begin(), sd.end());
    for (size_t i = 0; i + 1 < sd.size(); ++i)
      if (sd[i + 1].first < sd[i].first * sd[i].second)
        return fail(COMET_ERR_INVALID_STRIDE, "output dimensions overlap in memory");
  }
  if (total == 0) return COMET_OK;
  if (!out || (alpha != 0.0 && !in)) return fail(COMET_ERR_NULL_POINTER, "NULL tensor pointer");
  PermuteDesc d = make_permute(lo, so, li, si, eo);
  PermuteLaunch pl{};
  pl.ndim = (int)d.ext.size();
  for (int i = 0; i < pl.ndim; ++i) {
    pl.ext[i] = d.ext[i];
    pl.s_in[i] = alpha == 0.0 ? 0 : d.s_in[i];
    pl.s_out[i] = d.s_out[i];
  }
  pl.in = alpha == 0.0 ? out : in;
  pl.out = out;
  pl.alpha = alpha;
  pl.beta = beta;
  pl.dtype = dtype == COMET_F64 ? 0 : 1;
  if (dtype == COMET_F32) {
    pl.alpha = double(float(alpha));
    pl.beta = double(float(beta));
  }
  if (alpha == 0.0) {
    // out = beta * out: a permutation of out onto itself is the identity
    for (int i = 0; i < pl.ndim; ++i) pl.s_in[i] = pl.s_out[i];
    pl.alpha = 0.0;
  }
  HIP_TRY(launch_permute(pl, static_cast<hipStream_t>(stream)), "permute launch");
  return COMET_OK;
}

comet_status_t comet_chain_plan(const char *spec, const int64_t *extents, char *buf, size_t len) {
  if (!buf || !len) return fail(COMET_ERR_NULL_POINTER, "buf is NULL");
  ChainPlan cp;
  Status st = chain_plan(spec, extents, cp);
  if (!st.ok()) return fail(st);
  const std::string js = chain_json(cp);
  std::strncpy(buf, js.c_str(), len - 1);
  buf[len - 1] = 0;
  if (js.size() + 1 > len) return fail(COMET_ERR_WORKSPACE, "chain plan buffer too small");
  return COMET_OK;
}

namespace {
// per-(device, stream) buffers for the intermediates of comet_contract_chain,
// and the lock held from the buffer's acquisition until every step of the
// chain is enqueued (comet_contract takes g_mu itself, so this is another one)
std::map<WsKey, DeviceWorkspace> g_chain_ws;
std::mutex g_chain_mu;
}  // namespace

comet_status_t comet_contract_chain(const char *spec, const int64_t *extents, comet_dtype_t dtype,
                                    comet_compute_t compute, double alpha, int n, const void *const *operands,
                                    const int64_t *const *strides, double beta, void *C,
                                    const int64_t *strides_C, void *stream) {
  ChainPlan cp;
  Status st = chain_plan(spec, extents, cp);
  if (!st.ok()) return fail(st);
  if (n != int(cp.operands.size())) return fail(COMET_ERR_INVALID_SPEC, "operand count does not match the spec");
  if (!operands) return fail(COMET_ERR_NULL_POINTER, "operands is NULL");
  if (dtype != COMET_F64 && dtype != COMET_F32) return fail(COMET_ERR_UNSUPPORTED, "unknown dtype");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return fail(COMET_ERR_UNSUPPORTED, "comet_contract_chain allocates; it cannot run under capture");
  auto ext_of = [&](char ch) {
    return cp.extents[std::find(cp.labels.begin(), cp.labels.end(), ch) - cp.labels.begin()];
  };
  // intermediates: dense, one allocation
  const size_t es = elem_size(dtype);
  std::vector<size_t> off(cp.steps.size(), 0);
  size_t total = 0;
  for (size_t i = 0; i + 1 < cp.steps.size(); ++i) {
    size_t cnt = 1;
    for (char ch : cp.steps[i].out_labels) cnt *= size_t(ext_of(ch));
    off[i] = total;
    total += align256(std::max<size_t>(cnt, 1) * es);
  }
  char *inter = nullptr;
  std::unique_lock<std::mutex> lk(g_chain_mu);
  DeviceWorkspace *w = nullptr;
  if (total > 0) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    w = &g_chain_ws[WsKey(dev, s)];
    comet_status_t rc = ws_acquire(*w, total, s);
    if (rc != COMET_OK) return rc;
    inter = static_cast<char *>(w->ptr);
  }
  const int ns = int(cp.steps.size());
  std::vector<const void *> ptr(size_t(n) + size_t(ns), nullptr);
  std::vector<const int64_t *> str(size_t(n) + size_t(ns), nullptr);
  for (int i = 0; i < n; ++i) {
    ptr[i] = operands[i];
    str[i] = strides ? strides[i] : nullptr;
  }
  for (int i = 0; i < ns; ++i) {
    const ChainStep &stp = cp.steps[i];
    const bool last = i == ns - 1;
    std::string seen;
    std::vector<int64_t> ext;
    for (char ch : stp.spec)
      if (ch != '=' && ch != '*' && seen.find(ch) == std::string::npos) {
        seen += ch;
        ext.push_back(ext_of(ch));
      }
    void *out = last ? C : static_cast<void *>(inter + off[i]);
    comet_status_t rc = comet_contract(stp.spec.c_str(), ext.data(), dtype, compute, last ? alpha : 1.0,
                                       ptr[stp.left], str[stp.left], ptr[stp.right], str[stp.right],
                                       last ? beta : 0.0, out, last ? strides_C : nullptr, stream);
    if (rc != COMET_OK) {
      if (w) (void)ws_release(*w, s);
      return rc;
    }
    ptr[n + i] = out;
    str[n + i] = nullptr;
  }
  return w ? ws_release(*w, s) : COMET_OK;
}

comet_status_t comet_fill(int rank, const int64_t *extents, comet_dtype_t dtype, double value, void *out,
                          const int64_t *strides, void *stream) {
  if (rank < 0 || rank > COMET_MAX_RANK) return fail(COMET_ERR_INVALID_SHAPE, "rank must be within 0..12");
  if (dtype != COMET_F64 && dtype != COMET_F32) return fail(COMET_ERR_UNSUPPORTED, "unknown dtype");
  if (rank > 0 && !extents) return fail(COMET_ERR_NULL_POINTER, "extents is NULL");
  std::vector<int64_t> e(extents, extents + rank);
  int64_t total = 1;
  for (int64_t x : e) {
    if (x < 0) return fail(COMET_ERR_INVALID_SHAPE, "negative extent");
    if (__builtin_mul_overflow(total, x, &total)) return fail(COMET_ERR_INVALID_SHAPE, "size overflows int64");
  }
  std::vector<int64_t> st = strides ? std::vector<int64_t>(strides, strides + rank) : dense_strides(e);
  for (int64_t x : st)
    if (x < 0) return fail(COMET_ERR_INVALID_STRIDE, "negative stride");
  if (total == 0) return COMET_OK;   // an empty tensor: strides do not matter
  {
    std::vector<std::pair<int64_t, int64_t>> sd;
    for (int p = 0; p < rank; ++p) {
      if (e[p] <= 1) continue;
      if (st[p] == 0) return fail(COMET_ERR_INVALID_STRIDE, "stride 0 on a dimension of extent > 1");
      sd.push_back({st[p], e[p]});
    }
    std::sort(sd.begin(), sd.end());
    for (size_t i = 0; i + 1 < sd.size(); ++i)
      if (sd[i + 1].first < sd[i].first * sd[i].second)
        return fail(COMET_ERR_INVALID_STRIDE, "dimensions overlap in memory");
  }
  if (!out) return fail(COMET_ERR_NULL_POINTER, "out is NULL");
  // the stream form of the permute kernel with nothing read: out = fill
  PermuteLaunch pl{};
  pl.ndim = rank;
  for (int i = 0; i < rank; ++i) {
    pl.ext[i] = e[i];
    pl.s_in[i] = st[i];
    pl.s_out[i] = st[i];
  }
  pl.in = out;
  pl.out = out;
  pl.alpha = 0.0;
  pl.beta = 0.0;
  pl.dtype = dtype == COMET_F64 ? 0 : 1;
  pl.fill = dtype == COMET_F32 ? double(float(value)) : value;
  HIP_TRY(launch_permute(pl, static_cast<hipStream_t>(stream)), "fill launch");
  return COMET_OK;
}

comet_status_t comet_batch_create(comet_batch_t *batch, int n, const comet_problem_t *problems, comet_dtype_t dtype,
                                  comet_compute_t compute) {
  if (!batch) return fail(COMET_ERR_NULL_POINTER, "batch is NULL");
  if (n < 0) return fail(COMET_ERR_INVALID_SHAPE, "negative problem count");
  if (n > 0 && !problems) return fail(COMET_ERR_NULL_POINTER, "problems is NULL");
  std::unique_ptr<comet_batch_s> b(new comet_batch_s());
  b->dtype = dtype;
  std::vector<Analysis> an(n);
  for (int i = 0; i < n; ++i) {
    const comet_problem_t &pr = problems[i];
    Status st = analyze(pr.spec, pr.extents, pr.strides_A, pr.strides_B, pr.strides_C, dtype, compute,
                        COMET_PATH_GETT, g_split_slices, an[i], g_int8_slices);
    if (!st.ok()) return fail(st.code, "problem " + std::to_string(i) + ": " + st.msg);
    const Analysis &a = an[i];
    int mode;
    if (a.compute == COMET_COMPUTE_SPLIT_BF16X3 && dtype == COMET_F32)
      mode = 1;
    else if ((a.compute == COMET_COMPUTE_F64 && dtype == COMET_F64) || (a.compute == COMET_COMPUTE_F32 && dtype == COMET_F32))
      mode = 0;
    else
      return fail(COMET_ERR_UNSUPPORTED, "batch: compute must be the storage type's native MFMA, or BF16x3 on FP32");
    if (i == 0) b->mode = mode;
    if (a.empty_out) continue;
    if (!pr.C) return fail(COMET_ERR_NULL_POINTER, "problem " + std::to_string(i) + ": C is NULL");
    const bool reads = pr.alpha != 0.0 && !a.empty_sum;
    if (reads && (!pr.A || !pr.B)) return fail(COMET_ERR_NULL_POINTER, "problem " + std::to_string(i) + ": A or B is NULL");
    if (reads && (pr.C == pr.A || pr.C == pr.B))
      return fail(COMET_ERR_UNSUPPORTED, "problem " + std::to_string(i) + ": C aliases an input");
  }
  // dense copies of one operand of each element-load problem (COMET_BATCH_COPY=0
  // keeps the element-load kernel for them)
  const int VEC = dtype == COMET_F64 ? 2 : 4;
  std::vector<BatchCopy> copies(n);
  std::vector<size_t> copy_off(n, 0);
  size_t copy_bytes = 0;
  {
    const char *env = std::getenv("COMET_BATCH_COPY");
    const bool allow = !(env && *env && std::atoi(env) == 0);
    for (int i = 0; allow && i < n; ++i) {
      const Analysis &a = an[i];
      const comet_problem_t &pr = problems[i];
      if (a.empty_out || a.empty_sum || pr.alpha == 0.0) continue;
      if (tables_vec_ok(a.offAm, a.offAk, a.layoutA, a.runAm, a.runAk, VEC) &&
          tables_vec_ok(a.offBn, a.offBk, a.layoutB, a.runBn, a.runBk, VEC))
        continue;
      Analysis na;
      if (batch_copy_choice(pr, a, dtype, compute, VEC, na, copies[i])) {
        an[i] = na;
        copy_off[i] = copy_bytes;
        copy_bytes += align256(size_t(copies[i].count) * elem_size(dtype));
      }
    }
  }
  // one descriptor per batch entry of each problem (a problem without batch
  // labels has one); device buffer: descriptors, work items, then every
  // problem's six tables and its C batch table
  std::vector<int64_t> first(n + 1, 0);
  for (int i = 0; i < n; ++i) first[i + 1] = first[i] + (an[i].empty_out ? 1 : an[i].nb);
  const int64_t nd = first[n];
  constexpr int64_t kMaxEntries = int64_t(1) << 22;   // descriptors held on the host and the device
  if (nd > kMaxEntries) return fail(COMET_ERR_UNSUPPORTED, "batch has more than 2^22 problems and batch entries");
  std::vector<BatchDesc> descs(static_cast<size_t>(nd));
  std::vector<size_t> tab_off(n, 0);
  std::vector<char> live(size_t(nd), 0);   // descriptors with work (some output and a nonzero product)
  for (int i = 0; i < n; ++i) {
    const Analysis &a = an[i];
    if (a.empty_out || a.empty_sum || problems[i].alpha == 0.0) continue;
    for (int64_t e = 0; e < a.nb; ++e) live[size_t(first[i] + e)] = 1;
  }
  size_t bytes = align256(sizeof(BatchDesc) * std::max<int64_t>(nd, 1));
  for (int i = 0; i < n; ++i) {
    tab_off[i] = bytes;
    const Analysis &a = an[i];
    for (const std::vector<int64_t> *v : {&a.offAm, &a.offAk, &a.offBk, &a.offBn, &a.offCm, &a.offCn, &a.offCx})
      bytes += align256(std::max<size_t>(v->size(), 1) * sizeof(int64_t));
  }
  const size_t es = elem_size(dtype);
  const int dt = dtype == COMET_F64 ? 0 : 1;
  // descriptors (table pointers are filled in once the buffer exists)
  std::vector<std::vector<char>> host_tabs(n);
  for (int i = 0; i < n; ++i) {
    const Analysis &a = an[i];
    const comet_problem_t &pr = problems[i];
    const double alpha = dtype == COMET_F32 ? double(float(pr.alpha)) : pr.alpha;
    const double beta = dtype == COMET_F32 ? double(float(pr.beta)) : pr.beta;
    // a copied operand: its pointer is set once the copy buffer exists (256-byte aligned)
    const void *oA = copies[i].which == 0 ? reinterpret_cast<const void *>(uintptr_t(256)) : pr.A;
    const void *oB = copies[i].which == 1 ? reinterpret_cast<const void *>(uintptr_t(256)) : pr.B;
    const void *pa = a.swapped ? oB : oA, *pb = a.swapped ? oA : oB;
    const bool vec_tables = tables_vec_ok(a.offAm, a.offAk, a.layoutA, a.runAm, a.runAk, VEC) &&
                            tables_vec_ok(a.offBn, a.offBk, a.layoutB, a.runBn, a.runBk, VEC);
    for (int64_t e = 0; e < (a.empty_out ? 1 : a.nb); ++e) {
      BatchDesc &d = descs[size_t(first[i] + e)];
      const bool bx = !a.offAx.empty() && !a.empty_out;
      d.A = pa ? static_cast<const char *>(pa) + (bx ? a.offAx[e] * es : 0) : nullptr;
      d.B = pb ? static_cast<const char *>(pb) + (bx ? a.offBx[e] * es : 0) : nullptr;
      d.C = pr.C ? static_cast<char *>(pr.C) + (bx ? a.offCx[e] * es : 0) : nullptr;
      d.M = a.m;
      d.N = a.n;
      d.K = a.k;
      d.alpha = alpha;
      d.beta = beta;
      const bool vec = vec_tables && reinterpret_cast<uintptr_t>(d.A) % 16 == 0 &&
                       reinterpret_cast<uintptr_t>(d.B) % 16 == 0;
      d.variant = a.layoutA * 2 + a.layoutB + (vec ? 0 : 4);
      d.cls = 0;
    }
  }
  // tile class of every live descriptor: the autotuner's, else the model's
  comet_status_t crc = batch_choose_classes(an, first, live, descs, dt, b->mode);
  if (crc != COMET_OK) return crc;
  {
    const char *env = std::getenv("COMET_BATCH_CLASS");
    if (!(env && *env) && tune_cache().mode() != 0)
      for (size_t j = 0; j < live.size(); ++j) b->tuned += live[j] ? 1 : 0;
  }
  int64_t total = 0;
  for (int64_t j = 0; j < nd; ++j) {
    BatchDesc &d = descs[size_t(j)];
    int bm, bn;
    batch_class_shape(d.cls, &bm, &bn);
    d.tilesN = int((d.N + bn - 1) / bn);
    if (live[size_t(j)]) total += ((d.M + bm - 1) / bm) * d.tilesN;
  }
  // the device work counters are ints that every persistent workgroup
  // increments once more after a queue is drained: keep total + grid below
  // 2^31 (the grid is at most one workgroup per CU slot, far below kMaxGrid)
  constexpr int64_t kMaxGrid = int64_t(1) << 20;
  if (total > int64_t(INT32_MAX) - kMaxGrid)
    return fail(COMET_ERR_UNSUPPORTED, "batch has more than 2^31 - 2^20 output tiles");
  const size_t items_off = bytes;
  bytes += align256(sizeof(BatchItem) * std::max<int64_t>(total, 1));
  HIP_TRY(hipGetDevice(&b->device), "hipGetDevice");
  HIP_TRY(hipMalloc(&b->dbuf, bytes), "hipMalloc(batch)");
  if (copy_bytes > 0) {
    HIP_TRY(hipMalloc(&b->pbuf, copy_bytes), "hipMalloc(batch copies)");
    for (int i = 0; i < n; ++i) {
      const BatchCopy &cp = copies[i];
      if (cp.which < 0) continue;
      char *dst = static_cast<char *>(b->pbuf) + copy_off[i];
      const Analysis &a = an[i];
      const bool dst_is_A = (cp.which == 0) != a.swapped;   // after the A/B exchange
      BatchDesc &d = descs[size_t(first[i])];
      if (dst_is_A)
        d.A = dst;
      else
        d.B = dst;
      // the copy: out[order] = in[original labels, caller strides]
      const comet_problem_t &pr = problems[i];
      const std::string &lx = cp.which == 0 ? a.spec_a : a.spec_b;
      const int64_t *given = cp.which == 0 ? pr.strides_A : pr.strides_B;
      std::vector<int64_t> ex;
      for (char ch : lx) ex.push_back(cp.ext[cp.order.find(ch)]);
      const std::vector<int64_t> sin = given ? std::vector<int64_t>(given, given + lx.size()) : dense_strides(ex);
      const PermuteDesc pd = make_permute(cp.order, dense_strides(cp.ext), lx, sin, cp.ext);
      PermuteLaunch pl{};
      pl.ndim = int(pd.ext.size());
      for (int q = 0; q < pl.ndim; ++q) {
        pl.ext[q] = pd.ext[q];
        pl.s_in[q] = pd.s_in[q];
        pl.s_out[q] = pd.s_out[q];
      }
      pl.in = cp.which == 0 ? pr.A : pr.B;
      pl.out = dst;
      pl.alpha = 1.0;
      pl.beta = 0.0;
      pl.dtype = dtype == COMET_F64 ? 0 : 1;
      b->perms.push_back(pl);
    }
  }
  std::vector<char> host(bytes, 0);
  char *dev = static_cast<char *>(b->dbuf);
  for (int i = 0; i < n; ++i) {
    const Analysis &a = an[i];
    const comet_problem_t &pr = problems[i];
    size_t off = tab_off[i];
    const int64_t *ptr[7];
    int k = 0;
    for (const std::vector<int64_t> *v : {&a.offAm, &a.offAk, &a.offBk, &a.offBn, &a.offCm, &a.offCn, &a.offCx}) {
      if (!v->empty()) std::memcpy(host.data() + off, v->data(), v->size() * sizeof(int64_t));
      ptr[k++] = reinterpret_cast<const int64_t *>(dev + off);
      off += align256(std::max<size_t>(v->size(), 1) * sizeof(int64_t));
    }
    for (int64_t e = 0; e < (a.empty_out ? 1 : a.nb); ++e)
      descs[size_t(first[i] + e)].t = GettTables{ptr[0], ptr[1], ptr[2], ptr[3], ptr[4], ptr[5]};
    if (!a.empty_out && (a.empty_sum || pr.alpha == 0.0)) {
      const double beta = dtype == COMET_F32 ? double(float(pr.beta)) : pr.beta;
      b->scales.push_back({pr.C, ptr[4], ptr[5], a.m, a.n, beta, a.offCx.empty() ? nullptr : ptr[6], a.nb});
    }
  }
  // queues: whole descriptors to the least-loaded queue, heaviest first
  // (longest processing time first); in each queue the heaviest first, and
  // a descriptor's tiles in groups of kGroup tile rows, so that the
  // workgroups working at one time share operand rows and columns
  std::vector<int64_t> order;
  std::vector<double> cost(size_t(nd), 0.0);
  for (int64_t j = 0; j < nd; ++j) {
    if (!live[size_t(j)]) continue;
    order.push_back(j);
    const BatchDesc &d = descs[size_t(j)];
    int bm, bn;
    batch_class_shape(d.cls, &bm, &bn);
    cost[size_t(j)] = double((d.M + bm - 1) / bm) * double(d.tilesN) * bm * bn * double(d.K);
  }
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return cost[size_t(x)] > cost[size_t(y)]; });
  std::vector<std::vector<int64_t>> qlist(kBatchQueues);
  std::vector<double> load(kBatchQueues, 0.0);
  for (int64_t j : order) {
    const int qmin = int(std::min_element(load.begin(), load.end()) - load.begin());
    qlist[size_t(qmin)].push_back(j);
    load[size_t(qmin)] += cost[size_t(j)];
  }
  BatchItem *items = reinterpret_cast<BatchItem *>(host.data() + items_off);
  constexpr int kGroup = 4;
  int64_t w = 0;
  for (int qi = 0; qi < kBatchQueues; ++qi) {
    b->queues.off[qi] = w;
    for (int64_t j : qlist[size_t(qi)]) {
      const BatchDesc &d = descs[size_t(j)];
      int bm, bn;
      batch_class_shape(d.cls, &bm, &bn);
      const int64_t tm_ = (d.M + bm - 1) / bm, tn_ = d.tilesN;
      for (int64_t id = 0; id < tm_ * tn_; ++id) {
        const int64_t per = kGroup * tn_, group = id / per, first_row = group * kGroup;
        const int64_t gsize = std::min<int64_t>(kGroup, tm_ - first_row);
        const int64_t in = id - group * per;
        const int64_t tm = first_row + in % gsize, tn = in / gsize;
        items[w++] = BatchItem{int(j), int(tm * tn_ + tn)};
      }
    }
  }
  b->queues.off[kBatchQueues] = w;
  if (nd > 0 && n > 0) std::memcpy(host.data(), descs.data(), sizeof(BatchDesc) * size_t(nd));
  HIP_TRY(hipMemcpy(b->dbuf, host.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy(batch)");
  b->descs = reinterpret_cast<const BatchDesc *>(dev);
  b->items = reinterpret_cast<const BatchItem *>(dev + items_off);
  b->total = total;
  b->classes.assign(kBatchClasses, 0);
  for (int64_t j : order) b->classes[size_t(descs[size_t(j)].cls)] += 1;
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, b->device), "hipGetDeviceProperties");
  const int64_t resident = int64_t(prop.multiProcessorCount) * batch_blocks_per_cu(dt, b->mode);
  b->grid = int(std::max<int64_t>(1, std::min<int64_t>(total, resident)));
  *batch = b.release();
  return COMET_OK;
}

comet_status_t comet_batch_workspace_size(comet_batch_t batch, size_t *bytes) {
  if (!batch || !bytes) return fail(COMET_ERR_NULL_POINTER, "NULL argument");
  *bytes = 256;   // the work counter
  return COMET_OK;
}

comet_status_t comet_batch_execute(comet_batch_t batch, void *workspace, size_t ws_bytes, void *stream) {
  if (!batch) return fail(COMET_ERR_NULL_POINTER, "batch is NULL");
  if (!workspace || ws_bytes < 256) return fail(COMET_ERR_WORKSPACE, "batch workspace needs 256 bytes");
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (const auto &sc : batch->scales)
    HIP_TRY(launch_scale(sc.C, batch->dtype == COMET_F64 ? 0 : 1, sc.offCm, sc.offCn, sc.m, sc.n, sc.beta, s,
                         sc.offCb, sc.nb),
            "batch scale");
  for (const PermuteLaunch &pl : batch->perms) HIP_TRY(launch_permute(pl, s), "batch operand copy");
  HIP_TRY(launch_batch(batch->descs, batch->items, batch->queues, static_cast<int *>(workspace),
                       batch->dtype == COMET_F64 ? 0 : 1, batch->mode, batch->grid, s),
          "batch launch");
  return COMET_OK;
}

comet_status_t comet_batch_describe(comet_batch_t batch, char *buf, size_t len) {
  if (!batch || !buf || !len) return fail(COMET_ERR_NULL_POINTER, "NULL argument");
  std::string js = "{\"tiles\":" + std::to_string(batch->total) + ",\"grid\":" + std::to_string(batch->grid) +
                   ",\"mode\":" + std::to_string(batch->mode) + ",\"classes\":[";
  for (size_t c = 0; c < batch->classes.size(); ++c) js += (c ? "," : "") + std::to_string(batch->classes[c]);
  js += "],\"queues\":[";
  for (int q = 0; q < kBatchQueues; ++q)
    js += (q ? "," : "") + std::to_string(batch->queues.off[q + 1] - batch->queues.off[q]);
  js += "],\"tuned\":" + std::to_string(batch->tuned) + ",\"copies\":" + std::to_string(batch->perms.size()) + "}";
  std::strncpy(buf, js.c_str(), len - 1);
  buf[len - 1] = 0;
  if (js.size() + 1 > len) return fail(COMET_ERR_WORKSPACE, "describe buffer too small");
  return COMET_OK;
}

comet_status_t comet_batch_destroy(comet_batch_t batch) {
  delete batch;
  return COMET_OK;
}

comet_status_t comet_autotune(const char *cache_path, int mode) {
  if (mode < 0 || mode > 2) return fail(COMET_ERR_UNSUPPORTED, "autotune mode must be 0, 1 or 2");
  TuneCache &tc = tune_cache();
  {
    std::lock_guard<std::mutex> lk(tc.mutex());
    tc.configure(cache_path ? std::string(cache_path) : std::string(), mode);
  }
  // plans made under another tuning mode are not reused by the convenience call
  return COMET_OK;
}

}  // extern "C"
