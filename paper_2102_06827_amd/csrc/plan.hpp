// plan.hpp -- host-side analysis of one binary contraction: parsing, validation,
// label classification and fusion, offset tables and the lowering choice.
// No HIP calls here, so everything in this file also runs on a machine
// without a GPU (comet_analyze).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "comet.h"

namespace comet {

// Label classes.  A contraction C = A * B is the matrix product of A viewed as
// an M x K matrix and B viewed as K x N (the TTGT flattening of Section 2):
// M = free labels of A, N = free labels of B, K = summation labels.  A label
// in all three tensors (X, a batch label) indexes C, A and B alike and is not
// summed: the contraction is one such matrix product per batch entry.
enum LabelClass { CLS_M = 0, CLS_N = 1, CLS_K = 2, CLS_X = 3 };

// A (possibly fused) dimension of the index space.  `labels` holds the
// original labels it stands for, outermost first; strides are in elements and
// are 0 in a tensor that does not hold the dimension.
struct Dim {
  std::string labels;
  int64_t ext = 1;
  int64_t sA = 0, sB = 0, sC = 0;
  int cls = CLS_M;
};

struct Status {
  comet_status_t code = COMET_OK;
  std::string msg;
  bool ok() const { return code == COMET_OK; }
  static Status error(comet_status_t c, const std::string &m) { return Status{c, m}; }
};

// Operand layout inside the fused gather kernel: which matrix dimension the
// operand is contiguous along in memory.
enum OperandLayout { LAYOUT_K_CONTIG = 0, LAYOUT_MN_CONTIG = 1 };

// One tensor permutation (TTGT transposes; the permute entry point): out[q] =
// in[perm applied], described by the common dims with both strides.
struct PermuteDesc {
  std::vector<int64_t> ext;       // dims in output order, outermost first
  std::vector<int64_t> s_in;      // input element stride of each dim
  std::vector<int64_t> s_out;     // output element stride of each dim
};

struct TTGTChoice {
  bool swap = false;              // A and B exchanged before flattening
  std::string a_order;            // label order of the permuted A (the matrix A_p)
  std::string b_order;            // label order of the permuted B (B_p)
  std::string c_order;            // label order of the product C_p
  bool a_copy = true, b_copy = true, c_copy = true;   // permute needed at all
  int64_t cost = 0;               // the Section 6 position weights of this flattening
  double model_us = 0.0;          // the MI355X time model of its permutes and product
};

struct Analysis {
  // inputs
  std::string spec_c, spec_a, spec_b;     // label strings as given
  comet_dtype_t dtype = COMET_F64;
  comet_compute_t compute = COMET_COMPUTE_DEFAULT;   // resolved (never DEFAULT)
  comet_path_t path = COMET_PATH_GETT;               // resolved (never AUTO)
  std::vector<char> labels;               // distinct labels, extents order
  std::vector<int64_t> extents;
  std::vector<int64_t> strA, strB, strC;  // per position of each tensor
  int64_t sizeA = 0, sizeB = 0, sizeC = 0;    // element span (max offset + 1)

  // after classification (and the A/B swap, if any)
  bool swapped = false;                   // A, B exchanged so C's unit label is in N
  std::vector<Dim> M, N, K;               // outermost first; fused, extent-1 dims dropped
  std::vector<Dim> X;                     // batch labels, same conventions
  int64_t m = 1, n = 1, k = 1;            // flattened sizes
  int64_t nb = 1;                         // batch entries (product of the X extents)
  bool empty_out = false;                 // m, n or nb == 0: nothing to do
  bool empty_sum = false;                 // k == 0: C = beta * C

  // offset tables (elements), one entry per flattened index
  std::vector<int64_t> offAm, offAk, offBk, offBn, offCm, offCn;
  // per batch entry: base offset of its slice of A, B and C (empty without
  // batch labels; A and B after the exchange, like the tables above)
  std::vector<int64_t> offAx, offBx, offCx;
  // contiguous-run widths (1, 2, 4 or 8) of each operand along each class
  int runAm = 1, runAk = 1, runBk = 1, runBn = 1, runCm = 1, runCn = 1;
  OperandLayout layoutA = LAYOUT_K_CONTIG, layoutB = LAYOUT_K_CONTIG;
  bool tables32 = true;                   // every offset fits in int32

  // tile shape of the gather kernel (index into the kernel's variant list)
  int tile = 0;
  // stream-K: the last sk_tiles output tiles are split along K over
  // sk_blocks workgroups (0: every tile is computed whole)
  int sk_tiles = 0, sk_blocks = 0;
  // nonzero: the balanced schedule instead of stream-K -- the first
  // even_whole tiles whole (full rounds of the whole-tile kernel), then the
  // sk_tiles leftover tiles cut into sk_blocks summation pieces
  int even = 0, even_whole = 0;
  // > 0: the persistent kernel with this many workgroups (short summations)
  int persist = 0;
  // > 0: the short-summation kernel (stores overlapped with the next tile's
  // products) with this many workgroups
  int shortk = 0;
  // matrix-vector products (M == 1): 1 the matrix is read along its free
  // index, 2 along the summation; the summation cut into gemv_split
  // slabs of gemv_slab indices
  int gemv = 0;
  int gemv_split = 0;
  int64_t gemv_slab = 0;
  int split_slices = 5;

  TTGTChoice ttgt;
};

// Parse "C=A*B".  Fills spec_c/a/b and the distinct label list.
Status parse_spec(const char *spec, Analysis &an);

// Full host analysis.  `split_slices` applies to SPLIT_BF16, `int8_slices`
// to SPLIT_INT8.
Status analyze(const char *spec, const int64_t *extents, const int64_t *strides_A,
               const int64_t *strides_B, const int64_t *strides_C, comet_dtype_t dtype,
               comet_compute_t compute, comet_path_t path, int split_slices, Analysis &an,
               int int8_slices = 6);

// TTGT permutation choice (Section 6, "Optimal permutation for TTGT").  By
// default every valid flattening is ranked by the MI355X time model
// (ttgt_model_us) and the fastest wins; with COMET_TTGT_MODEL=weights, or
// when the label groups have more than kTTGTModelMax orders together, the
// published cost model decides instead: the flattenings that keep each label
// group in the order of a tensor holding it, costed by the positions of the
// dimensions they move.
TTGTChoice choose_ttgt(const Analysis &an);
constexpr int64_t kTTGTModelMax = 512;
// Every valid TTGT flattening (each order of the M, N and K label groups, each
// operand stored K-major or not, with and without exchanging A and B), with
// its Section 6 cost and its modelled time, fastest by the model first.  The
// autotuner times them.
std::vector<TTGTChoice> ttgt_candidates(const Analysis &an);
// Modelled time of one flattening on MI355X, in microseconds: each permute
// launch it needs at its kernel class's measured rate (C's read with beta !=
// 0 included), plus the product at a rate from its FLOP and output bytes,
// raised by the measured penalty of the operand layouts it gives the gather
// kernel.
double ttgt_model_us(const Analysis &an, const TTGTChoice &ch);
int64_t ttgt_cost(const std::string &orig, const std::string &perm, int64_t weight);

// Describe the permutation `in_labels` (with strides) -> `out_labels` (with
// strides) as a PermuteDesc over the output's dims, fusing dims that are
// consecutive in both.
PermuteDesc make_permute(const std::string &out_labels, const std::vector<int64_t> &out_strides,
                         const std::string &in_labels, const std::vector<int64_t> &in_strides,
                         const std::vector<int64_t> &ext_by_out);

// Largest v in {8,4,2,1} such that the table is made of runs off[t..t+v) =
// off[t] + 0..v-1 starting at every multiple of v, and v divides its length.
int contiguous_run(const std::vector<int64_t> &off);

std::string describe_json(const Analysis &an);

size_t elem_size(comet_dtype_t dt);

}  // namespace comet
