// chain.hpp -- multi-operand contraction chains (Section 5, ta.mult / ta.set;
// Section 6, "Multi-Operand Expression"): the order of pairwise contractions,
// chosen as the binary tree with the fewest algorithmic operations.  Host only.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "plan.hpp"

namespace comet {

constexpr int kChainMaxOperands = 8;

// One pairwise contraction of the chain.  Operands 0..n-1 are the inputs,
// n.. the intermediates in the order the steps produce them; the last step
// produces the output.
struct ChainStep {
  int left = 0, right = 0;     // operand indices
  std::string spec;            // "T=X*Y" in the chain's labels
  std::string out_labels;      // labels of the step's result, outermost first
  double flops = 0.0;          // 2 * product of the extents of every label the step touches
};

struct ChainPlan {
  std::string out;                       // output labels
  std::vector<std::string> operands;     // input labels
  std::vector<char> labels;              // distinct labels, first appearance scanning out, operands
  std::vector<int64_t> extents;          // per entry of `labels`
  std::vector<ChainStep> steps;          // the chosen order
  double flops = 0.0;                    // its total
  double natural_flops = 0.0;            // left to right: ((A1 A2) A3) ...
};

// Parse "C=A1*A2*...*An" (2 <= n <= kChainMaxOperands; every label in at
// least two of the tensors) with one extent per distinct label, in order of
// first appearance scanning C then the operands, and choose the order.
Status chain_plan(const char *spec, const int64_t *extents, ChainPlan &plan);

std::string chain_json(const ChainPlan &plan);

}  // namespace comet
