// chain.cpp -- order of a multi-operand contraction chain (Section 6,
// "Multi-Operand Expression": every grouping gives the same result, the
// number of operations differs, and the ordering with the fewest is chosen
// and lowered to a sequence of binary contractions, Section 5's ta.mult).
//
// The search is a dynamic program over subsets of operands: the intermediate
// of a subset S keeps the labels of S that also occur outside S (in another
// operand or the output); contracting the intermediates of S1 and S2 = S \ S1
// costs 2 * prod(extents of labels(I(S1)) u labels(I(S2))); best(S) is the
// cheapest split.  This visits every binary tree without listing them.
#include "chain.hpp"

#include <algorithm>
#include <cstdio>
#include <functional>
#include <limits>
#include <sstream>

namespace comet {

namespace {

bool is_label(char ch) { return (ch >= 'a' && ch <= 'z') || (ch >= 'A' && ch <= 'Z'); }

}  // namespace

Status chain_plan(const char *spec, const int64_t *extents, ChainPlan &plan) {
  plan = ChainPlan();
  if (!spec) return Status::error(COMET_ERR_NULL_POINTER, "spec is NULL");
  std::vector<std::string> parts(1);
  bool eq = false;
  for (const char *p = spec; *p; ++p) {
    const char ch = *p;
    if (ch == ' ' || ch == '\t' || ch == '\n') continue;
    if (ch == '=') {
      if (eq) return Status::error(COMET_ERR_INVALID_SPEC, "unexpected '=' in chain spec");
      eq = true;
      parts.emplace_back();
      continue;
    }
    if (ch == '*') {
      if (!eq) return Status::error(COMET_ERR_INVALID_SPEC, "unexpected '*' in chain spec");
      parts.emplace_back();
      continue;
    }
    if (!is_label(ch))
      return Status::error(COMET_ERR_INVALID_SPEC, std::string("bad character '") + ch + "' in chain spec");
    std::string &t = parts.back();
    if (t.find(ch) != std::string::npos)
      return Status::error(COMET_ERR_INVALID_SPEC, std::string("label '") + ch + "' repeated in one tensor");
    if ((int)t.size() >= COMET_MAX_RANK) return Status::error(COMET_ERR_INVALID_SPEC, "tensor rank above 12");
    t += ch;
  }
  const int n = int(parts.size()) - 1;
  if (!eq || n < 2) return Status::error(COMET_ERR_INVALID_SPEC, "chain spec must read C=A1*A2[*...]");
  if (n > kChainMaxOperands) return Status::error(COMET_ERR_UNSUPPORTED, "more than 8 operands");
  for (int i = 1; i <= n; ++i)
    if (parts[i].empty()) return Status::error(COMET_ERR_INVALID_SPEC, "an operand without labels");
  plan.out = parts[0];
  plan.operands.assign(parts.begin() + 1, parts.end());
  for (const std::string &t : parts)
    for (char ch : t)
      if (std::find(plan.labels.begin(), plan.labels.end(), ch) == plan.labels.end()) plan.labels.push_back(ch);
  // a label in more than two tensors becomes a batch label of the steps
  // whose operands both hold it while a third tensor still needs it
  for (char ch : plan.labels) {
    int cnt = 0;
    for (const std::string &t : parts) cnt += t.find(ch) != std::string::npos;
    if (cnt < 2) return Status::error(COMET_ERR_INVALID_SPEC, std::string("label '") + ch + "' appears once");
  }
  if (!plan.labels.empty() && !extents) return Status::error(COMET_ERR_NULL_POINTER, "extents is NULL");
  for (size_t i = 0; i < plan.labels.size(); ++i) {
    if (extents[i] < 0) return Status::error(COMET_ERR_INVALID_SHAPE, "negative extent");
    plan.extents.push_back(extents[i]);
  }
  // label sets as bit masks over plan.labels
  const int L = int(plan.labels.size());
  if (L > 62) return Status::error(COMET_ERR_UNSUPPORTED, "too many labels");
  auto mask_of = [&](const std::string &t) {
    uint64_t m = 0;
    for (char ch : t) m |= uint64_t(1) << (std::find(plan.labels.begin(), plan.labels.end(), ch) - plan.labels.begin());
    return m;
  };
  std::vector<uint64_t> opm(n);
  for (int i = 0; i < n; ++i) opm[i] = mask_of(plan.operands[i]);
  const uint64_t outm = mask_of(plan.out);
  auto prod = [&](uint64_t m) {
    double p = 1.0;
    for (int b = 0; b < L; ++b)
      if (m >> b & 1) p *= double(plan.extents[b]);
    return p;
  };
  const int full = (1 << n) - 1;
  // labels of the intermediate of subset S: those of S's operands that also
  // occur in an operand outside S or in the output
  std::vector<uint64_t> inter(1 << n, 0);
  for (int S = 1; S <= full; ++S) {
    uint64_t in = 0, outside = outm;
    for (int i = 0; i < n; ++i) (S >> i & 1 ? in : outside) |= opm[i];
    inter[S] = in & outside;
  }
  const double inf = std::numeric_limits<double>::infinity();
  std::vector<double> best(1 << n, inf);
  std::vector<int> split(1 << n, 0);
  for (int i = 0; i < n; ++i) best[1 << i] = 0.0;
  for (int S = 1; S <= full; ++S) {
    if ((S & (S - 1)) == 0) continue;
    // every split into two non-empty parts, each unordered pair once
    for (int S1 = (S - 1) & S; S1 > 0; S1 = (S1 - 1) & S) {
      const int S2 = S ^ S1;
      if (S1 < S2) continue;
      const double c = best[S1] + best[S2] + 2.0 * prod(inter[S1] | inter[S2]);
      if (c < best[S]) {
        best[S] = c;
        split[S] = S1;
      }
    }
  }
  plan.flops = best[full];
  // left to right
  {
    double f = 0.0;
    int S = 1;
    for (int i = 1; i < n; ++i) {
      f += 2.0 * prod(inter[S] | inter[1 << i]);
      S |= 1 << i;
    }
    plan.natural_flops = f;
  }
  // emit the steps of the chosen tree, children before parents
  std::vector<int> id(1 << n, -1);
  for (int i = 0; i < n; ++i) id[1 << i] = i;
  int next = n;
  // labels of an intermediate, ordered as in the output, then by first
  // appearance in the chain's operands
  auto order = [&](uint64_t m) {
    std::string s;
    for (char ch : plan.out)
      if (m >> (std::find(plan.labels.begin(), plan.labels.end(), ch) - plan.labels.begin()) & 1) s += ch;
    for (const std::string &t : plan.operands)
      for (char ch : t) {
        const int b = int(std::find(plan.labels.begin(), plan.labels.end(), ch) - plan.labels.begin());
        if ((m >> b & 1) && s.find(ch) == std::string::npos) s += ch;
      }
    return s;
  };
  std::vector<std::string> labels_of(size_t(n) + size_t(n), "");
  for (int i = 0; i < n; ++i) labels_of[i] = plan.operands[i];
  std::function<int(int)> emit = [&](int S) -> int {
    if (id[S] >= 0) return id[S];
    const int S1 = split[S], S2 = S ^ S1;
    const int a = emit(S1), b = emit(S2);
    ChainStep st;
    st.left = a;
    st.right = b;
    st.out_labels = S == full ? plan.out : order(inter[S]);
    st.spec = st.out_labels + "=" + labels_of[a] + "*" + labels_of[b];
    st.flops = 2.0 * prod(inter[S1] | inter[S2]);
    plan.steps.push_back(st);
    id[S] = next;
    labels_of[next] = st.out_labels;
    return next++;
  };
  emit(full);
  return Status{};
}

std::string chain_json(const ChainPlan &plan) {
  std::ostringstream o;
  char buf[64];
  auto num = [&](double x) {
    std::snprintf(buf, sizeof buf, "%.17g", x);
    return std::string(buf);
  };
  o << "{\"out\":\"" << plan.out << "\",\"operands\":[";
  for (size_t i = 0; i < plan.operands.size(); ++i) o << (i ? "," : "") << "\"" << plan.operands[i] << "\"";
  o << "],\"flops\":" << num(plan.flops) << ",\"natural_flops\":" << num(plan.natural_flops) << ",\"steps\":[";
  for (size_t i = 0; i < plan.steps.size(); ++i) {
    const ChainStep &s = plan.steps[i];
    o << (i ? "," : "") << "{\"left\":" << s.left << ",\"right\":" << s.right << ",\"spec\":\"" << s.spec
      << "\",\"flops\":" << num(s.flops) << "}";
  }
  o << "]}";
  return o.str();
}

}  // namespace comet
