// planner_driver.cpp -- runs the host planner (plan.cpp, chain.cpp) under the
// address and undefined-behaviour sanitizers.  Each input line is
//   p <spec> <extents...>            analyze + both TTGT searches + description
//   s <spec> <extents...> | <strides of A> | <strides of B> | <strides of C>
//   c <chain spec> <extents...>      chain planning
// Results are printed (status codes and sizes) so that the test can also
// compare them with the library's own analysis.
#include <cstdio>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "chain.hpp"
#include "plan.hpp"

using namespace comet;

static std::vector<int64_t> read_ints(std::istringstream &in) {
  std::vector<int64_t> v;
  std::string tok;
  while (in >> tok) {
    if (tok == "|") break;
    v.push_back(std::stoll(tok));
  }
  return v;
}

int main() {
  std::string line;
  long n = 0;
  while (std::getline(std::cin, line)) {
    std::istringstream in(line);
    std::string kind, spec;
    if (!(in >> kind >> spec)) continue;
    std::vector<int64_t> ext = read_ints(in);
    if (kind == "c") {
      ChainPlan cp;
      Status st = chain_plan(spec.c_str(), ext.data(), cp);
      std::printf("c %d %zu\n", int(st.code), st.ok() ? chain_json(cp).size() : size_t(0));
    } else {
      std::vector<int64_t> sa, sb, sc;
      if (kind == "s") {
        sa = read_ints(in);
        sb = read_ints(in);
        sc = read_ints(in);
      }
      for (int dt = 0; dt < 2; ++dt) {
        for (int cp : {0, 3, 6}) {
          Analysis an;
          Status st = analyze(spec.c_str(), ext.empty() ? nullptr : ext.data(), sa.empty() ? nullptr : sa.data(),
                              sb.empty() ? nullptr : sb.data(), sc.empty() ? nullptr : sc.data(),
                              comet_dtype_t(dt), comet_compute_t(cp), COMET_PATH_AUTO, 5, an, 6);
          if (!st.ok()) {
            std::printf("p %d\n", int(st.code));
            continue;
          }
          size_t cands = 0;
          if (an.X.empty() && !an.empty_out) {
            TTGTChoice c = choose_ttgt(an);
            cands = ttgt_candidates(an).size();
            (void)c;
          }
          std::printf("p 0 %lld %lld %lld %zu %zu\n", (long long)an.m, (long long)an.n, (long long)an.k, cands,
                      describe_json(an).size());
        }
      }
    }
    ++n;
  }
  std::fprintf(stderr, "%ld lines\n", n);
  return 0;
}
