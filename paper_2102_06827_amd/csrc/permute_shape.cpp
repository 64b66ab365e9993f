// permute_shape.cpp -- classification of a permutation onto the permute
// kernels (flat walk, row stream, LDS transpose) and its time model.
#include "permute_shape.hpp"

#include <algorithm>
#include <cmath>

namespace comet {

PermShape permute_shape(int ndim, const int64_t *ext, const int64_t *s_in, const int64_t *s_out, bool reads) {
  PermShape s;
  s.total = 1;
  for (int k = 0; k < ndim; ++k) s.total *= ext[k];
  if (s.total == 0) return s;
  std::vector<PermDim> &d = s.d;
  for (int k = 0; k < ndim; ++k)
    if (ext[k] != 1) d.push_back({ext[k], s_in[k], s_out[k]});
  // fuse pairs that are contiguous in both tensors (the faster dimension
  // continues into the slower one on both sides)
  bool merged = true;
  while (merged) {
    merged = false;
    for (size_t f = 0; f < d.size() && !merged; ++f)
      for (size_t g = 0; g < d.size() && !merged; ++g) {
        if (f == g) continue;
        if (d[g].si == d[f].si * d[f].ext && d[g].so == d[f].so * d[f].ext) {
          d[f].ext *= d[g].ext;
          d.erase(d.begin() + g);
          merged = true;
        }
      }
  }
  const int n = (int)d.size();
  for (int k = 0; k < n; ++k) {
    if (s.uo < 0 || d[k].so < d[s.uo].so) s.uo = k;
    if (s.ui < 0 || d[k].si < d[s.ui].si) s.ui = k;
  }
  if (!reads) s.ui = s.uo;
  if (n == 1 && d[0].so == 1 && (!reads || d[0].si == 1)) {
    s.kind = PERM_FLAT;
    return s;
  }
  if (n == 0 || s.ui == s.uo) {
    s.kind = PERM_STREAM;
    return s;
  }
  s.kind = PERM_TILED;
  std::vector<bool> used(n, false);
  used[s.ui] = used[s.uo] = true;
  s.gi = {s.ui};
  s.go = {s.uo};
  s.EI = d[s.ui].ext;
  s.EO = d[s.uo].ext;
  auto grow = [&](std::vector<int> &g, int64_t &E, bool input) {
    while (E < kPermTile) {
      const PermDim &last = d[g.back()];
      int next = -1;
      for (int k = 0; k < n; ++k) {
        if (used[k]) continue;
        if (input ? d[k].si == last.si * last.ext : d[k].so == last.so * last.ext) {
          next = k;
          break;
        }
      }
      if (next < 0) break;
      used[next] = true;
      g.push_back(next);
      E *= d[next].ext;
    }
  };
  grow(s.gi, s.EI, true);
  grow(s.go, s.EO, false);
  for (int k = 0; k < n; ++k)
    if (!used[k]) s.rest.push_back(k);
  std::sort(s.rest.begin(), s.rest.end(), [&](int x, int y) { return d[x].so < d[y].so; });
  return s;
}

double permute_time_us(const PermShape &s, int elem_bytes, bool reads_out) {
  if (s.kind == PERM_EMPTY) return 0.0;
  const double bytes = double(s.total) * elem_bytes * (reads_out ? 3.0 : 2.0);
  // TB/s of each kernel class and the fixed cost of a launch, fitted to the
  // permute kernels' times over all 352 flattenings of two CCSD-like FP64
  // contractions (75 MB to 1 GB per tensor) on MI355X
  double tbs = 5.1;
  if (s.kind == PERM_FLAT) {
    tbs = 5.5;
  } else if (s.kind == PERM_STREAM) {
    // rows of fewer than 32 elements fill fewer whole cache lines per wave
    tbs = s.d.empty() || s.d[s.uo].ext >= kPermTile ? 5.5 : 4.8;
  } else {
    // a partly filled tile leaves lanes idle: a half-filled one ran at
    // 4.0 TB/s against 5.1 for a full one
    const double fill = double(std::min<int64_t>(s.EI, kPermTile)) * double(std::min<int64_t>(s.EO, kPermTile)) /
                        double(kPermTile * kPermTile);
    tbs = 5.1 * std::pow(fill, 0.35);
  }
  return 3.3 + bytes / (tbs * 1e6);
}

}  // namespace comet
