// plan.cpp -- host analysis of a binary contraction (no HIP calls).
//
// Parsing and validation follow the label rules of Section 2: summation
// indices appear in both inputs and not in the output; free indices appear in
// one input and the output.  A label in all three tensors is a batch label:
// it selects one slice of C, A and B, and each slice is an ordinary
// contraction of the other labels.  Label fusion is the index merging of the TTGT
// flattening (Section 2: consecutive indices merged into one matrix index);
// here it is done only where the merged index is still one stride in every
// tensor holding it.  The TTGT permutation is picked by the cost model of
// Section 6 ("Optimal permutation for TTGT").
#include "plan.hpp"
#include "permute_shape.hpp"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <set>
#include <sstream>

namespace comet {

size_t elem_size(comet_dtype_t dt) { return dt == COMET_F64 ? 8 : 4; }

static bool is_label(char ch) { return (ch >= 'a' && ch <= 'z') || (ch >= 'A' && ch <= 'Z'); }

Status parse_spec(const char *spec, Analysis &an) {
  if (!spec) return Status::error(COMET_ERR_NULL_POINTER, "spec is NULL");
  std::string parts[3];
  int part = 0;
  for (const char *p = spec; *p; ++p) {
    char ch = *p;
    if (ch == ' ' || ch == '\t' || ch == '\n') continue;
    if (ch == '=') {
      if (part != 0) return Status::error(COMET_ERR_INVALID_SPEC, "unexpected '=' in spec");
      part = 1;
      continue;
    }
    if (ch == '*') {
      if (part != 1) return Status::error(COMET_ERR_INVALID_SPEC, "unexpected '*' in spec");
      part = 2;
      continue;
    }
    if (!is_label(ch))
      return Status::error(COMET_ERR_INVALID_SPEC, std::string("bad character '") + ch + "' in spec");
    if (parts[part].find(ch) != std::string::npos)
      return Status::error(COMET_ERR_INVALID_SPEC, std::string("label '") + ch + "' repeated in one tensor");
    if ((int)parts[part].size() >= COMET_MAX_RANK)
      return Status::error(COMET_ERR_INVALID_SPEC, "tensor rank above COMET_MAX_RANK");
    parts[part] += ch;
  }
  if (part != 2) return Status::error(COMET_ERR_INVALID_SPEC, "spec must read C=A*B");
  an.spec_c = parts[0];
  an.spec_a = parts[1];
  an.spec_b = parts[2];
  an.labels.clear();
  for (int t = 0; t < 3; ++t)
    for (char ch : parts[t])
      if (std::find(an.labels.begin(), an.labels.end(), ch) == an.labels.end()) an.labels.push_back(ch);
  for (char ch : an.labels) {
    int cnt = (an.spec_c.find(ch) != std::string::npos) + (an.spec_a.find(ch) != std::string::npos) +
              (an.spec_b.find(ch) != std::string::npos);
    if (cnt < 2)
      return Status::error(COMET_ERR_INVALID_SPEC, std::string("label '") + ch + "' appears in only one tensor");
  }
  return Status{};
}

static bool mul_ok(int64_t a, int64_t b, int64_t *out) { return !__builtin_mul_overflow(a, b, out); }
static bool add_ok(int64_t a, int64_t b, int64_t *out) { return !__builtin_add_overflow(a, b, out); }

// element span of a tensor (max offset + 1), 0 if empty; false on overflow
static bool tensor_span(const std::vector<int64_t> &ext, const std::vector<int64_t> &str, int64_t *span) {
  int64_t hi = 0;
  for (size_t i = 0; i < ext.size(); ++i) {
    if (ext[i] == 0) {
      *span = 0;
      return true;
    }
  }
  for (size_t i = 0; i < ext.size(); ++i) {
    int64_t t;
    if (!mul_ok(ext[i] - 1, str[i], &t) || !add_ok(hi, t, &hi)) return false;
  }
  return add_ok(hi, 1, span);
}

static Status strides_for(const std::string &labs, const std::vector<int64_t> &ext_of, const Analysis &an,
                          const int64_t *given, std::vector<int64_t> &out, const char *name) {
  out.assign(labs.size(), 0);
  std::vector<int64_t> ext(labs.size());
  for (size_t p = 0; p < labs.size(); ++p) {
    auto it = std::find(an.labels.begin(), an.labels.end(), labs[p]);
    ext[p] = ext_of[it - an.labels.begin()];
  }
  if (given) {
    for (size_t p = 0; p < labs.size(); ++p) {
      if (given[p] < 0)
        return Status::error(COMET_ERR_INVALID_STRIDE, std::string("negative stride in ") + name);
      out[p] = given[p];
    }
  } else {
    int64_t s = 1;
    for (int p = (int)labs.size() - 1; p >= 0; --p) {
      out[p] = s;
      if (ext[p] > 0 && !mul_ok(s, ext[p], &s))
        return Status::error(COMET_ERR_INVALID_SHAPE, std::string("size of ") + name + " overflows int64");
    }
  }
  int64_t span;
  if (!tensor_span(ext, out, &span))
    return Status::error(COMET_ERR_INVALID_SHAPE, std::string("extent of ") + name + " overflows int64");
  return Status{};
}

int contiguous_run(const std::vector<int64_t> &off) {
  const int64_t n = (int64_t)off.size();
  for (int v = 8; v > 1; v /= 2) {
    if (n % v) continue;
    bool ok = true;
    for (int64_t t = 0; t < n && ok; t += v)
      for (int i = 1; i < v; ++i)
        if (off[t + i] != off[t] + i) {
          ok = false;
          break;
        }
    if (ok) return v;
  }
  return 1;
}

static void build_table(const std::vector<Dim> &dims, int which, std::vector<int64_t> &out) {
  int64_t total = 1;
  for (const Dim &d : dims) total *= d.ext;
  out.assign((size_t)total, 0);
  if (total == 0) return;
  std::vector<int64_t> idx(dims.size(), 0);
  int64_t cur = 0;
  auto stride = [&](const Dim &d) { return which == 0 ? d.sA : which == 1 ? d.sB : d.sC; };
  for (int64_t t = 0; t < total; ++t) {
    out[(size_t)t] = cur;
    for (int i = (int)dims.size() - 1; i >= 0; --i) {
      if (++idx[i] < dims[i].ext) {
        cur += stride(dims[i]);
        break;
      }
      cur -= (dims[i].ext - 1) * stride(dims[i]);
      idx[i] = 0;
    }
  }
}

// Fuse neighbours (outer d1, inner d2) where every tensor holding them has
// stride(d1) == stride(d2) * ext(d2).
static void fuse(std::vector<Dim> &dims, bool useA, bool useB, bool useC) {
  bool changed = true;
  while (changed) {
    changed = false;
    for (size_t i = 0; i + 1 < dims.size(); ++i) {
      Dim &o = dims[i], &in = dims[i + 1];
      bool ok = (!useA || o.sA == in.sA * in.ext) && (!useB || o.sB == in.sB * in.ext) &&
                (!useC || o.sC == in.sC * in.ext);
      if (ok) {
        Dim f = in;
        f.labels = o.labels + in.labels;
        f.ext = o.ext * in.ext;
        dims[i] = f;
        dims.erase(dims.begin() + i + 1);
        changed = true;
        break;
      }
    }
  }
}

static int64_t min_stride(const std::vector<Dim> &dims, int which) {
  int64_t best = INT64_MAX;
  for (const Dim &d : dims) {
    int64_t s = which == 0 ? d.sA : which == 1 ? d.sB : d.sC;
    best = std::min(best, s);
  }
  return best;
}

static void sort_by(std::vector<Dim> &dims, int primary, int secondary) {
  auto key = [](const Dim &d, int w) { return w == 0 ? d.sA : w == 1 ? d.sB : d.sC; };
  std::stable_sort(dims.begin(), dims.end(), [&](const Dim &x, const Dim &y) {
    int64_t px = key(x, primary), py = key(y, primary);
    if (px != py) return px > py;
    return key(x, secondary) > key(y, secondary);
  });
}

int64_t ttgt_cost(const std::string &orig, const std::string &perm, int64_t weight) {
  // A dimension that leaves its place costs more the further out it sat:
  // row-major storage makes moving the outer dimensions the expensive part.
  int64_t r = (int64_t)orig.size(), c = 0;
  for (int64_t p = 0; p < r; ++p)
    if (p >= (int64_t)perm.size() || orig[p] != perm[p]) c += weight * (r - p);
  return c;
}

static std::string labels_in(const std::string &order_src, const std::string &set) {
  std::string r;
  for (char ch : order_src)
    if (set.find(ch) != std::string::npos) r += ch;
  return r;
}

static bool dense_rowmajor(const std::vector<int64_t> &ext, const std::vector<int64_t> &str) {
  int64_t s = 1;
  for (int p = (int)ext.size() - 1; p >= 0; --p) {
    if (ext[p] != 1 && str[p] != s) return false;
    s *= ext[p];
  }
  return true;
}

static TTGTChoice choose_ttgt_weights(const Analysis &an) {
  const std::string &c = an.spec_c, &a = an.spec_a, &b = an.spec_b;
  std::string Mset, Nset, Kset;
  for (char ch : a) (c.find(ch) != std::string::npos ? Mset : Kset) += ch;
  for (char ch : b)
    if (c.find(ch) != std::string::npos) Nset += ch;
  // candidate orders of each label group: as it sits in either tensor holding it
  std::vector<std::string> Mo{labels_in(a, Mset), labels_in(c, Mset)};
  std::vector<std::string> No{labels_in(b, Nset), labels_in(c, Nset)};
  std::vector<std::string> Ko{labels_in(a, Kset), labels_in(b, Kset)};
  auto uniq = [](std::vector<std::string> &v) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  };
  uniq(Mo);
  uniq(No);
  uniq(Ko);
  auto ext_of = [&](char ch) {
    return an.extents[std::find(an.labels.begin(), an.labels.end(), ch) - an.labels.begin()];
  };
  auto exts = [&](const std::string &s) {
    std::vector<int64_t> e;
    for (char ch : s) e.push_back(ext_of(ch));
    return e;
  };
  bool denseA = dense_rowmajor(exts(a), an.strA), denseB = dense_rowmajor(exts(b), an.strB),
       denseC = dense_rowmajor(exts(c), an.strC);
  TTGTChoice best;
  bool have = false;
  for (int swap = 0; swap < 2; ++swap)
    for (const auto &mo : Mo)
      for (const auto &no : No)
        for (const auto &ko : Ko)
          for (int la = 0; la < 2; ++la)
            for (int lb = 0; lb < 2; ++lb) {
              // left operand rows x K, right operand K x cols; the product is
              // rows x cols.  Without the exchange rows = M (from A), cols = N.
              std::string rows = swap ? no : mo, cols = swap ? mo : no;
              std::string left = la ? ko + rows : rows + ko;     // la: left stored K-major
              std::string right = lb ? cols + ko : ko + cols;    // lb: right stored N-major
              std::string prod = rows + cols;
              std::string ap = swap ? right : left, bp = swap ? left : right;
              int64_t cost = ttgt_cost(a, ap, 1) * (ap == a && denseA ? 0 : 1) +
                             ttgt_cost(b, bp, 1) * (bp == b && denseB ? 0 : 1) +
                             ttgt_cost(c, prod, 2) * (prod == c && denseC ? 0 : 1);
              // a copy of a dense tensor in its own order is free; a strided
              // one must still be packed, charged as moving everything
              if (ap == a && !denseA) cost += ttgt_cost(a, std::string(a.size(), '#'), 1);
              if (bp == b && !denseB) cost += ttgt_cost(b, std::string(b.size(), '#'), 1);
              if (prod == c && !denseC) cost += ttgt_cost(c, std::string(c.size(), '#'), 2);
              TTGTChoice ch;
              ch.swap = swap;
              ch.a_order = ap;
              ch.b_order = bp;
              ch.c_order = prod;
              ch.a_copy = !(ap == a && denseA);
              ch.b_copy = !(bp == b && denseB);
              ch.c_copy = !(prod == c && denseC);
              ch.cost = cost;
              std::string key = ap + "|" + bp + "|" + prod + (swap ? "1" : "0");
              std::string bkey = best.a_order + "|" + best.b_order + "|" + best.c_order + (best.swap ? "1" : "0");
              if (!have || cost < best.cost || (cost == best.cost && key < bkey)) {
                best = ch;
                have = true;
              }
            }
  return best;
}

double ttgt_model_us(const Analysis &an, const TTGTChoice &ch) {
  auto ext_of = [&](char ch_) {
    return an.extents[std::find(an.labels.begin(), an.labels.end(), ch_) - an.labels.begin()];
  };
  // dense row-major stride of `label` in `order`
  auto dense = [&](const std::string &order, char label) {
    int64_t st = 1;
    for (size_t p = order.size(); p-- > 0;) {
      if (order[p] == label) return st;
      st *= ext_of(order[p]);
    }
    return int64_t(0);
  };
  const int es = (int)elem_size(an.dtype);
  double t = 0.0;
  // one permute from `src` (strides given, or dense when null) to `dst` (the same)
  auto perm = [&](const std::string &src, const std::vector<int64_t> *ssrc, const std::string &dst,
                  const std::vector<int64_t> *sdst, bool reads_out) {
    std::vector<int64_t> e, si, so;
    for (size_t p = 0; p < src.size(); ++p) {
      e.push_back(ext_of(src[p]));
      si.push_back(ssrc ? (*ssrc)[p] : dense(src, src[p]));
      const size_t q = dst.find(src[p]);
      so.push_back(sdst ? (*sdst)[q] : dense(dst, src[p]));
    }
    t += permute_time_us(permute_shape((int)e.size(), e.data(), si.data(), so.data(), true), es, reads_out);
  };
  if (ch.a_copy) perm(an.spec_a, &an.strA, ch.a_order, nullptr, false);
  if (ch.b_copy) perm(an.spec_b, &an.strB, ch.b_order, nullptr, false);
  // a plan serves any beta: the output permute is costed with its read of C
  if (ch.c_copy) perm(ch.c_order, nullptr, an.spec_c, &an.strC, true);
  // the product: FLOP at 65 (FP64) or 120 (FP32) TFLOP/s, or its output at
  // 5 TB/s written (and read), whichever is longer
  double M = 1, N = 1, K = 1;
  for (char l : an.spec_a) (an.spec_c.find(l) != std::string::npos ? M : K) *= double(ext_of(l));
  for (char l : an.spec_b)
    if (an.spec_c.find(l) != std::string::npos) N *= double(ext_of(l));
  const double rate = an.dtype == COMET_F64 ? 65e12 : 120e12;
  double g = std::max(2.0 * M * N * K / rate, 2.0 * es * M * N / 5e12) * 1e6;
  // the gather kernel's left operand holds the product's row labels and its
  // right operand its column labels; measured on the CCSD-like product:
  // +2% when the left operand's unit stride is not along the summation,
  // +1.7% when the right operand's unit stride is along it
  if (!ch.c_order.empty()) {
    const bool a_left = an.spec_a.find(ch.c_order[0]) != std::string::npos;
    const std::string &left = a_left ? ch.a_order : ch.b_order;
    const std::string &right = a_left ? ch.b_order : ch.a_order;
    auto in_k = [&](char l) { return an.spec_c.find(l) == std::string::npos; };
    if (!left.empty() && !in_k(left.back())) g *= 1.02;
    if (!right.empty() && in_k(right.back())) g *= 1.017;
  }
  return t + g;
}

static int64_t orders_of(size_t n) {
  int64_t f = 1;
  for (size_t k = 2; k <= n; ++k) f *= int64_t(k);
  return f;
}

TTGTChoice choose_ttgt(const Analysis &an) {
  const std::string &c = an.spec_c, &a = an.spec_a, &b = an.spec_b;
  size_t nm = 0, nn = 0, nk = 0;
  for (char ch : a) (c.find(ch) != std::string::npos ? nm : nk) += 1;
  for (char ch : b)
    if (c.find(ch) != std::string::npos) nn += 1;
  const char *env = std::getenv("COMET_TTGT_MODEL");
  const bool weights = env && std::strcmp(env, "weights") == 0;
  if (weights || nm > 8 || nn > 8 || nk > 8 || orders_of(nm) * orders_of(nn) * orders_of(nk) > kTTGTModelMax) {
    TTGTChoice ch = choose_ttgt_weights(an);
    ch.model_us = ttgt_model_us(an, ch);
    return ch;
  }
  return ttgt_candidates(an).front();
}

std::vector<TTGTChoice> ttgt_candidates(const Analysis &an) {
  const std::string &c = an.spec_c, &a = an.spec_a, &b = an.spec_b;
  std::string Mset, Nset, Kset;
  for (char ch : a) (c.find(ch) != std::string::npos ? Mset : Kset) += ch;
  for (char ch : b)
    if (c.find(ch) != std::string::npos) Nset += ch;
  auto perms = [](std::string x) {
    std::vector<std::string> v;
    std::sort(x.begin(), x.end());
    do v.push_back(x);
    while (std::next_permutation(x.begin(), x.end()));
    return v;
  };
  auto ext_of = [&](char ch) {
    return an.extents[std::find(an.labels.begin(), an.labels.end(), ch) - an.labels.begin()];
  };
  auto exts = [&](const std::string &s) {
    std::vector<int64_t> e;
    for (char ch : s) e.push_back(ext_of(ch));
    return e;
  };
  const bool denseA = dense_rowmajor(exts(a), an.strA), denseB = dense_rowmajor(exts(b), an.strB),
             denseC = dense_rowmajor(exts(c), an.strC);
  std::vector<TTGTChoice> out;
  std::set<std::string> seen;
  for (const auto &mo : perms(Mset))
    for (const auto &no : perms(Nset))
      for (const auto &ko : perms(Kset))
        for (int swap = 0; swap < 2; ++swap)
          for (int la = 0; la < 2; ++la)
            for (int lb = 0; lb < 2; ++lb) {
              const std::string rows = swap ? no : mo, cols = swap ? mo : no;
              const std::string left = la ? ko + rows : rows + ko;
              const std::string right = lb ? cols + ko : ko + cols;
              TTGTChoice ch;
              ch.swap = swap;
              ch.a_order = swap ? right : left;
              ch.b_order = swap ? left : right;
              ch.c_order = rows + cols;
              const std::string key = ch.a_order + "|" + ch.b_order + "|" + ch.c_order;
              if (!seen.insert(key).second) continue;
              ch.a_copy = !(ch.a_order == a && denseA);
              ch.b_copy = !(ch.b_order == b && denseB);
              ch.c_copy = !(ch.c_order == c && denseC);
              ch.cost = (ch.a_copy ? ttgt_cost(a, ch.a_order == a ? std::string(a.size(), '#') : ch.a_order, 1) : 0) +
                        (ch.b_copy ? ttgt_cost(b, ch.b_order == b ? std::string(b.size(), '#') : ch.b_order, 1) : 0) +
                        (ch.c_copy ? ttgt_cost(c, ch.c_order == c ? std::string(c.size(), '#') : ch.c_order, 2) : 0);
              ch.model_us = ttgt_model_us(an, ch);
              out.push_back(ch);
            }
  std::stable_sort(out.begin(), out.end(), [](const TTGTChoice &x, const TTGTChoice &y) {
    if (x.model_us != y.model_us) return x.model_us < y.model_us;
    return x.cost < y.cost;
  });
  return out;
}

PermuteDesc make_permute(const std::string &out_labels, const std::vector<int64_t> &out_strides,
                         const std::string &in_labels, const std::vector<int64_t> &in_strides,
                         const std::vector<int64_t> &ext_by_out) {
  PermuteDesc d;
  for (size_t p = 0; p < out_labels.size(); ++p) {
    if (ext_by_out[p] == 1) continue;
    size_t q = in_labels.find(out_labels[p]);
    d.ext.push_back(ext_by_out[p]);
    d.s_out.push_back(out_strides[p]);
    d.s_in.push_back(in_strides[q]);
  }
  // fuse dims consecutive in both
  bool changed = true;
  while (changed) {
    changed = false;
    for (size_t i = 0; i + 1 < d.ext.size(); ++i) {
      if (d.s_out[i] == d.s_out[i + 1] * d.ext[i + 1] && d.s_in[i] == d.s_in[i + 1] * d.ext[i + 1]) {
        d.ext[i] *= d.ext[i + 1];
        d.s_out[i] = d.s_out[i + 1];
        d.s_in[i] = d.s_in[i + 1];
        d.ext.erase(d.ext.begin() + i + 1);
        d.s_out.erase(d.s_out.begin() + i + 1);
        d.s_in.erase(d.s_in.begin() + i + 1);
        changed = true;
        break;
      }
    }
  }
  return d;
}

Status analyze(const char *spec, const int64_t *extents, const int64_t *strides_A, const int64_t *strides_B,
               const int64_t *strides_C, comet_dtype_t dtype, comet_compute_t compute, comet_path_t path,
               int split_slices, Analysis &an, int int8_slices) {
  an = Analysis();
  Status st = parse_spec(spec, an);
  if (!st.ok()) return st;
  if (dtype != COMET_F64 && dtype != COMET_F32) return Status::error(COMET_ERR_UNSUPPORTED, "unknown dtype");
  if (compute < COMET_COMPUTE_DEFAULT || compute > COMET_COMPUTE_SPLIT_INT8)
    return Status::error(COMET_ERR_UNSUPPORTED, "unknown compute mode");
  if (path < COMET_PATH_AUTO || path > COMET_PATH_TTGT) return Status::error(COMET_ERR_UNSUPPORTED, "unknown path");
  an.dtype = dtype;
  an.compute = compute == COMET_COMPUTE_DEFAULT ? (dtype == COMET_F64 ? COMET_COMPUTE_F64 : COMET_COMPUTE_F32)
                                                : compute;
  an.split_slices = compute == COMET_COMPUTE_SPLIT_INT8 ? int8_slices : split_slices;
  if (!an.labels.empty() && !extents) return Status::error(COMET_ERR_NULL_POINTER, "extents is NULL");
  an.extents.assign(extents, extents + an.labels.size());
  for (size_t i = 0; i < an.labels.size(); ++i)
    if (an.extents[i] < 0)
      return Status::error(COMET_ERR_INVALID_SHAPE, std::string("negative extent for label '") + an.labels[i] + "'");
  st = strides_for(an.spec_a, an.extents, an, strides_A, an.strA, "A");
  if (!st.ok()) return st;
  st = strides_for(an.spec_b, an.extents, an, strides_B, an.strB, "B");
  if (!st.ok()) return st;
  st = strides_for(an.spec_c, an.extents, an, strides_C, an.strC, "C");
  if (!st.ok()) return st;

  auto ext_of = [&](char ch) {
    return an.extents[std::find(an.labels.begin(), an.labels.end(), ch) - an.labels.begin()];
  };
  auto stride_in = [&](const std::string &labs, const std::vector<int64_t> &s, char ch) -> int64_t {
    size_t p = labs.find(ch);
    return p == std::string::npos ? 0 : s[p];
  };
  // C must not overlap itself
  {
    std::vector<std::pair<int64_t, int64_t>> sd;   // (stride, extent)
    for (size_t p = 0; p < an.spec_c.size(); ++p) {
      int64_t e = ext_of(an.spec_c[p]);
      if (e <= 1) continue;
      if (an.strC[p] == 0)
        return Status::error(COMET_ERR_INVALID_STRIDE, "C has stride 0 on a dimension of extent > 1");
      sd.push_back({an.strC[p], e});
    }
    std::sort(sd.begin(), sd.end());
    for (size_t i = 0; i + 1 < sd.size(); ++i) {
      int64_t need;
      if (!mul_ok(sd[i].first, sd[i].second, &need) || sd[i + 1].first < need)
        return Status::error(COMET_ERR_INVALID_STRIDE, "C dimensions overlap in memory");
    }
  }
  {
    std::vector<int64_t> e;
    for (char ch : an.spec_a) e.push_back(ext_of(ch));
    tensor_span(e, an.strA, &an.sizeA);
    e.clear();
    for (char ch : an.spec_b) e.push_back(ext_of(ch));
    tensor_span(e, an.strB, &an.sizeB);
    e.clear();
    for (char ch : an.spec_c) e.push_back(ext_of(ch));
    tensor_span(e, an.strC, &an.sizeC);
  }

  auto in_all = [&](char ch) {
    return an.spec_a.find(ch) != std::string::npos && an.spec_b.find(ch) != std::string::npos &&
           an.spec_c.find(ch) != std::string::npos;
  };
  // classify; exchange A and B when C's smallest-stride matrix dimension
  // comes from A
  {
    int64_t best = INT64_MAX;
    char unit = 0;
    for (size_t p = 0; p < an.spec_c.size(); ++p) {
      if (ext_of(an.spec_c[p]) <= 1 || in_all(an.spec_c[p])) continue;
      if (an.strC[p] < best) {
        best = an.strC[p];
        unit = an.spec_c[p];
      }
    }
    an.swapped = unit && an.spec_a.find(unit) != std::string::npos;
  }
  const std::string &la = an.swapped ? an.spec_b : an.spec_a;
  const std::string &lb = an.swapped ? an.spec_a : an.spec_b;
  const std::vector<int64_t> &sa = an.swapped ? an.strB : an.strA;
  const std::vector<int64_t> &sb = an.swapped ? an.strA : an.strB;
  for (char ch : an.labels) {
    Dim d;
    d.labels = std::string(1, ch);
    d.ext = ext_of(ch);
    d.sA = stride_in(la, sa, ch);
    d.sB = stride_in(lb, sb, ch);
    d.sC = stride_in(an.spec_c, an.strC, ch);
    bool inA = la.find(ch) != std::string::npos, inB = lb.find(ch) != std::string::npos;
    d.cls = in_all(ch) ? CLS_X : (inA && inB) ? CLS_K : inA ? CLS_M : CLS_N;
    int64_t &tot = d.cls == CLS_M ? an.m : d.cls == CLS_N ? an.n : d.cls == CLS_K ? an.k : an.nb;
    tot *= d.ext;
    if (d.ext == 1) continue;
    (d.cls == CLS_M ? an.M : d.cls == CLS_N ? an.N : d.cls == CLS_K ? an.K : an.X).push_back(d);
  }
  an.empty_out = an.m == 0 || an.n == 0 || an.nb == 0;
  an.empty_sum = an.k == 0;
  const int64_t kTableCap = int64_t(1) << 28;
  if (an.m > kTableCap || an.n > kTableCap || an.k > kTableCap || an.nb > kTableCap)
    return Status::error(COMET_ERR_UNSUPPORTED, "a flattened matrix or batch dimension exceeds 2^28");

  // dimension order inside each class (outermost first, last fastest)
  bool a_m_contig = !an.M.empty() && (an.K.empty() || min_stride(an.M, 0) < min_stride(an.K, 0));
  bool b_n_contig = !an.N.empty() && (an.K.empty() || min_stride(an.N, 1) < min_stride(an.K, 1));
  if (a_m_contig) sort_by(an.M, 0, 2); else sort_by(an.M, 2, 0);
  if (b_n_contig) sort_by(an.N, 1, 2); else sort_by(an.N, 2, 1);
  // K follows the operand that reads along K; when both do, the one with the
  // smaller stride there, and on a tie the larger operand (the other one's
  // scattered reads then cost little: the GEMV-like "ia=dn*inad" reads its
  // 75 MB operand in runs of 96 instead of one element per row)
  bool k_by_a;
  if (a_m_contig) {
    k_by_a = false;
  } else if (b_n_contig) {
    k_by_a = true;
  } else {
    const int64_t ka = min_stride(an.K, 0), kb = min_stride(an.K, 1);
    const int64_t size0 = an.swapped ? an.sizeB : an.sizeA, size1 = an.swapped ? an.sizeA : an.sizeB;
    k_by_a = ka < kb || (ka == kb && size0 >= size1);
  }
  if (k_by_a) sort_by(an.K, 0, 1);
  else sort_by(an.K, 1, 0);
  fuse(an.M, true, false, true);
  fuse(an.N, false, true, true);
  fuse(an.K, true, true, false);
  // batch entries in C's memory order
  sort_by(an.X, 2, 0);
  fuse(an.X, true, true, true);

  if (!an.empty_out) {
    if (!an.X.empty()) {
      build_table(an.X, 0, an.offAx);
      build_table(an.X, 1, an.offBx);
      build_table(an.X, 2, an.offCx);
    }
    build_table(an.M, 0, an.offAm);
    build_table(an.M, 2, an.offCm);
    build_table(an.N, 1, an.offBn);
    build_table(an.N, 2, an.offCn);
    if (!an.empty_sum) {
      build_table(an.K, 0, an.offAk);
      build_table(an.K, 1, an.offBk);
    }
    an.runAm = contiguous_run(an.offAm);
    an.runCm = contiguous_run(an.offCm);
    an.runBn = contiguous_run(an.offBn);
    an.runCn = contiguous_run(an.offCn);
    if (!an.empty_sum) {
      an.runAk = contiguous_run(an.offAk);
      an.runBk = contiguous_run(an.offBk);
    }
    an.layoutA = an.runAm > an.runAk ? LAYOUT_MN_CONTIG : LAYOUT_K_CONTIG;
    an.layoutB = an.runBn > an.runBk ? LAYOUT_MN_CONTIG : LAYOUT_K_CONTIG;
    auto maxv = [](const std::vector<int64_t> &v) { return v.empty() ? 0 : *std::max_element(v.begin(), v.end()); };
    const int64_t lim = int64_t(1) << 31;
    an.tables32 = maxv(an.offAm) + maxv(an.offAk) < lim && maxv(an.offBk) + maxv(an.offBn) < lim &&
                  maxv(an.offCm) + maxv(an.offCn) < lim;
  }

  bool native = an.compute == COMET_COMPUTE_F64 || an.compute == COMET_COMPUTE_F32;
  comet_path_t p = path;
  if (p == COMET_PATH_AUTO) {
    const char *env = std::getenv("COMET_FORCE_PATH");
    p = (env && std::strcmp(env, "ttgt") == 0 && native && an.X.empty()) ? COMET_PATH_TTGT : COMET_PATH_GETT;
  }
  if (p == COMET_PATH_TTGT && !native)
    return Status::error(COMET_ERR_UNSUPPORTED, "the TTGT path runs the native FP64/FP32 products only");
  if (p == COMET_PATH_TTGT && !an.X.empty())
    return Status::error(COMET_ERR_UNSUPPORTED, "the TTGT path has no batch labels (use the GETT path)");
  an.path = p;
  if (an.path == COMET_PATH_TTGT) an.ttgt = choose_ttgt(an);
  return Status{};
}

static void json_dims(std::ostringstream &o, const char *name, const std::vector<Dim> &dims) {
  o << "\"" << name << "\":[";
  for (size_t i = 0; i < dims.size(); ++i) {
    const Dim &d = dims[i];
    o << (i ? "," : "") << "{\"labels\":\"" << d.labels << "\",\"ext\":" << d.ext << ",\"sA\":" << d.sA
      << ",\"sB\":" << d.sB << ",\"sC\":" << d.sC << "}";
  }
  o << "]";
}

std::string describe_json(const Analysis &an) {
  static const char *cnames[] = {"default", "f64", "f32", "split_bf16", "split_bf16x3", "split_fp16x2", "split_int8"};
  std::ostringstream o;
  o << "{\"spec\":\"" << an.spec_c << "=" << an.spec_a << "*" << an.spec_b << "\"";
  o << ",\"dtype\":\"" << (an.dtype == COMET_F64 ? "f64" : "f32") << "\"";
  o << ",\"compute\":\"" << cnames[an.compute] << "\"";
  o << ",\"path\":\"" << (an.path == COMET_PATH_TTGT ? "ttgt" : "gett") << "\"";
  o << ",\"swapped\":" << (an.swapped ? "true" : "false");
  o << ",\"m\":" << an.m << ",\"n\":" << an.n << ",\"k\":" << an.k << ",\"nb\":" << an.nb;
  o << ",";
  json_dims(o, "X", an.X);
  o << ",";
  json_dims(o, "M", an.M);
  o << ",";
  json_dims(o, "N", an.N);
  o << ",";
  json_dims(o, "K", an.K);
  o << ",\"runs\":{\"Am\":" << an.runAm << ",\"Ak\":" << an.runAk << ",\"Bk\":" << an.runBk << ",\"Bn\":" << an.runBn
    << ",\"Cm\":" << an.runCm << ",\"Cn\":" << an.runCn << "}";
  o << ",\"layoutA\":\"" << (an.layoutA == LAYOUT_K_CONTIG ? "k" : "m") << "\"";
  o << ",\"layoutB\":\"" << (an.layoutB == LAYOUT_K_CONTIG ? "k" : "n") << "\"";
  o << ",\"tables32\":" << (an.tables32 ? "true" : "false");
  o << ",\"tile\":" << an.tile << ",\"sk_tiles\":" << an.sk_tiles << ",\"sk_blocks\":" << an.sk_blocks << ",\"even\":" << an.even << ",\"even_whole\":" << an.even_whole << ",\"persist\":" << an.persist
    << ",\"shortk\":" << an.shortk << ",\"gemv\":" << an.gemv << ",\"gemv_split\":" << an.gemv_split;
  o << ",\"split_slices\":" << an.split_slices;
  o << ",\"empty_out\":" << (an.empty_out ? "true" : "false") << ",\"empty_sum\":" << (an.empty_sum ? "true" : "false");
  if (an.path == COMET_PATH_TTGT) {
    const TTGTChoice &t = an.ttgt;
    o << ",\"ttgt\":{\"swap\":" << (t.swap ? "true" : "false") << ",\"A\":\"" << t.a_order << "\",\"B\":\""
      << t.b_order << "\",\"C\":\"" << t.c_order << "\",\"copyA\":" << (t.a_copy ? "true" : "false")
      << ",\"copyB\":" << (t.b_copy ? "true" : "false") << ",\"copyC\":" << (t.c_copy ? "true" : "false")
      << ",\"cost\":" << t.cost << ",\"model_us\":" << t.model_us << "}";
  }
  o << "}";
  return o.str();
}

}  // namespace comet
