// tune.cpp -- JSON cache of autotuned tile shapes (host only).
//
// File format (one object; unknown or malformed content makes the whole file
// ignored and rewritten):
//   {"format": "comet-tune-2", "entries": {"<key>": {"tile": 3, "path": 1, "us": 1234.5, "ttgt": ""}, ...}}
#include "tune.hpp"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>

#include "comet.h"

namespace comet {

namespace {
const char *kFormat = "comet-tune-2";
const char *kKernelVersion = "k11";   // bump when kernels change in a way that invalidates timings

int bucket(int64_t x) {
  int b = 0;
  while ((int64_t(1) << b) < x && b < 62) ++b;
  return b;
}

std::string default_path() {
  const char *env = std::getenv("COMET_TUNE_CACHE");
  if (env && *env) return env;
  const char *home = std::getenv("HOME");
  return std::string(home ? home : ".") + "/.cache/comet_tune.json";
}

// minimal parser for the flat format written by save()
bool parse(const std::string &text, std::map<std::string, TuneEntry> &out) {
  if (text.find(std::string("\"format\": \"") + kFormat + "\"") == std::string::npos) return false;
  size_t p = text.find("\"entries\"");
  if (p == std::string::npos) return false;
  p = text.find('{', p);
  if (p == std::string::npos) return false;
  ++p;
  for (;;) {
    while (p < text.size() && (text[p] == ' ' || text[p] == '\n' || text[p] == ',')) ++p;
    if (p >= text.size()) return false;
    if (text[p] == '}') return true;
    if (text[p] != '"') return false;
    size_t q = text.find('"', p + 1);
    if (q == std::string::npos) return false;
    std::string key = text.substr(p + 1, q - p - 1);
    size_t o = text.find('{', q);
    size_t c = text.find('}', q);
    if (o == std::string::npos || c == std::string::npos || c < o) return false;
    std::string body = text.substr(o + 1, c - o - 1);
    TuneEntry e;
    int tile = -1, path = -1;
    double us = -1;
    if (std::sscanf(body.c_str(), " \"tile\": %d, \"path\": %d, \"us\": %lf", &tile, &path, &us) != 3) return false;
    if (tile < 0 || path < COMET_PATH_GETT || path > COMET_PATH_TTGT || !(us >= 0)) return false;
    e.tile = tile;
    e.path = path;
    e.us = us;
    const size_t tq = body.find("\"ttgt\": \"");
    if (tq != std::string::npos) {
      const size_t t0 = tq + 9, t1 = body.find('"', t0);
      if (t1 == std::string::npos) return false;
      e.ttgt = body.substr(t0, t1 - t0);
      for (char ch : e.ttgt)
        if (!((ch >= 'a' && ch <= 'z') || (ch >= 'A' && ch <= 'Z') || ch == '|')) return false;
    }
    out[key] = e;
    p = c + 1;
  }
}
}  // namespace

// The cache starts in the mode COMET_AUTOTUNE names ("off", "on" = time
// missing classes and reuse the cache, "force" = time every class again), at
// COMET_TUNE_CACHE or ~/.cache/comet_tune.json; comet_autotune() changes it.
TuneCache &tune_cache() {
  static TuneCache c;
  static bool init = [] {
    const char *env = std::getenv("COMET_AUTOTUNE");
    if (env && *env) {
      const std::string v(env);
      const int mode = (v == "on" || v == "1") ? 1 : (v == "force" || v == "2") ? 2 : 0;
      if (mode) c.configure(std::string(), mode);
    }
    return true;
  }();
  (void)init;
  return c;
}

void TuneCache::configure(const std::string &path, int mode) {
  path_ = path.empty() ? default_path() : path;
  mode_ = mode;
  entries_.clear();
  if (mode_ == 1) load();
}

void TuneCache::load() {
  std::ifstream f(path_);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  std::map<std::string, TuneEntry> m;
  if (parse(ss.str(), m)) entries_ = m;   // corrupt: start empty, rewritten on the next store
}

void TuneCache::save() const {
  std::string tmp = path_ + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\"format\": \"" << kFormat << "\", \"entries\": {";
    bool first = true;
    char buf[256];
    for (const auto &kv : entries_) {
      std::snprintf(buf, sizeof buf, "{\"tile\": %d, \"path\": %d, \"us\": %.3f, \"ttgt\": \"%s\"}", kv.second.tile,
                    kv.second.path, kv.second.us, kv.second.ttgt.c_str());
      f << (first ? "\n" : ",\n") << "  \"" << kv.first << "\": " << buf;
      first = false;
    }
    f << "\n}}\n";
  }
  std::rename(tmp.c_str(), path_.c_str());
}

bool TuneCache::lookup(const std::string &key, TuneEntry *e) {
  auto it = entries_.find(key);
  if (it == entries_.end()) return false;
  *e = it->second;
  return true;
}

void TuneCache::store(const std::string &key, const TuneEntry &e) {
  entries_[key] = e;
  save();
}

std::string tune_key(const Analysis &an, const std::string &arch) {
  std::ostringstream k;
  k << arch << "/" << kKernelVersion << "/" << (an.dtype == COMET_F64 ? "f64" : "f32")
    << "/c" << int(an.compute) << "/L" << int(an.layoutA) << int(an.layoutB) << "/r" << an.runAm << an.runAk
    << an.runBk << an.runBn << an.runCn << "/s" << (an.swapped ? 1 : 0) << "/m" << bucket(an.m) << "n" << bucket(an.n)
    << "k" << bucket(an.k) << "b" << bucket(an.nb);
  return k.str();
}

std::string batch_tune_key(int dtype, int mode, int variant, int64_t m, int64_t n, int64_t k,
                           const std::string &arch) {
  std::ostringstream o;
  o << "batch/" << arch << "/" << kKernelVersion << "/" << (dtype == 0 ? "f64" : "f32") << "/x" << mode << "/v"
    << variant << "/m" << bucket(m) << "n" << bucket(n) << "k" << bucket(k);
  return o.str();
}

}  // namespace comet
