// tune.hpp -- the autotuner's cache: which tile variant and lowering ran
// fastest for a class of contractions.  Timing itself happens in api.cpp,
// which owns plans and launches.
#pragma once

#include <map>
#include <mutex>
#include <string>

#include "plan.hpp"

namespace comet {

struct TuneEntry {
  int tile = 0;
  int path = COMET_PATH_GETT;
  double us = 0.0;
  std::string ttgt;   // for path TTGT: "A order|B order|C order" of the fastest flattening
};

class TuneCache {
 public:
  // mode 0: off; 1: use the cache, time classes it lacks; 2: re-time all
  void configure(const std::string &path, int mode);
  int mode() const { return mode_; }
  bool lookup(const std::string &key, TuneEntry *e);
  void store(const std::string &key, const TuneEntry &e);
  std::mutex &mutex() { return mu_; }
  const std::string &path() const { return path_; }
  size_t size() const { return entries_.size(); }

 private:
  void load();
  void save() const;
  std::mutex mu_;
  std::string path_;
  int mode_ = 0;
  std::map<std::string, TuneEntry> entries_;
};

TuneCache &tune_cache();

// Problem class of a planned contraction: `arch` (device architecture and
// runtime version, supplied by the caller), the kernel version, operand layouts and contiguous runs, the A/B exchange, and
// the flattened sizes bucketed by powers of two.
std::string tune_key(const Analysis &an, const std::string &arch);

// Problem class of one batched problem: `arch`, the kernel version, storage
// dtype (0 FP64, 1 FP32), batch mode (0 native, 1 fused BF16x3), layout
// variant and the flattened sizes bucketed by powers of two.  The cache
// entry's `tile` holds the batch tile class.
std::string batch_tune_key(int dtype, int mode, int variant, int64_t m, int64_t n, int64_t k,
                           const std::string &arch);

}  // namespace comet
