// split.hip -- placeholder until the slice kernels land.
#include "split.hpp"

namespace comet {

Status split_prepare(const Analysis &, SplitPlan &) {
  return Status::error(COMET_ERR_UNSUPPORTED, "split compute modes are not built yet");
}

hipError_t split_execute(const Analysis &, const SplitPlan &, const GettTables &, double, const void *, const void *,
                         double, void *, void *, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace comet
