// Instantiation of the matrix-core kernels for split BF16 operands (hi + lo,
// three products per product).
#include "tuned_kern.hpp"

namespace seis {

hipError_t pred_dispatch_bf16x3(int N, const LaunchCfg& c, const TArgs& a, int64_t e0, int64_t e1, const Sched& sc,
                                hipStream_t s) {
  return pred_dispatch<OpBF16X3>(N, c, a, e0, e1, sc, s);
}

hipError_t corr_dispatch_bf16x3(int N, const LaunchCfg& c, const TArgs& a, int64_t e0, int64_t e1, hipStream_t s) {
  return corr_dispatch<OpBF16X3>(N, c, a, e0, e1, s);
}

}  // namespace seis
