// Tuned (MFMA) element kernels.
#include "tuned.hpp"

namespace seis {

hipError_t tuned_build(TunedData& t, const Model& M, int precision, const DevData<double>& d64,
                       const DevData<float>& d32, int tile, std::vector<void*>& owned, int64_t& bytes) {
  (void)t; (void)M; (void)precision; (void)d64; (void)d32; (void)tile; (void)owned; (void)bytes;
  return hipErrorNotSupported;
}
hipError_t tuned_predict(const TunedData&, int, int, int64_t, int64_t, int, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t tuned_correct(const TunedData&, int, int, int64_t, int64_t, int, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace seis
