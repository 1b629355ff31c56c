// Tuned (MFMA) element kernels: interface used by the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

#include "device.hpp"
#include "model.hpp"

namespace seis {

struct TunedData {
  int ready = 0;
  int N = 0;
  int precision = 0;
  int tile = 0;
  DevData<double> d64{};
  DevData<float> d32{};
};

hipError_t tuned_build(TunedData& t, const Model& M, int precision, const DevData<double>& d64,
                       const DevData<float>& d32, int tile, std::vector<void*>& owned, int64_t& bytes);
hipError_t tuned_predict(const TunedData& t, int precision, int N, int64_t e0, int64_t ne, int parity,
                         hipStream_t s);
hipError_t tuned_correct(const TunedData& t, int precision, int N, int64_t e0, int64_t ne, int parity,
                         hipStream_t s);

}  // namespace seis
