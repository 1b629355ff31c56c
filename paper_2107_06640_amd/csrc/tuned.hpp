// Tuned (matrix-core) element kernels: interface used by the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

#include "device.hpp"
#include "model.hpp"

namespace seis {

// Arguments of the tuned kernels (device pointers; FP32 state).
struct TArgs {
  float* Q;             // tiled [E][B][9]
  float* In;            // tiled [E][4][Bf][9]
  const float* G;       // [E][9]
  const float* mat;     // [E][3]
  const float* RCm;     // [E][4][12] own-trace flux coefficients
  const float* RCp;     // [E][4][12] neighbour-trace flux coefficients
  const int32_t* tgt;   // [E][4]
  const int8_t* mode;   // [E][4]
  const int8_t* hperm;  // [E][4]
  const int32_t* pinv;  // [6][Bf]
  const int32_t* gslot; // [E]
  float* gD;            // [F_g][N+1][B][9]
  float* Ib;            // tiled [E][B][9]: time-integrated predictor I~ = Q + J, parked by the predictor
  const void* ref;      // reference matrices K | E | L in operand precision
  int ref_bytes;
};

// Launch configuration of one tuned kernel.
struct LaunchCfg {
  int waves = 4;  // wavefronts per work-group (16 elements each): 2 or 4
  int cap = 0;    // work-groups per compute unit of a persistent grid; 0 = one work-group per 16*waves elements
  int remap = 0;  // 1: XCD-contiguous work-group order
  int split = 2;  // corrector: passes over the output rows (1 or 2)
};

struct TunedData {
  int ready = 0;
  int N = 0;
  int precision = 0;
  LaunchCfg pc{}, cc{};  // predictor, corrector
  int fixed = 0;         // configuration fixed by the caller (options.tile)
  int source = 0;        // 0 default or fixed, 1 measured at set-up, 2 read from the tuning cache
  TArgs a{};
  std::vector<int64_t> iface_start;   // per cluster: first element handled by the plain kernels
  DevData<double> d64{};
  DevData<float> d32{};
};

hipError_t tuned_build(TunedData& t, const Model& M, int precision, const DevData<double>& d64,
                       const DevData<float>& d32, int tile, std::vector<void*>& owned, int64_t& bytes);
// Elements [e0, ei) go to the matrix-core kernels, [ei, e1) (neighbours in
// another LTS cluster) to the plain kernels.
hipError_t tuned_predict(const TunedData& t, int precision, int N, int64_t e0, int64_t ei, int64_t e1, int parity,
                         hipStream_t s);
hipError_t tuned_correct(const TunedData& t, int precision, int N, int64_t e0, int64_t ei, int64_t e1, int parity,
                         hipStream_t s);
// Choose pc and cc for the largest cluster's matrix-core range [e0, ei) by
// timing the candidates on the (zero) state left by set-up, or read them from
// the tuning cache. The state stays zero: every kernel is linear.
hipError_t tuned_autotune(TunedData& t, const Model& M, hipStream_t s);

}  // namespace seis
