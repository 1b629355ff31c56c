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
  const int32_t* mh4;   // [E]: byte f = mode | hperm << 2 of face f
  const int32_t* pinv;  // [6][Bf]
  const int32_t* dslot; // [E] slot of the stored time derivatives, -1 none
  float* gD;            // [slots][N+1][B][9] time derivatives (gravity faces, then hand-over to finer neighbours)
  const float* Ef;      // [4][Bf][B] face-trace matrices (FP32)
  float* H2;            // [n_half2][Bf][9] second-half traces for finer neighbours
  const int32_t* half2; // [E][4] writer: second-half slot, -1 none
  const int32_t* rhalf2;// [E][4] reader: second-half slot, -1 none
  const int32_t* fix_list;  // element * 4 + face of the faces handing over to a finer neighbour
  const int32_t* h2_list;   // element * 4 + face of the faces reading a second-half slot
  float* Ib;            // tiled [E][B][9]: time-integrated predictor I~ = Q + J, parked by the predictor
  const int32_t* gac;   // [ceil(E/16)]: 1 where every element of the 16-element group is acoustic
                        // (run in the 4-quantity form), else 0
  const void* ref;      // reference matrices K | E | L in operand precision
  int ref_bytes;
};

// Launch configuration of one tuned kernel.
struct LaunchCfg {
  int waves = 4;  // wavefronts per work-group (16 elements each): 2 or 4
  int cap = 0;    // work-groups per compute unit of a persistent grid; 0 = one work-group per 16*waves elements
  int remap = 0;  // 1: XCD-contiguous work-group order
  int split = 2;  // corrector: passes over the output rows (1 or 2)
  int variant = 0;  // predictor shape: FP32 0 = I~ parked in LDS as far as it fits, 1 = in HBM;
                    // BF16 0 = 16x16x16 products, 1 = 16x16x32 products over two row tiles
};

struct TunedData {
  int ready = 0;
  int N = 0;
  int precision = 0;
  LaunchCfg pc{}, cc{};  // predictor, corrector
  int fixed = 0;         // configuration fixed by the caller (options.tile)
  int source = 0;        // 0 default or fixed, 1 measured at set-up, 2 read from the tuning cache
  int64_t mc_min = 0;    // clusters with fewer elements run on the plain FP32 kernels
  int64_t n_acoustic_groups = 0;  // 16-element groups run in the 4-quantity form
  TArgs a{};
  std::vector<int64_t> fix_start, h2_start;  // per cluster: ranges of fix_list and h2_list
  DevData<double> d64{};
  DevData<float> d32{};
};

// Matrix-core launches of one precision (tuned_f32.hip, tuned_bf16.hip).
hipError_t pred_dispatch_f32(int N, const LaunchCfg& c, const TArgs& a, int64_t e0, int64_t e1, const Sched& sc,
                             hipStream_t s);
hipError_t pred_dispatch_bf16(int N, const LaunchCfg& c, const TArgs& a, int64_t e0, int64_t e1, const Sched& sc,
                              hipStream_t s);
hipError_t corr_dispatch_f32(int N, const LaunchCfg& c, const TArgs& a, int64_t e0, int64_t e1, hipStream_t s);
hipError_t corr_dispatch_bf16(int N, const LaunchCfg& c, const TArgs& a, int64_t e0, int64_t e1, hipStream_t s);
hipError_t pred_dispatch_bf16x3(int N, const LaunchCfg& c, const TArgs& a, int64_t e0, int64_t e1, const Sched& sc,
                                hipStream_t s);
hipError_t corr_dispatch_bf16x3(int N, const LaunchCfg& c, const TArgs& a, int64_t e0, int64_t e1, hipStream_t s);

// acoustic: nonzero runs 16-element groups of acoustic elements in the
// 4-quantity form.
hipError_t tuned_build(TunedData& t, const Model& M, int precision, const DevData<double>& d64,
                       const DevData<float>& d32, int tile, int acoustic, std::vector<void*>& owned,
                       int64_t& bytes);
// Clusters c0..c1 = elements [e0, e1) (a launch may span several clusters;
// sc gives each element's step parity). FP64 runs the plain kernels, and so
// does a range of fewer than mc_min elements (in FP32). Otherwise the
// matrix-core predictor handles every element; faces handing over to a finer
// neighbour are then rewritten with the first- and second-half traces, and
// before the corrector the second-half traces of the clusters on the second
// step of their pair are copied into the inbox of the finer elements that
// read them.
hipError_t tuned_predict(const TunedData& t, int precision, int N, int c0, int c1, int64_t e0, int64_t e1,
                         const Sched& sc, hipStream_t s);
hipError_t tuned_correct(const TunedData& t, int precision, int N, int c0, int c1, int64_t e0, int64_t e1,
                         const Sched& sc, hipStream_t s);
// Choose pc and cc for the largest cluster by
// timing the candidates on the (zero) state left by set-up, or read them from
// the tuning cache. The state stays zero: every kernel is linear.
hipError_t tuned_autotune(TunedData& t, const Model& M, hipStream_t s);

}  // namespace seis
