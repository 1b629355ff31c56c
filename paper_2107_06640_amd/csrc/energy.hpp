// Energy and field norms of the state: device data and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace seis {

// Number of FP64 values one work-group leaves in the partial-sum buffer, and
// the largest work-group count a launch uses (the grid strides over the
// element groups beyond it).
constexpr int kEnergyValues = 12;
constexpr int kEnergyMaxGroups = 1024;

// FP64 per-element and per-face weights of the energy (library order).
struct EnergyData {
  int64_t E = 0, Fg = 0;
  int B = 0, nq = 0;
  const double* absdet = nullptr;  // [E]   |det J|
  const double* lmr = nullptr;     // [E][3] lambda, mu, rho
  const double* gcoef = nullptr;   // [F_g] rho g A of the gravity face
  const double* tw = nullptr;      // [nq]  face rule weights (sum 1/2)
  const double* eta = nullptr;     // [F_g][nq]
};

// Work-groups of one energy launch for E elements (at most kEnergyMaxGroups).
int energy_groups(int64_t E);

// Partial sums of the energy into partial[groups][kEnergyValues], then their
// sum into out[kEnergyValues] (device). Q is the tiled state of the handle
// (FP64 or FP32). partial must hold energy_groups(E) * kEnergyValues doubles.
hipError_t launch_energy(const EnergyData& d, const double* Q64, const float* Q32, double* partial, double* out,
                         hipStream_t s);

// The library's fixed partial-sum buffer on the current device (for callers
// that cannot allocate). energy_scratch_init() looks its address up once per
// device and must run, with that device current, before energy_scratch().
hipError_t energy_scratch_init();
double* energy_scratch();
constexpr int64_t kEnergyScratchValues = int64_t(kEnergyMaxGroups) * kEnergyValues;

}  // namespace seis
