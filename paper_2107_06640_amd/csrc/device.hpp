// Device-side data of one handle and the kernel launchers.
//
// Layout in HBM (library element order, clusters contiguous):
//   Q     [E][B][9]        modal coefficients (compute type)
//   G     [E][9]           dt_c * dxi_d/dx_e (row d)          -- scaled star matrices are
//   mat   [E][3]           lambda, mu, 1/rho                     rebuilt from these on the fly
//   Fm,Fp [E][4][81]       2 A_i dt_c / |J| * F-+ (row p, column r)
//   In    [E][4][Bf][9]    time-integrated neighbour traces received at face nodes,
//                          divided by the receiver's dt (its own node numbering)
//   H2    [n_half2][Bf][9] second-half traces from a coarser neighbour
//   gD    [F_g][N+1][B][9] scaled time derivatives of elements with a gravity face
//   eta   [F_g][nq]        FP64 sea-surface displacement
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace seis {

// Position in the rate-2 LTS schedule (Sec. 4.4): the sub-step of the macro
// step and the element ranges of the clusters (library order, cluster c is
// [cstart[c], cstart[c+1])). An element of cluster c is on the second step of
// a pair of its steps when (sub >> c) & 1; the hand-over to a coarser
// neighbour and the reading of second-half traces depend on it. A launch may
// span several clusters, so the kernels take it per element.
struct Sched {
  static constexpr int kMax = 16;
  int sub = 0;
  int C = 1;
  int64_t cstart[kMax + 1] = {};
  __host__ __device__ __forceinline__ int parity(int64_t e) const {
    int c = 0;
#pragma unroll
    for (int k = 1; k < kMax; ++k) c = (k < C && e >= cstart[k]) ? k : c;
    return (sub >> c) & 1;
  }
};

template <typename T>
struct DevData {
  int64_t E;
  T* Q;
  const T* G;
  const T* mat;
  const T* Fm;
  const T* Fp;
  T* In;
  T* H2;
  const int32_t* tgt;
  const int8_t* mode;
  const int8_t* hperm;
  const int32_t* half2;
  const int32_t* rhalf2;
  const int32_t* gslot;
  const int32_t* dslot;  // [E] slot of the stored time derivatives (gravity faces, fault faces, ...), -1 none
  T* gD;
  // reference matrices (compute type)
  const T* K;   // [3][B][B]
  const T* Ef;  // [4][Bf][B]
  const T* Lf;  // [4][B][Bf]
  const int32_t* perm;  // [6][Bf]
  // gravity (FP64)
  const double* Eg;     // [4][nq][B]
  const double* Lg;     // [4][B][nq]
  const int32_t* g_elem;
  const int8_t* g_face;
  const double* g_par;  // [F_g][8]
  double* eta;          // [F_g][nq]
  double g;
};

// Plain kernels: one work-group per element, FP64 or FP32.
template <typename T>
hipError_t launch_predict_plain(int N, const DevData<T>& d, int64_t e0, int64_t ne, const Sched& sc, hipStream_t s);
template <typename T>
hipError_t launch_correct_plain(int N, const DevData<T>& d, int64_t e0, int64_t ne, const Sched& sc, hipStream_t s);
// Gravity faces listed in glist[0..ng) (FP64 ODE and lift).
template <typename T>
hipError_t launch_gravity(int N, const DevData<T>& d, const int32_t* glist, int64_t ng, hipStream_t s);

}  // namespace seis
