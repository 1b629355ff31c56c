// The velocity-stress flux operator on the device.
//
// apply_A(e, v) = A_e v with A_x, A_y, A_z the Jacobians of
// q_t + A q_x + B q_y + C q_z = 0 (Sec. 3 PDE, Sec. 4.1 linear form), written
// out component by component (quantity order s_xx s_yy s_zz s_xy s_yz s_xz v_x v_y v_z).
// The scaled star matrix of an element is A*_d = sum_e G[d][e] A_e with
// G = dt * dxi/dx, so neither A_e nor A*_d is ever stored.
#pragma once

#include <hip/hip_runtime.h>

namespace seis {

// out_p = (sum_e c_e A_e) v for the combination c = (cx, cy, cz).
template <typename T>
__device__ __forceinline__ void apply_star(T cx, T cy, T cz, T lam, T mu, T rinv, const T v[9], T out[9]) {
  // the minus signs are carried by the coefficients: negation is exact, so
  // this equals -(l2m cx vx + ...) etc. bit for bit, without sign flips
  const T nl2m = -(lam + T(2) * mu), nlam = -lam, nmu = -mu, nr = -rinv;
  const T vx = v[6], vy = v[7], vz = v[8];
  out[0] = nl2m * cx * vx + nlam * cy * vy + nlam * cz * vz;
  out[1] = nlam * cx * vx + nl2m * cy * vy + nlam * cz * vz;
  out[2] = nlam * cx * vx + nlam * cy * vy + nl2m * cz * vz;
  out[3] = nmu * (cx * vy + cy * vx);
  out[4] = nmu * (cy * vz + cz * vy);
  out[5] = nmu * (cx * vz + cz * vx);
  out[6] = nr * (cx * v[0] + cy * v[3] + cz * v[5]);
  out[7] = nr * (cx * v[3] + cy * v[1] + cz * v[4]);
  out[8] = nr * (cx * v[5] + cy * v[4] + cz * v[2]);
}

// out_p = sum_e (A_e w_e)_p for three vectors w_x, w_y, w_z (physical gradient components).
template <typename T>
__device__ __forceinline__ T grad_op(int p, T lam, T mu, T rinv, const T* wx, const T* wy, const T* wz) {
  const T l2m = lam + T(2) * mu;
  switch (p) {
    case 0: return -(l2m * wx[6] + lam * wy[7] + lam * wz[8]);
    case 1: return -(lam * wx[6] + l2m * wy[7] + lam * wz[8]);
    case 2: return -(lam * wx[6] + lam * wy[7] + l2m * wz[8]);
    case 3: return -mu * (wx[7] + wy[6]);
    case 4: return -mu * (wy[8] + wz[7]);
    case 5: return -mu * (wx[8] + wz[6]);
    case 6: return -rinv * (wx[0] + wy[3] + wz[5]);
    case 7: return -rinv * (wx[3] + wy[1] + wz[4]);
    default: return -rinv * (wx[5] + wy[4] + wz[2]);
  }
}

__host__ __device__ constexpr int nbasis(int N) { return (N + 1) * (N + 2) * (N + 3) / 6; }
__host__ __device__ constexpr int nface(int N) { return (N + 1) * (N + 2) / 2; }

}  // namespace seis
