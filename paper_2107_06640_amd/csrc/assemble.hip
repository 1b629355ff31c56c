// FP64 assembly of the per-element and per-face operators on the GPU.
#include "assemble.hpp"

namespace seis {

namespace {

__device__ void mul9(const double* a, const double* b, double* c) {
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) {
      double s = 0.0;
      for (int k = 0; k < 9; ++k) s += a[i * 9 + k] * b[k * 9 + j];
      c[i * 9 + j] = s;
    }
}

// One thread per face: the flux operators of the face (Sec. 4.2, numerical
// flux F- q- + F+ q+ with F-+ = T A- G-+ T^-1, scaled by 2 A dt / |J|), the
// pointwise middle-state coefficients of the same flux, and (face 0 thread)
// the element's scaled inverse Jacobian and material.
template <typename T>
__global__ __launch_bounds__(64) void k_assemble(AsmInput in, AsmOutput<T> out) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= in.E * 4) return;
  const int64_t e = id >> 2;
  const int f = int(id & 3);
  const double lam = in.lmr[e * 3 + 0], mu = in.lmr[e * 3 + 1], rho = in.lmr[e * 3 + 2];
  const double dt = in.dt[e];
  if (f == 0) {
    for (int i = 0; i < 9; ++i) out.G[e * 9 + i] = (T)(dt * in.Jinv[e * 9 + i]);
    out.mat[e * 3 + 0] = (T)lam;
    out.mat[e * 3 + 1] = (T)mu;
    out.mat[e * 3 + 2] = (T)(1.0 / rho);
  }
  const int kind = in.kind[id];
  const double scale = 2.0 * in.area[id] * dt / in.absdet[e];
  const double zpm = sqrt((lam + 2 * mu) * rho), zsm = sqrt(mu * rho);
  double zpp = zpm, zsp = zsm;
  const bool paired = kind == 0 || kind == 1;
  if (paired) {
    const int64_t e2 = in.nbk[id];
    const double l2 = in.lmr[e2 * 3 + 0], m2 = in.lmr[e2 * 3 + 1], r2 = in.lmr[e2 * 3 + 2];
    zpp = sqrt((l2 + 2 * m2) * r2);
    zsp = sqrt(m2 * r2);
  }
  const double n[3] = {in.nrm[id * 3 + 0], in.nrm[id * 3 + 1], in.nrm[id * 3 + 2]};
  if (out.Fm) {
    double A[81], Tr[81], Ti[81], Gm[81], Gp[81], X[81], Y[81];
    jacobian_x(lam, mu, rho, A);
    rotation(n, Tr, Ti);
    middle_state(zpm, zsm, zpp, zsp, Gm, Gp);
    if (kind == 4 || kind == 5 || kind == 6) {
      // ghost w+ = diag(m) w-: velocity flipped (wall; a prescribed velocity
      // adds 2 v_b, which the inbox supplies) or stress flipped (free surface)
      for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) {
          const double m = (kind != 5) ? (c >= 6 ? -1.0 : 1.0) : (c < 6 ? -1.0 : 1.0);
          Gm[r * 9 + c] += Gp[r * 9 + c] * m;
        }
    }
    T* fm = out.Fm + id * 81;
    T* fp = out.Fp + id * 81;
    if (kind == 2) {  // gravity face: the eta ODE supplies the whole flux
      for (int i = 0; i < 81; ++i) fm[i] = fp[i] = (T)0;
    } else if (kind == 7) {
      // fault face: the friction kernel supplies the middle state w^b in the
      // inbox; the flux is T A T^-1 w^b (A reads only the components of w^b
      // that the middle state sets)
      mul9(Tr, A, Y);
      mul9(Y, Ti, X);
      for (int i = 0; i < 81; ++i) {
        fm[i] = (T)0;
        fp[i] = (T)(scale * X[i]);
      }
    } else {
      mul9(A, Gm, X);
      mul9(Tr, X, Y);
      mul9(Y, Ti, X);
      for (int i = 0; i < 81; ++i) fm[i] = (T)(scale * X[i]);
      if (paired || kind == 6) {
        mul9(A, Gp, X);
        mul9(Tr, X, Y);
        mul9(Y, Ti, X);
        for (int i = 0; i < 81; ++i) fp[i] = (T)(scale * X[i]);
      } else {
        for (int i = 0; i < 81; ++i) fp[i] = (T)0;
      }
    }
  }
  if (out.RCm) {
    double cm[8], cp[8];
    pointwise_coeffs(kind, zpm, zsm, zpp, zsp, scale, cm, cp);
    float* rm = out.RCm + id * 12;
    float* rp = out.RCp + id * 12;
    for (int d = 0; d < 3; ++d) rm[d] = rp[d] = (float)n[d];
    for (int i = 0; i < 8; ++i) {
      rm[3 + i] = (float)cm[i];
      rp[3 + i] = (float)cp[i];
    }
    rm[11] = rp[11] = 0.0f;
  }
}

}  // namespace

template <typename T>
hipError_t launch_assemble(const AsmInput& in, const AsmOutput<T>& out, hipStream_t s) {
  if (in.E <= 0) return hipSuccess;
  const int64_t n = in.E * 4;
  hipLaunchKernelGGL(k_assemble<T>, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, in, out);
  return hipGetLastError();
}

template hipError_t launch_assemble<double>(const AsmInput&, const AsmOutput<double>&, hipStream_t);
template hipError_t launch_assemble<float>(const AsmInput&, const AsmOutput<float>&, hipStream_t);

}  // namespace seis
