// Assembly of the per-element and per-face operators of the update in FP64
// on the GPU (Sec. 4.1 semi-discrete form, Sec. 4.2 numerical flux, Sec. 4.3
// ghost states).
//
// Inputs are per element in library order (geometry computed on the host
// while validating and clustering the mesh); outputs are written in the
// compute type of the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace seis {

struct AsmInput {
  int64_t E;
  const double* Jinv;   // [E][9]   d xi_d / d x_e (row d)
  const double* absdet; // [E]      |det J|
  const double* dt;     // [E]      time step of the element's cluster
  const double* lmr;    // [E][3]   lambda, mu, rho
  const double* nrm;    // [E][4][3] outward unit normals
  const double* area;   // [E][4]
  const int8_t* kind;   // [E][4]   face kinds (seis.h)
  const int64_t* nbk;   // [E][4]   neighbour element (library order), -1 on physical boundaries
};

template <typename T>
struct AsmOutput {
  T* G;        // [E][9]    dt * Jinv
  T* mat;      // [E][3]    lambda, mu, 1/rho
  T* Fm;       // [E][4][81] 2 A dt/|J| * T A- G- T^-1 (own trace), nullable
  T* Fp;       // [E][4][81] 2 A dt/|J| * T A- G+ T^-1 (neighbour trace), nullable
  float* RCm;  // [E][4][12] pointwise middle-state coefficients, own trace, nullable
  float* RCp;  // [E][4][12] pointwise middle-state coefficients, neighbour trace, nullable
};

template <typename T>
hipError_t launch_assemble(const AsmInput& in, const AsmOutput<T>& out, hipStream_t s);

// --------------------------------------------------------------------------
// Building blocks, usable on host and device. Matrices are 9x9 row-major,
// quantities ordered s_xx, s_yy, s_zz, s_xy, s_yz, s_xz, v_x, v_y, v_z.

// x-direction Jacobian A of q_t + A q_x + B q_y + C q_z = 0 (Sec. 3 and 4.1):
// stress rows -(lambda delta_ij + mu (...)) dv/dx, velocity rows -(1/rho) ds_xj/dx.
__host__ __device__ inline void jacobian_x(double lam, double mu, double rho, double A[81]) {
  for (int i = 0; i < 81; ++i) A[i] = 0.0;
  A[0 * 9 + 6] = -(lam + 2 * mu);
  A[1 * 9 + 6] = -lam;
  A[2 * 9 + 6] = -lam;
  A[3 * 9 + 7] = -mu;
  A[5 * 9 + 8] = -mu;
  A[6 * 9 + 0] = -1.0 / rho;
  A[7 * 9 + 3] = -1.0 / rho;
  A[8 * 9 + 5] = -1.0 / rho;
}

// T(n) of the rotational invariance A-hat = T A T^-1 (Sec. 4.2): block-diagonal
// with the stress transformation (R s R^T in Voigt form) and R = [n s t].
__host__ __device__ inline void rotation(const double n[3], double T[81], double Ti[81]) {
  double e[3] = {0, 0, 0};
  int k = 0;
  for (int d = 1; d < 3; ++d)
    if (fabs(n[d]) < fabs(n[k])) k = d;
  e[k] = 1.0;
  const double en = e[0] * n[0] + e[1] * n[1] + e[2] * n[2];
  double s[3] = {e[0] - en * n[0], e[1] - en * n[1], e[2] - en * n[2]};
  const double ns = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
  for (int d = 0; d < 3; ++d) s[d] /= ns;
  const double t[3] = {n[1] * s[2] - n[2] * s[1], n[2] * s[0] - n[0] * s[2], n[0] * s[1] - n[1] * s[0]};
  double R[3][3];
  for (int d = 0; d < 3; ++d) {
    R[d][0] = n[d];
    R[d][1] = s[d];
    R[d][2] = t[d];
  }
  const int vi[6] = {0, 1, 2, 0, 1, 0}, vj[6] = {0, 1, 2, 1, 2, 2};
  for (int i = 0; i < 81; ++i) T[i] = Ti[i] = 0.0;
  for (int a = 0; a < 6; ++a) {
    // unit Voigt tensor a, rotated forward (R E R^T) and back (R^T E R)
    for (int b = 0; b < 6; ++b) {
      const int i = vi[b], j = vj[b];
      double g, l;
      if (vi[a] == vj[a]) {
        const int p = vi[a];
        g = R[i][p] * R[j][p];
        l = R[p][i] * R[p][j];
      } else {
        const int p = vi[a], q = vj[a];
        g = R[i][p] * R[j][q] + R[i][q] * R[j][p];
        l = R[p][i] * R[q][j] + R[q][i] * R[p][j];
      }
      T[b * 9 + a] = g;
      Ti[b * 9 + a] = l;
    }
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T[(6 + i) * 9 + 6 + j] = R[i][j];
      Ti[(6 + i) * 9 + 6 + j] = R[j][i];
    }
}

// Middle state of the rotated Riemann problem, w^b = Gm w- + Gp w+
// (Sec. 4.2, eigen-decomposition and boundary state). Rows of components the
// flux does not read stay zero.
__host__ __device__ inline void middle_state(double zpm, double zsm, double zpp, double zsp, double Gm[81],
                                             double Gp[81]) {
  for (int i = 0; i < 81; ++i) Gm[i] = Gp[i] = 0.0;
  const double c = zpm * zpp / (zpm + zpp);
  Gm[0 * 9 + 0] = 1.0 - c / zpp;
  Gm[0 * 9 + 6] = -c;
  Gp[0 * 9 + 0] = c / zpp;
  Gp[0 * 9 + 6] = c;
  Gm[6 * 9 + 6] = 1.0 - c / zpm;
  Gm[6 * 9 + 0] = -c / (zpp * zpm);
  Gp[6 * 9 + 0] = c / (zpp * zpm);
  Gp[6 * 9 + 6] = c / zpm;
  const int pa[2] = {3, 5}, pb[2] = {7, 8};
  for (int k = 0; k < 2; ++k) {
    const int a = pa[k], b = pb[k];
    if (zsm > 0.0 && zsp > 0.0) {
      const double cs = zsm * zsp / (zsm + zsp);
      Gm[a * 9 + a] = 1.0 - cs / zsp;
      Gm[a * 9 + b] = -cs;
      Gp[a * 9 + a] = cs / zsp;
      Gp[a * 9 + b] = cs;
      Gm[b * 9 + b] = 1.0 - cs / zsm;
      Gm[b * 9 + a] = -cs / (zsp * zsm);
      Gp[b * 9 + a] = cs / (zsp * zsm);
      Gp[b * 9 + b] = cs / zsm;
    } else if (zsm > 0.0) {  // elastic '-', acoustic '+': zero shear traction
      Gm[b * 9 + b] = 1.0;
      Gm[b * 9 + a] = -1.0 / zsm;
    }
    // acoustic '-': the tangential state is multiplied by mu- = 0 in the flux
  }
}

// Middle-state coefficients of the pointwise Godunov solver (Sec. 4.2) in the
// physical frame, scaled by s: with s_n = n.s.n, t_t = s n - s_n n,
// v_n = v.n, v_t = v - v_n n of a trace,
//   s_n^b = c0 s_n + c1 v_n,  v_n^b = c2 s_n + c3 v_n,
//   t_t^b = c4 t_t + c5 v_t,  v_t^b = c6 t_t + c7 v_t
// summed over the own trace (cm) and the neighbour trace (cp); the flux is
// then A-hat^-(n) applied to (v^b, traction s_n^b n + t_t^b). Ghost states of
// physical boundaries (Sec. 4.3) are folded into cm. A fault face (kind 7)
// receives its middle state itself (the friction kernel writes it where the
// neighbour trace would be): cm = 0 and cp the identity.
__host__ __device__ inline void pointwise_coeffs(int kind, double zpm, double zsm, double zpp, double zsp,
                                                 double s, double cm[8], double cp[8]) {
  for (int i = 0; i < 8; ++i) cm[i] = cp[i] = 0.0;
  if (kind == 2) return;  // gravity surface: handled by the eta ODE
  if (kind == 7) {
    cp[0] = cp[3] = cp[4] = cp[7] = s;
    return;
  }
  const double c1 = zpm * zpp / (zpm + zpp);
  double a[8], b[8];
  a[0] = 1.0 - c1 / zpp; a[1] = -c1; b[0] = c1 / zpp; b[1] = c1;
  a[2] = -c1 / (zpp * zpm); a[3] = 1.0 - c1 / zpm; b[2] = c1 / (zpp * zpm); b[3] = c1 / zpm;
  if (zsm > 0.0 && zsp > 0.0) {
    const double ct = zsm * zsp / (zsm + zsp);
    a[4] = 1.0 - ct / zsp; a[5] = -ct; b[4] = ct / zsp; b[5] = ct;
    a[6] = -ct / (zsp * zsm); a[7] = 1.0 - ct / zsm; b[6] = ct / (zsp * zsm); b[7] = ct / zsm;
  } else if (zsm > 0.0) {
    a[4] = a[5] = b[4] = b[5] = 0.0;
    a[6] = -1.0 / zsm; a[7] = 1.0; b[6] = b[7] = 0.0;
  } else {
    for (int i = 4; i < 8; ++i) a[i] = b[i] = 0.0;
  }
  if (kind == 0 || kind == 1) {
    for (int i = 0; i < 8; ++i) { cm[i] = s * a[i]; cp[i] = s * b[i]; }
    return;
  }
  // ghost traces: absorbing 0; wall: same traction, velocity flipped; free:
  // traction flipped; prescribed velocity: as the wall, plus 2 v_b, which
  // reaches the flux through the neighbour coefficients and the inbox
  double gs = 0.0, gv = 0.0;
  if (kind == 4 || kind == 6) { gs = 1.0; gv = -1.0; }
  if (kind == 5) { gs = -1.0; gv = 1.0; }
  for (int i = 0; i < 8; i += 2) {
    cm[i] = s * (a[i] + gs * b[i]);
    cm[i + 1] = s * (a[i + 1] + gv * b[i + 1]);
  }
  if (kind == 6)
    for (int i = 0; i < 8; ++i) cp[i] = s * b[i];
}

}  // namespace seis
