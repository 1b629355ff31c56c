// Dynamic-rupture fault faces (Sec. 3, fault boundary condition): where the
// shear traction reaches the frictional strength the two sides slip, and the
// face flux of each side is that of the friction-limited middle state.
//
// With n the normal from the '-' to the '+' side, the normal stress and
// normal velocity of the middle state are those of the welded interface
// (Godunov state, Sec. 4.2); the shear traction follows from the S-wave
// characteristics of the two sides,
//   tau^b = tau- + Zs- (v-^b - v-_t) = tau+ - Zs+ (v+^b - v+_t),
// which without slip gives tau_lock = eta (tau-/Zs- + tau+/Zs+ + v+_t - v-_t),
// eta = Zs- Zs+ / (Zs- + Zs+). The total shear traction T = tau0 + tau_lock
// (tau0 the fault's background traction) is kept when |T| <= tau_S, else
// scaled to the strength tau_S = C + f(psi) max(0, -(s0 + s^b)), and the slip
// rate is V = (tau_lock - tau^b) / eta, parallel to T. Friction laws, per face:
//  * linear slip weakening (the benchmark's law, Sec. 6.2):
//    f = mu_s - (mu_s - mu_d) min(psi / D_c, 1), psi the slip path;
//  * rate and state with fast velocity weakening (the Palu run's law):
//    f(V, psi) = a asinh(V / (2 V0) exp(psi / a)), the fault always slides
//    with |T| - eta V = f(V, psi) max(0, -(s0 + s^b)) (solved for V by
//    safeguarded Newton), and over the time the point stands for, h, the
//    state relaxes at that V: psi <- psi_ss + (psi - psi_ss) exp(-V h / L),
//    psi_ss(V) = a ln(2 V0 / V sinh(f_ss(V) / a)),
//    f_ss(V) = f_w + (f0 - (b - a) ln(V / V0) - f_w) / (1 + (V / V_w)^8)^(1/8).
//
// Over an element step the traces of both sides come from their stored time
// derivatives, at the N + 1 Gauss-Legendre points of the step, in order; psi
// advances by the point's weight times |V| after each point. The law is
// applied at the face nodes (the equispaced lattice); the time average of
// each side's middle state is written into that side's inbox, where the
// corrector reads it with identity middle-state coefficients (the face's
// own-trace coefficients are zero). Arithmetic in FP64.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace seis {

// per face: s0, tau0 (x, y, z), then the law's parameters, the law at [15]:
//   slip weakening (0): mu_s, mu_d, D_c, C
//   rate and state (1): a, b, L, V0, f0, f_w, V_w, psi0
constexpr int kFaultParams = 16;
constexpr int kLawSlipWeakening = 0, kLawRateState = 1;
constexpr int kFaultState = 11;  // slip (3), slip path, slip rate (3), shear traction (3), normal stress

struct FaultArgs {
  const int64_t* elem;    // [F] '-' element (library order)
  const int8_t* face;     // [F]
  const int64_t* pelem;   // [F] '+' element
  const int8_t* pface;    // [F]
  const int8_t* perm;     // [F] node map index: '-' node m is '+' node pinv[perm][m]
  const double* geo;      // [F][8]: n, Zp-, Zs-, Zp+, Zs+, dt
  const double* par;      // [F][kFaultParams]
  double* state;          // [F][Bf][kFaultState]
  const double* E;        // [4][Bf][B] basis at the face nodes
  const int32_t* pinv;    // [6][Bf]
  const int32_t* dslot;   // [E] slot of the stored time derivatives
  const double* tq;       // [N+1] Gauss-Legendre points on [0, 1]
  const double* tw;       // [N+1] their weights (sum 1)
};

// Fault faces [f0, f0 + nf): middle states into both inboxes, state updated.
// gD: stored time derivatives [slots][N+1][B][9]; In: inbox (FP64 or FP32).
template <typename T>
hipError_t launch_fault(int N, const FaultArgs& a, const T* gD, T* In, int64_t f0, int64_t nf, hipStream_t s);

}  // namespace seis
