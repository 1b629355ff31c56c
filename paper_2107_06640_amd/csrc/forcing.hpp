// Prescribed bottom velocity from a seafloor-uplift history (the forcing of
// the surrogate's runs): on faces of kind 6 the ghost state is the wall's
// (same traction, velocity flipped) plus 2 v_b, v_b = (0, 0, du/dt) with
//   u(x, y, t) = sum_j A_j exp(-((x - x_j)^2 + (y - y_j)^2) / (2 w_j^2)) S(t / T_j),
//   S(s) = 0 (s <= 0), s - sin(2 pi s) / (2 pi) (0 < s < 1), 1 (s >= 1).
// The flux is linear in the ghost, so its v_b part is a neighbour trace: the
// time integral of 2 v_b over the element's step, 2 (u(t1) - u(t0)), divided
// by the step (the inbox convention), written into the face's inbox before
// the corrector. The inbox holds a degree-N polynomial on the face (its nodal
// values), so the forcing enters as its L2 projection onto P_N, taken with a
// high-order face rule: the face integral of the flux against the basis is
// then the exact one (up to that rule's error).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace seis {

constexpr int kMaxUpliftSources = 16;

struct ForcingArgs {
  const int64_t* elem;     // [F_v] library element
  const int8_t* face;      // [F_v]
  const double* dt;        // [F_v] the element's step
  const double* xy;        // [F_v][nqf][2] points of the projection rule
  const double* proj;      // [Bf][nqf] nodal values of the projection
  int nqf;
  const double* src;       // [1 + 5 kMaxUpliftSources]: count, then (A, x, y, w, T) per source
  const int64_t* macro;    // completed macro steps since seis_write (device counter)
  int Bf;
  int FT;
  int macro_len;           // sub-steps per macro step, 2^(C-1)
  double dt_min;
  int sub;                 // sub-step of the correctors (set per launch)
};

// Inbox of faces [f0, f0 + nf) for the correctors ending at the end of
// sub-step sub of the current macro step. In: FP64 or FP32 inbox.
template <typename T>
hipError_t launch_forcing(const ForcingArgs& a, T* In, int64_t f0, int64_t nf, int sub, hipStream_t s);

// macro += 1 (one thread), at the end of a macro step (so that a captured
// macro step replays with the right time).
hipError_t launch_tick(int64_t* macro, hipStream_t s);

}  // namespace seis
