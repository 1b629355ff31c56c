// Output of the solution at points: receivers at given physical points, and
// the sea surface and the elastic-acoustic interface at the face rule of the
// sea-surface height (Sec. 6.2 writes receivers every 0.01 s and both surfaces
// every 0.1 s).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "model.hpp"

namespace seis {

struct PointSet {
  int64_t n = 0;
  std::vector<double> xyz;           // [n][3]
  std::vector<int64_t> elem_caller;  // [n]
  double* phi = nullptr;             // device [n][B]: basis values at the point's reference coordinates
  int32_t* elem = nullptr;           // device [n]: element, library order
  bool sea = false;                  // the sea-surface set (the points of eta)
};

// Element (the lowest caller id among those containing the point, within
// 1e-9 in barycentric coordinates) and reference coordinates of n points.
// Returns an empty string, or an error message for a point outside the mesh.
std::string locate_points(const Model& M, int64_t n, const double* xyz, std::vector<int64_t>& elem_caller,
                          std::vector<double>& xi);

// Host part of a set: the points, their elements and basis values.
// which: 0 given points (located), 1 sea surface (eta points of the gravity
// faces, eta order), 2 elastic-acoustic interface (elastic side).
std::string build_points(const Model& M, int which, int64_t n, const double* xyz, PointSet& ps,
                         std::vector<double>& phi, std::vector<int32_t>& elem_lib);

// out[r][p] = sum_l phi[r][l] Q[elem[r]][l][p] (FP64); eta_out[r] = eta[r] if eta_out.
hipError_t launch_sample(const PointSet& ps, int B, const double* Q64, const float* Q32, const double* eta,
                         double* out, double* eta_out, hipStream_t s);

}  // namespace seis
