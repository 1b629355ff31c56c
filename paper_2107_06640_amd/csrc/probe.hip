// Output of the solution at points (see probe.hpp).
#include "probe.hpp"

#include <algorithm>
#include <cmath>
#include <sstream>

#include "layout.hpp"
#include "refelem.hpp"

namespace seis {

namespace {

// x0 and the inverse of J = [x1-x0, x2-x0, x3-x0] of a caller element
void element_map(const Model& M, int64_t e, double x0[3], double Ji[9]) {
  const double* X[4];
  for (int v = 0; v < 4; ++v) X[v] = M.xyz.data() + 3 * M.tet[e * 4 + v];
  double J[9];
  for (int d = 0; d < 3; ++d)
    for (int c = 0; c < 3; ++c) J[d * 3 + c] = X[c + 1][d] - X[0][d];  // J[row d][col c]
  const double det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                     J[2] * (J[3] * J[7] - J[4] * J[6]);
  Ji[0] = (J[4] * J[8] - J[5] * J[7]) / det;
  Ji[1] = (J[2] * J[7] - J[1] * J[8]) / det;
  Ji[2] = (J[1] * J[5] - J[2] * J[4]) / det;
  Ji[3] = (J[5] * J[6] - J[3] * J[8]) / det;
  Ji[4] = (J[0] * J[8] - J[2] * J[6]) / det;
  Ji[5] = (J[2] * J[3] - J[0] * J[5]) / det;
  Ji[6] = (J[3] * J[7] - J[4] * J[6]) / det;
  Ji[7] = (J[1] * J[6] - J[0] * J[7]) / det;
  Ji[8] = (J[0] * J[4] - J[1] * J[3]) / det;
  for (int d = 0; d < 3; ++d) x0[d] = X[0][d];
}

template <typename T>
__global__ __launch_bounds__(256) void k_sample(const T* Q, int RT, int B, const int32_t* elem, const double* phi,
                                                int64_t n, double* out, const double* eta, double* eta_out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n * 9) return;
  const int64_t r = i / 9;
  const int p = int(i % 9);
  const int64_t e = elem[r];
  double acc = 0.0;
  for (int l = 0; l < B; ++l) acc += phi[r * B + l] * (double)Q[qidx(e, l, p, RT)];
  out[i] = acc;
  if (p == 0 && eta_out) eta_out[r] = eta[r];
}

}  // namespace

std::string locate_points(const Model& M, int64_t n, const double* xyz, std::vector<int64_t>& elem_caller,
                          std::vector<double>& xi) {
  const int64_t E = M.E, nv = (int64_t)M.xyz.size() / 3;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < nv; ++v)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], M.xyz[3 * v + d]);
      hi[d] = std::max(hi[d], M.xyz[3 * v + d]);
    }
  double L = 0.0;
  for (int d = 0; d < 3; ++d) L = std::max(L, hi[d] - lo[d]);
  const double pad = 1e-9 * L;
  // uniform grid of about one element per cell; each element is listed in
  // every cell its (slightly widened) bounding box touches
  double vol = 1.0;
  for (int d = 0; d < 3; ++d) vol *= std::max(hi[d] - lo[d], 1e-12 * L);
  const double hc = std::cbrt(vol / double(E));
  int nc[3];
  double cs[3];
  for (int d = 0; d < 3; ++d) {
    nc[d] = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (int64_t)std::llround((hi[d] - lo[d]) / hc)));
    cs[d] = std::max(hi[d] - lo[d], 1e-12 * L) / nc[d];
  }
  auto cell_of = [&](double x, int d) {
    const int c = (int)std::floor((x - lo[d]) / cs[d]);
    return std::min(std::max(c, 0), nc[d] - 1);
  };
  const int64_t ncell = int64_t(nc[0]) * nc[1] * nc[2];
  // cell range of every element's widened bounding box
  std::vector<int> crange(E * 6);
  for (int64_t e = 0; e < E; ++e)
    for (int d = 0; d < 3; ++d) {
      double a = 1e300, b = -1e300;
      for (int v = 0; v < 4; ++v) {
        const double x = M.xyz[3 * M.tet[e * 4 + v] + d];
        a = std::min(a, x);
        b = std::max(b, x);
      }
      crange[6 * e + 2 * d] = cell_of(a - pad, d);
      crange[6 * e + 2 * d + 1] = cell_of(b + pad, d);
    }
  // element lists per cell (counts, offsets, fill)
  std::vector<int64_t> start(ncell + 1, 0);
  auto for_cells = [&](int64_t e, auto fn) {
    const int* cr = crange.data() + 6 * e;
    for (int i = cr[0]; i <= cr[1]; ++i)
      for (int j = cr[2]; j <= cr[3]; ++j)
        for (int k = cr[4]; k <= cr[5]; ++k) fn((int64_t(i) * nc[1] + j) * nc[2] + k);
  };
  for (int64_t e = 0; e < E; ++e) for_cells(e, [&](int64_t c) { start[c + 1]++; });
  for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
  std::vector<int64_t> fill(start.begin(), start.end() - 1), list(start[ncell]);
  for (int64_t e = 0; e < E; ++e) for_cells(e, [&](int64_t c) { list[fill[c]++] = e; });
  // each point: the lowest element id among the candidates of its cell that contain it
  elem_caller.assign(n, -1);
  xi.assign(n * 3, 0.0);
  for (int64_t r = 0; r < n; ++r) {
    const double* x = xyz + 3 * r;
    const int64_t c = (int64_t(cell_of(x[0], 0)) * nc[1] + cell_of(x[1], 1)) * nc[2] + cell_of(x[2], 2);
    int64_t best = -1;
    double bxi[3] = {0, 0, 0};
    for (int64_t q = start[c]; q < start[c + 1]; ++q) {
      const int64_t e = list[q];
      if (best >= 0 && e >= best) continue;
      double x0[3], Ji[9], rx[3];
      element_map(M, e, x0, Ji);
      for (int d = 0; d < 3; ++d)
        rx[d] = Ji[d * 3 + 0] * (x[0] - x0[0]) + Ji[d * 3 + 1] * (x[1] - x0[1]) + Ji[d * 3 + 2] * (x[2] - x0[2]);
      const double b0 = 1.0 - rx[0] - rx[1] - rx[2];
      if (b0 >= -1e-9 && rx[0] >= -1e-9 && rx[1] >= -1e-9 && rx[2] >= -1e-9) {
        best = e;
        for (int d = 0; d < 3; ++d) bxi[d] = rx[d];
      }
    }
    if (best < 0) {
      std::ostringstream os;
      os << "point " << r << " (" << x[0] << ", " << x[1] << ", " << x[2] << ") is outside the mesh";
      return os.str();
    }
    elem_caller[r] = best;
    for (int d = 0; d < 3; ++d) xi[3 * r + d] = bxi[d];
  }
  return "";
}

std::string build_points(const Model& M, int which, int64_t n, const double* xyz, PointSet& ps,
                         std::vector<double>& phi, std::vector<int32_t>& elem_lib) {
  const int B = M.B;
  std::vector<double> xi;
  std::vector<double> pts;
  std::vector<int64_t> ec;
  if (which == 0) {
    pts.assign(xyz, xyz + 3 * n);
    const std::string e = locate_points(M, n, xyz, ec, xi);
    if (!e.empty()) return e;
  } else {
    // faces of the set in output order: (library element, local face)
    std::vector<std::pair<int64_t, int>> faces;
    if (which == 1)
      for (size_t f = 0; f < M.g_elem.size(); ++f) faces.push_back({M.g_elem[f], M.g_face[f]});
    else
      for (size_t f = 0; f < M.floor_elem.size(); ++f) faces.push_back({M.floor_elem[f], M.floor_face[f]});
    const int nq = M.nq;
    n = (int64_t)faces.size() * nq;
    pts.resize(3 * n);
    xi.resize(3 * n);
    ec.resize(n);
    for (size_t f = 0; f < faces.size(); ++f) {
      const int64_t e = M.old_of_new[faces[f].first];
      double x0[3], Ji[9];
      element_map(M, e, x0, Ji);
      const double* X[4];
      for (int v = 0; v < 4; ++v) X[v] = M.xyz.data() + 3 * M.tet[e * 4 + v];
      for (int q = 0; q < nq; ++q) {
        const int64_t r = (int64_t)f * nq + q;
        double* rx = xi.data() + 3 * r;
        face_to_ref(faces[f].second, M.ref.eta_st[2 * q], M.ref.eta_st[2 * q + 1], rx);
        for (int d = 0; d < 3; ++d)
          pts[3 * r + d] = X[0][d] + (X[1][d] - X[0][d]) * rx[0] + (X[2][d] - X[0][d]) * rx[1] +
                           (X[3][d] - X[0][d]) * rx[2];
        ec[r] = e;
      }
    }
  }
  ps.n = n;
  ps.xyz = pts;
  ps.elem_caller = ec;
  ps.sea = which == 1;
  phi.assign(n * B, 0.0);
  elem_lib.assign(n, 0);
  for (int64_t r = 0; r < n; ++r) {
    dubiner(M.N, xi.data() + 3 * r, phi.data() + r * B, nullptr);
    elem_lib[r] = int32_t(M.new_of_old[ec[r]]);
  }
  return "";
}

hipError_t launch_sample(const PointSet& ps, int B, const double* Q64, const float* Q32, const double* eta,
                         double* out, double* eta_out, hipStream_t s) {
  if (ps.n <= 0) return hipSuccess;
  const int RT = row_tiles(B);
  const unsigned grid = (unsigned)((ps.n * 9 + 255) / 256);
  if (Q64)
    hipLaunchKernelGGL(k_sample<double>, dim3(grid), dim3(256), 0, s, Q64, RT, B, ps.elem, ps.phi, ps.n, out, eta,
                       eta_out);
  else
    hipLaunchKernelGGL(k_sample<float>, dim3(grid), dim3(256), 0, s, Q32, RT, B, ps.elem, ps.phi, ps.n, out, eta,
                       eta_out);
  return hipGetLastError();
}

}  // namespace seis
