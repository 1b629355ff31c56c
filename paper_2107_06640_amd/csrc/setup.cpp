// Mesh set-up of the library (host, FP64): validation, geometry, face
// matching, Godunov flux matrices, LTS clusters and element order.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>
#include <sstream>

#include "model.hpp"

namespace seis {

namespace {

const int FACE_V[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

using M9 = std::array<double, 81>;

M9 zero9() {
  M9 m;
  m.fill(0.0);
  return m;
}
M9 mul9(const M9& a, const M9& b) {
  M9 c = zero9();
  for (int i = 0; i < 9; ++i)
    for (int k = 0; k < 9; ++k) {
      const double v = a[i * 9 + k];
      if (v == 0.0) continue;
      for (int j = 0; j < 9; ++j) c[i * 9 + j] += v * b[k * 9 + j];
    }
  return c;
}

// x-direction Jacobian of the velocity-stress system (Sec. 3 PDE written as
// q_t + A q_x + ... = 0): stress rows pick up -(lambda delta_ij + mu ...) dv/dx,
// velocity rows -(1/rho) d s_xj / dx.
M9 jacobian_x(double lam, double mu, double rho) {
  M9 A = zero9();
  A[0 * 9 + 6] = -(lam + 2 * mu);
  A[1 * 9 + 6] = -lam;
  A[2 * 9 + 6] = -lam;
  A[3 * 9 + 7] = -mu;
  A[5 * 9 + 8] = -mu;
  A[6 * 9 + 0] = -1.0 / rho;
  A[7 * 9 + 3] = -1.0 / rho;
  A[8 * 9 + 5] = -1.0 / rho;
  return A;
}

// T(n) of the rotational invariance A-hat = T A T^-1 (Sec. 4.2): block-diagonal
// with the stress transformation (R s R^T in Voigt form) and R = [n s t].
void rotation(const double n[3], M9& T, M9& Tinv) {
  double e[3] = {0, 0, 0};
  int k = 0;
  for (int d = 1; d < 3; ++d)
    if (std::fabs(n[d]) < std::fabs(n[k])) k = d;
  e[k] = 1.0;
  const double en = e[0] * n[0] + e[1] * n[1] + e[2] * n[2];
  double s[3] = {e[0] - en * n[0], e[1] - en * n[1], e[2] - en * n[2]};
  const double ns = std::sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
  for (int d = 0; d < 3; ++d) s[d] /= ns;
  const double t[3] = {n[1] * s[2] - n[2] * s[1], n[2] * s[0] - n[0] * s[2], n[0] * s[1] - n[1] * s[0]};
  double R[3][3];
  for (int d = 0; d < 3; ++d) {
    R[d][0] = n[d];
    R[d][1] = s[d];
    R[d][2] = t[d];
  }
  const int vi[6] = {0, 1, 2, 0, 1, 0}, vj[6] = {0, 1, 2, 1, 2, 2};
  T = zero9();
  Tinv = zero9();
  for (int a = 0; a < 6; ++a) {
    double Ea[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    Ea[vi[a]][vj[a]] = 1.0;
    Ea[vj[a]][vi[a]] = 1.0;
    double G[3][3], L[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double g = 0.0, l = 0.0;
        for (int p = 0; p < 3; ++p)
          for (int q = 0; q < 3; ++q) {
            g += R[i][p] * Ea[p][q] * R[j][q];  // R E R^T
            l += R[p][i] * Ea[p][q] * R[q][j];  // R^T E R
          }
        G[i][j] = g;
        L[i][j] = l;
      }
    for (int b = 0; b < 6; ++b) {
      T[b * 9 + a] = G[vi[b]][vj[b]];
      Tinv[b * 9 + a] = L[vi[b]][vj[b]];
    }
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T[(6 + i) * 9 + 6 + j] = R[i][j];
      Tinv[(6 + i) * 9 + 6 + j] = R[j][i];
    }
}

// Middle state of the rotated Riemann problem, w^b = Gm w- + Gp w+
// (Sec. 4.2, eigen-decomposition and boundary state). Rows of components the
// flux does not read stay zero.
void middle_state(double zpm, double zsm, double zpp, double zsp, M9& Gm, M9& Gp) {
  Gm = zero9();
  Gp = zero9();
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
    // acoustic '-': tangential state is multiplied by mu- = 0 in the flux
  }
}

// Middle-state coefficients of the pointwise Godunov solver (Sec. 4.2) in the
// physical frame, scaled by s: with s_n = n.s.n, t_t = s n - s_n n,
// v_n = v.n, v_t = v - v_n n of a trace,
//   s_n^b = c0 s_n + c1 v_n,  v_n^b = c2 s_n + c3 v_n,
//   t_t^b = c4 t_t + c5 v_t,  v_t^b = c6 t_t + c7 v_t
// summed over the own trace (cm) and the neighbour trace (cp); the flux is
// then A-hat^-(n) applied to (v^b, traction s_n^b n + t_t^b). Ghost states of
// physical boundaries are folded into cm.
void pointwise_coeffs(int kind, double zpm, double zsm, double zpp, double zsp, double s, double cm[8],
                      double cp[8]) {
  for (int i = 0; i < 8; ++i) cm[i] = cp[i] = 0.0;
  if (kind == 2) return;  // gravity surface: handled by the eta ODE
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
  // ghost traces: absorbing 0; wall: same traction, velocity flipped; free: traction flipped
  double gs = 0.0, gv = 0.0;
  if (kind == 4) { gs = 1.0; gv = -1.0; }
  if (kind == 5) { gs = -1.0; gv = 1.0; }
  for (int i = 0; i < 8; i += 2) {
    cm[i] = s * (a[i] + gs * b[i]);
    cm[i + 1] = s * (a[i + 1] + gv * b[i + 1]);
  }
}

struct FaceKey {
  int64_t k[3];
  int64_t id;  // element * 4 + face
};

bool key_less(const FaceKey& a, const FaceKey& b) {
  for (int i = 0; i < 3; ++i)
    if (a.k[i] != b.k[i]) return a.k[i] < b.k[i];
  return a.id < b.id;
}
bool key_eq(const FaceKey& a, const FaceKey& b) {
  return a.k[0] == b.k[0] && a.k[1] == b.k[1] && a.k[2] == b.k[2];
}

}  // namespace

std::string build_model(int64_t nv, const double* xyz, int64_t E, const int64_t* tet, const int8_t* face_kind,
                        const double period[3], const double* rho, const double* lam, const double* mu, int N,
                        double cfl, double g, int max_clusters, Model& M) {
  std::ostringstream err;
  if (nv <= 0 || E <= 0 || !xyz || !tet || !face_kind || !rho || !lam || !mu) return "null or empty mesh/material array";
  if (N < 2 || N > 6) return "order out of range (3..7)";
  if (!(cfl > 0.0) || !(g >= 0.0)) return "cfl must be > 0 and g >= 0";
  if (max_clusters < 1 || max_clusters > 16) return "max_clusters must be in 1..16";
  if (E > (int64_t(1) << 29)) return "too many elements";
  for (int64_t e = 0; e < E; ++e) {
    for (int v = 0; v < 4; ++v)
      if (tet[e * 4 + v] < 0 || tet[e * 4 + v] >= nv) {
        err << "element " << e << ": vertex id out of range";
        return err.str();
      }
    for (int f = 0; f < 4; ++f)
      if (face_kind[e * 4 + f] < 0 || face_kind[e * 4 + f] > 5) {
        err << "element " << e << ": bad face kind";
        return err.str();
      }
    if (!(rho[e] > 0.0) || !(mu[e] >= 0.0) || !(lam[e] + 2.0 * mu[e] > 0.0)) {
      err << "element " << e << ": bad material";
      return err.str();
    }
  }
  M.ref = build_reference(N);
  const RefElement& R = M.ref;
  M.N = N;
  M.B = R.B;
  M.Bf = R.Bf;
  M.nq = R.nq;
  M.E = E;
  M.g = g;

  // ---- geometry (old order)
  std::vector<double> Jinv(E * 9), absdet(E), area(E * 4), normal(E * 12), h(E), cent(E * 12);
  double Lscale = 0.0;
  for (int64_t i = 0; i < nv * 3; ++i) Lscale = std::max(Lscale, std::fabs(xyz[i]));
  Lscale = std::max(Lscale, 1.0);
  for (int64_t e = 0; e < E; ++e) {
    const double* X[4];
    for (int v = 0; v < 4; ++v) X[v] = xyz + 3 * tet[e * 4 + v];
    double J[3][3];
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < 3; ++c) J[d][c] = X[c + 1][d] - X[0][d];
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    double emax = 0.0;
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < 3; ++c) emax = std::max(emax, std::fabs(J[d][c]));
    if (!(std::fabs(det) > 1e-12 * emax * emax * emax)) {
      err << "element " << e << " is degenerate";
      return err.str();
    }
    absdet[e] = std::fabs(det);
    // inverse: Jinv[d][x] = d xi_d / d x
    double* Ji = &Jinv[e * 9];
    Ji[0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    Ji[1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[3] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    Ji[4] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[5] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[6] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    Ji[7] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[8] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    double asum = 0.0;
    for (int f = 0; f < 4; ++f) {
      const double* A = X[FACE_V[f][0]];
      const double* Bp = X[FACE_V[f][1]];
      const double* Cp = X[FACE_V[f][2]];
      const double u[3] = {Bp[0] - A[0], Bp[1] - A[1], Bp[2] - A[2]};
      const double w[3] = {Cp[0] - A[0], Cp[1] - A[1], Cp[2] - A[2]};
      double cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
      const double nrm = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
      for (int d = 0; d < 3; ++d) cr[d] /= nrm;
      const double* O = X[f];
      const double side = cr[0] * (O[0] - A[0]) + cr[1] * (O[1] - A[1]) + cr[2] * (O[2] - A[2]);
      if (side > 0)
        for (int d = 0; d < 3; ++d) cr[d] = -cr[d];
      for (int d = 0; d < 3; ++d) {
        normal[e * 12 + f * 3 + d] = cr[d];
        cent[e * 12 + f * 3 + d] = (A[d] + Bp[d] + Cp[d]) / 3.0;
      }
      area[e * 4 + f] = 0.5 * nrm;
      asum += 0.5 * nrm;
    }
    h[e] = 6.0 * (absdet[e] / 6.0) / asum;  // insphere diameter
  }

  // ---- face matching (old order): nb[e*4+f] = e2*4+f2, vertex map sigma, shift
  std::vector<int64_t> nb(E * 4, -1);
  std::vector<double> shift(E * 12, 0.0);
  {
    std::vector<FaceKey> keys;
    keys.reserve(E * 4);
    for (int64_t e = 0; e < E; ++e)
      for (int f = 0; f < 4; ++f)
        if (face_kind[e * 4 + f] == 0) {
          FaceKey k;
          for (int a = 0; a < 3; ++a) k.k[a] = tet[e * 4 + FACE_V[f][a]];
          std::sort(k.k, k.k + 3);
          k.id = e * 4 + f;
          keys.push_back(k);
        }
    std::sort(keys.begin(), keys.end(), key_less);
    size_t i = 0;
    while (i < keys.size()) {
      if (i + 1 < keys.size() && key_eq(keys[i], keys[i + 1]) &&
          !(i + 2 < keys.size() && key_eq(keys[i], keys[i + 2]))) {
        nb[keys[i].id] = keys[i + 1].id;
        nb[keys[i + 1].id] = keys[i].id;
        i += 2;
      } else {
        err << "interior face of element " << keys[i].id / 4 << " (face " << keys[i].id % 4
            << ") is not shared by exactly two elements";
        return err.str();
      }
    }
    // periodic faces: centroids reduced modulo the period, quantised
    std::vector<FaceKey> pk;
    const double q = 1e-7 * Lscale;
    for (int64_t e = 0; e < E; ++e)
      for (int f = 0; f < 4; ++f)
        if (face_kind[e * 4 + f] == 1) {
          FaceKey k;
          for (int d = 0; d < 3; ++d) {
            double c = cent[e * 12 + f * 3 + d];
            if (period[d] > 0.0) {
              c = std::fmod(c, period[d]);
              if (c < 0) c += period[d];
              if (std::fabs(c - period[d]) < 1e-9 * Lscale) c = 0.0;
            }
            k.k[d] = (int64_t)std::llround(c / q);
          }
          k.id = e * 4 + f;
          pk.push_back(k);
        }
    std::sort(pk.begin(), pk.end(), key_less);
    i = 0;
    while (i < pk.size()) {
      if (i + 1 < pk.size() && key_eq(pk[i], pk[i + 1]) && !(i + 2 < pk.size() && key_eq(pk[i], pk[i + 2]))) {
        const int64_t a = pk[i].id, b = pk[i + 1].id;
        nb[a] = b;
        nb[b] = a;
        for (int d = 0; d < 3; ++d) {
          const double s = cent[(b / 4) * 12 + (b % 4) * 3 + d] - cent[(a / 4) * 12 + (a % 4) * 3 + d];
          shift[a * 3 + d] = s;
          shift[b * 3 + d] = -s;
        }
        i += 2;
      } else {
        err << "periodic face of element " << pk[i].id / 4 << " (face " << pk[i].id % 4 << ") has no partner";
        return err.str();
      }
    }
  }
  // vertex map of each matched face: my face vertex a == neighbour face vertex sigma[a]
  std::vector<int8_t> hmap(E * 4, 0);
  for (int64_t id = 0; id < E * 4; ++id) {
    if (nb[id] < 0) continue;
    const int64_t e = id / 4, f = id % 4, e2 = nb[id] / 4, f2 = nb[id] % 4;
    int sigma[3] = {-1, -1, -1};
    for (int a = 0; a < 3; ++a) {
      const int64_t va = tet[e * 4 + FACE_V[f][a]];
      for (int b = 0; b < 3; ++b) {
        const int64_t vb = tet[e2 * 4 + FACE_V[f2][b]];
        bool same;
        if (face_kind[id] == 0) {
          same = (va == vb);
        } else {
          double d2 = 0.0;
          for (int d = 0; d < 3; ++d) {
            const double x = xyz[3 * va + d] + shift[id * 3 + d] - xyz[3 * vb + d];
            d2 += x * x;
          }
          same = d2 < 1e-18 * Lscale * Lscale;
        }
        if (same) sigma[a] = b;
      }
    }
    const int hh = vertex_map_index(R, sigma);
    if (hh < 0) {
      err << "face " << f << " of element " << e << ": vertices do not match its neighbour's";
      return err.str();
    }
    hmap[id] = (int8_t)hh;
  }

  // ---- gravity faces: acoustic, horizontal, outward normal +z, one per element
  for (int64_t e = 0; e < E; ++e) {
    int cnt = 0;
    for (int f = 0; f < 4; ++f)
      if (face_kind[e * 4 + f] == 2) {
        ++cnt;
        if (mu[e] != 0.0) {
          err << "gravity face on elastic element " << e;
          return err.str();
        }
        if (!(normal[e * 12 + f * 3 + 2] > 1.0 - 1e-9)) {
          err << "gravity face of element " << e << " does not face +z";
          return err.str();
        }
      }
    if (cnt > 1) {
      err << "element " << e << " has more than one gravity face";
      return err.str();
    }
  }

  // ---- time steps and rate-2 clusters (Sec. 4.4)
  std::vector<double> dtk(E);
  double dmin = 1e300;
  for (int64_t e = 0; e < E; ++e) {
    const double cp = std::sqrt((lam[e] + 2 * mu[e]) / rho[e]);
    dtk[e] = cfl / (2 * N + 1) * h[e] / cp;
    dmin = std::min(dmin, dtk[e]);
  }
  std::vector<int32_t> cl(E);
  for (int64_t e = 0; e < E; ++e) {
    int c = (int)std::floor(std::log2(dtk[e] / dmin));
    c = std::max(0, std::min(c, max_clusters - 1));
    cl[e] = c;
  }
  for (bool changed = true; changed;) {
    changed = false;
    for (int64_t id = 0; id < E * 4; ++id) {
      if (nb[id] < 0) continue;
      const int64_t e = id / 4, e2 = nb[id] / 4;
      if (cl[e] > cl[e2] + 1) {
        cl[e] = cl[e2] + 1;
        changed = true;
      }
    }
  }
  int C = 1;
  for (int64_t e = 0; e < E; ++e) C = std::max(C, cl[e] + 1);
  M.C = C;
  M.dt_min = dmin;
  M.dt_c.resize(C);
  for (int c = 0; c < C; ++c) M.dt_c[c] = std::ldexp(dmin, c);
  M.cluster_old = cl;

  // ---- element order: by cluster; inside a cluster, elements with a
  // neighbour in another cluster last (stable)
  std::vector<int8_t> iface(E, 0);
  for (int64_t id = 0; id < E * 4; ++id)
    if (nb[id] >= 0 && cl[nb[id] / 4] != cl[id / 4]) iface[id / 4] = 1;
  M.old_of_new.resize(E);
  std::iota(M.old_of_new.begin(), M.old_of_new.end(), 0);
  std::stable_sort(M.old_of_new.begin(), M.old_of_new.end(), [&](int64_t a, int64_t b) {
    if (cl[a] != cl[b]) return cl[a] < cl[b];
    return iface[a] < iface[b];
  });
  M.new_of_old.resize(E);
  for (int64_t k = 0; k < E; ++k) M.new_of_old[M.old_of_new[k]] = k;
  M.cluster_start.assign(C + 1, 0);
  for (int64_t e = 0; e < E; ++e) M.cluster_start[cl[e] + 1]++;
  for (int c = 0; c < C; ++c) M.cluster_start[c + 1] += M.cluster_start[c];
  M.iface_start.assign(C, 0);
  for (int c = 0; c < C; ++c) {
    int64_t k = M.cluster_start[c];
    while (k < M.cluster_start[c + 1] && !iface[M.old_of_new[k]]) ++k;
    M.iface_start[c] = k;
  }

  // ---- per element data (new order)
  M.G.assign(E * 9, 0.0);
  M.mat.assign(E * 3, 0.0);
  M.Fm.assign(E * 4 * 81, 0.0);
  M.Fp.assign(E * 4 * 81, 0.0);
  M.RCm.assign(E * 4 * 12, 0.0);
  M.RCp.assign(E * 4 * 12, 0.0);
  M.tgt.assign(E * 4, -1);
  M.mode.assign(E * 4, MODE_NONE);
  M.hperm.assign(E * 4, 0);
  M.half2.assign(E * 4, -1);
  M.rhalf2.assign(E * 4, -1);
  M.gslot.assign(E, -1);
  int64_t nh2 = 0;
  for (int64_t k = 0; k < E; ++k) {
    const int64_t e = M.old_of_new[k];
    const double dt = M.dt_c[cl[e]];
    for (int i = 0; i < 9; ++i) M.G[k * 9 + i] = dt * Jinv[e * 9 + i];
    M.mat[k * 3 + 0] = lam[e];
    M.mat[k * 3 + 1] = mu[e];
    M.mat[k * 3 + 2] = 1.0 / rho[e];
    const double zpm = std::sqrt((lam[e] + 2 * mu[e]) * rho[e]), zsm = std::sqrt(mu[e] * rho[e]);
    const M9 A = jacobian_x(lam[e], mu[e], rho[e]);
    for (int f = 0; f < 4; ++f) {
      const int64_t id = e * 4 + f;
      const int kind = face_kind[id];
      const double scale = 2.0 * area[id] * dt / absdet[e];
      M9 T, Ti, Gm, Gp, Fm = zero9(), Fp = zero9();
      rotation(&normal[id * 3], T, Ti);
      if (kind == 0 || kind == 1) {
        const int64_t e2 = nb[id] / 4;
        const double zpp = std::sqrt((lam[e2] + 2 * mu[e2]) * rho[e2]), zsp = std::sqrt(mu[e2] * rho[e2]);
        middle_state(zpm, zsm, zpp, zsp, Gm, Gp);
        Fm = mul9(mul9(T, mul9(A, Gm)), Ti);
        Fp = mul9(mul9(T, mul9(A, Gp)), Ti);
      } else if (kind == 3 || kind == 4 || kind == 5) {
        middle_state(zpm, zsm, zpm, zsm, Gm, Gp);
        if (kind == 4 || kind == 5) {
          // ghost w+ = diag(m) w-, with m flipping velocity (wall) or stress (free surface)
          for (int r = 0; r < 9; ++r)
            for (int c = 0; c < 9; ++c) {
              const double m = (kind == 4) ? (c >= 6 ? -1.0 : 1.0) : (c < 6 ? -1.0 : 1.0);
              Gm[r * 9 + c] += Gp[r * 9 + c] * m;
            }
        }
        Fm = mul9(mul9(T, mul9(A, Gm)), Ti);
      }
      for (int i = 0; i < 81; ++i) {
        M.Fm[(k * 4 + f) * 81 + i] = scale * Fm[i];
        M.Fp[(k * 4 + f) * 81 + i] = scale * Fp[i];
      }
      double zpp = zpm, zsp = zsm;
      if (kind == 0 || kind == 1) {
        const int64_t e2 = nb[id] / 4;
        zpp = std::sqrt((lam[e2] + 2 * mu[e2]) * rho[e2]);
        zsp = std::sqrt(mu[e2] * rho[e2]);
      }
      double cm[8], cp[8];
      pointwise_coeffs(kind, zpm, zsm, zpp, zsp, scale, cm, cp);
      double* rm = &M.RCm[(k * 4 + f) * 12];
      double* rp = &M.RCp[(k * 4 + f) * 12];
      for (int d = 0; d < 3; ++d) rm[d] = rp[d] = normal[id * 3 + d];
      for (int i = 0; i < 8; ++i) {
        rm[3 + i] = cm[i];
        rp[3 + i] = cp[i];
      }
    }
  }
  // writer-side hand-over of each face: element J (new kn) face j writes into neighbour K's face i
  for (int64_t kn = 0; kn < E; ++kn) {
    const int64_t e = M.old_of_new[kn];
    for (int f = 0; f < 4; ++f) {
      const int64_t id = e * 4 + f;
      if (nb[id] < 0) continue;
      const int64_t e2 = nb[id] / 4, f2 = nb[id] % 4;
      const int64_t k2 = M.new_of_old[e2];
      M.tgt[kn * 4 + f] = int32_t(k2 * 4 + f2);
      // node map for the receiving face: its vertex a == my vertex sigma'[a]
      M.hperm[kn * 4 + f] = hmap[nb[id]];
      const int dc = cl[e2] - cl[e];
      if (dc == 0) M.mode[kn * 4 + f] = MODE_SAME;
      else if (dc == -1) {
        M.mode[kn * 4 + f] = MODE_FINER;
        M.half2[kn * 4 + f] = int32_t(nh2);
        M.rhalf2[k2 * 4 + f2] = int32_t(nh2);
        ++nh2;
      } else if (dc == 1) M.mode[kn * 4 + f] = MODE_COARSER;
      else return "cluster normalisation failed";
    }
  }
  M.n_half2 = nh2;

  // ---- gravity faces, ABI order = sorted by (caller element, face)
  for (int64_t e = 0; e < E; ++e)
    for (int f = 0; f < 4; ++f)
      if (face_kind[e * 4 + f] == 2) {
        const int64_t id = e * 4 + f;
        const int64_t kn = M.new_of_old[e];
        M.gslot[kn] = int32_t(M.g_elem.size());
        M.g_elem.push_back(kn);
        M.g_face.push_back(int8_t(f));
        const double zp = std::sqrt(lam[e] * rho[e]);
        const double par[8] = {2.0 * area[id] / absdet[e], normal[id * 3], normal[id * 3 + 1], normal[id * 3 + 2],
                               zp, rho[e] * g / zp, lam[e], M.dt_c[cl[e]]};
        for (int p = 0; p < 8; ++p) M.g_par.push_back(par[p]);
      }
  M.g_order.resize(M.g_elem.size());
  std::iota(M.g_order.begin(), M.g_order.end(), 0);
  return "";
}

}  // namespace seis
