// Mesh set-up of the library (host, FP64): validation, geometry, face
// matching, LTS clusters, element order and the inputs of the operator
// assembly, which runs on the GPU.
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
  if (N < 1 || N > 7) return "order out of range (2..8)";
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
      if (face_kind[e * 4 + f] < 0 || face_kind[e * 4 + f] > 7) {
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
        if (face_kind[e * 4 + f] == 0 || face_kind[e * 4 + f] == 7) {
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
        if (face_kind[keys[i].id] != face_kind[keys[i + 1].id]) {
          err << "fault face of element " << keys[i].id / 4 << " (face " << keys[i].id % 4
              << ") meets a face that is not a fault face";
          return err.str();
        }
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
        if (face_kind[id] == 0 || face_kind[id] == 7) {
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

  // ---- fault faces: elastic on both sides
  for (int64_t id = 0; id < E * 4; ++id)
    if (face_kind[id] == 7 && !(mu[id / 4] > 0.0)) {
      err << "fault face on acoustic element " << id / 4;
      return err.str();
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
  // neighbours differ by at most one cluster; the two sides of a fault face
  // share one (the friction law couples them pointwise in time)
  for (bool changed = true; changed;) {
    changed = false;
    for (int64_t id = 0; id < E * 4; ++id) {
      if (nb[id] < 0) continue;
      const int64_t e = id / 4, e2 = nb[id] / 4;
      const int up = face_kind[id] == 7 ? 0 : 1;
      if (cl[e] > cl[e2] + up) {
        cl[e] = cl[e2] + up;
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
  // neighbour in another cluster last, so that the hand-over branches of the
  // matrix-core kernels diverge in few element groups, and inside each of
  // those the acoustic elements first, so that whole 16-element groups are
  // acoustic (the 4-quantity form); stable otherwise
  std::vector<int8_t> iface(E, 0);
  for (int64_t id = 0; id < E * 4; ++id)
    if (nb[id] >= 0 && cl[nb[id] / 4] != cl[id / 4]) iface[id / 4] = 1;
  M.old_of_new.resize(E);
  std::iota(M.old_of_new.begin(), M.old_of_new.end(), 0);
  std::stable_sort(M.old_of_new.begin(), M.old_of_new.end(), [&](int64_t a, int64_t b) {
    if (cl[a] != cl[b]) return cl[a] < cl[b];
    if (iface[a] != iface[b]) return iface[a] < iface[b];
    return (mu[a] > 0.0) < (mu[b] > 0.0);
  });
  M.new_of_old.resize(E);
  for (int64_t k = 0; k < E; ++k) M.new_of_old[M.old_of_new[k]] = k;
  M.cluster_start.assign(C + 1, 0);
  for (int64_t e = 0; e < E; ++e) M.cluster_start[cl[e] + 1]++;
  for (int c = 0; c < C; ++c) M.cluster_start[c + 1] += M.cluster_start[c];

  // ---- per element inputs of the operator assembly (new order)
  M.a_Jinv.resize(E * 9);
  M.a_absdet.resize(E);
  M.a_dt.resize(E);
  M.a_lmr.resize(E * 3);
  M.a_nrm.resize(E * 12);
  M.a_area.resize(E * 4);
  M.a_kind.resize(E * 4);
  M.a_nbk.assign(E * 4, -1);
  M.tgt.assign(E * 4, -1);
  M.mode.assign(E * 4, MODE_NONE);
  M.hperm.assign(E * 4, 0);
  M.half2.assign(E * 4, -1);
  M.rhalf2.assign(E * 4, -1);
  M.gslot.assign(E, -1);
  int64_t nh2 = 0;
  for (int64_t k = 0; k < E; ++k) {
    const int64_t e = M.old_of_new[k];
    for (int i = 0; i < 9; ++i) M.a_Jinv[k * 9 + i] = Jinv[e * 9 + i];
    M.a_absdet[k] = absdet[e];
    M.a_dt[k] = M.dt_c[cl[e]];
    M.a_lmr[k * 3 + 0] = lam[e];
    M.a_lmr[k * 3 + 1] = mu[e];
    M.a_lmr[k * 3 + 2] = rho[e];
    for (int f = 0; f < 4; ++f) {
      const int64_t id = e * 4 + f;
      for (int d = 0; d < 3; ++d) M.a_nrm[k * 12 + f * 3 + d] = normal[id * 3 + d];
      M.a_area[k * 4 + f] = area[id];
      M.a_kind[k * 4 + f] = face_kind[id];
      if (nb[id] >= 0) M.a_nbk[k * 4 + f] = M.new_of_old[nb[id] / 4];
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
      // node map for the receiving face: its vertex a == my vertex sigma'[a]
      M.hperm[kn * 4 + f] = hmap[nb[id]];
      if (face_kind[id] == 7) continue;  // fault: the friction kernel fills both inboxes
      M.tgt[kn * 4 + f] = int32_t(k2 * 4 + f2);
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
        M.g_coef.push_back(rho[e] * g * area[id]);
      }
  // ---- elastic-acoustic interface faces (elastic side), for output
  for (int64_t e = 0; e < E; ++e) {
    if (!(mu[e] > 0.0)) continue;
    for (int f = 0; f < 4; ++f) {
      const int64_t id = e * 4 + f;
      if (nb[id] >= 0 && mu[nb[id] / 4] == 0.0) {
        M.floor_elem.push_back(M.new_of_old[e]);
        M.floor_face.push_back(int8_t(f));
      }
    }
  }
  // ---- prescribed-velocity faces, grouped by cluster (library order inside)
  M.vface_start.assign(C + 1, 0);
  for (int c = 0; c < C; ++c) {
    M.vface_start[c] = (int64_t)M.v_elem.size();
    for (int64_t kn = M.cluster_start[c]; kn < M.cluster_start[c + 1]; ++kn) {
      const int64_t e = M.old_of_new[kn];
      for (int f = 0; f < 4; ++f) {
        if (face_kind[e * 4 + f] != 6) continue;
        M.v_elem.push_back(kn);
        M.v_face.push_back(int8_t(f));
        M.v_dt.push_back(M.dt_c[c]);
        const double* X[4];
        for (int v = 0; v < 4; ++v) X[v] = xyz + 3 * tet[e * 4 + v];
        for (int m = 0; m < R.nqf; ++m) {
          double xi[3];
          face_to_ref(f, R.fproj_st[2 * m], R.fproj_st[2 * m + 1], xi);
          for (int d = 0; d < 2; ++d)
            M.v_xy.push_back(X[0][d] + (X[1][d] - X[0][d]) * xi[0] + (X[2][d] - X[0][d]) * xi[1] +
                             (X[3][d] - X[0][d]) * xi[2]);
        }
      }
    }
  }
  M.vface_start[C] = (int64_t)M.v_elem.size();
  // ---- fault faces from their '-' side (the smaller caller element id),
  // grouped by cluster (ABI order = by caller (element, face) of that side)
  {
    std::vector<std::pair<int64_t, int>> fl;  // caller (element, face)
    for (int64_t e = 0; e < E; ++e)
      for (int f = 0; f < 4; ++f)
        if (face_kind[e * 4 + f] == 7 && nb[e * 4 + f] / 4 > e) fl.push_back({e, f});
    M.fault_start.assign(C + 1, 0);
    std::vector<std::vector<int64_t>> by_c(C);
    for (int64_t k = 0; k < (int64_t)fl.size(); ++k) by_c[cl[fl[k].first]].push_back(k);
    M.fault_abi.assign(fl.size(), 0);
    for (int c = 0; c < C; ++c) {
      M.fault_start[c] = (int64_t)M.f_elem.size();
      for (int64_t k : by_c[c]) {
        const int64_t e = fl[k].first, id = e * 4 + fl[k].second;
        const int64_t e2 = nb[id] / 4;
        M.fault_abi[k] = (int64_t)M.f_elem.size();
        M.f_elem.push_back(M.new_of_old[e]);
        M.f_face.push_back(int8_t(fl[k].second));
        M.f_pelem.push_back(M.new_of_old[e2]);
        M.f_pface.push_back(int8_t(nb[id] % 4));
        M.f_perm.push_back(hmap[nb[id]]);
        const double zpm = std::sqrt((lam[e] + 2 * mu[e]) * rho[e]), zsm = std::sqrt(mu[e] * rho[e]);
        const double zpp = std::sqrt((lam[e2] + 2 * mu[e2]) * rho[e2]), zsp = std::sqrt(mu[e2] * rho[e2]);
        const double geo[8] = {normal[id * 3], normal[id * 3 + 1], normal[id * 3 + 2], zpm, zsm, zpp, zsp,
                               M.dt_c[cl[e]]};
        for (int p = 0; p < 8; ++p) M.f_geo.push_back(geo[p]);
        const double* X[4];
        for (int v = 0; v < 4; ++v) X[v] = xyz + 3 * tet[e * 4 + v];
        for (int m = 0; m < R.Bf; ++m) {
          double xi[3];
          face_to_ref(fl[k].second, R.node_st[2 * m], R.node_st[2 * m + 1], xi);
          for (int d = 0; d < 3; ++d)
            M.f_xyz.push_back(X[0][d] + (X[1][d] - X[0][d]) * xi[0] + (X[2][d] - X[0][d]) * xi[1] +
                              (X[3][d] - X[0][d]) * xi[2]);
        }
      }
    }
    M.fault_start[C] = (int64_t)M.f_elem.size();
  }
  M.xyz.assign(xyz, xyz + nv * 3);
  M.tet.assign(tet, tet + E * 4);
  M.g_order.resize(M.g_elem.size());
  std::iota(M.g_order.begin(), M.g_order.end(), 0);

  // ---- derivative slots and the per-cluster face lists of the LTS hand-over
  M.dslot.assign(E, -1);
  int64_t nd = (int64_t)M.g_elem.size();
  for (int64_t k = 0; k < E; ++k) M.dslot[k] = M.gslot[k];
  std::vector<char> on_fault(E, 0);
  for (size_t k = 0; k < M.f_elem.size(); ++k) on_fault[M.f_elem[k]] = on_fault[M.f_pelem[k]] = 1;
  for (int64_t k = 0; k < E; ++k) {
    bool finer = false;
    for (int f = 0; f < 4; ++f) finer = finer || M.mode[k * 4 + f] == MODE_FINER;
    if ((finer || on_fault[k]) && M.dslot[k] < 0) M.dslot[k] = int32_t(nd++);
  }
  M.n_dslot = nd;
  for (size_t k = 0; k < M.f_elem.size(); ++k)
    if (M.dslot[M.f_elem[k]] < 0 || M.dslot[M.f_pelem[k]] < 0) return "fault element without a derivative slot";
  M.fix_start.assign(C + 1, 0);
  M.h2_start.assign(C + 1, 0);
  for (int c = 0; c < C; ++c) {
    M.fix_start[c] = (int64_t)M.fix_list.size();
    M.h2_start[c] = (int64_t)M.h2_list.size();
    for (int64_t k = M.cluster_start[c]; k < M.cluster_start[c + 1]; ++k)
      for (int f = 0; f < 4; ++f) {
        if (M.mode[k * 4 + f] == MODE_FINER) M.fix_list.push_back(int32_t(k * 4 + f));
        if (M.rhalf2[k * 4 + f] >= 0) M.h2_list.push_back(int32_t(k * 4 + f));
      }
  }
  M.fix_start[C] = (int64_t)M.fix_list.size();
  M.h2_start[C] = (int64_t)M.h2_list.size();
  return "";
}

}  // namespace seis
