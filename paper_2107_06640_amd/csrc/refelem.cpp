// Reference-element integrals of the library (host, FP64). See refelem.hpp.
//
// The basis is evaluated in a division-free form so that it can be sampled on
// faces, edges and vertices of the reference element: with s = 1 - y - z and
// t = 1 - z,
//   phi_pqr = H_p^(0,0)(2x - s, s) H_q^(2p+1,0)(2y - t, t) P_r^(2p+2q+2,0)(2z - 1) / sqrt(n_pqr)
// where H_n^(a,b)(u, w) = w^n P_n^(a,b)(u / w) is the homogenised Jacobi
// polynomial (its three-term recurrence carries powers of w instead of a
// division) and n_pqr = 1 / (2 (2p+1)(p+q+1)(2p+2q+2r+3)) is the squared norm.
// Gradients use forward-mode dual numbers through the same recurrences.
#include "refelem.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace seis {

namespace {

struct Dual {
  double v = 0, d[3] = {0, 0, 0};
  Dual() = default;
  Dual(double c) : v(c) {}
};
inline Dual operator+(const Dual& a, const Dual& b) {
  Dual r(a.v + b.v);
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
inline Dual operator-(const Dual& a, const Dual& b) {
  Dual r(a.v - b.v);
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
inline Dual operator*(const Dual& a, const Dual& b) {
  Dual r(a.v * b.v);
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
inline Dual operator*(double s, const Dual& a) {
  Dual r(s * a.v);
  for (int i = 0; i < 3; ++i) r.d[i] = s * a.d[i];
  return r;
}

// Homogenised Jacobi polynomials H_0..H_n at (u, w): w^k P_k^(a,b)(u/w).
void hjacobi(int n, double a, double b, const Dual& u, const Dual& w, std::vector<Dual>& H) {
  H.assign(n + 1, Dual(0.0));
  H[0] = Dual(1.0);
  if (n == 0) return;
  H[1] = 0.5 * ((a - b) * w + (a + b + 2.0) * u);
  for (int k = 1; k < n; ++k) {
    const double s = 2.0 * k + a + b;
    const double a1 = 2.0 * (k + 1) * (k + a + b + 1) * s;
    const double a2 = (s + 1) * (a * a - b * b);
    const double a3 = s * (s + 1) * (s + 2);
    const double a4 = 2.0 * (k + a) * (k + b) * (s + 2);
    H[k + 1] = (1.0 / a1) * ((a2 * w + a3 * u) * H[k] - a4 * (w * w) * H[k - 1]);
  }
}

double jacobi_p(int n, double a, double b, double x, double* dp) {
  // value and derivative of P_n^(a,b)(x) by the recurrence
  double p0 = 1.0, p1 = 0.5 * (a - b + (a + b + 2.0) * x);
  double d0 = 0.0, d1 = 0.5 * (a + b + 2.0);
  if (n == 0) {
    if (dp) *dp = 0.0;
    return 1.0;
  }
  for (int k = 1; k < n; ++k) {
    const double s = 2.0 * k + a + b;
    const double a1 = 2.0 * (k + 1) * (k + a + b + 1) * s;
    const double a2 = (s + 1) * (a * a - b * b);
    const double a3 = s * (s + 1) * (s + 2);
    const double a4 = 2.0 * (k + a) * (k + b) * (s + 2);
    const double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
    const double d2 = ((a2 + a3 * x) * d1 + a3 * p1 - a4 * d0) / a1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  if (dp) *dp = d1;
  return p1;
}

struct PQR { int p, q, r; };

std::vector<PQR> ordering(int N) {
  std::vector<PQR> idx;
  for (int p = 0; p <= N; ++p)
    for (int q = 0; p + q <= N; ++q)
      for (int r = 0; p + q + r <= N; ++r) idx.push_back({p, q, r});
  std::sort(idx.begin(), idx.end(), [](const PQR& A, const PQR& B) {
    const int da = A.p + A.q + A.r, db = B.p + B.q + B.r;
    if (da != db) return da < db;
    if (A.r != B.r) return A.r < B.r;
    if (A.q != B.q) return A.q < B.q;
    return A.p < B.p;
  });
  return idx;
}

// Plain LU solve with partial pivoting of A X = Bm (A n x n, Bm n x m, row-major).
void lu_solve(int n, std::vector<double> A, std::vector<double>& Bm, int m) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) throw std::runtime_error("singular Vandermonde matrix");
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
      for (int k = 0; k < m; ++k) std::swap(Bm[c * m + k], Bm[piv * m + k]);
    }
    for (int r = c + 1; r < n; ++r) {
      const double f = A[r * n + c] / A[c * n + c];
      if (f == 0.0) continue;
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      for (int k = 0; k < m; ++k) Bm[r * m + k] -= f * Bm[c * m + k];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    for (int k = 0; k < m; ++k) {
      double s = Bm[c * m + k];
      for (int j = c + 1; j < n; ++j) s -= A[c * n + j] * Bm[j * m + k];
      Bm[c * m + k] = s / A[c * n + c];
    }
  }
}

// Orthogonal (unnormalised) basis of P_N on the triangle {s, t >= 0, s + t <= 1}.
void triangle_basis(int N, double s, double t, std::vector<double>& out) {
  out.clear();
  std::vector<Dual> Ha;
  Dual u(2.0 * s - (1.0 - t)), w(1.0 - t);
  hjacobi(N, 0.0, 0.0, u, w, Ha);
  for (int b = 0; b <= N; ++b)
    for (int a = 0; a + b <= N; ++a) {
      const double pb = jacobi_p(b, 2.0 * a + 1.0, 0.0, 2.0 * t - 1.0, nullptr);
      out.push_back(Ha[a].v * pb);
    }
}

const double REF_V[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
const int FACE_V[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

}  // namespace

void face_to_ref(int i, double s, double t, double xi[3]) {
  const double* a = REF_V[FACE_V[i][0]];
  const double* b = REF_V[FACE_V[i][1]];
  const double* c = REF_V[FACE_V[i][2]];
  for (int d = 0; d < 3; ++d) xi[d] = a[d] + s * (b[d] - a[d]) + t * (c[d] - a[d]);
}

int n_basis(int N) { return (N + 1) * (N + 2) * (N + 3) / 6; }
int n_face_nodes(int N) { return (N + 1) * (N + 2) / 2; }

void gauss_jacobi(int n, double alpha, double beta, std::vector<double>& x, std::vector<double>& w) {
  // Newton iteration with deflation from Chebyshev starting points.
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int k = 0; k < n; ++k) {
    double r = -std::cos((2.0 * k + 1.0) * M_PI / (2.0 * n));
    if (k > 0) r = 0.5 * (r + x[k - 1]);
    for (int it = 0; it < 200; ++it) {
      double dp;
      const double p = jacobi_p(n, alpha, beta, r, &dp);
      double sum = 0.0;
      for (int j = 0; j < k; ++j) sum += 1.0 / (r - x[j]);
      const double delta = -p / (dp - sum * p);
      r += delta;
      if (std::fabs(delta) < 1e-16) break;
    }
    x[k] = r;
  }
  std::sort(x.begin(), x.end());
  const double c = std::pow(2.0, alpha + beta + 1.0) * std::exp(std::lgamma(n + alpha + 1.0) +
                   std::lgamma(n + beta + 1.0) - std::lgamma(n + alpha + beta + 1.0) - std::lgamma(n + 1.0));
  for (int k = 0; k < n; ++k) {
    double dp;
    jacobi_p(n, alpha, beta, x[k], &dp);
    w[k] = c / ((1.0 - x[k] * x[k]) * dp * dp);
  }
}

void dubiner(int N, const double xi[3], double* val, double* grad) {
  Dual X(xi[0]), Y(xi[1]), Z(xi[2]);
  X.d[0] = 1.0; Y.d[1] = 1.0; Z.d[2] = 1.0;
  const Dual one(1.0);
  const Dual s = one - Y - Z, t = one - Z;
  const Dual c = 2.0 * Z - one;
  std::vector<Dual> Hp, Hq, Pr;
  hjacobi(N, 0.0, 0.0, 2.0 * X - s, s, Hp);
  const auto idx = ordering(N);
  for (size_t l = 0; l < idx.size(); ++l) {
    const int p = idx[l].p, q = idx[l].q, r = idx[l].r;
    hjacobi(q, 2.0 * p + 1.0, 0.0, 2.0 * Y - t, t, Hq);
    hjacobi(r, 2.0 * p + 2.0 * q + 2.0, 0.0, c, one, Pr);
    const double nrm = 1.0 / (2.0 * (2 * p + 1) * (p + q + 1) * (2 * p + 2 * q + 2 * r + 3));
    const Dual f = (1.0 / std::sqrt(nrm)) * (Hp[p] * Hq[q] * Pr[r]);
    val[l] = f.v;
    if (grad)
      for (int d = 0; d < 3; ++d) grad[l * 3 + d] = f.d[d];
  }
}

int vertex_map_index(const RefElement& r, const int sigma[3]) {
  for (int h = 0; h < 6; ++h)
    if (r.sigma[h][0] == sigma[0] && r.sigma[h][1] == sigma[1] && r.sigma[h][2] == sigma[2]) return h;
  return -1;
}

RefElement build_reference(int N) {
  if (N < 1 || N > 7) throw std::runtime_error("degree out of range");
  RefElement R;
  R.N = N;
  R.B = n_basis(N);
  R.Bf = n_face_nodes(N);
  const int B = R.B, Bf = R.Bf;

  // volume rule exact to degree 2N+1
  std::vector<double> ga, wa, gb, wb, gc, wc;
  const int nv = N + 1;
  gauss_jacobi(nv, 0.0, 0.0, ga, wa);
  gauss_jacobi(nv, 1.0, 0.0, gb, wb);
  gauss_jacobi(nv, 2.0, 0.0, gc, wc);
  R.K.assign(3 * B * B, 0.0);
  std::vector<double> val(B), grad(3 * B);
  for (int i = 0; i < nv; ++i)
    for (int j = 0; j < nv; ++j)
      for (int k = 0; k < nv; ++k) {
        const double a = ga[i], b = gb[j], c = gc[k];
        const double xi[3] = {(1 + a) * (1 - b) * (1 - c) / 8.0, (1 + b) * (1 - c) / 4.0, (1 + c) / 2.0};
        const double w = wa[i] * wb[j] * wc[k] / 64.0;
        dubiner(N, xi, val.data(), grad.data());
        for (int d = 0; d < 3; ++d)
          for (int kk = 0; kk < B; ++kk)
            for (int l = 0; l < B; ++l) R.K[(d * B + kk) * B + l] += w * grad[kk * 3 + d] * val[l];
      }

  // face lattice nodes and their Lagrange basis
  std::vector<std::array<int, 2>> nodes;
  for (int b = 0; b <= N; ++b)
    for (int a = 0; a + b <= N; ++a) nodes.push_back({a, b});
  std::vector<double> V(Bf * Bf);  // V[m][j] = psi_j(node m)
  std::vector<double> psi;
  for (int m = 0; m < Bf; ++m) {
    triangle_basis(N, double(nodes[m][0]) / N, double(nodes[m][1]) / N, psi);
    for (int j = 0; j < Bf; ++j) V[m * Bf + j] = psi[j];
  }
  // triangle rule exact to degree 2N+1 (also the eta points)
  std::vector<double> ta, twa, tb, twb;
  gauss_jacobi(N + 1, 0.0, 0.0, ta, twa);
  gauss_jacobi(N + 1, 1.0, 0.0, tb, twb);
  const int nq = (N + 1) * (N + 1);
  R.nq = nq;
  R.eta_st.resize(2 * nq);
  std::vector<double> tw(nq);
  for (int j = 0; j <= N; ++j)
    for (int i = 0; i <= N; ++i) {
      const int q = j * (N + 1) + i;
      R.eta_st[2 * q] = (1 + ta[i]) * (1 - tb[j]) / 4.0;
      R.eta_st[2 * q + 1] = (1 + tb[j]) / 2.0;
      tw[q] = twa[i] * twb[j] / 8.0;
    }
  // Lagrange basis at the rule points: ell(q)[m] solves V^T ell = psi(q)
  std::vector<double> rhs(Bf * nq);
  for (int q = 0; q < nq; ++q) {
    triangle_basis(N, R.eta_st[2 * q], R.eta_st[2 * q + 1], psi);
    for (int j = 0; j < Bf; ++j) rhs[j * nq + q] = psi[j];
  }
  std::vector<double> VT(Bf * Bf);
  for (int m = 0; m < Bf; ++m)
    for (int j = 0; j < Bf; ++j) VT[j * Bf + m] = V[m * Bf + j];
  lu_solve(Bf, VT, rhs, nq);  // rhs[m][q] = ell_m(point q)
  R.tw = tw;
  {
    // projection of a sampled face function onto P_N, evaluated at the nodes
    const int n1 = N + 10;
    std::vector<double> fa, fwa, fb, fwb;
    gauss_jacobi(n1, 0.0, 0.0, fa, fwa);
    gauss_jacobi(n1, 1.0, 0.0, fb, fwb);
    const int nqf = n1 * n1;
    R.nqf = nqf;
    R.fproj_st.resize(2 * nqf);
    std::vector<double> Psi(nqf * Bf), M(Bf * Bf, 0.0), rhs(Bf * nqf);
    for (int j = 0; j < n1; ++j)
      for (int i = 0; i < n1; ++i) {
        const int q = j * n1 + i;
        const double s = (1 + fa[i]) * (1 - fb[j]) / 4.0, t = (1 + fb[j]) / 2.0, w = fwa[i] * fwb[j] / 8.0;
        R.fproj_st[2 * q] = s;
        R.fproj_st[2 * q + 1] = t;
        triangle_basis(N, s, t, psi);
        for (int k = 0; k < Bf; ++k) {
          Psi[q * Bf + k] = psi[k];
          rhs[k * nqf + q] = w * psi[k];
        }
        for (int k = 0; k < Bf; ++k)
          for (int l = 0; l < Bf; ++l) M[k * Bf + l] += w * psi[k] * psi[l];
      }
    lu_solve(Bf, M, rhs, nqf);  // rhs = M^-1 Psi^T W
    R.fproj.assign(Bf * nqf, 0.0);
    for (int m = 0; m < Bf; ++m)
      for (int k = 0; k < Bf; ++k)
        for (int q = 0; q < nqf; ++q) R.fproj[m * nqf + q] += V[m * Bf + k] * rhs[k * nqf + q];
  }
  R.node_st.resize(2 * Bf);
  for (int m = 0; m < Bf; ++m) {
    R.node_st[2 * m] = double(nodes[m][0]) / N;
    R.node_st[2 * m + 1] = double(nodes[m][1]) / N;
  }

  R.E.assign(4 * Bf * B, 0.0);
  R.L.assign(4 * B * Bf, 0.0);
  R.Eg.assign(4 * nq * B, 0.0);
  R.Lg.assign(4 * B * nq, 0.0);
  for (int f = 0; f < 4; ++f) {
    for (int m = 0; m < Bf; ++m) {
      double xi[3];
      face_to_ref(f, double(nodes[m][0]) / N, double(nodes[m][1]) / N, xi);
      dubiner(N, xi, val.data(), nullptr);
      for (int l = 0; l < B; ++l) R.E[(f * Bf + m) * B + l] = val[l];
    }
    for (int q = 0; q < nq; ++q) {
      double xi[3];
      face_to_ref(f, R.eta_st[2 * q], R.eta_st[2 * q + 1], xi);
      dubiner(N, xi, val.data(), nullptr);
      for (int l = 0; l < B; ++l) {
        R.Eg[(f * nq + q) * B + l] = val[l];
        R.Lg[(f * B + l) * nq + q] = tw[q] * val[l];
        for (int m = 0; m < Bf; ++m) R.L[(f * B + l) * Bf + m] += tw[q] * val[l] * rhs[m * nq + q];
      }
    }
  }

  // vertex maps and node permutations
  int h = 0;
  int s3[3] = {0, 1, 2};
  do {
    R.sigma[h] = {s3[0], s3[1], s3[2]};
    ++h;
  } while (std::next_permutation(s3, s3 + 3));
  R.perm.assign(6 * Bf, -1);
  for (int hh = 0; hh < 6; ++hh)
    for (int m = 0; m < Bf; ++m) {
      const int beta[3] = {N - nodes[m][0] - nodes[m][1], nodes[m][0], nodes[m][1]};
      int bp[3];
      for (int a = 0; a < 3; ++a) bp[R.sigma[hh][a]] = beta[a];
      for (int m2 = 0; m2 < Bf; ++m2)
        if (nodes[m2][0] == bp[1] && nodes[m2][1] == bp[2]) R.perm[hh * Bf + m] = m2;
    }
  R.pinv.assign(6 * Bf, -1);
  for (int hh = 0; hh < 6; ++hh)
    for (int m = 0; m < Bf; ++m) R.pinv[hh * Bf + R.perm[hh * Bf + m]] = m;
  return R;
}

}  // namespace seis
