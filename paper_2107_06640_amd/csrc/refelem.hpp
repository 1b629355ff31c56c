// Reference-element data of the library (host, FP64).
//
// The DG method maps every element to the reference tetrahedron and uses
// precomputed reference integrals instead of per-element quadrature
// (Sec. 4.1). This file builds those integrals for the orthonormal Dubiner
// basis (the basis is fixed by the ABI in include/seis.h):
//
//   K[d][k][l]   = int_ref d(phi_k)/d(xi_d) phi_l            stiffness, B x B
//   E[i][m][l]   = phi_l(node m of face i)                    trace at face nodes, Bf x B
//   L[i][k][m]   = int_tri phi_k(face i) ell_m               lift, B x Bf
//   Eg[i][q][l]  = phi_l(eta point q of face i)              gravity face, nq x B
//   Lg[i][k][q]  = w_q phi_k(eta point q of face i)          gravity lift, B x nq
//
// Face nodes are the equispaced lattice (a/N, b/N), a + b <= N, of the face
// parameter triangle; ell_m is the Lagrange basis of P_N on it. The lattice is
// invariant under permutations of the triangle's vertices, so the two sides of
// a face see the same physical nodes and only their numbering differs
// (perm[h][m], one table per vertex permutation h).
#pragma once

#include <array>
#include <vector>

namespace seis {

struct RefElement {
  int N = 0, B = 0, Bf = 0, nq = 0;
  std::vector<double> K;   // [3][B][B]
  std::vector<double> E;   // [4][Bf][B]
  std::vector<double> L;   // [4][B][Bf]
  std::vector<double> Eg;  // [4][nq][B]
  std::vector<double> Lg;  // [4][B][nq]
  std::vector<double> eta_st;  // [nq][2] face parameters of the eta points
  std::vector<double> tw;      // [nq] weights of the face rule at the eta points (sum 1/2)
  std::vector<double> node_st; // [Bf][2] face parameters of the face nodes
  // L2 projection onto P_N of a face of a function sampled at a high-order
  // face rule (N + 10 Gauss points per collapsed direction), as nodal values:
  // nodal[m] = sum_q fproj[m][q] f(point q)
  int nqf = 0;
  std::vector<double> fproj_st; // [nqf][2] face parameters of the rule's points
  std::vector<double> fproj;    // [Bf][nqf]
  std::vector<int> perm;   // [6][Bf]: neighbour node index for node m under vertex map h
  std::vector<int> pinv;   // [6][Bf]: inverse of perm[h]
  std::array<std::array<int, 3>, 6> sigma{};  // the 6 vertex maps: my face vertex a -> neighbour's sigma[a]
};

int n_basis(int N);
int n_face_nodes(int N);

// Build all reference matrices for degree N (1 <= N <= 7).
RefElement build_reference(int N);

// Gauss-Jacobi nodes and weights on [-1, 1] for weight (1-x)^alpha (1+x)^beta.
void gauss_jacobi(int n, double alpha, double beta, std::vector<double>& x, std::vector<double>& w);

// Orthonormal Dubiner basis values (and reference gradients if grad != nullptr,
// layout [B][3]) at a point of the closed reference tetrahedron.
void dubiner(int N, const double xi[3], double* val, double* grad);

// Reference coordinates of the point (s, t) of face i (opposite vertex i,
// parametrised by its other vertices in ascending order).
void face_to_ref(int i, double s, double t, double xi[3]);

// Index of the vertex map sigma (as in RefElement::sigma), or -1.
int vertex_map_index(const RefElement& r, const int sigma[3]);

}  // namespace seis
