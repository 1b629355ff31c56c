// Host-side model of a mesh after set-up (FP64), in the library's element
// order: elements are grouped by LTS cluster (cluster c occupies
// [cluster_start[c], cluster_start[c+1])), keeping the caller's relative
// order inside a cluster.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "refelem.hpp"

namespace seis {

// Face exchange modes of the writer side (see the predictor kernels).
enum FaceMode : int8_t {
  MODE_NONE = 0,     // physical boundary: nothing is handed over
  MODE_SAME = 1,     // neighbour in the same cluster: full-step integral
  MODE_FINER = 2,    // neighbour one cluster finer: first and second half-step integrals
  MODE_COARSER = 3,  // neighbour one cluster coarser: half of the integral, accumulated over two steps
};

struct Model {
  int N = 0, B = 0, Bf = 0, nq = 0;
  int64_t E = 0;
  int C = 1;                           // number of clusters
  double dt_min = 0.0;
  std::vector<double> dt_c;            // [C]
  std::vector<int64_t> cluster_start;  // [C+1]
  std::vector<int64_t> new_of_old;     // [E]
  std::vector<int64_t> old_of_new;     // [E]
  std::vector<int32_t> cluster_old;    // [E], caller order

  // per element inputs of the operator assembly (library order, FP64; see assemble.hpp)
  std::vector<double> a_Jinv;          // [E][9]
  std::vector<double> a_absdet;        // [E]
  std::vector<double> a_dt;            // [E]
  std::vector<double> a_lmr;           // [E][3] lambda, mu, rho
  std::vector<double> a_nrm;           // [E][4][3]
  std::vector<double> a_area;          // [E][4]
  std::vector<int8_t> a_kind;          // [E][4]
  std::vector<int64_t> a_nbk;          // [E][4] neighbour (library order), -1 none
  std::vector<int32_t> tgt;            // [E][4] writer: K*4 + i of the receiving face, -1 none
  std::vector<int8_t> mode;            // [E][4] writer FaceMode
  std::vector<int8_t> hperm;           // [E][4] writer node map index (0..5)
  std::vector<int32_t> half2;          // [E][4] writer MODE_FINER: slot of the second half
  std::vector<int32_t> rhalf2;         // [E][4] reader: slot read on odd sub-steps, -1 none
  int64_t n_half2 = 0;

  // gravity faces (library element order of their elements, sorted by caller (element, face))
  std::vector<int64_t> g_elem;         // [F_g] library element id
  std::vector<int8_t> g_face;          // [F_g]
  std::vector<double> g_par;           // [F_g][8]: scale 2A/|J|, n_x, n_y, n_z, Z, a = rho g / Z, lambda, dt
  std::vector<double> g_coef;          // [F_g] rho g A of the face (surface energy weight)
  std::vector<int32_t> gslot;          // [E] gravity face index of an element, -1 none
  std::vector<int64_t> g_order;        // [F_g]: ABI position of library gravity face f
  // stored time derivatives: gravity elements use their gravity face index,
  // elements handing over to a finer neighbour (and without a gravity face)
  // the slots after those
  std::vector<int32_t> dslot;          // [E] derivative slot, -1 none
  int64_t n_dslot = 0;
  // per cluster c, entries [start[c], start[c+1]) of element * 4 + face:
  std::vector<int32_t> fix_list;       // faces handing over to a finer neighbour (MODE_FINER)
  std::vector<int64_t> fix_start;      // [C+1]
  std::vector<int32_t> h2_list;        // faces that read a second-half slot on odd sub-steps
  std::vector<int64_t> h2_start;       // [C+1]
  double g = 9.81;

  // prescribed-velocity faces (uplift forcing), library element order,
  // grouped by cluster ([vface_start[c], vface_start[c+1]))
  std::vector<int64_t> v_elem;
  std::vector<int8_t> v_face;
  std::vector<double> v_dt;            // [F_v] the element's time step
  std::vector<double> v_xy;            // [F_v][nqf][2] x, y of the face's projection rule points
  std::vector<int64_t> vface_start;    // [C+1]

  // the mesh as given (caller order), kept for locating output points
  std::vector<double> xyz;             // [nv][3]
  std::vector<int64_t> tet;            // [E][4]
  // elastic-acoustic interface faces seen from the elastic side, ordered by
  // (caller element, local face); element ids in library order
  std::vector<int64_t> floor_elem;
  std::vector<int8_t> floor_face;

  // dynamic-rupture fault faces (kind 7), seen from their '-' side (the
  // element with the smaller caller id), grouped by cluster
  // ([fault_start[c], fault_start[c+1])); element ids in library order
  std::vector<int64_t> f_elem, f_pelem;  // '-' and '+' elements
  std::vector<int8_t> f_face, f_pface;   // their local faces
  std::vector<int8_t> f_perm;            // node map: '-' node m is '+' node perm[f_perm][m]
  std::vector<double> f_geo;             // [F][8]: n (from - to +), Zp-, Zs-, Zp+, Zs+, dt
  std::vector<double> f_xyz;             // [F][Bf][3] face nodes ('-' numbering)
  std::vector<int64_t> fault_start;      // [C+1]
  std::vector<int64_t> fault_abi;        // [F]: library position of the ABI's fault face k

  RefElement ref;
};

// Build the model. Returns an empty string on success, else an error message.
std::string build_model(int64_t nv, const double* xyz, int64_t E, const int64_t* tet, const int8_t* face_kind,
                        const double period[3], const double* rho, const double* lam, const double* mu, int N,
                        double cfl, double g, int max_clusters, Model& M);

}  // namespace seis
