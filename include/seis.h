/*
 * seis.h -- C ABI of the MI355X element-update library for the ADER-DG
 * discretisation of the coupled elastic-acoustic system with a gravity sea
 * surface (Krenz et al., "3D Acoustic-Elastic Coupling with Gravity", SC'21).
 *
 * Problem (Sec. 3 and Sec. 4.1): q_t + A q_x + B q_y + C q_z = 0 for
 * q = (s_xx, s_yy, s_zz, s_xy, s_yz, s_xz, v_x, v_y, v_z) on conforming
 * tetrahedra with element-constant (rho, lambda, mu); mu = 0 elements are
 * the acoustic ocean (s = -p I). Faces use the exact Godunov flux of the
 * elastic-acoustic Riemann problem (Sec. 4.2); boundaries are imposed
 * through ghost states (Sec. 4.3); the sea surface z = 0 carries the
 * displacement eta through p' = rho g eta, d eta/dt = u_z (Sec. 3, gravity
 * boundary condition; Sec. 4.3, coupled ODE). Elements are stepped with the
 * ADER predictor-corrector (Sec. 4.1) and rate-2 clustered local time
 * stepping (Sec. 4.4).
 *
 * Conventions fixed by this ABI
 *   - Order O = N + 1 (convergence order); N is the polynomial degree, and
 *     each element carries B = (N+1)(N+2)(N+3)/6 modal coefficients per
 *     quantity (Sec. 4.1, basis dimension). Supported: 3 <= O <= 7.
 *   - Basis: orthonormal Dubiner basis on the reference tetrahedron
 *     {x,y,z >= 0, x+y+z <= 1} mapped by x = X0 + [X1-X0, X2-X0, X3-X0] xi from
 *     the element's vertices in the caller's order (either orientation).
 *     phi_pqr = P_p(a) ((1-b)/2)^p P_q^(2p+1,0)(b) ((1-c)/2)^(p+q) P_r^(2p+2q+2,0)(c),
 *     a = 2x/(1-y-z) - 1, b = 2y/(1-z) - 1, c = 2z - 1, normalised to unit L2
 *     norm on the reference element, ordered by (p+q+r, r, q, p).
 *   - DOFs at the boundary: FP64 [E][B][9], caller's element order.
 *   - Face i of an element is opposite its local vertex i, parametrised by
 *     its vertices in ascending local order.
 *   - eta: FP64 [F_g][(N+1)^2]. Gravity faces are ordered by (element,
 *     local face); the points are the collapsed Gauss rule on the face,
 *     s = (1+a_i)(1-b_j)/4, t = (1+b_j)/2 (a: Gauss-Legendre, b:
 *     Gauss-Jacobi(1,0), N+1 points each), point index j*(N+1)+i.
 *
 * Errors: every int-returning call returns SEIS_OK (0) or a negative code;
 * seis_last_error() gives the message. No call aborts or throws across the
 * ABI. A handle is not thread-safe: serialise calls on one handle.
 */
#ifndef SEIS_H
#define SEIS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SEIS_OK = 0,
  SEIS_EINVAL = -1,  /* bad argument, degenerate element, unmatched face, ... */
  SEIS_ENOMEM = -2,  /* host or device allocation failed */
  SEIS_EDEVICE = -3, /* HIP error (message kept) or no gfx950 device */
  SEIS_EORDER = -4,  /* call out of schedule order (see seis_predict/seis_correct) */
  SEIS_ERANGE = -5   /* cluster id or element id out of range */
};

/* Face kinds, face i opposite local vertex i. */
enum {
  SEIS_FACE_INTERIOR = 0,  /* matched by its three vertex ids */
  SEIS_FACE_PERIODIC = 1,  /* matched by centroid modulo period[] */
  SEIS_FACE_GRAVITY = 2,   /* sea surface z = 0 with gravity (Sec. 4.3); acoustic elements only */
  SEIS_FACE_ABSORBING = 3, /* zero ghost state */
  SEIS_FACE_WALL = 4,      /* rigid wall: ghost v+ = -v-, same stress */
  SEIS_FACE_FREE = 5,      /* traction-free surface (g = 0): ghost s+ = -s-, same velocity */
  SEIS_FACE_VELOCITY = 6,  /* prescribed velocity v_b = (0, 0, du/dt) of the uplift history set by
                              seis_set_uplift: ghost v+ = 2 v_b - v-, same stress */
  SEIS_FACE_FAULT = 7      /* dynamic-rupture fault (Sec. 3, friction boundary condition): an interior
                              face between two elastic elements, kind 7 on both sides, matched by its
                              vertex ids; see seis_set_fault. Its two elements share an LTS cluster. */
};

/* Precision of the element update's operands. SEIS_BF16_SPLIT: every operand
 * of a matrix-core product is split into two BF16 numbers, x = hi + lo with
 * hi = bf16(x) and lo = bf16(x - hi), and each product is formed from three
 * BF16 products (hi hi + hi lo + lo hi) with FP32 accumulation: about 16
 * significant bits per operand, near FP32 accuracy on the BF16 matrix cores. */
enum { SEIS_FP64 = 0, SEIS_FP32 = 1, SEIS_BF16 = 2, SEIS_BF16_SPLIT = 3 };
enum { SEIS_KERNEL_TUNED = 0, SEIS_KERNEL_PLAIN = 1 };

typedef struct seis_t seis_t; /* opaque; owns all device memory */

/* Mesh description. All arrays are host memory owned by the caller and are
 * copied during seis_setup. */
typedef struct {
  int64_t n_vertices;
  const double *xyz;       /* [n_vertices][3], metres */
  int64_t n_elements;
  const int64_t *tet;      /* [n_elements][4] vertex ids, any orientation */
  const int8_t *face_kind; /* [n_elements][4], SEIS_FACE_* */
  double period[3];        /* periodic box lengths, 0 = not periodic */
} seis_mesh_t;

/* Per-element material (Sec. 3): density, Lame parameters; mu == 0 is acoustic. */
typedef struct {
  const double *rho;
  const double *lambda;
  const double *mu;
} seis_materials_t;

typedef struct {
  int precision;    /* SEIS_FP64 / SEIS_FP32 / SEIS_BF16 / SEIS_BF16_SPLIT (operands; FP32 accumulation) */
  int kernel;       /* SEIS_KERNEL_TUNED (default) or SEIS_KERNEL_PLAIN; FP64 has no
                       matrix-core form and always runs the plain kernels */
  double cfl;       /* C in dt_K = C/(2N+1) h_K / c_p,K (Sec. 4.4); default 0.35 */
  double g;         /* gravitational acceleration (Sec. 3); default 9.81 */
  int max_clusters; /* rate-2 LTS clusters (Sec. 4.4); 1 = global time stepping */
  void *stream;     /* hipStream_t to launch on; NULL = the default stream */
  int tile;         /* elements per work-group for the tuned kernels (32: 2 wavefronts, 64: 4);
                       0 = autotuned: at set-up the launch configurations and the predictor's
                       shape (FP32: I~ parked in LDS or in HBM; BF16: 16x16x16 or 16x16x32
                       matrix-core products) are timed on the largest cluster and the fastest
                       kept, cached per (kernel sources, device, order, precision, size class)
                       in the file $SEIS_TUNE_CACHE (default $HOME/.cache/seis/tune.txt).
                       SEIS_TUNE=0 in the environment disables tuning;
                       SEIS_TUNE=w,cap,remap,w,cap,remap[,split[,shape]] fixes it. */
  int graph;        /* nonzero: seis_step captures its macro step into a hipGraph at its first
                       call and replays that graph afterwards (one launch per macro step) */
  int mc_min;       /* tuned kernels, FP32/BF16: a cluster with fewer elements than this runs on
                       the plain FP32 kernels instead of the matrix cores (a matrix-core
                       wavefront works through its 16 elements in sequence, so a tiny cluster is
                       bound by that latency there). Default 2048; 0 puts every cluster on the
                       matrix cores. Must be >= 0. */
  int fused;        /* nonzero (default): seis_step launches each phase of a sub-step once over every
                       cluster due in it (the due clusters 0..k are one element range, Sec. 4.4), the
                       predictor over the range on the matrix cores when it has at least mc_min
                       elements, else on the plain FP32 kernels; 0: one launch per cluster, each
                       cluster's kernel chosen by its own size. seis_predict/seis_correct always work
                       per cluster. */
  int acoustic;     /* tuned kernels, FP32/BF16: nonzero (default) runs each 16-element group whose
                       elements are all acoustic (mu = 0) in the 4-quantity form (Sec. 4.1: the stress
                       is -p I there): s_xx = -p and the velocity are integrated, s_yy and s_zz are
                       stored equal to s_xx and the shear components as zero, and the face fluxes of
                       such an element read the neighbour's full nine-quantity trace (elastic at the
                       seafloor). The state of an acoustic element is then taken to be isotropic:
                       s_yy, s_zz and the shear components written by seis_write are not read there.
                       Set-up orders the acoustic elements of a cluster together. 0: the
                       nine-quantity embedding everywhere. */
} seis_options_t;

typedef struct {
  int order;            /* O = N + 1 */
  int n_basis;          /* B */
  int n_face_nodes;     /* (N+1)(N+2)/2 */
  int n_eta_points;     /* (N+1)^2 */
  int precision;
  int kernel;
  int n_clusters;
  int64_t n_elements;
  int64_t n_gravity_faces;
  double dt_min;        /* smallest element time step; cluster c steps 2^c dt_min */
  double time;          /* simulated time of the last completed macro step */
  int64_t cluster_size[16];
  int64_t updates_per_macro_step; /* sum_c n_c 2^(C-1-c) */
  int64_t device_bytes;
  int launch[8];        /* matrix-core launch configuration of the predictor, then the corrector:
                           wavefronts per work-group, work-groups per CU of a persistent grid
                           (0 = one work-group per 16 x wavefronts elements), XCD-contiguous order;
                           [6] the corrector's passes over its output rows; [7] options.mc_min */
  int launch_source;    /* 0 default or fixed (options.tile, SEIS_TUNE), 1 measured at set-up,
                           2 read from the tuning cache */
  int fused;            /* options.fused */
  int shape;            /* the predictor's shape: FP32 0 = I~ parked in LDS as far as it fits,
                           1 = in HBM; BF16 0 = 16x16x16 products, 1 = 16x16x32 products */
  int64_t n_acoustic_groups; /* 16-element groups run in the 4-quantity form (options.acoustic) */
  int64_t n_fault_faces; /* SEIS_FACE_FAULT faces, each counted once (seis_set_fault) */
} seis_info_t;

/* Default options: FP64, tuned kernels, cfl 0.35, g 9.81, GTS, default stream,
 * eager launches (no graph), mc_min 2048, fused sub-step launches, 4-quantity
 * acoustic groups. */
void seis_default_options(seis_options_t *opt);

/* Build the solver for a mesh (Sec. 4.1-4.4): validate, match faces,
 * assemble geometry, element Jacobians and the per-face Godunov flux
 * matrices F-, F+ (Sec. 4.2, bilinear rewrite of the numerical flux) in FP64,
 * assign LTS clusters, allocate device state (all zero: Q = 0, eta = 0).
 * order: O = N + 1 in [2, 8] with the plain kernels, [3, 7] with the
 * matrix-core kernels ([3, 6] with split BF16 operands); fault faces need
 * O <= 7. opt may be NULL (defaults). On success *out owns the handle; free
 * it with seis_destroy.
 * Errors: SEIS_EINVAL (degenerate element, unmatched interior or periodic
 * face, gravity face not acoustic or not horizontal with outward normal +z,
 * more than one gravity face per element, order outside the kernels' range),
 * SEIS_ENOMEM, SEIS_EDEVICE. */
int seis_setup(const seis_mesh_t *mesh, const seis_materials_t *mat, int order,
               const seis_options_t *opt, seis_t **out);

/* Copy state from host FP64: dofs [E][B][9] (caller order) and/or eta
 * [F_g][(N+1)^2]; either may be NULL to keep the current value. Resets the
 * schedule to the start of a macro step and the simulated time to 0. */
int seis_write(seis_t *h, const double *dofs, const double *eta);

/* Uplift history driving the SEIS_FACE_VELOCITY faces (a seafloor uplift,
 * the input of a one-way linked tsunami model, Sec. 2; here prescribed at the
 * bottom of the solid): n <= 16 sources src [n][5] = (A [m], x_c, y_c [m],
 * w [m] > 0, T [s] > 0),
 *   u(x, y, t) = sum_j A_j exp(-((x - x_j)^2 + (y - y_j)^2) / (2 w_j^2)) S(t / T_j),
 *   S(s) = 0 for s <= 0, s - sin(2 pi s)/(2 pi) for 0 < s < 1, 1 for s >= 1,
 * with t the simulated time since the last seis_write. The faces impose the
 * velocity (0, 0, du/dt) weakly through the ghost state; over an element's
 * step the ghost contributes the exact time integral 2 (u(t1) - u(t0)).
 * Synchronises the stream; n = 0 removes the forcing. Errors: SEIS_EINVAL. */
int seis_set_uplift(seis_t *h, int n, const double *src);

enum {
  SEIS_FRICTION_SLIP_WEAKENING = 0, /* linear slip weakening (the benchmark's law, Sec. 6.2) */
  SEIS_FRICTION_RATE_STATE = 1      /* rate and state, fast velocity weakening (the Palu run's law) */
};

/* Friction of the SEIS_FACE_FAULT faces (Sec. 3, fault boundary condition:
 * |tau| <= tau_S, slip parallel to tau where |tau| = tau_S). A fault face is
 * listed once, from its '-' side, the element with the smaller id; n points
 * from '-' to '+'; faces are ordered by ('-' element, local face); n must
 * equal seis_info's n_fault_faces. params, host memory, per face first
 *   s0       background normal stress (Pa, negative in compression),
 *   tau0[3]  background traction (Pa; its normal part is ignored),
 * then, for law SEIS_FRICTION_SLIP_WEAKENING ([n][8]):
 *   mu_s, mu_d, D_c  f = mu_s - (mu_s - mu_d) min(psi / D_c, 1), psi the slip
 *            path (m), D_c > 0,
 *   C        cohesion (Pa, >= 0; INFINITY keeps the face locked);
 *   strength tau_S = C + f max(0, -(s0 + s)) with s the normal stress of the
 *   elements' state; the fault slips where |tau0 + tau| would exceed it;
 * or, for law SEIS_FRICTION_RATE_STATE ([n][12]):
 *   a, b, L, V0, f0, f_w, V_w, psi0 of f(V, psi) = a asinh(V / (2 V0) e^(psi / a)),
 *   dpsi/dt = -(V / L)(psi - psi_ss(V)), psi_ss(V) = a ln(2 V0 / V sinh(f_ss(V) / a)),
 *   f_ss(V) = f_w + (f0 - (b - a) ln(V / V0) - f_w) / (1 + (V / V_w)^8)^(1/8);
 *   psi0 the initial state; the fault always slides, with
 *   |tau0 + tau| = f(|V|, psi) max(0, -(s0 + s)) + eta |V|.
 * The law is applied at the fault's points at the Gauss-Legendre points of
 * each step (the state advanced after each). Until this is called every
 * fault face is locked (a welded interface). Puts the fault at rest (no
 * slip, psi = 0 or psi0). Errors: SEIS_EINVAL (n, law, a parameter out of
 * range). */
int seis_set_fault(seis_t *h, int64_t n, int law, const double *params);

/* Fault state at the fault's points: out [n_fault_faces][(N+1)(N+2)/2][14]
 * (host, caller-owned), per point: x, y, z, slip (3, m, v+ - v- integrated
 * over time), psi (the slip path, m, or the rate-and-state state), slip rate
 * V (3, m/s, at the last time point of the last step), total shear traction
 * tau0 + tau (3, Pa), total normal stress s0 + s (Pa). Points are the face's
 * equispaced lattice nodes; match them by their coordinates. seis_write and
 * seis_set_fault put the fault at rest. Synchronises the stream. */
int seis_fault_read(seis_t *h, double *out);

/* ADER predictor of every element of cluster c for its next step (Sec. 4.1,
 * Taylor expansion; Cauchy-Kowalevski procedure), its time integral, the
 * element-local part of the corrector (volume term and local flux term of the
 * semi-discrete form, Sec. 4.1 and 4.2) and the gravity surface faces of the
 * cluster (per-point eta ODE and time-integrated boundary state, Sec. 4.3).
 * It also hands each face neighbour the time-integrated trace it needs.
 * Errors: SEIS_ERANGE (bad c), SEIS_EORDER (cluster c already predicted and
 * not yet corrected). */
int seis_predict(seis_t *h, int c);

/* Neighbour flux term of the corrector for cluster c (Sec. 4.2, F+ q+ part),
 * completing the step of cluster c; advances its time by 2^c dt_min.
 * Errors: SEIS_ERANGE, SEIS_EORDER (c not predicted, or a neighbour cluster
 * has not yet predicted the interval c needs). */
int seis_correct(seis_t *h, int c);

/* One LTS macro step (2^(C-1) sub-steps of dt_min): in sub-step s the
 * predictors of the clusters with s mod 2^c == 0, then the correctors of the
 * clusters with (s+1) mod 2^c == 0 (Sec. 4.4). Launches asynchronously on the
 * handle's stream. With options.graph set, the first call captures these
 * launches into a hipGraph (on a private stream) and every later call
 * launches that graph on the handle's stream. Kernel timings cannot be read
 * from inside a graph: while profiling is on (seis_profile) the step is
 * launched eagerly. */
int seis_step(seis_t *h);

/* Run n macro steps (same as calling seis_step n times). */
int seis_run(seis_t *h, int n);

/* Copy state to host FP64 (synchronises the stream first): dofs [E][B][9]
 * in caller element order and/or eta [F_g][(N+1)^2]; either may be NULL.
 * Errors: SEIS_EORDER if a cluster is between predict and correct. */
int seis_read(seis_t *h, double *dofs, double *eta);

/* Read only the DOFs of n elements (caller ids) into dofs [n][B][9]. */
int seis_read_elements(seis_t *h, const int64_t *ids, int64_t n, double *dofs);

/* Summary of the handle (sizes, clusters, time step). */
int seis_info(const seis_t *h, seis_info_t *info);

/* Cluster of every element, caller order: out [E]. */
int seis_cluster_of(const seis_t *h, int32_t *out);

/* Per-kernel timing for measurement: with enable != 0 every kernel launch of
 * the handle is bracketed by HIP events on the handle's stream and the
 * totals are cleared; enable == 0 stops recording. */
int seis_profile(seis_t *h, int enable);

/* Totals since profiling was enabled, for the kernel kinds
 * [0] predictor, [1] gravity face, [2] corrector, [3] fault face (arrays of
 * 4): elapsed ms, number of launches and number of elements (gravity and
 * fault: faces) processed. Any pointer may be NULL. Synchronises the stream. */
int seis_profile_read(seis_t *h, double *ms, int64_t *launches, int64_t *elements);

/* Output at points (Sec. 6.2 writes receivers every 0.01 s, and the sea
 * surface and the elastic-acoustic interface every 0.1 s of simulated time).
 * A point set is fixed once; seis_sample then evaluates the current state at
 * its points on the device, so that a time series is one sample after each
 * macro step of the right length (all clusters are at the same time only
 * between macro steps). Two sets are built in:
 *   SEIS_POINTS_SEA_SURFACE: the eta points of every gravity face, in the
 *     order of the eta array (faces by (element, local face), points by the
 *     face rule documented above), evaluated in the acoustic element;
 *   SEIS_POINTS_SEAFLOOR: the same face rule on every elastic-acoustic face,
 *     evaluated in its elastic element; faces ordered by (caller element of
 *     the elastic side, local face). */
enum { SEIS_POINTS_SEA_SURFACE = -1, SEIS_POINTS_SEAFLOOR = -2 };

/* Define a set of n receivers at physical points xyz [n][3] (host, FP64,
 * copied). Each point is evaluated in the element that contains it (within
 * 1e-9 in barycentric coordinates); of several (a point on a shared face,
 * edge or vertex) the one with the lowest caller id. *id receives the set's
 * id (0, 1, ... in order of definition). Allocates device memory for the
 * set's basis values (n x B doubles), freed by seis_destroy.
 * Errors: SEIS_EINVAL (NULL argument, n <= 0, a point outside the mesh). */
int seis_points(seis_t *h, int64_t n, const double *xyz, int *id);

/* Size of a point set and (each nullable, host) its points [n][3] and the
 * caller id of the element each point is evaluated in [n]. For a built-in
 * set the first call builds it (host work and a device allocation).
 * Errors: SEIS_ERANGE (no such set). */
int seis_points_info(seis_t *h, int id, int64_t *n, double *xyz, int64_t *element);

/* The nine quantities (order above) at the points of set id from the
 * current state, out: DEVICE pointer [n][9] FP64, asynchronous on the
 * handle's stream. eta (DEVICE [n], nullable) receives the sea-surface
 * height at the points; only for SEIS_POINTS_SEA_SURFACE. Launches one
 * kernel and allocates nothing once the set exists (a built-in set is built
 * at its first use: call seis_points_info first when capturing a graph).
 * Errors: SEIS_EINVAL, SEIS_ERANGE, SEIS_EORDER (between a prediction and its
 * correction), SEIS_EDEVICE. */
int seis_sample(seis_t *h, int id, double *out, double *eta);

/* Energy and field norms of the current state (Sec. 3: the velocity-stress
 * system with the gravitational sea surface, whose energy
 *   E = sum_K int_K (rho |v|^2 / 2 + W(s)) + int_surface rho g eta^2 / 2
 * the continuous model conserves and the upwind scheme does not increase;
 * W = (s:s - lambda/(3 lambda + 2 mu) (tr s)^2) / (4 mu) in an elastic element,
 * p^2 / (2 lambda) with p = -tr s / 3 in an acoustic one).
 * out: DEVICE pointer to 12 doubles, written asynchronously on the handle's
 * stream (synchronise before reading it):
 *   out[0] = E, out[1] = the volume part, out[2] = the surface part,
 *   out[3 + p] = int |q_p|^2 over the mesh, p = 0..8 (quantity order above).
 * Computed in FP64 from the stored state (FP64, or FP32 widened). The sums
 * go through a partial-sum buffer (12 doubles per work-group, at most 1024
 * work-groups) that this call allocates on the device at its first use on
 * the handle and keeps until seis_destroy. Errors: SEIS_EINVAL (NULL
 * argument), SEIS_EORDER (between a prediction and its correction),
 * SEIS_EDEVICE. */
int seis_energy(seis_t *h, double *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as seis_energy, bit for bit, but the partial sums live in a fixed
 * device array of the library (1024 x 12 doubles = 96 KiB on each GPU the
 * library runs on, held until the process ends), so the call allocates
 * nothing. Every call on one GPU shares that array: calls that overlap on one
 * GPU (two streams, or two handles on different streams) race on it and must
 * be serialised by the caller. The array is fully rewritten by each call, so
 * nothing has to be cleared between calls. Errors: as seis_energy, and
 * SEIS_EDEVICE when no handle was set up with the current device,
 * SEIS_ERANGE if the partial sums would exceed the array (cannot happen with
 * at most 1024 work-groups, checked anyway). */
int seis_energy_noalloc(seis_t *h, double *out);

/* Synchronise the handle's stream. */
int seis_sync(seis_t *h);

/* Free all memory of the handle (NULL is ignored). */
void seis_destroy(seis_t *h);

/* Message of the last error on this handle (or of the last failed
 * seis_setup when h is NULL). Never NULL. */
const char *seis_last_error(const seis_t *h);

#ifdef __cplusplus
}
#endif

#endif /* SEIS_H */
