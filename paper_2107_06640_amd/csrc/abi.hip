// C ABI of the library (see include/seis.h): handle, device buffers,
// schedule bookkeeping and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/seis.h"
#include "assemble.hpp"
#include "device.hpp"
#include "energy.hpp"
#include "fault.hpp"
#include "forcing.hpp"
#include "layout.hpp"
#include "model.hpp"
#include "probe.hpp"
#include "tuned.hpp"

using namespace seis;

namespace {

std::mutex g_err_mu;
std::string g_setup_error = "no error";

struct Buffers {
  std::vector<void*> ptrs;
  int64_t bytes = 0;
  template <typename X>
  hipError_t alloc(X** p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    void* q = nullptr;
    hipError_t st = hipMalloc(&q, n * sizeof(X));
    if (st != hipSuccess) return st;
    ptrs.push_back(q);
    bytes += int64_t(n * sizeof(X));
    *p = static_cast<X*>(q);
    return hipSuccess;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

}  // namespace

struct seis_t {
  Model M;
  int precision = SEIS_FP64;
  int kernel = SEIS_KERNEL_TUNED;
  int tile = 0;
  hipStream_t stream = nullptr;
  Buffers buf;
  DevData<double> d64{};
  DevData<float> d32{};
  TunedData tuned{};
  int32_t* glist = nullptr;             // gravity faces grouped by cluster
  std::vector<int64_t> gstart;          // [C+1]
  std::string err = "no error";
  // schedule cursor inside the current macro step
  int sub = 0;                          // sub-step index
  std::vector<int> predicted;           // per cluster, predicted in this sub-step
  std::vector<int> corrected;
  int64_t macro_done = 0;
  // per-kernel event timing
  bool prof = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec { int kind; hipEvent_t a, b; int64_t n; };
  std::vector<Rec> recs;
  double tot_ms[4] = {0, 0, 0, 0};
  int64_t tot_launch[4] = {0, 0, 0, 0}, tot_elem[4] = {0, 0, 0, 0};
  // energy and field norms: FP64 weights, and the partial sums of seis_energy
  // (allocated at its first call)
  EnergyData en{};
  double* en_partial = nullptr;
  // prescribed-velocity faces: forcing data, the source buffer and the
  // device count of completed macro steps (the forcing's clock)
  ForcingArgs forcing{};
  // dynamic-rupture faces: friction data, parameters and state on the device
  FaultArgs fault{};
  double* fault_par = nullptr;
  double* fault_state = nullptr;
  std::vector<double> fault_par_host;  // [F][kFaultParams], library order
  double* uplift_src = nullptr;
  int64_t* macro_dev = nullptr;
  // output point sets: seis_points (ids 0, 1, ...), and the sea surface and
  // the seafloor (built at their first use)
  std::vector<PointSet> psets;
  PointSet sea_set, floor_set;
  bool sea_built = false, floor_built = false;
  // seis_step launches one kernel per phase per sub-step over every due
  // cluster (options.fused), else one per cluster
  bool fused = true;
  // hipGraph of one macro step (options.graph)
  bool use_graph = false;
  hipStream_t cap = nullptr;            // private capture stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
};

namespace {

int fail(seis_t* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

int hip_fail(seis_t* h, hipError_t st, const char* where) {
  return fail(h, SEIS_EDEVICE, std::string(where) + ": " + hipGetErrorString(st));
}

#define HIPCHK(h, call, where)                      \
  do {                                              \
    hipError_t _st = (call);                        \
    if (_st != hipSuccess) return hip_fail(h, _st, where); \
  } while (0)

template <typename X, typename Y>
hipError_t upload(Buffers& b, X** dst, const std::vector<Y>& src) {
  hipError_t st = b.alloc(dst, src.size());
  if (st != hipSuccess) return st;
  if (src.empty()) return hipSuccess;
  std::vector<X> tmp(src.begin(), src.end());
  return hipMemcpy(*dst, tmp.data(), tmp.size() * sizeof(X), hipMemcpyHostToDevice);
}

bool due_predict(int s, int c) { return (s % (1 << c)) == 0; }
bool due_correct(int s, int c) { return ((s + 1) % (1 << c)) == 0; }

template <typename T>
int build_dev(seis_t* h, DevData<T>& d) {
  Model& M = h->M;
  Buffers& b = h->buf;
  const int64_t E = M.E;
  const int B = M.B, Bf = M.Bf, N = M.N;
  d.E = E;
  d.g = M.g;
  T *Q, *G, *mat, *Fm, *Fp, *In, *H2, *gD, *K, *Ef, *Lf;
  const int RT = row_tiles(B), FT = row_tiles(Bf);
  HIPCHK(h, b.alloc(&Q, q_size(E, RT)), "alloc Q");
  HIPCHK(h, hipMemset(Q, 0, q_size(E, RT) * sizeof(T)), "memset Q");
  // operators: filled on the device by the assembly kernel
  HIPCHK(h, b.alloc(&G, E * 9), "alloc G");
  HIPCHK(h, b.alloc(&mat, E * 3), "alloc mat");
  HIPCHK(h, b.alloc(&Fm, E * 4 * 81), "alloc Fm");
  HIPCHK(h, b.alloc(&Fp, E * 4 * 81), "alloc Fp");
  HIPCHK(h, b.alloc(&In, in_size(E, FT)), "alloc In");
  HIPCHK(h, hipMemset(In, 0, in_size(E, FT) * sizeof(T)), "memset In");
  HIPCHK(h, b.alloc(&H2, std::max<int64_t>(M.n_half2, 1) * Bf * 9), "alloc H2");
  HIPCHK(h, hipMemset(H2, 0, std::max<int64_t>(M.n_half2, 1) * Bf * 9 * sizeof(T)), "memset H2");
  const int64_t Fg = (int64_t)M.g_elem.size();
  HIPCHK(h, b.alloc(&gD, std::max<int64_t>(std::max<int64_t>(Fg, M.n_dslot), 1) * (N + 1) * B * 9), "alloc gD");
  HIPCHK(h, upload(b, &K, M.ref.K), "upload K");
  HIPCHK(h, upload(b, &Ef, M.ref.E), "upload E");
  HIPCHK(h, upload(b, &Lf, M.ref.L), "upload L");
  d.Q = Q; d.G = G; d.mat = mat; d.Fm = Fm; d.Fp = Fp; d.In = In; d.H2 = H2; d.gD = gD;
  d.K = K; d.Ef = Ef; d.Lf = Lf;
  return SEIS_OK;
}

template <typename T>
void share_common(const DevData<double>& c, DevData<T>& d) {
  d.tgt = c.tgt; d.mode = c.mode; d.hperm = c.hperm; d.half2 = c.half2; d.rhalf2 = c.rhalf2;
  d.gslot = c.gslot; d.dslot = c.dslot; d.perm = c.perm; d.Eg = c.Eg; d.Lg = c.Lg; d.g_elem = c.g_elem; d.g_face = c.g_face;
  d.g_par = c.g_par; d.eta = c.eta;
}

int build_common(seis_t* h, DevData<double>& c) {
  Model& M = h->M;
  Buffers& b = h->buf;
  int32_t *tgt, *half2, *rhalf2, *gslot, *dslot, *perm, *gelem;
  int8_t *mode, *hperm, *gface;
  double *Eg, *Lg, *gpar, *eta;
  HIPCHK(h, upload(b, &tgt, M.tgt), "upload tgt");
  HIPCHK(h, upload(b, &mode, M.mode), "upload mode");
  HIPCHK(h, upload(b, &hperm, M.hperm), "upload hperm");
  HIPCHK(h, upload(b, &half2, M.half2), "upload half2");
  HIPCHK(h, upload(b, &rhalf2, M.rhalf2), "upload rhalf2");
  HIPCHK(h, upload(b, &gslot, M.gslot), "upload gslot");
  HIPCHK(h, upload(b, &dslot, M.dslot), "upload dslot");
  HIPCHK(h, upload(b, &perm, M.ref.perm), "upload perm");
  HIPCHK(h, upload(b, &Eg, M.ref.Eg), "upload Eg");
  HIPCHK(h, upload(b, &Lg, M.ref.Lg), "upload Lg");
  std::vector<int32_t> ge(M.g_elem.begin(), M.g_elem.end());
  HIPCHK(h, upload(b, &gelem, ge), "upload g_elem");
  HIPCHK(h, upload(b, &gface, M.g_face), "upload g_face");
  HIPCHK(h, upload(b, &gpar, M.g_par), "upload g_par");
  const int64_t Fg = (int64_t)M.g_elem.size();
  HIPCHK(h, b.alloc(&eta, std::max<int64_t>(Fg, 1) * M.nq), "alloc eta");
  HIPCHK(h, hipMemset(eta, 0, std::max<int64_t>(Fg, 1) * M.nq * sizeof(double)), "memset eta");
  // gravity faces grouped by cluster
  std::vector<int32_t> gl;
  h->gstart.assign(M.C + 1, 0);
  for (int cc = 0; cc < M.C; ++cc) {
    h->gstart[cc] = (int64_t)gl.size();
    for (int64_t f = 0; f < Fg; ++f) {
      const int64_t e = M.g_elem[f];
      if (e >= M.cluster_start[cc] && e < M.cluster_start[cc + 1]) gl.push_back(int32_t(f));
    }
  }
  h->gstart[M.C] = (int64_t)gl.size();
  HIPCHK(h, upload(b, &h->glist, gl), "upload glist");
  {
    int64_t* ve;
    int8_t* vf;
    double *vdt, *vxy, *vpr;
    HIPCHK(h, upload(b, &ve, M.v_elem), "upload velocity faces");
    HIPCHK(h, upload(b, &vf, M.v_face), "upload velocity faces");
    HIPCHK(h, upload(b, &vdt, M.v_dt), "upload velocity faces");
    HIPCHK(h, upload(b, &vxy, M.v_xy), "upload velocity face points");
    HIPCHK(h, upload(b, &vpr, M.ref.fproj), "upload face projection");
    HIPCHK(h, b.alloc(&h->uplift_src, 1 + 5 * kMaxUpliftSources), "alloc uplift sources");
    HIPCHK(h, hipMemset(h->uplift_src, 0, sizeof(double) * (1 + 5 * kMaxUpliftSources)), "clear uplift sources");
    HIPCHK(h, b.alloc(&h->macro_dev, 1), "alloc macro counter");
    HIPCHK(h, hipMemset(h->macro_dev, 0, sizeof(int64_t)), "clear macro counter");
    h->forcing = ForcingArgs{ve, vf, vdt, vxy, vpr, M.ref.nqf, h->uplift_src, h->macro_dev, M.Bf, row_tiles(M.Bf),
                             1 << (M.C - 1), M.dt_min, 0};
  }
  {
    // fault faces: geometry, parameters (a locked fault: infinite cohesion) and state
    const int64_t F = (int64_t)M.f_elem.size();
    int64_t *fe, *fpe;
    int8_t *ff, *fpf, *fpm;
    double *fg, *fE, *tq, *tw;
    int32_t *pinv;
    HIPCHK(h, upload(b, &fe, M.f_elem), "upload fault faces");
    HIPCHK(h, upload(b, &ff, M.f_face), "upload fault faces");
    HIPCHK(h, upload(b, &fpe, M.f_pelem), "upload fault faces");
    HIPCHK(h, upload(b, &fpf, M.f_pface), "upload fault faces");
    HIPCHK(h, upload(b, &fpm, M.f_perm), "upload fault faces");
    HIPCHK(h, upload(b, &fg, M.f_geo), "upload fault geometry");
    std::vector<double> par(std::max<int64_t>(F, 1) * kFaultParams, 0.0);
    for (int64_t k = 0; k < F; ++k) {
      par[k * kFaultParams + 6] = 1.0;
      par[k * kFaultParams + 7] = INFINITY;
    }
    HIPCHK(h, upload(b, &h->fault_par, par), "upload fault parameters");
    h->fault_par_host = par;
    const int64_t ns = std::max<int64_t>(F, 1) * M.Bf * kFaultState;
    HIPCHK(h, b.alloc(&h->fault_state, ns), "alloc fault state");
    HIPCHK(h, hipMemset(h->fault_state, 0, ns * sizeof(double)), "clear fault state");
    HIPCHK(h, upload(b, &fE, M.ref.E), "upload face traces");
    HIPCHK(h, upload(b, &pinv, M.ref.pinv), "upload node maps");
    std::vector<double> gx, gw;
    gauss_jacobi(M.N + 1, 0.0, 0.0, gx, gw);
    for (size_t j = 0; j < gx.size(); ++j) {
      gx[j] = 0.5 * (gx[j] + 1.0);
      gw[j] *= 0.5;
    }
    HIPCHK(h, upload(b, &tq, gx), "upload time points");
    HIPCHK(h, upload(b, &tw, gw), "upload time weights");
    h->fault = FaultArgs{fe, ff, fpe, fpf, fpm, fg, h->fault_par, h->fault_state, fE, pinv, dslot, tq, tw};
  }
  {
    double *ad, *lmr, *gc, *tw;
    HIPCHK(h, upload(b, &ad, M.a_absdet), "upload absdet");
    HIPCHK(h, upload(b, &lmr, M.a_lmr), "upload materials");
    HIPCHK(h, upload(b, &gc, M.g_coef), "upload surface weights");
    HIPCHK(h, upload(b, &tw, M.ref.tw), "upload face weights");
    h->en = EnergyData{M.E, Fg, M.B, M.nq, ad, lmr, gc, tw, eta};
  }
  c.tgt = tgt; c.mode = mode; c.hperm = hperm; c.half2 = half2; c.rhalf2 = rhalf2; c.gslot = gslot;
  c.dslot = dslot;
  c.perm = perm; c.Eg = Eg; c.Lg = Lg; c.g_elem = gelem; c.g_face = gface; c.g_par = gpar; c.eta = eta;
  c.g = M.g;
  return SEIS_OK;
}

// FP64 assembly of G, material, F-+ and the pointwise flux coefficients on the
// device (assemble.hpp); the host inputs are released afterwards.
int assemble_ops(seis_t* h) {
  Model& M = h->M;
  Buffers tmp;
  double *Ji, *ad, *dt, *lmr, *nrm, *area;
  int8_t* kind;
  int64_t* nbk;
  auto bail = [&](hipError_t st, const char* w) {
    tmp.release();
    return hip_fail(h, st, w);
  };
  hipError_t st = upload(tmp, &Ji, M.a_Jinv);
  if (st == hipSuccess) st = upload(tmp, &ad, M.a_absdet);
  if (st == hipSuccess) st = upload(tmp, &dt, M.a_dt);
  if (st == hipSuccess) st = upload(tmp, &lmr, M.a_lmr);
  if (st == hipSuccess) st = upload(tmp, &nrm, M.a_nrm);
  if (st == hipSuccess) st = upload(tmp, &area, M.a_area);
  if (st == hipSuccess) st = upload(tmp, &kind, M.a_kind);
  if (st == hipSuccess) st = upload(tmp, &nbk, M.a_nbk);
  if (st != hipSuccess) return bail(st, "upload assembly inputs");
  const AsmInput in{M.E, Ji, ad, dt, lmr, nrm, area, kind, nbk};
  const bool tuned = h->kernel == SEIS_KERNEL_TUNED && h->precision != SEIS_FP64;
  float* rcm = tuned ? const_cast<float*>(h->tuned.a.RCm) : nullptr;
  float* rcp = tuned ? const_cast<float*>(h->tuned.a.RCp) : nullptr;
  if (h->precision == SEIS_FP64) {
    DevData<double>& d = h->d64;
    const AsmOutput<double> out{const_cast<double*>(d.G), const_cast<double*>(d.mat), const_cast<double*>(d.Fm),
                                const_cast<double*>(d.Fp), nullptr, nullptr};
    st = launch_assemble(in, out, nullptr);
  } else {
    DevData<float>& d = h->d32;
    const AsmOutput<float> out{const_cast<float*>(d.G), const_cast<float*>(d.mat), const_cast<float*>(d.Fm),
                               const_cast<float*>(d.Fp), rcm, rcp};
    st = launch_assemble(in, out, nullptr);
  }
  if (st == hipSuccess) st = hipDeviceSynchronize();
  if (st != hipSuccess) return bail(st, "operator assembly");
  tmp.release();
  std::vector<double>().swap(M.a_Jinv);
  std::vector<double>().swap(M.a_absdet);
  std::vector<double>().swap(M.a_dt);
  std::vector<double>().swap(M.a_lmr);
  std::vector<double>().swap(M.a_nrm);
  std::vector<double>().swap(M.a_area);
  std::vector<int8_t>().swap(M.a_kind);
  std::vector<int64_t>().swap(M.a_nbk);
  return SEIS_OK;
}

hipEvent_t next_event(seis_t* h) {
  if (h->used == h->pool.size()) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return nullptr;
    h->pool.push_back(ev);
  }
  return h->pool[h->used++];
}

// fold recorded event pairs into the totals
hipError_t fold_list(seis_t* h, const std::vector<seis_t::Rec>& recs) {
  if (recs.empty()) return hipSuccess;
  hipError_t st = hipEventSynchronize(recs.back().b);
  if (st != hipSuccess) return st;
  for (const auto& r : recs) {
    float ms = 0.0f;
    st = hipEventElapsedTime(&ms, r.a, r.b);
    if (st != hipSuccess) return st;
    h->tot_ms[r.kind] += ms;
    h->tot_launch[r.kind] += 1;
    h->tot_elem[r.kind] += r.n;
  }
  return hipSuccess;
}

hipError_t fold_profile(seis_t* h) {
  hipError_t st = fold_list(h, h->recs);
  h->recs.clear();
  h->used = 0;
  return st;
}

// launch fn() bracketed by events when profiling
template <typename F>
hipError_t timed(seis_t* h, int kind, int64_t n, F fn) {
  if (!h->prof || n <= 0) return fn();
  if (h->used + 2 > 4096) {
    hipError_t st = fold_profile(h);
    if (st != hipSuccess) return st;
  }
  hipEvent_t a = next_event(h), b = next_event(h);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t st = hipEventRecord(a, h->stream);
  if (st != hipSuccess) return st;
  st = fn();
  if (st != hipSuccess) return st;
  st = hipEventRecord(b, h->stream);
  if (st != hipSuccess) return st;
  h->recs.push_back({kind, a, b, n});
  return hipSuccess;
}

// Faults at rest: no slip, slip rates zero, the friction state at its start
// (slip path 0; the rate-and-state state psi0 of the face).
int reset_faults(seis_t* h) {
  const Model& M = h->M;
  const int64_t F = (int64_t)M.f_elem.size();
  if (F == 0) return SEIS_OK;
  std::vector<double> st(F * M.Bf * kFaultState, 0.0);
  for (int64_t f = 0; f < F; ++f) {
    const double* q = h->fault_par_host.data() + f * kFaultParams;
    if (q[15] == double(kLawRateState))
      for (int m = 0; m < M.Bf; ++m) st[(f * M.Bf + m) * kFaultState + 3] = q[11];
  }
  HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
  HIPCHK(h, hipMemcpy(h->fault_state, st.data(), st.size() * sizeof(double), hipMemcpyHostToDevice),
         "reset fault state");
  return SEIS_OK;
}

Sched make_sched(const seis_t* h) {
  Sched sc;
  sc.sub = h->sub;
  sc.C = h->M.C;
  for (int c = 0; c <= h->M.C; ++c) sc.cstart[c] = h->M.cluster_start[c];
  return sc;
}

// Predictors of clusters c0..c1 (consecutive, so one element range) at the
// current sub-step, then their gravity faces.
int do_predict(seis_t* h, int c0, int c1) {
  Model& M = h->M;
  const int64_t e0 = M.cluster_start[c0], ne = M.cluster_start[c1 + 1] - e0;
  const Sched sc = make_sched(h);
  hipError_t st = hipSuccess;
  const int32_t* gl = h->glist + h->gstart[c0];
  const int64_t ng = h->gstart[c1 + 1] - h->gstart[c0];
  const int N = M.N;
  st = timed(h, 0, ne, [&]() -> hipError_t {
    if (h->kernel == SEIS_KERNEL_PLAIN) {
      if (h->precision == SEIS_FP64) return launch_predict_plain<double>(N, h->d64, e0, ne, sc, h->stream);
      return launch_predict_plain<float>(N, h->d32, e0, ne, sc, h->stream);
    }
    return tuned_predict(h->tuned, h->precision, N, c0, c1, e0, e0 + ne, sc, h->stream);
  });
  // gravity faces, then fault faces (both read the stored time derivatives)
  if (st == hipSuccess)
    st = timed(h, 1, ng, [&]() -> hipError_t {
      if (h->precision == SEIS_FP64) return launch_gravity<double>(N, h->d64, gl, ng, h->stream);
      return launch_gravity<float>(N, h->d32, gl, ng, h->stream);
    });
  const int64_t f0 = M.fault_start[c0], nf = M.fault_start[c1 + 1] - f0;
  if (st == hipSuccess)
    st = timed(h, 3, nf, [&]() -> hipError_t {
      if (h->precision == SEIS_FP64) return launch_fault<double>(N, h->fault, h->d64.gD, h->d64.In, f0, nf, h->stream);
      return launch_fault<float>(N, h->fault, h->d32.gD, h->d32.In, f0, nf, h->stream);
    });
  if (st != hipSuccess) return hip_fail(h, st, "predict launch");
  return SEIS_OK;
}

int do_correct(seis_t* h, int c0, int c1) {
  Model& M = h->M;
  const int64_t e0 = M.cluster_start[c0], ne = M.cluster_start[c1 + 1] - e0;
  const Sched sc = make_sched(h);
  const int N = M.N;
  hipError_t st = timed(h, 2, ne, [&]() -> hipError_t {
    // uplift forcing of the prescribed-velocity faces of these clusters
    const int64_t v0 = M.vface_start[c0], nv = M.vface_start[c1 + 1] - v0;
    if (nv > 0) {
      const hipError_t sf = h->precision == SEIS_FP64
                                ? launch_forcing<double>(h->forcing, h->d64.In, v0, nv, h->sub, h->stream)
                                : launch_forcing<float>(h->forcing, h->d32.In, v0, nv, h->sub, h->stream);
      if (sf != hipSuccess) return sf;
    }
    if (h->kernel == SEIS_KERNEL_PLAIN) {
      if (h->precision == SEIS_FP64) return launch_correct_plain<double>(N, h->d64, e0, ne, sc, h->stream);
      return launch_correct_plain<float>(N, h->d32, e0, ne, sc, h->stream);
    }
    return tuned_correct(h->tuned, h->precision, N, c0, c1, e0, e0 + ne, sc, h->stream);
  });
  if (st != hipSuccess) return hip_fail(h, st, "correct launch");
  return SEIS_OK;
}

void reset_cursor(seis_t* h) {
  h->sub = 0;
  h->predicted.assign(h->M.C, 0);
  h->corrected.assign(h->M.C, 0);
}

bool mid_step(const seis_t* h) {
  if (h->sub != 0) return true;
  for (int c = 0; c < h->M.C; ++c)
    if (h->predicted[c]) return true;
  return false;
}

// advance the cursor once every due predict and correct of the sub-step ran
void maybe_advance(seis_t* h) {
  const int C = h->M.C;
  for (int c = 0; c < C; ++c) {
    if (h->M.cluster_start[c + 1] == h->M.cluster_start[c]) continue;
    if (due_predict(h->sub, c) && !h->predicted[c]) return;
    if (due_correct(h->sub, c) && !h->corrected[c]) return;
  }
  for (int c = 0; c < C; ++c) {
    if (due_correct(h->sub, c)) {
      h->predicted[c] = 0;
      h->corrected[c] = 0;
    }
  }
  h->sub++;
  if (h->sub == (1 << (C - 1))) {
    h->sub = 0;
    h->macro_done++;
    (void)launch_tick(h->macro_dev, h->stream);
  }
}

int step_eager(seis_t* h);
int step_graph(seis_t* h);

}  // namespace

extern "C" {

void seis_default_options(seis_options_t* o) {
  if (!o) return;
  o->precision = SEIS_FP64;
  o->kernel = SEIS_KERNEL_TUNED;
  o->cfl = 0.35;
  o->g = 9.81;
  o->max_clusters = 1;
  o->stream = nullptr;
  o->tile = 0;
  o->graph = 0;
  o->mc_min = 2048;
  o->fused = 1;
  o->acoustic = 1;
}

int seis_setup(const seis_mesh_t* mesh, const seis_materials_t* mat, int order, const seis_options_t* opt,
               seis_t** out) {
  auto setup_fail = [&](int code, const std::string& msg) {
    std::lock_guard<std::mutex> lk(g_err_mu);
    g_setup_error = msg;
    return code;
  };
  if (!out) return setup_fail(SEIS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!mesh || !mat) return setup_fail(SEIS_EINVAL, "mesh or materials is NULL");
  seis_options_t o;
  seis_default_options(&o);
  if (opt) o = *opt;
  if (o.precision < SEIS_FP64 || o.precision > SEIS_BF16_SPLIT) return setup_fail(SEIS_EINVAL, "bad precision");
  if (o.kernel != SEIS_KERNEL_TUNED && o.kernel != SEIS_KERNEL_PLAIN) return setup_fail(SEIS_EINVAL, "bad kernel");
  if (o.precision == SEIS_BF16_SPLIT && order > 6)
    return setup_fail(SEIS_EINVAL, "split BF16 supports orders 3..6 (its two LDS images of order 7 exceed a CU)");
  if (o.kernel == SEIS_KERNEL_PLAIN && (o.precision == SEIS_BF16 || o.precision == SEIS_BF16_SPLIT))
    return setup_fail(SEIS_EINVAL, "BF16 operands need the tuned (MFMA) kernels");
  if (order < 2 || order > 8) return setup_fail(SEIS_EINVAL, "order must be in 2..8");
  if (o.kernel == SEIS_KERNEL_TUNED && o.precision != SEIS_FP64 && (order < 3 || order > 7))
    return setup_fail(SEIS_EINVAL, "the matrix-core kernels support orders 3..7 (orders 2 and 8: kernel plain)");
  if (o.mc_min < 0) return setup_fail(SEIS_EINVAL, "mc_min must be >= 0");
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return setup_fail(SEIS_EDEVICE, "no HIP device");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return setup_fail(SEIS_EDEVICE, std::string("kernels are built for gfx950, device is ") + prop.gcnArchName);
  {
    const hipError_t st = energy_scratch_init();
    if (st != hipSuccess)
      return setup_fail(SEIS_EDEVICE, std::string("scratch address: ") + hipGetErrorString(st));
  }
  seis_t* h = new (std::nothrow) seis_t();
  if (!h) return setup_fail(SEIS_ENOMEM, "host allocation failed");
  std::string e;
  try {
    e = build_model(mesh->n_vertices, mesh->xyz, mesh->n_elements, mesh->tet, mesh->face_kind, mesh->period,
                    mat->rho, mat->lambda, mat->mu, order - 1, o.cfl, o.g, o.max_clusters, h->M);
  } catch (const std::bad_alloc&) {
    delete h;
    return setup_fail(SEIS_ENOMEM, "host allocation failed during set-up");
  } catch (const std::exception& ex) {
    delete h;
    return setup_fail(SEIS_EINVAL, ex.what());
  }
  if (!e.empty()) {
    delete h;
    return setup_fail(SEIS_EINVAL, e);
  }
  if (!h->M.f_elem.empty() && order > 7) {
    // both sides' stored derivatives of an order-8 face exceed a work-group's LDS
    delete h;
    return setup_fail(SEIS_EINVAL, "fault faces support orders 2..7");
  }
  h->precision = o.precision;
  h->kernel = o.kernel;
  h->tile = o.tile;
  h->stream = (hipStream_t)o.stream;
  h->use_graph = o.graph != 0;
  h->fused = o.fused != 0;
  h->tuned.mc_min = o.mc_min;
  int rc = build_common(h, h->d64);
  if (rc == SEIS_OK) {
    if (o.precision == SEIS_FP64) {
      rc = build_dev<double>(h, h->d64);
    } else {
      share_common(h->d64, h->d32);
      rc = build_dev<float>(h, h->d32);
    }
  }
  if (rc == SEIS_OK && o.kernel == SEIS_KERNEL_TUNED) {
    hipError_t st = tuned_build(h->tuned, h->M, h->precision, h->d64, h->d32, h->tile, o.acoustic != 0, h->buf.ptrs,
                                h->buf.bytes);
    if (st != hipSuccess) rc = hip_fail(h, st, "tuned set-up");
  }
  if (rc == SEIS_OK) rc = assemble_ops(h);
  if (rc == SEIS_OK && o.kernel == SEIS_KERNEL_TUNED) {
    hipError_t st = tuned_autotune(h->tuned, h->M, h->stream);
    if (st != hipSuccess) rc = hip_fail(h, st, "autotune");
  }
  if (rc == SEIS_OK) {
    hipError_t st = hipDeviceSynchronize();
    if (st != hipSuccess) rc = hip_fail(h, st, "set-up sync");
  }
  if (rc != SEIS_OK) {
    const std::string msg = h->err;
    h->buf.release();
    delete h;
    return setup_fail(rc, msg);
  }
  reset_cursor(h);
  *out = h;
  return SEIS_OK;
}

int seis_write(seis_t* h, const double* dofs, const double* eta) {
  if (!h) return SEIS_EINVAL;
  Model& M = h->M;
  HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
  if (dofs) {
    const int RT = row_tiles(M.B);
    const int64_t n = q_size(M.E, RT);
    const size_t row = (size_t)M.B * 9;
    std::vector<double> tmp(n, 0.0);
    for (int64_t k = 0; k < M.E; ++k) {
      const double* src = dofs + M.old_of_new[k] * row;
      for (int r = 0; r < M.B; ++r)
        for (int p = 0; p < 9; ++p) tmp[qidx(k, r, p, RT)] = src[r * 9 + p];
    }
    if (h->precision == SEIS_FP64) {
      HIPCHK(h, hipMemcpy(h->d64.Q, tmp.data(), n * sizeof(double), hipMemcpyHostToDevice), "write Q");
    } else {
      std::vector<float> tf(tmp.begin(), tmp.end());
      HIPCHK(h, hipMemcpy(h->d32.Q, tf.data(), n * sizeof(float), hipMemcpyHostToDevice), "write Q");
    }
  }
  if (eta && !M.g_elem.empty()) {
    HIPCHK(h, hipMemcpy(h->d64.eta, eta, M.g_elem.size() * M.nq * sizeof(double), hipMemcpyHostToDevice),
           "write eta");
  }
  // a written state starts a new run at time 0 (the clock of the uplift
  // forcing) with the faults at rest (no slip, the friction state initial)
  {
    const int rc = reset_faults(h);
    if (rc != SEIS_OK) return rc;
  }
  const int64_t zero = 0;
  HIPCHK(h, hipMemcpy(h->macro_dev, &zero, sizeof(zero), hipMemcpyHostToDevice), "reset macro counter");
  h->macro_done = 0;
  reset_cursor(h);
  return SEIS_OK;
}

int seis_set_fault(seis_t* h, int64_t n, int law, const double* params) {
  if (!h) return SEIS_EINVAL;
  const Model& M = h->M;
  const int64_t F = (int64_t)M.f_elem.size();
  if (n != F || (F > 0 && !params)) return fail(h, SEIS_EINVAL, "seis_set_fault: n must equal the number of fault faces");
  if (law != SEIS_FRICTION_SLIP_WEAKENING && law != SEIS_FRICTION_RATE_STATE)
    return fail(h, SEIS_EINVAL, "seis_set_fault: unknown friction law");
  const int np = law == SEIS_FRICTION_SLIP_WEAKENING ? 8 : 12;
  std::vector<double> par(std::max<int64_t>(F, 1) * kFaultParams, 0.0);
  for (int64_t k = 0; k < F; ++k) {
    const double* p = params + k * np;
    if (law == SEIS_FRICTION_SLIP_WEAKENING &&
        (!(p[4] >= 0.0) || !(p[5] >= 0.0) || !(p[6] > 0.0) || !(p[7] >= 0.0)))
      return fail(h, SEIS_EINVAL, "seis_set_fault: need mu_s, mu_d >= 0, D_c > 0, C >= 0");
    if (law == SEIS_FRICTION_RATE_STATE &&
        (!(p[4] > 0.0) || !(p[6] > 0.0) || !(p[7] > 0.0) || !(p[10] > 0.0) || !std::isfinite(p[5]) ||
         !std::isfinite(p[8]) || !std::isfinite(p[9]) || !std::isfinite(p[11])))
      return fail(h, SEIS_EINVAL, "seis_set_fault: need a, L, V0, V_w > 0 and finite b, f0, f_w, psi0");
    double* q = par.data() + M.fault_abi[k] * kFaultParams;
    for (int i = 0; i < np; ++i) q[i] = p[i];
    q[15] = law;
  }
  HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
  if (F > 0)
    HIPCHK(h, hipMemcpy(h->fault_par, par.data(), F * kFaultParams * sizeof(double), hipMemcpyHostToDevice),
           "write fault parameters");
  h->fault_par_host = par;
  return reset_faults(h);
}

int seis_fault_read(seis_t* h, double* out) {
  if (!h) return SEIS_EINVAL;
  const Model& M = h->M;
  const int64_t F = (int64_t)M.f_elem.size();
  if (F == 0) return SEIS_OK;
  if (!out) return SEIS_EINVAL;
  HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
  std::vector<double> st(F * M.Bf * kFaultState);
  HIPCHK(h, hipMemcpy(st.data(), h->fault_state, st.size() * sizeof(double), hipMemcpyDeviceToHost),
         "read fault state");
  for (int64_t k = 0; k < F; ++k) {
    const int64_t f = M.fault_abi[k];
    for (int m = 0; m < M.Bf; ++m) {
      double* o = out + (k * M.Bf + m) * (3 + kFaultState);
      for (int d = 0; d < 3; ++d) o[d] = M.f_xyz[(f * M.Bf + m) * 3 + d];
      for (int i = 0; i < kFaultState; ++i) o[3 + i] = st[(f * M.Bf + m) * kFaultState + i];
    }
  }
  return SEIS_OK;
}

int seis_set_uplift(seis_t* h, int n, const double* src) {
  if (!h || n < 0 || n > kMaxUpliftSources || (n > 0 && !src)) return SEIS_EINVAL;
  std::vector<double> buf(1 + 5 * kMaxUpliftSources, 0.0);
  buf[0] = n;
  for (int j = 0; j < n; ++j) {
    if (!(src[5 * j + 3] > 0.0) || !(src[5 * j + 4] > 0.0))
      return fail(h, SEIS_EINVAL, "uplift source width and rise time must be > 0");
    for (int k = 0; k < 5; ++k) buf[1 + 5 * j + k] = src[5 * j + k];
  }
  HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
  HIPCHK(h, hipMemcpy(h->uplift_src, buf.data(), buf.size() * sizeof(double), hipMemcpyHostToDevice),
         "write uplift sources");
  return SEIS_OK;
}

int seis_predict(seis_t* h, int c) {
  if (!h) return SEIS_EINVAL;
  if (c < 0 || c >= h->M.C) return fail(h, SEIS_ERANGE, "cluster id out of range");
  if (!due_predict(h->sub, c) || h->predicted[c])
    return fail(h, SEIS_EORDER, "cluster is not due for a prediction at this point of the LTS schedule");
  int rc = do_predict(h, c, c);
  if (rc != SEIS_OK) return rc;
  h->predicted[c] = 1;
  maybe_advance(h);
  return SEIS_OK;
}

int seis_correct(seis_t* h, int c) {
  if (!h) return SEIS_EINVAL;
  const int C = h->M.C;
  if (c < 0 || c >= C) return fail(h, SEIS_ERANGE, "cluster id out of range");
  if (!due_correct(h->sub, c) || h->corrected[c])
    return fail(h, SEIS_EORDER, "cluster is not due for a correction at this point of the LTS schedule");
  for (int cc = 0; cc < C; ++cc)
    if (h->M.cluster_start[cc + 1] > h->M.cluster_start[cc] && due_predict(h->sub, cc) && !h->predicted[cc])
      return fail(h, SEIS_EORDER, "all predictions of the sub-step must run before its corrections");
  if (!h->predicted[c]) return fail(h, SEIS_EORDER, "cluster has not been predicted for this step");
  int rc = do_correct(h, c, c);
  if (rc != SEIS_OK) return rc;
  h->corrected[c] = 1;
  maybe_advance(h);
  return SEIS_OK;
}

int seis_step(seis_t* h) {
  if (!h) return SEIS_EINVAL;
  if (mid_step(h)) return fail(h, SEIS_EORDER, "a macro step is in progress; finish it with seis_predict/seis_correct");
  if (h->use_graph) return step_graph(h);
  return step_eager(h);
}

int seis_run(seis_t* h, int n) {
  for (int i = 0; i < n; ++i) {
    int rc = seis_step(h);
    if (rc) return rc;
  }
  return SEIS_OK;
}

}  // extern "C"

namespace {

// One macro step with one launch per phase per sub-step: the clusters due in
// sub-step s are 0..k with k the largest c such that 2^c divides s (for the
// predictors) or s + 1 (for the correctors), so they form one element range
// (clusters are contiguous in library order) and one launch covers them all;
// each element takes its step parity from the schedule. Ordering between the
// phases stays at kernel boundaries on the stream.
int step_fused(seis_t* h) {
  const int C = h->M.C;
  auto top_due = [&](int s1) {
    int k = 0;
    while (k + 1 < C && s1 % (1 << (k + 1)) == 0) ++k;
    return k;
  };
  for (int s = 0; s < (1 << (C - 1)); ++s) {
    h->sub = s;
    int rc = do_predict(h, 0, top_due(s));
    if (rc == SEIS_OK) rc = do_correct(h, 0, top_due(s + 1));
    if (rc != SEIS_OK) {
      reset_cursor(h);
      return rc;
    }
  }
  reset_cursor(h);
  h->macro_done++;
  const hipError_t st = launch_tick(h->macro_dev, h->stream);
  if (st != hipSuccess) return hip_fail(h, st, "macro step counter");
  return SEIS_OK;
}

int step_eager(seis_t* h) {
  if (h->fused) return step_fused(h);
  const int C = h->M.C;
  for (int s = 0; s < (1 << (C - 1)); ++s) {
    for (int c = 0; c < C; ++c)
      if (due_predict(s, c)) {
        int rc = seis_predict(h, c);
        if (rc) return rc;
      }
    for (int c = 0; c < C; ++c)
      if (due_correct(s, c)) {
        int rc = seis_correct(h, c);
        if (rc) return rc;
      }
  }
  return SEIS_OK;
}

void drop_graph(seis_t* h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->gexec = nullptr;
  h->graph = nullptr;
}

// Capture the launches of one macro step on the private stream. The schedule
// cursor is restored afterwards: capturing runs nothing.
int capture_step(seis_t* h) {
  drop_graph(h);
  if (!h->cap) HIPCHK(h, hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking), "capture stream");
  const int sub = h->sub;
  const int64_t done = h->macro_done;
  const std::vector<int> pred = h->predicted, corr = h->corrected;
  hipStream_t user = h->stream;
  h->stream = h->cap;
  hipError_t st = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
  int rc = SEIS_OK;
  if (st == hipSuccess) rc = step_eager(h);
  hipGraph_t g = nullptr;
  const hipError_t se = st == hipSuccess ? hipStreamEndCapture(h->cap, &g) : st;
  h->stream = user;
  h->sub = sub;
  h->macro_done = done;
  h->predicted = pred;
  h->corrected = corr;
  if (rc != SEIS_OK || se != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    if (rc != SEIS_OK) return rc;
    return hip_fail(h, se, "graph capture");
  }
  h->graph = g;
  st = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
  if (st != hipSuccess) {
    drop_graph(h);
    return hip_fail(h, st, "graph instantiate");
  }
  return SEIS_OK;
}

// Graph replay of a macro step. Kernel timings cannot be read from inside a
// graph, so with profiling on the step is launched eagerly instead.
int step_graph(seis_t* h) {
  if (h->prof) return step_eager(h);
  if (!h->gexec) {
    int rc = capture_step(h);
    if (rc != SEIS_OK) return rc;
  }
  HIPCHK(h, hipGraphLaunch(h->gexec, h->stream), "graph launch");
  h->macro_done++;
  return SEIS_OK;
}

}  // namespace

extern "C" {

int seis_read(seis_t* h, double* dofs, double* eta) {
  if (!h) return SEIS_EINVAL;
  if (mid_step(h)) return fail(h, SEIS_EORDER, "state is between a prediction and its correction");
  Model& M = h->M;
  HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
  if (dofs) {
    const int RT = row_tiles(M.B);
    const int64_t n = q_size(M.E, RT);
    const size_t row = (size_t)M.B * 9;
    std::vector<double> tmp(n);
    if (h->precision == SEIS_FP64) {
      HIPCHK(h, hipMemcpy(tmp.data(), h->d64.Q, n * sizeof(double), hipMemcpyDeviceToHost), "read Q");
    } else {
      std::vector<float> tf(n);
      HIPCHK(h, hipMemcpy(tf.data(), h->d32.Q, n * sizeof(float), hipMemcpyDeviceToHost), "read Q");
      for (int64_t i = 0; i < n; ++i) tmp[i] = tf[i];
    }
    for (int64_t k = 0; k < M.E; ++k) {
      double* dst = dofs + M.old_of_new[k] * row;
      for (int r = 0; r < M.B; ++r)
        for (int p = 0; p < 9; ++p) dst[r * 9 + p] = tmp[qidx(k, r, p, RT)];
    }
  }
  if (eta && !M.g_elem.empty()) {
    HIPCHK(h, hipMemcpy(eta, h->d64.eta, M.g_elem.size() * M.nq * sizeof(double), hipMemcpyDeviceToHost),
           "read eta");
  }
  return SEIS_OK;
}

int seis_read_elements(seis_t* h, const int64_t* ids, int64_t n, double* dofs) {
  if (!h || (!ids && n > 0) || (!dofs && n > 0) || n < 0) return SEIS_EINVAL;
  if (mid_step(h)) return fail(h, SEIS_EORDER, "state is between a prediction and its correction");
  Model& M = h->M;
  HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
  const size_t row = (size_t)M.B * 9;
  const int RT = row_tiles(M.B);
  const int64_t gsz = (int64_t)RT * 36 * 64;  // values of one 16-element group
  std::vector<double> blk(gsz);
  std::vector<float> blkf(gsz);
  for (int64_t i = 0; i < n; ++i) {
    if (ids[i] < 0 || ids[i] >= M.E) return fail(h, SEIS_ERANGE, "element id out of range");
    const int64_t k = M.new_of_old[ids[i]];
    const int64_t base = (k >> 4) * gsz;
    if (h->precision == SEIS_FP64) {
      HIPCHK(h, hipMemcpy(blk.data(), h->d64.Q + base, gsz * sizeof(double), hipMemcpyDeviceToHost), "read element");
    } else {
      HIPCHK(h, hipMemcpy(blkf.data(), h->d32.Q + base, gsz * sizeof(float), hipMemcpyDeviceToHost), "read element");
      for (int64_t j = 0; j < gsz; ++j) blk[j] = blkf[j];
    }
    for (int r = 0; r < M.B; ++r)
      for (int p = 0; p < 9; ++p) dofs[i * row + r * 9 + p] = blk[qidx(k, r, p, RT) - base];
  }
  return SEIS_OK;
}

int seis_info(const seis_t* h, seis_info_t* info) {
  if (!h || !info) return SEIS_EINVAL;
  const Model& M = h->M;
  std::memset(info, 0, sizeof(*info));
  info->order = M.N + 1;
  info->n_basis = M.B;
  info->n_face_nodes = M.Bf;
  info->n_eta_points = M.nq;
  info->precision = h->precision;
  info->kernel = h->kernel;
  info->n_clusters = M.C;
  info->n_elements = M.E;
  info->n_gravity_faces = (int64_t)M.g_elem.size();
  info->dt_min = M.dt_min;
  info->time = double(h->macro_done) * double(1 << (M.C - 1)) * M.dt_min;
  int64_t upd = 0;
  for (int c = 0; c < M.C && c < 16; ++c) {
    info->cluster_size[c] = M.cluster_start[c + 1] - M.cluster_start[c];
    upd += info->cluster_size[c] << (M.C - 1 - c);
  }
  info->updates_per_macro_step = upd;
  info->device_bytes = h->buf.bytes;
  const LaunchCfg* lc[2] = {&h->tuned.pc, &h->tuned.cc};
  for (int k = 0; k < 2; ++k) {
    info->launch[3 * k + 0] = lc[k]->waves;
    info->launch[3 * k + 1] = lc[k]->cap;
    info->launch[3 * k + 2] = lc[k]->remap;
  }
  info->launch[6] = h->tuned.cc.split;
  info->launch[7] = h->tuned.mc_min;
  info->launch_source = h->tuned.source;
  info->fused = h->fused ? 1 : 0;
  info->shape = h->tuned.pc.variant;
  info->n_acoustic_groups = h->tuned.n_acoustic_groups;
  info->n_fault_faces = (int64_t)M.f_elem.size();
  return SEIS_OK;
}

int seis_cluster_of(const seis_t* h, int32_t* out) {
  if (!h || !out) return SEIS_EINVAL;
  std::memcpy(out, h->M.cluster_old.data(), h->M.E * sizeof(int32_t));
  return SEIS_OK;
}

int seis_profile(seis_t* h, int enable) {
  if (!h) return SEIS_EINVAL;
  HIPCHK(h, fold_profile(h), "profile");
  for (int k = 0; k < 4; ++k) {
    if (enable) {
      h->tot_ms[k] = 0.0;
      h->tot_launch[k] = 0;
      h->tot_elem[k] = 0;
    }
  }
  h->prof = enable != 0;
  return SEIS_OK;
}

int seis_profile_read(seis_t* h, double* ms, int64_t* launches, int64_t* elements) {
  if (!h) return SEIS_EINVAL;
  HIPCHK(h, fold_profile(h), "profile");
  for (int k = 0; k < 4; ++k) {
    if (ms) ms[k] = h->tot_ms[k];
    if (launches) launches[k] = h->tot_launch[k];
    if (elements) elements[k] = h->tot_elem[k];
  }
  return SEIS_OK;
}

}  // extern "C"

namespace {

int make_points(seis_t* h, int which, int64_t n, const double* xyz, PointSet& ps) {
  std::vector<double> phi;
  std::vector<int32_t> el;
  std::string e;
  try {
    e = build_points(h->M, which, n, xyz, ps, phi, el);
  } catch (const std::bad_alloc&) {
    return fail(h, SEIS_ENOMEM, "host allocation failed while locating points");
  }
  if (!e.empty()) return fail(h, SEIS_EINVAL, e);
  HIPCHK(h, upload(h->buf, &ps.phi, phi), "upload point basis values");
  HIPCHK(h, upload(h->buf, &ps.elem, el), "upload point elements");
  return SEIS_OK;
}

// the point set of id (building a built-in set at its first use), or null
PointSet* point_set(seis_t* h, int id, int* rc) {
  *rc = SEIS_OK;
  if (id == SEIS_POINTS_SEA_SURFACE || id == SEIS_POINTS_SEAFLOOR) {
    const bool sea = id == SEIS_POINTS_SEA_SURFACE;
    PointSet& ps = sea ? h->sea_set : h->floor_set;
    bool& built = sea ? h->sea_built : h->floor_built;
    if (!built) {
      *rc = make_points(h, sea ? 1 : 2, 0, nullptr, ps);
      if (*rc != SEIS_OK) return nullptr;
      built = true;
    }
    return &ps;
  }
  if (id < 0 || id >= (int)h->psets.size()) {
    *rc = fail(h, SEIS_ERANGE, "no such point set");
    return nullptr;
  }
  return &h->psets[id];
}

}  // namespace

extern "C" {

int seis_points(seis_t* h, int64_t n, const double* xyz, int* id) {
  if (!h || n <= 0 || !xyz || !id) return SEIS_EINVAL;
  PointSet ps;
  const int rc = make_points(h, 0, n, xyz, ps);
  if (rc != SEIS_OK) return rc;
  h->psets.push_back(std::move(ps));
  *id = (int)h->psets.size() - 1;
  return SEIS_OK;
}

int seis_points_info(seis_t* h, int id, int64_t* n, double* xyz, int64_t* element) {
  if (!h) return SEIS_EINVAL;
  int rc = SEIS_OK;
  PointSet* ps = point_set(h, id, &rc);
  if (!ps) return rc;
  if (n) *n = ps->n;
  if (xyz && ps->n) std::memcpy(xyz, ps->xyz.data(), sizeof(double) * 3 * ps->n);
  if (element && ps->n) std::memcpy(element, ps->elem_caller.data(), sizeof(int64_t) * ps->n);
  return SEIS_OK;
}

int seis_sample(seis_t* h, int id, double* out, double* eta) {
  if (!h || !out) return SEIS_EINVAL;
  if (mid_step(h)) return fail(h, SEIS_EORDER, "state is between a prediction and its correction");
  int rc = SEIS_OK;
  PointSet* ps = point_set(h, id, &rc);
  if (!ps) return rc;
  if (eta && !ps->sea) return fail(h, SEIS_EINVAL, "eta is only sampled on the sea-surface point set");
  const double* q64 = h->precision == SEIS_FP64 ? h->d64.Q : nullptr;
  const float* q32 = h->precision == SEIS_FP64 ? nullptr : h->d32.Q;
  HIPCHK(h, launch_sample(*ps, h->M.B, q64, q32, h->d64.eta, out, eta, h->stream), "sample launch");
  return SEIS_OK;
}

int seis_energy(seis_t* h, double* out) {
  if (!h || !out) return SEIS_EINVAL;
  if (mid_step(h)) return fail(h, SEIS_EORDER, "state is between a prediction and its correction");
  if (!h->en_partial) {
    void* p = nullptr;
    HIPCHK(h, hipMalloc(&p, sizeof(double) * energy_groups(h->M.E) * kEnergyValues), "alloc energy partials");
    h->en_partial = static_cast<double*>(p);
  }
  const double* q64 = h->precision == SEIS_FP64 ? h->d64.Q : nullptr;
  const float* q32 = h->precision == SEIS_FP64 ? nullptr : h->d32.Q;
  HIPCHK(h, launch_energy(h->en, q64, q32, h->en_partial, out, h->stream), "energy launch");
  return SEIS_OK;
}

int seis_energy_noalloc(seis_t* h, double* out) {
  if (!h || !out) return SEIS_EINVAL;
  if (mid_step(h)) return fail(h, SEIS_EORDER, "state is between a prediction and its correction");
  double* part = energy_scratch();
  if (!part)
    return fail(h, SEIS_EDEVICE, "the fixed scratch array has no address on the current device (seis_setup "
                                 "was not run with this device current)");
  const int64_t need = int64_t(energy_groups(h->M.E)) * kEnergyValues;
  if (need > kEnergyScratchValues)
    return fail(h, SEIS_ERANGE, "energy partial sums (" + std::to_string(need) +
                                    " values) exceed the fixed scratch array (" +
                                    std::to_string(kEnergyScratchValues) + " values)");
  const double* q64 = h->precision == SEIS_FP64 ? h->d64.Q : nullptr;
  const float* q32 = h->precision == SEIS_FP64 ? nullptr : h->d32.Q;
  HIPCHK(h, launch_energy(h->en, q64, q32, part, out, h->stream), "energy launch");
  return SEIS_OK;
}

int seis_sync(seis_t* h) {
  if (!h) return SEIS_EINVAL;
  HIPCHK(h, hipStreamSynchronize(h->stream), "sync");
  return SEIS_OK;
}

void seis_destroy(seis_t* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  drop_graph(h);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  for (hipEvent_t ev : h->pool) (void)hipEventDestroy(ev);
  if (h->en_partial) (void)hipFree(h->en_partial);
  h->buf.release();
  delete h;
}

const char* seis_last_error(const seis_t* h) {
  if (h) return h->err.c_str();
  std::lock_guard<std::mutex> lk(g_err_mu);
  return g_setup_error.c_str();
}

}  // extern "C"
