// Host side of the matrix-core kernels: reference-matrix images, set-up,
// per-cluster launches (with the LTS half-step fix-ups) and the autotuner.
// The kernels are in tuned_kern.hpp and are instantiated per operand
// precision in tuned_f32.hip and tuned_bf16.hip.
#include "tuned_kern.hpp"

#include <sys/stat.h>

#include <fstream>
#include <sstream>

namespace seis {

namespace {

// Half-step fix-up of the faces handing over to a finer neighbour (one
// work-group per face of list): the predictor wrote the full-step trace V;
// the finer neighbour needs the traces of the first and of the second half of
// this element's step, each over its own step: the first half
// h1 = E_f I~_h with I~_h = sum_k D~k 2^-k / (k+1) (from the stored
// derivatives) goes to the inbox, the second half 2 V - h1 to its slot.
template <int N>
__global__ __launch_bounds__(64) void k_finer_fixup(TArgs a, const int32_t* list) {
  constexpr int B = nbasis(N), Bf = nface(N), FT = row_tiles(Bf);
  __shared__ float sIh[B * 9];
  const int id = list[blockIdx.x];
  const int64_t e = id >> 2;
  const int f = id & 3;
  const float* D = a.gD + (int64_t)a.dslot[e] * (N + 1) * B * 9;
  for (int i = threadIdx.x; i < B * 9; i += 64) {
    float acc = 0.0f, w = 1.0f;
    for (int k = 0; k <= N; ++k) {
      acc += w / float(k + 1) * D[k * B * 9 + i];
      w *= 0.5f;
    }
    sIh[i] = acc;
  }
  __syncthreads();
  const int32_t tg = a.tgt[e * 4 + f];
  const int h = a.hperm[e * 4 + f];
  const int slot = a.half2[e * 4 + f];
  for (int i = threadIdx.x; i < Bf * 9; i += 64) {
    const int m = i / 9, p = i % 9;
    const float* Em = a.Ef + ((int64_t)f * Bf + m) * B;
    float h1 = 0.0f;
    for (int l = 0; l < B; ++l) h1 += Em[l] * sIh[l * 9 + p];
    const int mr = a.pinv[h * Bf + m];
    float* dst = a.In + inidx(tg >> 2, tg & 3, mr, p, FT);
    const float v = *dst;
    *dst = h1;
    a.H2[((int64_t)slot * Bf + mr) * 9 + p] = 2.0f * v - h1;
  }
}

// Second-half traces into the inbox before the corrector of an odd sub-step
// (one work-group per face of list).
template <int N>
__global__ __launch_bounds__(64) void k_h2_to_in(TArgs a, const int32_t* list) {
  constexpr int Bf = nface(N), FT = row_tiles(Bf);
  const int id = list[blockIdx.x];
  const int64_t e = id >> 2;
  const int f = id & 3;
  const int slot = a.rhalf2[e * 4 + f];
  for (int i = threadIdx.x; i < Bf * 9; i += 64) {
    const int m = i / 9, p = i % 9;
    a.In[inidx(e, f, m, p, FT)] = a.H2[((int64_t)slot * Bf + m) * 9 + p];
  }
}

template <int N>
hipError_t launch_fixup(const TArgs& a, const int32_t* list, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finer_fixup<N>, dim3((unsigned)n), dim3(64), 0, s, a, list);
  return hipGetLastError();
}

template <int N>
hipError_t launch_h2(const TArgs& a, const int32_t* list, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_h2_to_in<N>, dim3((unsigned)n), dim3(64), 0, s, a, list);
  return hipGetLastError();
}

hipError_t fixup_dispatch(int N, const TArgs& a, const int32_t* list, int64_t n, hipStream_t s) {
  switch (N) {
    case 2: return launch_fixup<2>(a, list, n, s);
    case 3: return launch_fixup<3>(a, list, n, s);
    case 4: return launch_fixup<4>(a, list, n, s);
    case 5: return launch_fixup<5>(a, list, n, s);
    case 6: return launch_fixup<6>(a, list, n, s);
  }
  return hipErrorInvalidValue;
}

hipError_t h2_dispatch(int N, const TArgs& a, const int32_t* list, int64_t n, hipStream_t s) {
  switch (N) {
    case 2: return launch_h2<2>(a, list, n, s);
    case 3: return launch_h2<3>(a, list, n, s);
    case 4: return launch_h2<4>(a, list, n, s);
    case 5: return launch_h2<5>(a, list, n, s);
    case 6: return launch_h2<6>(a, list, n, s);
  }
  return hipErrorInvalidValue;
}

template <typename X, typename Y>
hipError_t upload(std::vector<void*>& owned, int64_t& bytes, X** dst, const std::vector<Y>& src) {
  void* p = nullptr;
  const size_t n = std::max<size_t>(src.size(), 1);
  hipError_t st = hipMalloc(&p, n * sizeof(X));
  if (st != hipSuccess) return st;
  owned.push_back(p);
  bytes += int64_t(n * sizeof(X));
  *dst = static_cast<X*>(p);
  if (src.empty()) return hipSuccess;
  std::vector<X> tmp(src.size());
  for (size_t i = 0; i < src.size(); ++i) tmp[i] = (X)src[i];
  return hipMemcpy(p, tmp.data(), tmp.size() * sizeof(X), hipMemcpyHostToDevice);
}

// Host image of the LDS reference block (same layout as Lay<Op, N>).
template <class Op, int N>
std::vector<double> ref_image(const Model& M) {
  using L = Lay<Op, N>;
  const int B = L::B, Bf = L::Bf, B1 = L::B1;
  std::vector<double> r(L::total, 0.0);
  // position of state row k in the image: fragment order for BF16
  auto pos = [](int k) { return L::BF ? tile_perm(k) : k; };
  for (int d = 0; d < 3; ++d)
    for (int k = 0; k < B; ++k)
      for (int l = 0; l < B1; ++l) {
        const double v = M.ref.K[(d * B + k) * B + l];
        r[L::oK + (d * L::PB + pos(k)) * L::ldK + pos(l)] = v;
        if (L::BF) r[L::oT + (d * L::PB1 + pos(l)) * L::ldT + pos(k)] = v;
      }
  for (int f = 0; f < 4; ++f)
    for (int c = 0; c < 16 * L::FT; ++c) {
      const int m = node_of(c);
      if (m >= Bf) continue;  // padding slot: zero
      for (int k = 0; k < B; ++k) {
        r[L::oE + (f * 16 * L::FT + c) * L::ldE + pos(k)] = M.ref.E[(f * Bf + m) * B + k];
        r[L::oL + (f * L::PB + pos(k)) * L::ldL + c] = M.ref.L[(f * B + k) * Bf + m];
      }
    }
  return r;
}

template <class Op>
std::vector<double> ref_image_n(const Model& M, int& bytes) {
  switch (M.N) {
    case 2: bytes = Lay<Op, 2>::bytes; return ref_image<Op, 2>(M);
    case 3: bytes = Lay<Op, 3>::bytes; return ref_image<Op, 3>(M);
    case 4: bytes = Lay<Op, 4>::bytes; return ref_image<Op, 4>(M);
    case 5: bytes = Lay<Op, 5>::bytes; return ref_image<Op, 5>(M);
    default: bytes = Lay<Op, 6>::bytes; return ref_image<Op, 6>(M);
  }
}

}  // namespace

// matrix-core launches by precision: 1 FP32, 2 BF16, 3 split BF16
hipError_t pred_dispatch_any(int precision, int N, const LaunchCfg& c, const TArgs& a, int64_t e0, int64_t e1,
                             const Sched& sc, hipStream_t s) {
  if (precision == 1) return pred_dispatch_f32(N, c, a, e0, e1, sc, s);
  if (precision == 3) return pred_dispatch_bf16x3(N, c, a, e0, e1, sc, s);
  return pred_dispatch_bf16(N, c, a, e0, e1, sc, s);
}

hipError_t corr_dispatch_any(int precision, int N, const LaunchCfg& c, const TArgs& a, int64_t e0, int64_t e1,
                             hipStream_t s) {
  if (precision == 1) return corr_dispatch_f32(N, c, a, e0, e1, s);
  if (precision == 3) return corr_dispatch_bf16x3(N, c, a, e0, e1, s);
  return corr_dispatch_bf16(N, c, a, e0, e1, s);
}

hipError_t tuned_build(TunedData& t, const Model& M, int precision, const DevData<double>& d64,
                       const DevData<float>& d32, int tile, int acoustic, std::vector<void*>& owned,
                       int64_t& bytes) {
  t.N = M.N;
  t.precision = precision;
  t.d64 = d64;
  t.d32 = d32;
  t.fix_start = M.fix_start;
  t.h2_start = M.h2_start;
  if (tile > 0) {
    const int w = tile <= 32 ? 2 : 4;
    t.pc = LaunchCfg{w, 0, 0, 2};
    t.cc = LaunchCfg{w, 0, 0, 2};
    t.fixed = 1;
  }
  if (precision == 0) {  // FP64 runs the plain kernels
    t.ready = 1;
    return hipSuccess;
  }
  TArgs& a = t.a;
  a.Q = d32.Q;
  a.In = d32.In;
  a.G = d32.G;
  a.mat = d32.mat;
  a.tgt = d32.tgt;
  a.mode = d32.mode;
  a.hperm = d32.hperm;
  a.Ef = d32.Ef;
  a.H2 = d32.H2;
  a.half2 = d32.half2;
  a.rhalf2 = d32.rhalf2;
  a.gD = d32.gD;
  {
    const int64_t nJ = q_size(M.E, row_tiles(n_basis(M.N)));
    void* pj = nullptr;
    hipError_t sj = hipMalloc(&pj, nJ * sizeof(float));
    if (sj != hipSuccess) return sj;
    owned.push_back(pj);
    bytes += nJ * int64_t(sizeof(float));
    a.Ib = static_cast<float*>(pj);
  }
  // pointwise flux coefficients: filled by the operator assembly
  float* rc[2] = {nullptr, nullptr};
  for (int i = 0; i < 2; ++i) {
    void* p = nullptr;
    const int64_t n = M.E * 4 * 12;
    hipError_t sa = hipMalloc(&p, n * sizeof(float));
    if (sa != hipSuccess) return sa;
    owned.push_back(p);
    bytes += n * int64_t(sizeof(float));
    rc[i] = static_cast<float*>(p);
  }
  float *rcm = rc[0], *rcp = rc[1];
  int32_t* pinv;
  hipError_t st = upload(owned, bytes, &pinv, M.ref.pinv);
  if (st != hipSuccess) return st;
  a.RCm = rcm;
  a.RCp = rcp;
  a.pinv = pinv;
  {
    std::vector<int32_t> mh(M.E, 0);
    for (int64_t e = 0; e < M.E; ++e)
      for (int f = 0; f < 4; ++f) mh[e] |= ((M.mode[e * 4 + f] & 3) | (M.hperm[e * 4 + f] & 7) << 2) << (8 * f);
    int32_t* dm;
    st = upload(owned, bytes, &dm, mh);
    if (st != hipSuccess) return st;
    a.mh4 = dm;
  }
  {
    int32_t *ds, *fl, *hl;
    st = upload(owned, bytes, &ds, M.dslot);
    if (st == hipSuccess) st = upload(owned, bytes, &fl, M.fix_list);
    if (st == hipSuccess) st = upload(owned, bytes, &hl, M.h2_list);
    if (st != hipSuccess) return st;
    a.dslot = ds;
    a.fix_list = fl;
    a.h2_list = hl;
  }
  {
    // 16-element groups of acoustic elements (mu = 0) run in the 4-quantity
    // form; element order puts the acoustic elements of a cluster together
    const int64_t ng = (M.E + 15) / 16;
    std::vector<int32_t> gac(ng, 0);
    t.n_acoustic_groups = 0;
    for (int64_t gi = 0; gi < ng && acoustic; ++gi) {
      bool all = true;
      for (int64_t e = gi * 16; e < std::min<int64_t>(M.E, gi * 16 + 16); ++e) all = all && M.a_lmr[e * 3 + 1] == 0.0;
      gac[gi] = all ? 1 : 0;
      t.n_acoustic_groups += gac[gi];
    }
    int32_t* dg;
    st = upload(owned, bytes, &dg, gac);
    if (st != hipSuccess) return st;
    a.gac = dg;
  }
  // LDS image of the reference matrices (layout of Lay<Op, N>), padded to 16 bytes
  int lbytes = 0;
  if (precision == 1) {
    std::vector<double> ref = ref_image_n<OpF32>(M, lbytes);
    ref.resize(lbytes / 4, 0.0);
    float* r;
    st = upload(owned, bytes, &r, ref);
    a.ref = r;
  } else {
    // BF16: one image rounded to BF16; split BF16 (precision 3): the image of
    // hi = bf16(x), then the image of lo = bf16(x - hi)
    const bool split = precision == 3;
    std::vector<double> ref = split ? ref_image_n<OpBF16X3>(M, lbytes) : ref_image_n<OpBF16>(M, lbytes);
    std::vector<unsigned short> rb(lbytes / 2, 0);
    const size_t one = split ? rb.size() / 2 : rb.size();
    for (size_t i = 0; i < ref.size() && i < one; ++i) {
      const float x = (float)ref[i];
      rb[i] = f2bf(x);
      if (split) {
        const uint32_t u = uint32_t(rb[i]) << 16;
        float hi;
        std::memcpy(&hi, &u, 4);
        rb[one + i] = f2bf(x - hi);
      }
    }
    unsigned short* r;
    st = upload(owned, bytes, &r, rb);
    a.ref = r;
  }
  a.ref_bytes = lbytes;
  if (st != hipSuccess) return st;
  t.ready = 1;
  return hipSuccess;
}

hipError_t tuned_predict(const TunedData& t, int precision, int N, int c0, int c1, int64_t e0, int64_t e1,
                         const Sched& sc, hipStream_t s) {
  if (precision == 0) return launch_predict_plain<double>(N, t.d64, e0, e1 - e0, sc, s);
  if (e1 - e0 < t.mc_min) return launch_predict_plain<float>(N, t.d32, e0, e1 - e0, sc, s);
  hipError_t st = pred_dispatch_any(precision, N, t.pc, t.a, e0, e1, sc, s);
  if (st != hipSuccess) return st;
  const int64_t f0 = t.fix_start[c0], nf = t.fix_start[c1 + 1] - f0;
  return fixup_dispatch(N, t.a, t.a.fix_list + f0, nf, s);
}

hipError_t tuned_correct(const TunedData& t, int precision, int N, int c0, int c1, int64_t e0, int64_t e1,
                         const Sched& sc, hipStream_t s) {
  if (precision == 0) return launch_correct_plain<double>(N, t.d64, e0, e1 - e0, sc, s);
  if (e1 - e0 < t.mc_min) return launch_correct_plain<float>(N, t.d32, e0, e1 - e0, sc, s);
  // second-half traces into the inbox of the clusters on the second step of
  // their pair (h2_list is ordered by cluster): one launch per run of such
  // clusters
  for (int c = c0; c <= c1;) {
    if (!((sc.sub >> c) & 1)) {
      ++c;
      continue;
    }
    int c2 = c;
    while (c2 + 1 <= c1 && ((sc.sub >> (c2 + 1)) & 1)) ++c2;
    const int64_t h0 = t.h2_start[c], nh = t.h2_start[c2 + 1] - h0;
    hipError_t st = h2_dispatch(N, t.a, t.a.h2_list + h0, nh, s);
    if (st != hipSuccess) return st;
    c = c2 + 1;
  }
  return corr_dispatch_any(precision, N, t.cc, t.a, e0, e1, s);
}


namespace {

// ---------------------------------------------------------------------------
// Autotuner: candidate launch configurations are timed on the largest
// cluster's matrix-core range; the winner is kept per (kernel sources, device,
// order, precision, size class) in a text cache, one line per key:
//   <key> <waves> <cap> <remap> <waves> <cap> <remap> <split> <variant>
// (predictor, corrector, the corrector's passes over its output rows, the
// predictor's shape: FP32 LDS or HBM park of I~, BF16 16x16x16 or 16x16x32
// products). The cache is $SEIS_TUNE_CACHE, else $HOME/.cache/seis/tune.txt.
// SEIS_TUNE=0 disables tuning; SEIS_TUNE=w,cap,remap,w,cap,remap[,split[,variant]]
// fixes the configuration.

std::string cache_path() {
  const char* e = std::getenv("SEIS_TUNE_CACHE");
  if (e && *e) return e;
  const char* home = std::getenv("HOME");
  if (!home || !*home) return "";
  const std::string dir = std::string(home) + "/.cache/seis";
  ::mkdir((std::string(home) + "/.cache").c_str(), 0755);
  ::mkdir(dir.c_str(), 0755);
  return dir + "/tune.txt";
}

std::string tune_key(const TunedData& t, int64_t ngroups) {
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  for (char& c : arch)
    if (c == ' ' || c == ':') c = '_';
  int lg = 0;
  while ((int64_t(1) << (lg + 1)) <= ngroups) ++lg;
  std::ostringstream k;
  k << "v4/" << SEIS_SOURCE_HASH << "/" << arch << "/cu" << num_cus() << "/N" << t.N << "/p" << t.precision
    << "/g" << lg;
  return k.str();
}

bool valid(const LaunchCfg& c) {
  return (c.waves == 2 || c.waves == 4) && c.cap >= 0 && c.cap <= 8 && (c.remap == 0 || c.remap == 1) &&
         (c.split == 1 || c.split == 2) && (c.variant == 0 || c.variant == 1);
}

bool parse_cfg(const std::string& txt, LaunchCfg& p, LaunchCfg& c) {
  std::string t = txt;
  std::replace(t.begin(), t.end(), ',', ' ');
  std::istringstream in(t);
  LaunchCfg a, b;
  if (!(in >> a.waves >> a.cap >> a.remap >> b.waves >> b.cap >> b.remap)) return false;
  int sp = 2, var = 0;
  if (in >> sp) {
    b.split = sp;
    if (in >> var) a.variant = var;
  }
  if (!valid(a) || !valid(b)) return false;
  p = a;
  c = b;
  return true;
}

// average ms of n launches of fn after one warm-up launch
template <class F>
hipError_t time_launch(F fn, hipStream_t s, int n, float& ms) {
  hipEvent_t a, b;
  hipError_t st = hipEventCreate(&a);
  if (st != hipSuccess) return st;
  st = hipEventCreate(&b);
  if (st != hipSuccess) {
    (void)hipEventDestroy(a);
    return st;
  }
  st = fn();
  if (st == hipSuccess) st = hipEventRecord(a, s);
  for (int i = 0; i < n && st == hipSuccess; ++i) st = fn();
  if (st == hipSuccess) st = hipEventRecord(b, s);
  if (st == hipSuccess) st = hipEventSynchronize(b);
  if (st == hipSuccess) st = hipEventElapsedTime(&ms, a, b);
  ms /= float(n);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return st;
}

}  // namespace

hipError_t tuned_autotune(TunedData& t, const Model& M, hipStream_t s) {
  if (t.precision == 0 || t.fixed) return hipSuccess;
  const char* env = std::getenv("SEIS_TUNE");
  if (env && std::strcmp(env, "0") == 0) return hipSuccess;
  if (env && *env && parse_cfg(env, t.pc, t.cc)) {
    t.source = 0;
    return hipSuccess;
  }
  // the largest cluster
  int cbest = -1;
  int64_t nbest = 0;
  for (int c = 0; c < M.C; ++c) {
    const int64_t n = M.cluster_start[c + 1] - M.cluster_start[c];
    if (n > nbest) {
      nbest = n;
      cbest = c;
    }
  }
  if (cbest < 0 || nbest < 16 || nbest < t.mc_min) return hipSuccess;
  const int64_t e0 = M.cluster_start[cbest], ei = M.cluster_start[cbest + 1];
  const int64_t ngroups = ((ei - 1) >> 4) - (e0 >> 4) + 1;
  const std::string key = tune_key(t, ngroups);
  const std::string path = cache_path();
  if (!path.empty()) {
    std::ifstream in(path);
    std::string line;
    LaunchCfg p, c;
    bool hit = false;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      if (!(ls >> k) || k != key) continue;
      std::string rest;
      std::getline(ls, rest);
      if (parse_cfg(rest, p, c)) hit = true;
    }
    if (hit) {
      t.pc = p;
      t.cc = c;
      t.source = 2;
      return hipSuccess;
    }
  }
  const int reps = 2;
  LaunchCfg bp = t.pc, bc = t.cc;
  float tp = 1e30f, tc = 1e30f;
  for (int w : {4, 2})
    for (int cap : {0, 1, 2, 4})
      for (int rm : {0, 1}) {
        const LaunchCfg c{w, cap, rm, 2, 0};
        float ms = 0.0f;
        // predictor: both shapes of the precision (see LaunchCfg::variant;
        // split BF16 has one)
        for (int var = 0; var < (t.precision == 3 ? 1 : 2) && cap <= 2; ++var) {
          LaunchCfg cv = c;
          cv.variant = var;
          hipError_t st = time_launch(
              [&]() { return pred_dispatch_any(t.precision, t.N, cv, t.a, e0, ei, Sched{}, s); }, s, reps, ms);
          if (st != hipSuccess) return st;
          if (ms < tp) {
            tp = ms;
            bp = cv;
          }
        }
        for (int sp : {2, 1}) {
          LaunchCfg cs = c;
          cs.split = sp;
          hipError_t st = time_launch(
              [&]() { return corr_dispatch_any(t.precision, t.N, cs, t.a, e0, ei, s); }, s, reps, ms);
          if (st != hipSuccess) return st;
          if (ms < tc) {
            tc = ms;
            bc = cs;
          }
        }
      }
  t.pc = bp;
  t.cc = bc;
  t.source = 1;
  if (!path.empty()) {
    std::ofstream out(path, std::ios::app);
    if (out) out << key << ' ' << bp.waves << ' ' << bp.cap << ' ' << bp.remap << ' ' << bc.waves << ' ' << bc.cap
                 << ' ' << bc.remap << ' ' << bc.split << ' ' << bp.variant << '\n';
  }
  return hipSuccess;
}

}  // namespace seis
