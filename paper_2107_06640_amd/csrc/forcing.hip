// Uplift forcing of prescribed-velocity faces (see forcing.hpp).
#include "forcing.hpp"

#include "layout.hpp"

namespace seis {

namespace {

__device__ inline double ramp(double s) {
  const double twopi = 6.283185307179586476925286766559;
  if (s <= 0.0) return 0.0;
  if (s >= 1.0) return 1.0;
  return s - sin(twopi * s) / twopi;
}

// one work-group per face: the time integral of 2 v_b at the rule's points,
// then its projection at the nodes
template <typename T>
__global__ __launch_bounds__(256) void k_forcing(ForcingArgs a, T* In, int64_t f0) {
  __shared__ double du[400];
  const int64_t f = f0 + blockIdx.x;
  const double t1 = (double(*a.macro) * a.macro_len + a.sub + 1) * a.dt_min;
  const double dt = a.dt[f], t0 = t1 - dt;
  const int n = int(a.src[0]);
  for (int q = threadIdx.x; q < a.nqf; q += blockDim.x) {
    const double x = a.xy[(f * a.nqf + q) * 2], y = a.xy[(f * a.nqf + q) * 2 + 1];
    double d = 0.0;
    for (int j = 0; j < n && j < kMaxUpliftSources; ++j) {
      const double* s = a.src + 1 + 5 * j;
      const double dx = x - s[1], dy = y - s[2];
      d += s[0] * exp(-(dx * dx + dy * dy) / (2.0 * s[3] * s[3])) * (ramp(t1 / s[4]) - ramp(t0 / s[4]));
    }
    du[q] = 2.0 * d / dt;
  }
  __syncthreads();
  const int64_t e = a.elem[f];
  const int fc = a.face[f];
  for (int i = threadIdx.x; i < a.Bf * 9; i += blockDim.x) {
    const int m = i / 9, p = i % 9;
    double v = 0.0;
    if (p == 8)
      for (int q = 0; q < a.nqf; ++q) v += a.proj[m * a.nqf + q] * du[q];
    In[inidx(e, fc, m, p, a.FT)] = (T)v;
  }
}

__global__ void k_tick(int64_t* macro) {
  if (threadIdx.x == 0) *macro += 1;
}

}  // namespace

template <typename T>
hipError_t launch_forcing(const ForcingArgs& a, T* In, int64_t f0, int64_t nf, int sub, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  ForcingArgs b = a;
  b.sub = sub;
  hipLaunchKernelGGL(k_forcing<T>, dim3((unsigned)nf), dim3(256), 0, s, b, In, f0);
  return hipGetLastError();
}

hipError_t launch_tick(int64_t* macro, hipStream_t s) {
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, s, macro);
  return hipGetLastError();
}

template hipError_t launch_forcing<double>(const ForcingArgs&, double*, int64_t, int64_t, int, hipStream_t);
template hipError_t launch_forcing<float>(const ForcingArgs&, float*, int64_t, int64_t, int, hipStream_t);

}  // namespace seis
