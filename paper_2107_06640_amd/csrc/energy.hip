// Energy of the coupled system and L2 norms of the fields.
//
// The velocity-stress system with the gravitational sea surface (Sec. 3)
// conserves E = sum_K int_K (rho |v|^2 / 2 + W(s)) + int_surface rho g eta^2 / 2,
// with W the strain energy (s:s - lambda/(3 lambda + 2 mu) (tr s)^2) / (4 mu) of
// an elastic element and p^2 / (2 lambda), p = -tr s / 3, of an acoustic one.
// The basis is orthonormal on the reference element, so the integral of a
// quadratic form of q over K is |det J| times the sum of that form over the
// modal rows, and the surface term is 2 A sum_q w_q rho g eta_q^2 / 2 with the
// face rule of the eta points (weights summing to 1/2).
//
// One wavefront takes one 16-element group (lane el + 16 g holds rows
// 16 t + 4 v + g of element el, the layout of the state), a work-group of four
// wavefronts strides over the groups and then over the gravity faces, and
// leaves its kEnergyValues sums in a partial-sum buffer; one more work-group
// adds the partial sums in a fixed order, so the result is reproducible.
#include <mutex>

#include "energy.hpp"
#include "layout.hpp"

namespace seis {

namespace {

// Partial sums of the energy of callers that cannot allocate: one array per
// GPU for the life of the process, shared by every call on that GPU.
__device__ __align__(256) double scratch[kEnergyScratchValues];

constexpr int kDevices = 64;
double* g_scratch_ptr[kDevices] = {};
std::mutex g_scratch_mu;

constexpr int kThreads = 256;

__device__ __forceinline__ double warp_sum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// out values: [0] total, [1] volume (kinetic + strain), [2] surface, [3 + p] int q_p^2
template <typename T>
__global__ __launch_bounds__(kThreads) void k_energy_partial(EnergyData d, const T* Q, double* partial) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int el = lane & 15, g = lane >> 4;
  const int RT = row_tiles(d.B);
  const int64_t ngroups = (d.E + 15) >> 4;
  double acc[kEnergyValues];
  for (int i = 0; i < kEnergyValues; ++i) acc[i] = 0.0;
  for (int64_t grp = int64_t(blockIdx.x) * 4 + w; grp < ngroups; grp += int64_t(gridDim.x) * 4) {
    const int64_t e = grp * 16 + el;
    if (e >= d.E) continue;  // the padding elements of the last group
    double s2[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, tr2 = 0.0;
    for (int t = 0; t < RT; ++t)
      for (int v = 0; v < 4; ++v) {
        if (16 * t + 4 * v + g >= d.B) continue;
        const T* q = Q + (((grp * RT + t) * 4 + v) * 9) * 64 + lane;
        double x[9];
        for (int p = 0; p < 9; ++p) {
          x[p] = (double)q[p * 64];
          s2[p] += x[p] * x[p];
        }
        const double tr = x[0] + x[1] + x[2];
        tr2 += tr * tr;
      }
    const double lam = d.lmr[e * 3 + 0], mu = d.lmr[e * 3 + 1], rho = d.lmr[e * 3 + 2], J = d.absdet[e];
    const double ss = s2[0] + s2[1] + s2[2] + 2.0 * (s2[3] + s2[4] + s2[5]);
    const double W = mu > 0.0 ? (ss - lam / (3.0 * lam + 2.0 * mu) * tr2) / (4.0 * mu) : tr2 / (18.0 * lam);
    acc[1] += J * (0.5 * rho * (s2[6] + s2[7] + s2[8]) + W);
    for (int p = 0; p < 9; ++p) acc[3 + p] += J * s2[p];
  }
  for (int64_t f = int64_t(blockIdx.x) * kThreads + threadIdx.x; f < d.Fg; f += int64_t(gridDim.x) * kThreads) {
    double s = 0.0;
    for (int q = 0; q < d.nq; ++q) {
      const double h = d.eta[f * d.nq + q];
      s += d.tw[q] * h * h;
    }
    acc[2] += d.gcoef[f] * s;
  }
  __shared__ double red[4][kEnergyValues];
  for (int i = 1; i < kEnergyValues; ++i) {
    const double x = warp_sum(acc[i]);
    if (lane == 0) red[w][i] = x;
  }
  __syncthreads();
  if (threadIdx.x < kEnergyValues) {
    const int i = threadIdx.x;
    double x = 0.0;
    if (i > 0) x = red[0][i] + red[1][i] + red[2][i] + red[3][i];
    partial[int64_t(blockIdx.x) * kEnergyValues + i] = x;
  }
}

__global__ __launch_bounds__(kThreads) void k_energy_final(const double* partial, int groups, double* out) {
  __shared__ double red[kThreads / 64][kEnergyValues];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = 1; i < kEnergyValues; ++i) {
    double x = 0.0;
    for (int b = threadIdx.x; b < groups; b += kThreads) x += partial[int64_t(b) * kEnergyValues + i];
    x = warp_sum(x);
    if (lane == 0) red[w][i] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double v[kEnergyValues];
    for (int i = 1; i < kEnergyValues; ++i) v[i] = red[0][i] + red[1][i] + red[2][i] + red[3][i];
    v[0] = v[1] + v[2];
    for (int i = 0; i < kEnergyValues; ++i) out[i] = v[i];
  }
}

}  // namespace

int energy_groups(int64_t E) {
  const int64_t ngroups = (E + 15) >> 4;
  const int64_t want = (ngroups + 3) / 4;
  return int(want < 1 ? 1 : (want > kEnergyMaxGroups ? kEnergyMaxGroups : want));
}

hipError_t launch_energy(const EnergyData& d, const double* Q64, const float* Q32, double* partial, double* out,
                         hipStream_t s) {
  const int groups = energy_groups(d.E);
  if (Q64)
    hipLaunchKernelGGL(k_energy_partial<double>, dim3(groups), dim3(kThreads), 0, s, d, Q64, partial);
  else
    hipLaunchKernelGGL(k_energy_partial<float>, dim3(groups), dim3(kThreads), 0, s, d, Q32, partial);
  hipError_t st = hipGetLastError();
  if (st != hipSuccess) return st;
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kThreads), 0, s, partial, groups, out);
  return hipGetLastError();
}

hipError_t energy_scratch_init() {
  int dev = 0;
  hipError_t st = hipGetDevice(&dev);
  if (st != hipSuccess) return st;
  if (dev < 0 || dev >= kDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return hipSuccess;
  void* p = nullptr;
  st = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (st != hipSuccess) return st;
  g_scratch_ptr[dev] = static_cast<double*>(p);
  return hipSuccess;
}

double* energy_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[dev];
}

}  // namespace seis
