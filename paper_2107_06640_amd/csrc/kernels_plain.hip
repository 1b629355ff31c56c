// Plain element kernels: one work-group per element, every contraction a
// loop over shared memory and reference matrices read from global memory.
// They are the straightforward form of the update (the baseline the tuned
// kernels are measured against) and serve FP64 and FP32.
//
// Predictor (Sec. 4.1, Taylor expansion and Cauchy-Kowalevski procedure),
// with scaled derivatives Dk = dt^k/k! d^kQ/dt^k:
//   D0 = Q,  D(k+1) = -1/(k+1) sum_d (K^d)^T Dk (dt A*_d)^T
//   I~ = I/dt = sum_k Dk/(k+1)
// Element-local corrector part (Sec. 4.1 semi-discrete form; Sec. 4.2 flux):
//   Q += sum_d K^d I~ (dt A*_d)^T - sum_i L_i (F~-_i (E_i I~))
// where E_i evaluates traces at the face nodes and L_i lifts nodal values.
// Neighbour part (corrector): Q -= sum_i L_i (F~+_i In_i).
#include "device.hpp"
#include "elastic.hpp"
#include "layout.hpp"

namespace seis {

namespace {

// Threads per element: 256 for throughput; a launch over a few elements (a
// tiny LTS cluster) is bound by the latency of one work-group, so it uses 1024.
// The thread count is a launch parameter of one compiled kernel, not a
// template argument, so that an element's arithmetic (and its rounding) is
// the same whichever launch covers it.
constexpr int NT_WIDE = 256, NT_TALL = 1024, TALL_BELOW = 256;

template <typename T, int N>
__global__ __launch_bounds__(NT_TALL) void k_predict_plain(DevData<T> d, int64_t e0, Sched sc) {
  const int NT = blockDim.x;
  constexpr int B = nbasis(N), Bf = nface(N);
  constexpr int B1 = nbasis(N - 1);
  constexpr int RT = row_tiles(B), FT = row_tiles(Bf);
  const int64_t e = e0 + blockIdx.x;
  const int parity = sc.parity(e);
  const int tid = threadIdx.x;
  __shared__ T sD[B * 9], sI[B * 9], sIh[B * 9];
  __shared__ T sY[3 * B * 9];  // reused for the volume term
  __shared__ T sV[4 * Bf * 9], sVh[4 * Bf * 9];
  __shared__ T sG[9], sM[3];
  if (tid < 9) sG[tid] = d.G[e * 9 + tid];
  if (tid < 3) sM[tid] = d.mat[e * 3 + tid];
  const int gs = d.dslot[e];
  T* gD = gs >= 0 ? d.gD + (int64_t)gs * (N + 1) * B * 9 : nullptr;
  for (int i = tid; i < B * 9; i += NT) {
    const T q = d.Q[qidx(e, i / 9, i % 9, RT)];
    sD[i] = q;
    sI[i] = q;
    sIh[i] = q;
    if (gD) gD[i] = q;
  }
  __syncthreads();
  const T lam = sM[0], mu = sM[1], rinv = sM[2];
  T half = T(0.5);
  for (int k = 0; k < N; ++k) {
    const int nin = nbasis(N - k), nout = nbasis(N - k - 1);
    // Y_d = (K^d)^T D_k restricted to the non-zero rows
    for (int i = tid; i < 3 * nout * 9; i += NT) {
      const int dd = i / (nout * 9), m = (i / 9) % nout, r = i % 9;
      const T* Kd = d.K + (size_t)dd * B * B;
      T acc = T(0);
#pragma unroll 8
      for (int l = 0; l < nin; ++l) acc += Kd[l * B + m] * sD[l * 9 + r];
      sY[(dd * B + m) * 9 + r] = acc;
    }
    __syncthreads();
    const T f = T(-1) / T(k + 1);
    for (int i = tid; i < nout * 9; i += NT) {
      const int m = i / 9, p = i % 9;
      T wx[9], wy[9], wz[9];
      for (int r = 0; r < 9; ++r) {
        const T y0 = sY[(0 * B + m) * 9 + r], y1 = sY[(1 * B + m) * 9 + r], y2 = sY[(2 * B + m) * 9 + r];
        wx[r] = sG[0] * y0 + sG[3] * y1 + sG[6] * y2;
        wy[r] = sG[1] * y0 + sG[4] * y1 + sG[7] * y2;
        wz[r] = sG[2] * y0 + sG[5] * y1 + sG[8] * y2;
      }
      const T v = f * grad_op(p, lam, mu, rinv, wx, wy, wz);
      sD[i] = v;
      sI[i] += v / T(k + 2);
      sIh[i] += v * half / T(k + 2);
      if (gD) gD[(k + 1) * B * 9 + i] = v;
    }
    if (gD)
      for (int i = nout * 9 + tid; i < B * 9; i += NT) gD[(k + 1) * B * 9 + i] = T(0);
    half *= T(0.5);
    __syncthreads();
  }
  // traces at the face nodes: full step and first half step
  for (int i = tid; i < 4 * Bf * 9; i += NT) {
    const int f = i / (Bf * 9), m = (i / 9) % Bf, p = i % 9;
    const T* Em = d.Ef + ((size_t)f * Bf + m) * B;
    T a = T(0), b = T(0);
#pragma unroll 8
    for (int l = 0; l < B; ++l) {
      a += Em[l] * sI[l * 9 + p];
      b += Em[l] * sIh[l * 9 + p];
    }
    sV[i] = a;
    sVh[i] = b;
  }
  __syncthreads();
  // hand the traces to the neighbours (in their node numbering)
  for (int i = tid; i < 4 * Bf * 9; i += NT) {
    const int f = i / (Bf * 9), m = (i / 9) % Bf, p = i % 9;
    const int md = d.mode[e * 4 + f];
    if (md == 0) continue;
    const int32_t t = d.tgt[e * 4 + f];
    const int src = d.perm[d.hperm[e * 4 + f] * Bf + m];
    const T v = sV[(f * Bf + src) * 9 + p];
    T* dst = d.In + inidx(t >> 2, t & 3, m, p, FT);
    if (md == 1) {
      *dst = v;
    } else if (md == 2) {
      const T h1 = sVh[(f * Bf + src) * 9 + p];  // first half-step integral over the receiver's dt
      *dst = h1;
      d.H2[((int64_t)d.half2[e * 4 + f] * Bf + m) * 9 + p] = T(2) * v - h1;
    } else {
      *dst = parity ? *dst + T(0.5) * v : T(0.5) * v;
    }
  }
  // local flux at the nodes: F~-_f V_f (in place into sVh)
  __syncthreads();
  for (int i = tid; i < 4 * Bf * 9; i += NT) {
    const int f = i / (Bf * 9), m = (i / 9) % Bf, p = i % 9;
    const T* F = d.Fm + ((e * 4 + f) * 81 + p * 9);
    T a = T(0);
    for (int r = 0; r < 9; ++r) a += F[r] * sV[(f * Bf + m) * 9 + r];
    sVh[i] = a;
  }
  // volume: Z_d[l] = (dt A*_d) I~[l] for l < B1
  for (int i = tid; i < 3 * B1; i += NT) {
    const int dd = i / B1, l = i % B1;
    T out[9];
    apply_star(sG[dd * 3 + 0], sG[dd * 3 + 1], sG[dd * 3 + 2], lam, mu, rinv, &sI[l * 9], out);
    for (int p = 0; p < 9; ++p) sY[(dd * B + l) * 9 + p] = out[p];
  }
  __syncthreads();
  for (int i = tid; i < B * 9; i += NT) {
    const int kk = i / 9, p = i % 9;
    T acc = T(0);
    for (int dd = 0; dd < 3; ++dd) {
      const T* Kd = d.K + ((size_t)dd * B + kk) * B;
#pragma unroll 8
      for (int l = 0; l < B1; ++l) acc += Kd[l] * sY[(dd * B + l) * 9 + p];
    }
    for (int f = 0; f < 4; ++f) {
      const T* L = d.Lf + ((size_t)f * B + kk) * Bf;
#pragma unroll 8
      for (int m = 0; m < Bf; ++m) acc -= L[m] * sVh[(f * Bf + m) * 9 + p];
    }
    d.Q[qidx(e, kk, p, RT)] += acc;
  }
}

template <typename T, int N>
__global__ __launch_bounds__(NT_TALL) void k_correct_plain(DevData<T> d, int64_t e0, Sched sc) {
  const int NT = blockDim.x;
  constexpr int B = nbasis(N), Bf = nface(N);
  constexpr int RT = row_tiles(B), FT = row_tiles(Bf);
  const int64_t e = e0 + blockIdx.x;
  const int parity = sc.parity(e);
  const int tid = threadIdx.x;
  __shared__ T sW[4 * Bf * 9];
  for (int i = tid; i < 4 * Bf * 9; i += NT) {
    const int f = i / (Bf * 9), m = (i / 9) % Bf, p = i % 9;
    const int h2 = d.rhalf2[e * 4 + f];
    const T* F = d.Fp + ((e * 4 + f) * 81 + p * 9);
    T a = T(0);
    if (parity && h2 >= 0) {
      const T* src = d.H2 + ((int64_t)h2 * Bf + m) * 9;
      for (int r = 0; r < 9; ++r) a += F[r] * src[r];
    } else {
      for (int r = 0; r < 9; ++r) a += F[r] * d.In[inidx(e, f, m, r, FT)];
    }
    sW[i] = a;
  }
  __syncthreads();
  for (int i = tid; i < B * 9; i += NT) {
    const int kk = i / 9, p = i % 9;
    T acc = T(0);
    for (int f = 0; f < 4; ++f) {
      const T* L = d.Lf + ((size_t)f * B + kk) * Bf;
#pragma unroll 8
      for (int m = 0; m < Bf; ++m) acc += L[m] * sW[(f * Bf + m) * 9 + p];
    }
    d.Q[qidx(e, kk, p, RT)] -= acc;
  }
}

// Gravity face (Sec. 4.3): per point, the forcing f = v_n + p/Z of the
// predicted solution (p = -n.s.n), the ODE d eta/dt = f - a eta, dH/dt = eta
// integrated exactly through its Taylor series over the element's step, and
// the time-integrated boundary flux (stress rows -lambda (eta1 - eta0),
// velocity rows g H n) lifted with the face rule.
template <typename T, int N>
__global__ __launch_bounds__(256) void k_gravity(DevData<T> d, const int32_t* glist) {
  constexpr int B = nbasis(N);
  constexpr int RT = row_tiles(B);
  constexpr int nq = (N + 1) * (N + 1);
  const int gf = glist[blockIdx.x];
  const int tid = threadIdx.x;
  const int64_t e = d.g_elem[gf];
  const int face = d.g_face[gf];
  const double* par = d.g_par + gf * 8;
  const double scale = par[0], nx = par[1], ny = par[2], nz = par[3], Z = par[4], a = par[5], lam = par[6],
               dt = par[7];
  __shared__ T sD[(N + 1) * B * 9];
  __shared__ double sFm[nq][N + 1];
  __shared__ double sF[nq][2];
  // the element's scaled time derivatives, staged once (coalesced)
  const T* D = d.gD + (int64_t)gf * (N + 1) * B * 9;
  for (int i = tid; i < (N + 1) * B * 9; i += 256) sD[i] = D[i];
  __syncthreads();
  // trace of each derivative at each surface point: one (point, order) pair per thread
  for (int w = tid; w < nq * (N + 1); w += 256) {
    const int q = w / (N + 1), m = w % (N + 1);
    const double* Eq = d.Eg + ((size_t)face * nq + q) * B;
    double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 8
    for (int l = 0; l < B; ++l) {
      const double el = Eq[l];
#pragma unroll
      for (int p = 0; p < 9; ++p) v[p] += el * (double)sD[(m * B + l) * 9 + p];
    }
    const double tx = v[0] * nx + v[3] * ny + v[5] * nz;
    const double ty = v[3] * nx + v[1] * ny + v[4] * nz;
    const double tz = v[5] * nx + v[4] * ny + v[2] * nz;
    const double pm = -(tx * nx + ty * ny + tz * nz);
    sFm[q][m] = v[6] * nx + v[7] * ny + v[8] * nz + pm / Z;
  }
  __syncthreads();
  for (int q = tid; q < nq; q += 256) {
    const double eta0 = d.eta[(int64_t)gf * nq + q];
    double em = eta0, eta1 = eta0, H = eta0 * dt;
    for (int m = 0; m < N + 24; ++m) {
      const double fm = m <= N ? sFm[q][m] : 0.0;
      em = dt / (m + 1) * (fm - a * em);
      eta1 += em;
      H += em * dt / (m + 2);
    }
    d.eta[(int64_t)gf * nq + q] = eta1;
    sF[q][0] = -lam * (eta1 - eta0);
    sF[q][1] = d.g * H;
  }
  __syncthreads();
  // lift: rows of the three normal stresses (p < 3) and the velocities (p >= 6)
  const double nrm[3] = {nx, ny, nz};
  for (int i = tid; i < B * 6; i += 256) {
    const int kk = i / 6, j = i % 6;
    const int p = j < 3 ? j : j + 3;
    const double* Lq = d.Lg + ((size_t)face * B + kk) * nq;
    double acc = 0.0;
    if (p < 3) {
#pragma unroll 8
      for (int q = 0; q < nq; ++q) acc += Lq[q] * sF[q][0];
    } else {
#pragma unroll 8
      for (int q = 0; q < nq; ++q) acc += Lq[q] * sF[q][1] * nrm[p - 6];
    }
    d.Q[qidx(e, kk, p, RT)] -= (T)(scale * acc);
  }
}

template <typename T, int N>
hipError_t pred_n(const DevData<T>& d, int64_t e0, int64_t ne, const Sched& sc, hipStream_t s) {
  if (ne <= 0) return hipSuccess;
  if (ne < TALL_BELOW)
    hipLaunchKernelGGL((k_predict_plain<T, N>), dim3((unsigned)ne), dim3(NT_TALL), 0, s, d, e0, sc);
  else
    hipLaunchKernelGGL((k_predict_plain<T, N>), dim3((unsigned)ne), dim3(NT_WIDE), 0, s, d, e0, sc);
  return hipGetLastError();
}
template <typename T, int N>
hipError_t corr_n(const DevData<T>& d, int64_t e0, int64_t ne, const Sched& sc, hipStream_t s) {
  if (ne <= 0) return hipSuccess;
  if (ne < TALL_BELOW)
    hipLaunchKernelGGL((k_correct_plain<T, N>), dim3((unsigned)ne), dim3(NT_TALL), 0, s, d, e0, sc);
  else
    hipLaunchKernelGGL((k_correct_plain<T, N>), dim3((unsigned)ne), dim3(NT_WIDE), 0, s, d, e0, sc);
  return hipGetLastError();
}
template <typename T, int N>
hipError_t grav_n(const DevData<T>& d, const int32_t* glist, int64_t ng, hipStream_t s) {
  if (ng <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_gravity<T, N>), dim3((unsigned)ng), dim3(256), 0, s, d, glist);
  return hipGetLastError();
}

}  // namespace

#define SEIS_DISPATCH(FN, ...)                  \
  switch (N) {                                  \
    case 1: return FN<T, 1>(__VA_ARGS__);       \
    case 2: return FN<T, 2>(__VA_ARGS__);       \
    case 3: return FN<T, 3>(__VA_ARGS__);       \
    case 4: return FN<T, 4>(__VA_ARGS__);       \
    case 5: return FN<T, 5>(__VA_ARGS__);       \
    case 6: return FN<T, 6>(__VA_ARGS__);       \
    case 7: return FN<T, 7>(__VA_ARGS__);       \
    default: return hipErrorInvalidValue;       \
  }

template <typename T>
hipError_t launch_predict_plain(int N, const DevData<T>& d, int64_t e0, int64_t ne, const Sched& sc, hipStream_t s) {
  SEIS_DISPATCH(pred_n, d, e0, ne, sc, s)
}
template <typename T>
hipError_t launch_correct_plain(int N, const DevData<T>& d, int64_t e0, int64_t ne, const Sched& sc, hipStream_t s) {
  SEIS_DISPATCH(corr_n, d, e0, ne, sc, s)
}
template <typename T>
hipError_t launch_gravity(int N, const DevData<T>& d, const int32_t* glist, int64_t ng, hipStream_t s) {
  SEIS_DISPATCH(grav_n, d, glist, ng, s)
}

template hipError_t launch_predict_plain<double>(int, const DevData<double>&, int64_t, int64_t, const Sched&,
                                                 hipStream_t);
template hipError_t launch_predict_plain<float>(int, const DevData<float>&, int64_t, int64_t, const Sched&,
                                                hipStream_t);
template hipError_t launch_correct_plain<double>(int, const DevData<double>&, int64_t, int64_t, const Sched&,
                                                 hipStream_t);
template hipError_t launch_correct_plain<float>(int, const DevData<float>&, int64_t, int64_t, const Sched&,
                                                hipStream_t);
template hipError_t launch_gravity<double>(int, const DevData<double>&, const int32_t*, int64_t, hipStream_t);
template hipError_t launch_gravity<float>(int, const DevData<float>&, const int32_t*, int64_t, hipStream_t);

}  // namespace seis
