// Friction kernel of the dynamic-rupture faces (see fault.hpp).
#include "fault.hpp"

#include "elastic.hpp"
#include "layout.hpp"

namespace seis {

namespace {

// traction s n split into its normal and tangential parts, and the same for v
__device__ inline void split_state(const double* q, const double* n, double& sn, double* tt, double& vn,
                                   double* vt) {
  const double tx = q[0] * n[0] + q[3] * n[1] + q[5] * n[2];
  const double ty = q[3] * n[0] + q[1] * n[1] + q[4] * n[2];
  const double tz = q[5] * n[0] + q[4] * n[1] + q[2] * n[2];
  sn = tx * n[0] + ty * n[1] + tz * n[2];
  tt[0] = tx - sn * n[0];
  tt[1] = ty - sn * n[1];
  tt[2] = tz - sn * n[2];
  vn = q[6] * n[0] + q[7] * n[1] + q[8] * n[2];
  for (int d = 0; d < 3; ++d) vt[d] = q[6 + d] - vn * n[d];
}

// rate and state: the slip rate V in [0, T / eta] with
// T - eta V = sigma a asinh(V / (2 V0) e^(psi / a)), whose left side falls
// strictly with V; Newton steps kept inside a shrinking bracket (bisection
// where a step leaves it)
__device__ inline double rs_slip_rate(double T, double sigma, double eta, double psi, double a, double V0,
                                      double Vguess) {
  double lo = 0.0, hi = T / eta;
  const double c = exp(psi / a) / (2.0 * V0);
  double V = fmin(fmax(Vguess, lo), hi);
  for (int it = 0; it < 100; ++it) {
    const double x = c * V;
    const double g = T - eta * V - sigma * a * asinh(x);
    if (g > 0.0) lo = V; else hi = V;
    const double dg = -eta - sigma * a * c / sqrt(1.0 + x * x);
    double Vn = V - g / dg;
    if (!(Vn > lo && Vn < hi)) Vn = 0.5 * (lo + hi);
    if (fabs(Vn - V) <= 1e-15 * fmax(fabs(V), 1e-300) || hi - lo <= 1e-15 * fmax(hi, 1e-300)) {
      V = Vn;
      break;
    }
    V = Vn;
  }
  return V;
}

__device__ inline double rs_steady_state(double V, const double* r) {
  // r: a, b, L, V0, f0, f_w, V_w
  const double fLV = r[4] - (r[1] - r[0]) * log(V / r[3]);
  const double q = V / r[6], q2 = q * q, q4 = q2 * q2;
  const double fss = r[5] + (fLV - r[5]) / pow(1.0 + q4 * q4, 0.125);
  return r[0] * log(2.0 * r[3] / V * sinh(fss / r[0]));
}

// one work-group of kFaultThreads per fault face: the two elements' stored
// derivatives are staged in LDS with contiguous reads, their traces at the
// nodes formed by all threads, then thread m applies the law at node m
constexpr int kFaultThreads = 256;

template <typename T, int N>
__global__ __launch_bounds__(kFaultThreads) void k_fault(FaultArgs a, const T* gD, T* In, int64_t f0) {
  constexpr int B = nbasis(N), Bf = nface(N), FT = row_tiles(Bf);
  constexpr int ND = (N + 1) * B * 9;      // stored values per element
  __shared__ T sd[2][ND];                  // derivatives D~k of the two sides
  __shared__ double tr[2][N + 1][Bf][9];   // their traces at the nodes
  const int64_t f = f0 + blockIdx.x;
  const int64_t em = a.elem[f], ep = a.pelem[f];
  const int fm = a.face[f], fp = a.pface[f], h = a.perm[f];
  const T* Dm = gD + (int64_t)a.dslot[em] * ND;
  const T* Dp = gD + (int64_t)a.dslot[ep] * ND;
  for (int i = threadIdx.x; i < ND; i += blockDim.x) {
    sd[0][i] = Dm[i];
    sd[1][i] = Dp[i];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 2 * (N + 1) * Bf * 9; i += blockDim.x) {
    const int side = i / ((N + 1) * Bf * 9), r = i % ((N + 1) * Bf * 9);
    const int k = r / (Bf * 9), m = (r / 9) % Bf, p = r % 9;
    const int node = side == 0 ? m : a.pinv[h * Bf + m];
    const double* Em = a.E + ((int64_t)(side == 0 ? fm : fp) * Bf + node) * B;
    const T* D = &sd[side][k * B * 9 + p];
    double acc = 0.0;
#pragma unroll 8
    for (int l = 0; l < B; ++l) acc += Em[l] * (double)D[l * 9];
    tr[side][k][m][p] = acc;
  }
  __syncthreads();
  const int m = threadIdx.x;
  if (m >= Bf) return;
  const double* g = a.geo + f * 8;
  const double n[3] = {g[0], g[1], g[2]};
  const double zpm = g[3], zsm = g[4], zpp = g[5], zsp = g[6], dt = g[7];
  const double* pr = a.par + f * kFaultParams;
  const double s0 = pr[0];
  const double t0n = pr[1] * n[0] + pr[2] * n[1] + pr[3] * n[2];
  const double tau0[3] = {pr[1] - t0n * n[0], pr[2] - t0n * n[1], pr[3] - t0n * n[2]};
  const double mu_s = pr[4], mu_d = pr[5], dc = pr[6], coh = pr[7];
  const bool rate_state = pr[15] == double(kLawRateState);
  const double eta = zsm * zsp / (zsm + zsp);
  double* st = a.state + (f * Bf + m) * kFaultState;
  double slip[3] = {st[0], st[1], st[2]}, psi = st[3];
  double V[3] = {st[4], st[5], st[6]}, Tb[3] = {0.0, 0.0, 0.0}, Stot = 0.0;  // V: the last slip rate
  double as = 0.0, avn = 0.0, atau[3] = {0.0, 0.0, 0.0}, avm[3] = {0.0, 0.0, 0.0}, avp[3] = {0.0, 0.0, 0.0};
  // a real loop over the time points, the traces re-read from LDS in each
  // (an opaque offset keeps them from being hoisted into registers for the
  // whole loop, which would cost the occupancy of the trace phase)
#pragma unroll 1
  for (int j = 0; j <= N; ++j) {
    const double tj = a.tq[j], wj = a.tw[j];
    int z = 0;
    asm volatile("" : "+s"(z));
    const double* t0 = &tr[0][0][m][0] + z;
    const double* t1 = &tr[1][0][m][0] + z;
    double qm[9], qp[9];
    for (int p = 0; p < 9; ++p) {
      double x = 0.0, y = 0.0, pw = 1.0;
      for (int k = 0; k <= N; ++k) {  // q(t) = sum_k D~k (t / dt)^k
        x += pw * t0[k * Bf * 9 + p];
        y += pw * t1[k * Bf * 9 + p];
        pw *= tj;
      }
      qm[p] = x;
      qp[p] = y;
    }
    double snm, ttm[3], vnm, vtm[3], snp, ttp[3], vnp, vtp[3];
    split_state(qm, n, snm, ttm, vnm, vtm);
    split_state(qp, n, snp, ttp, vnp, vtp);
    const double s = (zpp * snm + zpm * snp + zpm * zpp * (vnp - vnm)) / (zpm + zpp);
    const double vn = (zpm * vnm + zpp * vnp + snp - snm) / (zpm + zpp);
    double lock[3], Ttot[3];
    for (int d = 0; d < 3; ++d) {
      lock[d] = eta * (ttm[d] / zsm + ttp[d] / zsp + vtp[d] - vtm[d]);
      Ttot[d] = tau0[d] + lock[d];
    }
    Stot = s0 + s;
    const double mag = sqrt(Ttot[0] * Ttot[0] + Ttot[1] * Ttot[1] + Ttot[2] * Ttot[2]);
    bool slips;
    double ratio;
    if (rate_state) {
      // always sliding, at the rate-dependent strength
      const double v = rs_slip_rate(mag, fmax(0.0, -Stot), eta, psi, pr[4], pr[7],
                                    sqrt(V[0] * V[0] + V[1] * V[1] + V[2] * V[2]));
      slips = true;
      ratio = mag > 0.0 ? (mag - eta * v) / mag : 1.0;
    } else {
      // below the strength the point is locked: tau = tau_lock, V = 0 exactly
      const double fr = mu_s - (mu_s - mu_d) * fmin(psi / dc, 1.0);
      const double strength = coh + fr * fmax(0.0, -Stot);
      slips = mag > strength;
      ratio = slips ? strength / mag : 1.0;
    }
    double speed2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      Tb[d] = ratio * Ttot[d];
      const double tau = slips ? Tb[d] - tau0[d] : lock[d];
      V[d] = slips ? (lock[d] - tau) / eta : 0.0;
      speed2 += V[d] * V[d];
      atau[d] += wj * tau;
      avm[d] += wj * (vtm[d] + (tau - ttm[d]) / zsm);
      avp[d] += wj * (vtp[d] - (tau - ttp[d]) / zsp);
      slip[d] += wj * dt * V[d];
    }
    as += wj * s;
    avn += wj * vn;
    const double speed = sqrt(speed2);
    if (!rate_state) {
      psi += wj * dt * speed;
    } else if (speed > 0.0) {
      const double pss = rs_steady_state(speed, pr + 4);
      psi = pss + (psi - pss) * exp(-speed * wj * dt / pr[6]);
    }
  }
  for (int d = 0; d < 3; ++d) {
    st[d] = slip[d];
    st[4 + d] = V[d];
    st[7 + d] = Tb[d];
  }
  st[3] = psi;
  st[10] = Stot;
  // time-averaged middle states: stress s n n + tau n + n tau, velocity vn n + v_t
  double sig[6];
  sig[0] = as * n[0] * n[0] + 2.0 * atau[0] * n[0];
  sig[1] = as * n[1] * n[1] + 2.0 * atau[1] * n[1];
  sig[2] = as * n[2] * n[2] + 2.0 * atau[2] * n[2];
  sig[3] = as * n[0] * n[1] + atau[0] * n[1] + atau[1] * n[0];
  sig[4] = as * n[1] * n[2] + atau[1] * n[2] + atau[2] * n[1];
  sig[5] = as * n[0] * n[2] + atau[0] * n[2] + atau[2] * n[0];
  const int mr = a.pinv[h * Bf + m];
  for (int p = 0; p < 6; ++p) {
    In[inidx(em, fm, m, p, FT)] = (T)sig[p];
    In[inidx(ep, fp, mr, p, FT)] = (T)sig[p];
  }
  for (int d = 0; d < 3; ++d) {
    In[inidx(em, fm, m, 6 + d, FT)] = (T)(avn * n[d] + avm[d]);
    In[inidx(ep, fp, mr, 6 + d, FT)] = (T)(avn * n[d] + avp[d]);
  }
}

}  // namespace

template <typename T>
hipError_t launch_fault(int N, const FaultArgs& a, const T* gD, T* In, int64_t f0, int64_t nf, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  if (!a.elem || !a.face || !a.pelem || !a.pface || !a.perm || !a.geo || !a.par || !a.state || !a.E || !a.pinv ||
      !a.dslot || !a.tq || !a.tw || !gD || !In)
    return hipErrorInvalidValue;
  switch (N) {
#define SEIS_F(NN) \
  case NN: hipLaunchKernelGGL((k_fault<T, NN>), dim3((unsigned)nf), dim3(kFaultThreads), 0, s, a, gD, In, f0); break;
    SEIS_F(1) SEIS_F(2) SEIS_F(3) SEIS_F(4) SEIS_F(5) SEIS_F(6)
#undef SEIS_F
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_fault<double>(int, const FaultArgs&, const double*, double*, int64_t, int64_t, hipStream_t);
template hipError_t launch_fault<float>(int, const FaultArgs&, const float*, float*, int64_t, int64_t, hipStream_t);

}  // namespace seis
