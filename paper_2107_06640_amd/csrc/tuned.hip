// Tuned element kernels on the CDNA4 matrix cores.
//
// A wavefront updates 16 elements. Every contraction with a reference matrix
// shared by all elements (stiffness K^d, face traces E_f, lifts L_f) is a
// matrix-core product C[16 x 16] += A[16 x k] B[k x 16] with the reference
// matrix as A (staged in LDS once per work-group) and the 16 elements as the
// 16 columns of B, one product per quantity. The element data stays in the
// output-fragment layout of those products (lane el + 16 g holds rows
// 16t + 4g + v of element el), which is directly the B-operand layout of the
// next product once the K index of A is permuted the same way, so the chain
// of contractions needs no data shuffles. Per-element 9x9 work (scaled star
// matrices, Godunov flux at the face nodes) is lane-local VALU work in FP32.
//
// Operand precisions: FP32 (v_mfma_f32_16x16x4_f32, K step of 4 rows) and
// BF16 (v_mfma_f32_16x16x16_bf16, K step of 16 rows); accumulation and the
// element state are FP32 in both.
//
// Algorithm (Sec. 4.1 and 4.2), scaled derivatives Dk = dt^k/k! d^kQ/dt^k:
//   predictor  D(k+1) = -1/(k+1) sum_d (K^d)^T (Dk (dt A*_d)^T)
//              I~ = sum_k Dk/(k+1)
//              Q += sum_d K^d (I~ (dt A*_d)^T) - sum_f L_f flux(E_f I~, own trace)
//              traces E_f I~ handed to the neighbours
//   corrector  Q -= sum_f L_f flux(neighbour trace)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>

#include "elastic.hpp"
#include "layout.hpp"
#include "tuned.hpp"

namespace seis {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

struct OpF32 {};
struct OpBF16 {};

template <int N>
struct Dim {
  static constexpr int B = nbasis(N), Bf = nface(N), B1 = nbasis(N - 1);
  static constexpr int RT = row_tiles(B), FT = row_tiles(Bf), RT1 = row_tiles(B1);
  static constexpr int nK = 3 * B * B1, nE = 4 * Bf * B, nL = 4 * B * Bf;
};

__host__ __device__ inline unsigned short f2bf(float x) {
  // round to nearest even
  unsigned int u;
  std::memcpy(&u, &x, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ s4 pack4(float a, float b, float c, float d) {
  s4 r;
  r[0] = (short)f2bf(a);
  r[1] = (short)f2bf(b);
  r[2] = (short)f2bf(c);
  r[3] = (short)f2bf(d);
  return r;
}

// (A_e u)_p for e = x, y, z: the three Jacobians of the velocity-stress
// system applied to a state u, component p.
template <int p>
__device__ __forceinline__ void flux_comp(const float* u, float lam, float mu, float rinv, float& ux, float& uy,
                                          float& uz) {
  const float l2m = lam + 2.0f * mu;
  if constexpr (p == 0) { ux = -l2m * u[6]; uy = -lam * u[7]; uz = -lam * u[8]; }
  if constexpr (p == 1) { ux = -lam * u[6]; uy = -l2m * u[7]; uz = -lam * u[8]; }
  if constexpr (p == 2) { ux = -lam * u[6]; uy = -lam * u[7]; uz = -l2m * u[8]; }
  if constexpr (p == 3) { ux = -mu * u[7]; uy = -mu * u[6]; uz = 0.0f; }
  if constexpr (p == 4) { ux = 0.0f; uy = -mu * u[8]; uz = -mu * u[7]; }
  if constexpr (p == 5) { ux = -mu * u[8]; uy = 0.0f; uz = -mu * u[6]; }
  if constexpr (p == 6) { ux = -rinv * u[0]; uy = -rinv * u[3]; uz = -rinv * u[5]; }
  if constexpr (p == 7) { ux = -rinv * u[3]; uy = -rinv * u[1]; uz = -rinv * u[4]; }
  if constexpr (p == 8) { ux = -rinv * u[5]; uy = -rinv * u[4]; uz = -rinv * u[2]; }
}

// Godunov flux A-hat^-(n) q^b at one face node (Sec. 4.2), with the middle
// state a linear map of the given trace: c = n_x, n_y, n_z, then the eight
// scaled coefficients of (s_n^b, v_n^b) from (s_n, v_n) and (t_t^b, v_t^b)
// from (t_t, v_t).
__device__ __forceinline__ void node_flux(const float* c, float lam, float mu, float rinv, const float* in,
                                          float* out) {
  const float nx = c[0], ny = c[1], nz = c[2];
  const float tx = in[0] * nx + in[3] * ny + in[5] * nz;
  const float ty = in[3] * nx + in[1] * ny + in[4] * nz;
  const float tz = in[5] * nx + in[4] * ny + in[2] * nz;
  const float sn = tx * nx + ty * ny + tz * nz;
  const float ttx = tx - sn * nx, tty = ty - sn * ny, ttz = tz - sn * nz;
  const float vn = in[6] * nx + in[7] * ny + in[8] * nz;
  const float vtx = in[6] - vn * nx, vty = in[7] - vn * ny, vtz = in[8] - vn * nz;
  const float snb = c[3] * sn + c[4] * vn;
  const float vnb = c[5] * sn + c[6] * vn;
  const float tbx = c[7] * ttx + c[8] * vtx, tby = c[7] * tty + c[8] * vty, tbz = c[7] * ttz + c[8] * vtz;
  const float vbx = c[9] * ttx + c[10] * vtx, vby = c[9] * tty + c[10] * vty, vbz = c[9] * ttz + c[10] * vtz;
  const float w = 2.0f * vnb;
  out[0] = -(lam * vnb + mu * (w * nx * nx + 2.0f * vbx * nx));
  out[1] = -(lam * vnb + mu * (w * ny * ny + 2.0f * vby * ny));
  out[2] = -(lam * vnb + mu * (w * nz * nz + 2.0f * vbz * nz));
  out[3] = -mu * (w * nx * ny + vbx * ny + vby * nx);
  out[4] = -mu * (w * ny * nz + vby * nz + vbz * ny);
  out[5] = -mu * (w * nx * nz + vbx * nz + vbz * nx);
  out[6] = -rinv * (snb * nx + tbx);
  out[7] = -rinv * (snb * ny + tby);
  out[8] = -rinv * (snb * nz + tbz);
}

template <class Op>
using RefT = typename std::conditional<std::is_same<Op, OpF32>::value, float, unsigned short>::type;

// A(i, k) of a stored reference block: row-major R[i][k] (TR = false) or
// R[k][i] (TR = true), ld columns, ni x nk entries. Indices are clamped into
// the block: clamped entries only meet zero B values or feed output rows that
// are discarded.
template <bool TR, class RT_>
__device__ __forceinline__ RT_ aref(const RT_* R, int ld, int ni, int nk, int i, int k) {
  i = min(i, ni - 1);
  k = min(k, nk - 1);
  return TR ? R[k * ld + i] : R[i * ld + k];
}

// acc[mt][p] += sum_k A(16 mt + el, k) X[k][p] over the input rows k < nrows,
// X held per lane as x[t][v][p] (row 16t + 4g + v).
template <class Op, bool TR, int NT, int MT, int P>
__device__ __forceinline__ void contract(f4 (&acc)[MT][P], const RefT<Op>* R, int ld, int ni, int nk,
                                         const float (&x)[NT][4][P], int nrows, int el, int g) {
  if constexpr (std::is_same<Op, OpF32>::value) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (16 * t + v >= nrows) continue;
        const int k = 16 * t + 4 * g + v;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const float a = aref<TR>(R, ld, ni, nk, 16 * mt + el, k);
#pragma unroll
          for (int p = 0; p < P; ++p) acc[mt][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, x[t][v][p], acc[mt][p], 0, 0, 0);
        }
      }
  } else {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (16 * t >= nrows) continue;
      const int k0 = 16 * t + 4 * g;
      s4 b[P];
#pragma unroll
      for (int p = 0; p < P; ++p) b[p] = pack4(x[t][0][p], x[t][1][p], x[t][2][p], x[t][3][p]);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        s4 a;
#pragma unroll
        for (int j = 0; j < 4; ++j) a[j] = (short)aref<TR>(R, ld, ni, nk, 16 * mt + el, k0 + j);
#pragma unroll
        for (int p = 0; p < P; ++p) acc[mt][p] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[p], acc[mt][p], 0, 0, 0);
      }
    }
  }
}

// dq[mt][p] += sum_l A(16 mt + el, l) (dt A*_d I~[l])_p over l < nrows: the
// star product of each input row is formed on the fly (lane-local) right
// before it enters the matrix core, so it is never stored for all rows.
template <class Op, int NT, int MT>
__device__ __forceinline__ void contract_star(f4 (&acc)[MT][9], const RefT<Op>* R, int ld, int ni, int nk,
                                              const float (&x)[NT][4][9], int nrows, const float* Gd, float lam,
                                              float mu, float rinv, int el, int g) {
  if constexpr (std::is_same<Op, OpF32>::value) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (16 * t + v >= nrows) continue;
        const int k = 16 * t + 4 * g + v;
        float z[9];
        apply_star(Gd[0], Gd[1], Gd[2], lam, mu, rinv, x[t][v], z);
        const bool ok = k < nrows;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const float a = aref<false>(R, ld, ni, nk, 16 * mt + el, k);
#pragma unroll
          for (int p = 0; p < 9; ++p)
            acc[mt][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, ok ? z[p] : 0.0f, acc[mt][p], 0, 0, 0);
        }
      }
  } else {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (16 * t >= nrows) continue;
      const int k0 = 16 * t + 4 * g;
      float z[4][9];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        apply_star(Gd[0], Gd[1], Gd[2], lam, mu, rinv, x[t][v], z[v]);
        if (k0 + v >= nrows)
#pragma unroll
          for (int p = 0; p < 9; ++p) z[v][p] = 0.0f;
      }
      s4 b[9];
#pragma unroll
      for (int p = 0; p < 9; ++p) b[p] = pack4(z[0][p], z[1][p], z[2][p], z[3][p]);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        s4 a;
#pragma unroll
        for (int j = 0; j < 4; ++j) a[j] = (short)aref<false>(R, ld, ni, nk, 16 * mt + el, k0 + j);
#pragma unroll
        for (int p = 0; p < 9; ++p) acc[mt][p] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[p], acc[mt][p], 0, 0, 0);
      }
    }
  }
}

// One Cauchy-Kowalevski step: D(K+1) from D(K), output quantity by quantity.
template <class Op, int N, int K, int RTI, int RTO>
__device__ __forceinline__ void ck_step(const float (&din)[RTI][4][9], float (&dout)[RTO][4][9],
                                        const RefT<Op>* sK, const float* G, float lam, float mu, float rinv,
                                        int el, int g) {
  constexpr int B = nbasis(N), B1 = nbasis(N - 1);
  constexpr int nin = nbasis(N - K), nout = nbasis(N - K - 1);
  const float fk = -1.0f / float(K + 1);
  auto body = [&](auto pc) {
    constexpr int p = decltype(pc)::value;
    f4 acc[RTO][1];
#pragma unroll
    for (int mt = 0; mt < RTO; ++mt) acc[mt][0] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      // z = (dt A*_d D(K))_p for the rows this lane holds
      float z[RTI][4][1];
#pragma unroll
      for (int t = 0; t < RTI; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float ux, uy, uz;
          flux_comp<p>(din[t][v], lam, mu, rinv, ux, uy, uz);
          z[t][v][0] = G[3 * d + 0] * ux + G[3 * d + 1] * uy + G[3 * d + 2] * uz;
        }
      // A(m, l) = K^d[l][m]: stored block K^d[l < B][m < B1]
      contract<Op, true, RTI, RTO, 1>(acc, sK + d * B * B1, B1, B1, B, z, nin, el, g);
    }
#pragma unroll
    for (int mt = 0; mt < RTO; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * mt + 4 * g + v;
        dout[mt][v][p] = row < nout ? fk * acc[mt][0][v] : 0.0f;
      }
  };
  body(std::integral_constant<int, 0>{});
  body(std::integral_constant<int, 1>{});
  body(std::integral_constant<int, 2>{});
  body(std::integral_constant<int, 3>{});
  body(std::integral_constant<int, 4>{});
  body(std::integral_constant<int, 5>{});
  body(std::integral_constant<int, 6>{});
  body(std::integral_constant<int, 7>{});
  body(std::integral_constant<int, 8>{});
}

// accumulate I~ += D(K+1)/(K+2)
template <int RT, int RTO>
__device__ __forceinline__ void accum(float (&I)[RT][4][9], const float (&d)[RTO][4][9], float w) {
#pragma unroll
  for (int t = 0; t < RTO; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int p = 0; p < 9; ++p) I[t][v][p] += w * d[t][v][p];
}

// store a derivative (rows held in x, zero beyond) for the gravity kernel
template <int N, int RTX>
__device__ __forceinline__ void store_deriv(float* dst, const float (&x)[RTX][4][9], int g) {
  constexpr int B = nbasis(N), RT = row_tiles(B);
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * t + 4 * g + v;
      if (row >= B) continue;
#pragma unroll
      for (int p = 0; p < 9; ++p) dst[row * 9 + p] = (t < RTX) ? x[t < RTX ? t : 0][v][p] : 0.0f;
    }
}

template <class Op, int N>
struct CK {
  // Runs the whole CK chain; I (holding D0 on entry) ends as I~.
  __device__ static void run(float (&I)[row_tiles(nbasis(N))][4][9], const RefT<Op>* sK, const float* G, float lam,
                             float mu, float rinv, int el, int g, float* gd) {
    constexpr int R0 = row_tiles(nbasis(N)), R1 = row_tiles(nbasis(N - 1));
    float d1[R1][4][9];
    if (gd) store_deriv<N>(gd, I, g);
    ck_step<Op, N, 0, R0, R1>(I, d1, sK, G, lam, mu, rinv, el, g);
    if (gd) store_deriv<N>(gd + 1 * nbasis(N) * 9, d1, g);
    accum(I, d1, 0.5f);
    if constexpr (N >= 2) {
      constexpr int R2 = row_tiles(nbasis(N - 2));
      float d2[R2][4][9];
      ck_step<Op, N, 1, R1, R2>(d1, d2, sK, G, lam, mu, rinv, el, g);
      if (gd) store_deriv<N>(gd + 2 * nbasis(N) * 9, d2, g);
      accum(I, d2, 1.0f / 3.0f);
      if constexpr (N >= 3) {
        constexpr int R3 = row_tiles(nbasis(N - 3));
        float d3[R3][4][9];
        ck_step<Op, N, 2, R2, R3>(d2, d3, sK, G, lam, mu, rinv, el, g);
        if (gd) store_deriv<N>(gd + 3 * nbasis(N) * 9, d3, g);
        accum(I, d3, 0.25f);
        if constexpr (N >= 4) {
          constexpr int R4 = row_tiles(nbasis(N - 4));
          float d4[R4][4][9];
          ck_step<Op, N, 3, R3, R4>(d3, d4, sK, G, lam, mu, rinv, el, g);
          if (gd) store_deriv<N>(gd + 4 * nbasis(N) * 9, d4, g);
          accum(I, d4, 0.2f);
          if constexpr (N >= 5) {
            constexpr int R5 = row_tiles(nbasis(N - 5));
            float d5[R5][4][9];
            ck_step<Op, N, 4, R4, R5>(d4, d5, sK, G, lam, mu, rinv, el, g);
            if (gd) store_deriv<N>(gd + 5 * nbasis(N) * 9, d5, g);
            accum(I, d5, 1.0f / 6.0f);
            if constexpr (N >= 6) {
              constexpr int R6 = row_tiles(nbasis(N - 6));
              float d6[R6][4][9];
              ck_step<Op, N, 5, R5, R6>(d5, d6, sK, G, lam, mu, rinv, el, g);
              if (gd) store_deriv<N>(gd + 6 * nbasis(N) * 9, d6, g);
              accum(I, d6, 1.0f / 7.0f);
            }
          }
        }
      }
    }
  }
};

template <class Op, int N, int W>
__global__ __launch_bounds__(64 * W) void k_predict_tuned(TArgs a, int64_t e0, int64_t e1, int parity) {
  using D = Dim<N>;
  constexpr int B = D::B, Bf = D::Bf, B1 = D::B1, RT = D::RT, FT = D::FT, RT1 = D::RT1;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  using R = RefT<Op>;
  R* sK = reinterpret_cast<R*>(lds_raw);
  R* sE = sK + D::nK;
  R* sL = sE + D::nE;
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.ref);
    uint32_t* dst = reinterpret_cast<uint32_t*>(lds_raw);
    const int n32 = a.ref_bytes / 4;
    for (int i = threadIdx.x; i < n32; i += 64 * W) dst[i] = src[i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, el = lane & 15, g = lane >> 4;
  const int64_t grp = (e0 >> 4) + (int64_t)blockIdx.x * W + w;
  if (grp > ((e1 - 1) >> 4)) return;
  const int64_t e = grp * 16 + el;
  const bool live = e >= e0 && e < e1;
  const int64_t ec = live ? e : e0;

  float G[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) G[i] = a.G[ec * 9 + i];
  const float lam = a.mat[ec * 3 + 0], mu = a.mat[ec * 3 + 1], rinv = a.mat[ec * 3 + 2];

  // load Q (one coalesced 256-byte access per register)
  float I[RT][4][9];
  const float* Qg = a.Q + grp * (int64_t)(RT * 36 * 64);
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const bool ok = 16 * t + 4 * g + v < B;
#pragma unroll
      for (int p = 0; p < 9; ++p) I[t][v][p] = ok ? Qg[((t * 4 + v) * 9 + p) * 64 + lane] : 0.0f;
    }

  const int gs = live ? a.gslot[e] : -1;
  float* gd = gs >= 0 ? a.gD + (int64_t)gs * (N + 1) * B * 9 : nullptr;
  CK<Op, N>::run(I, sK, G, lam, mu, rinv, el, g, gd);

  f4 dq[RT][9];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int p = 0; p < 9; ++p) dq[t][p] = f4{0.f, 0.f, 0.f, 0.f};

  // volume: dq += sum_d K^d (I~ (dt A*_d)^T), rows of I~ below B1
#pragma unroll
  for (int d = 0; d < 3; ++d)
    contract_star<Op, RT, RT>(dq, sK + d * B * B1, B1, B, B1, I, B1, G + 3 * d, lam, mu, rinv, el, g);

  // faces: traces at the nodes, hand-over, own-trace flux, lift
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    f4 va[FT][9];
#pragma unroll
    for (int t = 0; t < FT; ++t)
#pragma unroll
      for (int p = 0; p < 9; ++p) va[t][p] = f4{0.f, 0.f, 0.f, 0.f};
    contract<Op, false, RT, FT, 9>(va, sE + f * Bf * B, B, Bf, B, I, B, el, g);
    float V[FT][4][9];
#pragma unroll
    for (int t = 0; t < FT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const bool ok = 16 * t + 4 * g + v < Bf;
#pragma unroll
        for (int p = 0; p < 9; ++p) V[t][v][p] = ok ? va[t][p][v] : 0.0f;
      }
    const int md = live ? a.mode[ec * 4 + f] : 0;
    if (md != 0) {
      const int32_t tg = a.tgt[ec * 4 + f];
      const int h = a.hperm[ec * 4 + f];
#pragma unroll
      for (int t = 0; t < FT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int node = 16 * t + 4 * g + v;
          if (node >= Bf) continue;
          const int mr = a.pinv[h * Bf + node];
#pragma unroll
          for (int p = 0; p < 9; ++p) {
            float* dst = a.In + inidx(tg >> 2, tg & 3, mr, p, FT);
            if (md == 1) *dst = V[t][v][p];
            else *dst = parity ? *dst + 0.5f * V[t][v][p] : 0.5f * V[t][v][p];
          }
        }
    }
    float c[11];
#pragma unroll
    for (int i = 0; i < 11; ++i) c[i] = a.RCm[(ec * 4 + f) * 12 + i];
#pragma unroll
    for (int t = 0; t < FT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float out[9];
        node_flux(c, lam, mu, rinv, V[t][v], out);
#pragma unroll
        for (int p = 0; p < 9; ++p) V[t][v][p] = -out[p];
      }
    contract<Op, false, FT, RT, 9>(dq, sL + f * B * Bf, Bf, B, Bf, V, Bf, el, g);
  }

  // Q += dq
  if (live) {
    float* Qw = a.Q + grp * (int64_t)(RT * 36 * 64);
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (16 * t + 4 * g + v >= B) continue;
#pragma unroll
        for (int p = 0; p < 9; ++p) {
          const int idx = ((t * 4 + v) * 9 + p) * 64 + lane;
          Qw[idx] += dq[t][p][v];
        }
      }
  }
}

template <class Op, int N, int W>
__global__ __launch_bounds__(64 * W) void k_correct_tuned(TArgs a, int64_t e0, int64_t e1) {
  using D = Dim<N>;
  constexpr int B = D::B, Bf = D::Bf, RT = D::RT, FT = D::FT;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  using R = RefT<Op>;
  R* sL = reinterpret_cast<R*>(lds_raw);
  {
    // only the lifts are needed: they sit after K and E in the reference block
    const uint32_t* src = reinterpret_cast<const uint32_t*>(
        reinterpret_cast<const unsigned char*>(a.ref) + (D::nK + D::nE) * sizeof(R));
    uint32_t* dst = reinterpret_cast<uint32_t*>(lds_raw);
    const int n32 = (D::nL * (int)sizeof(R) + 3) / 4;
    for (int i = threadIdx.x; i < n32; i += 64 * W) dst[i] = src[i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, el = lane & 15, g = lane >> 4;
  const int64_t grp = (e0 >> 4) + (int64_t)blockIdx.x * W + w;
  if (grp > ((e1 - 1) >> 4)) return;
  const int64_t e = grp * 16 + el;
  const bool live = e >= e0 && e < e1;
  const int64_t ec = live ? e : e0;
  const float lam = a.mat[ec * 3 + 0], mu = a.mat[ec * 3 + 1], rinv = a.mat[ec * 3 + 2];

  f4 dq[RT][9];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int p = 0; p < 9; ++p) dq[t][p] = f4{0.f, 0.f, 0.f, 0.f};

#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const float* Ig = a.In + ((grp * 4 + f) * (int64_t)(FT * 36 * 64));
    float c[11];
#pragma unroll
    for (int i = 0; i < 11; ++i) c[i] = a.RCp[(ec * 4 + f) * 12 + i];
    float V[FT][4][9];
#pragma unroll
    for (int t = 0; t < FT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float in[9], out[9];
#pragma unroll
        for (int p = 0; p < 9; ++p) in[p] = Ig[((t * 4 + v) * 9 + p) * 64 + lane];
        node_flux(c, lam, mu, rinv, in, out);
        const bool ok = 16 * t + 4 * g + v < Bf;
#pragma unroll
        for (int p = 0; p < 9; ++p) V[t][v][p] = ok ? -out[p] : 0.0f;
      }
    contract<Op, false, FT, RT, 9>(dq, sL + f * B * Bf, Bf, B, Bf, V, Bf, el, g);
  }
  if (live) {
    float* Qw = a.Q + grp * (int64_t)(RT * 36 * 64);
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (16 * t + 4 * g + v >= B) continue;
#pragma unroll
        for (int p = 0; p < 9; ++p) {
          const int idx = ((t * 4 + v) * 9 + p) * 64 + lane;
          Qw[idx] += dq[t][p][v];
        }
      }
  }
}

template <class Op, int N>
int ref_bytes() {
  return (Dim<N>::nK + Dim<N>::nE + Dim<N>::nL) * (int)sizeof(RefT<Op>);
}

template <class Op, int N, int W>
hipError_t launch_pred(const TArgs& a, int64_t e0, int64_t e1, int parity, hipStream_t s) {
  if (e1 <= e0) return hipSuccess;
  const int64_t ng = ((e1 - 1) >> 4) - (e0 >> 4) + 1;
  const unsigned grid = (unsigned)((ng + W - 1) / W);
  const int lds = (ref_bytes<Op, N>() + 3) / 4 * 4;
  static bool attr = false;
  if (!attr) {
    hipError_t st = hipFuncSetAttribute((const void*)k_predict_tuned<Op, N, W>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (st != hipSuccess) return st;
    attr = true;
  }
  hipLaunchKernelGGL((k_predict_tuned<Op, N, W>), dim3(grid), dim3(64 * W), lds, s, a, e0, e1, parity);
  return hipGetLastError();
}

template <class Op, int N, int W>
hipError_t launch_corr(const TArgs& a, int64_t e0, int64_t e1, hipStream_t s) {
  if (e1 <= e0) return hipSuccess;
  const int64_t ng = ((e1 - 1) >> 4) - (e0 >> 4) + 1;
  const unsigned grid = (unsigned)((ng + W - 1) / W);
  const int lds = (Dim<N>::nL * (int)sizeof(RefT<Op>) + 3) / 4 * 4;
  static bool attr = false;
  if (!attr) {
    hipError_t st = hipFuncSetAttribute((const void*)k_correct_tuned<Op, N, W>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (st != hipSuccess) return st;
    attr = true;
  }
  hipLaunchKernelGGL((k_correct_tuned<Op, N, W>), dim3(grid), dim3(64 * W), lds, s, a, e0, e1);
  return hipGetLastError();
}

template <class Op>
hipError_t pred_dispatch(int N, int W, const TArgs& a, int64_t e0, int64_t e1, int parity, hipStream_t s) {
#define SEIS_P(NN, WW) \
  if (N == NN && W == WW) return launch_pred<Op, NN, WW>(a, e0, e1, parity, s);
  SEIS_P(2, 1) SEIS_P(2, 2) SEIS_P(2, 4)
  SEIS_P(3, 1) SEIS_P(3, 2) SEIS_P(3, 4)
  SEIS_P(4, 1) SEIS_P(4, 2) SEIS_P(4, 4)
  SEIS_P(5, 1) SEIS_P(5, 2) SEIS_P(5, 4)
  SEIS_P(6, 1) SEIS_P(6, 2) SEIS_P(6, 4)
#undef SEIS_P
  return hipErrorInvalidValue;
}

template <class Op>
hipError_t corr_dispatch(int N, int W, const TArgs& a, int64_t e0, int64_t e1, hipStream_t s) {
#define SEIS_C(NN, WW) \
  if (N == NN && W == WW) return launch_corr<Op, NN, WW>(a, e0, e1, s);
  SEIS_C(2, 1) SEIS_C(2, 2) SEIS_C(2, 4)
  SEIS_C(3, 1) SEIS_C(3, 2) SEIS_C(3, 4)
  SEIS_C(4, 1) SEIS_C(4, 2) SEIS_C(4, 4)
  SEIS_C(5, 1) SEIS_C(5, 2) SEIS_C(5, 4)
  SEIS_C(6, 1) SEIS_C(6, 2) SEIS_C(6, 4)
#undef SEIS_C
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

}  // namespace

hipError_t tuned_build(TunedData& t, const Model& M, int precision, const DevData<double>& d64,
                       const DevData<float>& d32, int tile, std::vector<void*>& owned, int64_t& bytes) {
  t.N = M.N;
  t.precision = precision;
  t.d64 = d64;
  t.d32 = d32;
  t.iface_start = M.iface_start;
  t.waves = tile > 0 ? std::max(1, std::min(4, tile / 16)) : 4;
  if (t.waves == 3) t.waves = 2;
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
  a.gslot = d32.gslot;
  a.gD = d32.gD;
  float *rcm, *rcp;
  int32_t* pinv;
  hipError_t st = upload(owned, bytes, &rcm, M.RCm);
  if (st == hipSuccess) st = upload(owned, bytes, &rcp, M.RCp);
  if (st == hipSuccess) st = upload(owned, bytes, &pinv, M.ref.pinv);
  if (st != hipSuccess) return st;
  a.RCm = rcm;
  a.RCp = rcp;
  a.pinv = pinv;
  // reference block: K^d[k < B][l < B1] for d = 0..2, E_f, L_f
  const int B = M.B, Bf = M.Bf, B1 = n_basis(M.N - 1);
  std::vector<double> ref;
  for (int d = 0; d < 3; ++d)
    for (int k = 0; k < B; ++k)
      for (int l = 0; l < B1; ++l) ref.push_back(M.ref.K[(d * B + k) * B + l]);
  ref.insert(ref.end(), M.ref.E.begin(), M.ref.E.end());
  ref.insert(ref.end(), M.ref.L.begin(), M.ref.L.end());
  if (precision == 1) {
    float* r;
    st = upload(owned, bytes, &r, ref);
    a.ref = r;
    a.ref_bytes = int(ref.size() * sizeof(float));
  } else {
    std::vector<unsigned short> rb(ref.size());
    for (size_t i = 0; i < ref.size(); ++i) rb[i] = f2bf((float)ref[i]);
    if (rb.size() % 2) rb.push_back(0);
    unsigned short* r;
    st = upload(owned, bytes, &r, rb);
    a.ref = r;
    a.ref_bytes = int(rb.size() * sizeof(unsigned short));
  }
  if (st != hipSuccess) return st;
  t.ready = 1;
  return hipSuccess;
}

hipError_t tuned_predict(const TunedData& t, int precision, int N, int64_t e0, int64_t ei, int64_t e1, int parity,
                         hipStream_t s) {
  if (precision == 0) return launch_predict_plain<double>(N, t.d64, e0, e1 - e0, parity, s);
  hipError_t st = precision == 1 ? pred_dispatch<OpF32>(N, t.waves, t.a, e0, ei, parity, s)
                                 : pred_dispatch<OpBF16>(N, t.waves, t.a, e0, ei, parity, s);
  if (st != hipSuccess) return st;
  return launch_predict_plain<float>(N, t.d32, ei, e1 - ei, parity, s);
}

hipError_t tuned_correct(const TunedData& t, int precision, int N, int64_t e0, int64_t ei, int64_t e1, int parity,
                         hipStream_t s) {
  if (precision == 0) return launch_correct_plain<double>(N, t.d64, e0, e1 - e0, parity, s);
  hipError_t st = precision == 1 ? corr_dispatch<OpF32>(N, t.waves, t.a, e0, ei, s)
                                 : corr_dispatch<OpBF16>(N, t.waves, t.a, e0, ei, s);
  if (st != hipSuccess) return st;
  return launch_correct_plain<float>(N, t.d32, ei, e1 - ei, parity, s);
}

}  // namespace seis
