// Kernels of the spectral neural-operator surrogate (include/fno.h): a general
// strided batched matrix product on the BF16 matrix cores and the elementwise
// and reduction kernels of training.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "../../include/fno.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// eight consecutive BF16 values from LDS as two 8-byte reads (rows are 8-byte aligned)
__device__ __forceinline__ bf8 lds8(const unsigned short* p) {
  const s4 lo = *reinterpret_cast<const s4*>(p), hi = *reinterpret_cast<const s4*>(p + 4);
  const s8 v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  return __builtin_bit_cast(bf8, v);
}

__device__ __forceinline__ unsigned short to_bf16(float x) {
  unsigned int u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf / nan kept
  u += 0x7fffu + ((u >> 16) & 1u);                                           // nearest even
  return (unsigned short)(u >> 16);
}

struct GemmArgs {
  int64_t M, N, K;
  float alpha;
  const float* A;
  int64_t sAb, sAm, sAk;
  const float* B;
  int64_t sBb, sBk, sBn;
  float* C;
  int64_t sCb, sCm, sCn;
  int64_t tiles_n;  // ceil(N / 64)
  int64_t tiles_m;  // ceil(M / 64)
  int64_t kchunk;   // K range of one split (multiple of 32)
  int atomic;       // add into C atomically (split K; C pre-scaled by beta)
  float beta;       // C = alpha A B + beta C (without split K); 0: C is not read
};

constexpr int BM = 64, BN = 64, BK = 32, LDK = BK + 4;  // LDS rows padded (8-byte aligned fragments)

// 256 threads, 4 wavefronts, each a 32 x 32 quarter of the 64 x 64 tile as
// 2 x 2 products v_mfma_f32_16x16x32_bf16 of gfx950 per 32-wide K step (A lane
// l: row l%16, eight k values 8(l/16)..+7; B lane l: the same eight k values,
// column l%16; C lane l: rows 4(l/16)+v, column l%16). A and B place each k
// value in the same (lane group, register slot), so the products pair the
// right entries whatever order the instruction gives the slots. Tiles of A
// and B are staged in LDS as BF16, both with k contiguous. C tiles with a
// unit stride are written through LDS, so that consecutive threads store
// consecutive addresses, with beta applied in the same pass.
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ unsigned short sA[BM][LDK];
  __shared__ unsigned short sB[BN][LDK];
  __shared__ float sC[BM][BN + 1];  // the output tile, for row- or column-contiguous writes
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // work-group -> (batch, row tile, column tile), column tiles fastest
  const int64_t bx = blockIdx.x;
  const int64_t tn = bx % g.tiles_n, tm = (bx / g.tiles_n) % g.tiles_m, b = bx / (g.tiles_n * g.tiles_m);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int64_t k_begin = (int64_t)blockIdx.z * g.kchunk;
  const int64_t k_end = k_begin + g.kchunk < g.K ? k_begin + g.kchunk : g.K;
  const float* A = g.A + b * g.sAb;
  const float* Bp = g.B + b * g.sBb;
  const bool a_kfast = g.sAk == 1, b_nfast = g.sBn == 1 && g.sBk != 1;
  const int wm = w >> 1, wn = w & 1;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  for (int64_t k0 = k_begin; k0 < k_end; k0 += BK) {
    // stage A (64 x 32) and B (32 x 64): 8 values per thread each; consecutive
    // threads walk the unit-stride index so global reads coalesce
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int idx = tid + 256 * i;
      int mm, kk;
      if (a_kfast) { mm = idx >> 5; kk = idx & 31; } else { mm = idx & 63; kk = idx >> 6; }
      const int64_t m = m0 + mm, k = k0 + kk;
      const float x = (m < g.M && k < k_end) ? A[m * g.sAm + k * g.sAk] : 0.0f;
      sA[mm][kk] = to_bf16(x);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int idx = tid + 256 * i;
      int nn, kk;
      if (b_nfast) { nn = idx & 63; kk = idx >> 6; } else { nn = idx >> 5; kk = idx & 31; }
      const int64_t n = n0 + nn, k = k0 + kk;
      const float x = (n < g.N && k < k_end) ? Bp[k * g.sBk + n * g.sBn] : 0.0f;
      sB[nn][kk] = to_bf16(x);
    }
    __syncthreads();
    {
      bf8 af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = lds8(&sA[wm * 32 + i * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = lds8(&sB[wn * 32 + j * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  float* C = g.C + b * g.sCb;
  if (g.atomic || (g.sCn != 1 && g.sCm != 1)) {
    // split K (atomic adds into the pre-scaled C) or a C with no unit stride
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + v;
          const int64_t n = n0 + wn * 32 + j * 16 + (lane & 15);
          if (m >= g.M || n >= g.N) continue;
          float* c = C + m * g.sCm + n * g.sCn;
          const float x = g.alpha * acc[i][j][v];
          if (g.atomic) atomicAdd(c, x);
          else *c = g.beta == 0.0f ? x : x + g.beta * *c;
        }
    return;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) sC[wm * 32 + i * 16 + 4 * (lane >> 4) + v][wn * 32 + j * 16 + (lane & 15)] = acc[i][j][v];
  __syncthreads();
  const bool rows = g.sCn == 1;  // else sCm == 1: walk m fastest
#pragma unroll 4
  for (int it = 0; it < BM * BN / 256; ++it) {
    const int f = tid + 256 * it;
    const int r = rows ? f >> 6 : f & 63, c = rows ? f & 63 : f >> 6;
    const int64_t m = m0 + r, n = n0 + c;
    if (m >= g.M || n >= g.N) continue;
    float* p = C + m * g.sCm + n * g.sCn;
    const float x = g.alpha * sC[r][c];
    *p = g.beta == 0.0f ? x : x + g.beta * *p;
  }
}

// C *= beta over the strided batch (beta = 0 writes zeros).
__global__ void k_scale_c(int64_t batch, int64_t M, int64_t N, float* C, int64_t sCb, int64_t sCm, int64_t sCn,
                          float beta) {
  const int64_t total = batch * M * N;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = i % N, m = (i / N) % M, b = i / (M * N);
    float* c = C + b * sCb + m * sCm + n * sCn;
    *c = beta == 0.0f ? 0.0f : beta * *c;
  }
}

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

__global__ void k_bias_act(int64_t n_outer, int64_t C, int64_t S, float* z, const float* bias, float* a, int act) {
  const int64_t total = n_outer * C * S;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    float x = z[i];
    if (bias) {
      x += bias[(i / S) % C];
      z[i] = x;
    }
    a[i] = act ? gelu(x) : x;
  }
}

__global__ void k_gelu_bwd(int64_t n, const float* z, const float* da, float* dz) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dz[i] = da[i] * gelu_d(z[i]);
}

// The same two kernels four values at a time (16-byte accesses), for arrays
// whose rows of S values start on 16-byte boundaries: the bias of a row is
// read once instead of dividing every index by S.
__global__ void k_bias_act4(int64_t rows, int64_t C, int64_t S4, f4* z, const float* bias, f4* a, int act) {
  for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
    const float bb = bias ? bias[r % C] : 0.0f;
    f4* zr = z + r * S4;
    f4* ar = a + r * S4;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < S4; j += (int64_t)gridDim.x * blockDim.x) {
      f4 x = zr[j];
      if (bias) {
        x += bb;
        if (ar != zr) zr[j] = x;
      }
      if (act) x = f4{gelu(x[0]), gelu(x[1]), gelu(x[2]), gelu(x[3])};
      ar[j] = x;
    }
  }
}
__global__ void k_gelu_bwd4(int64_t n4, const f4* z, const f4* da, f4* dz) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
    const f4 x = z[i], d = da[i];
    dz[i] = f4{d[0] * gelu_d(x[0]), d[1] * gelu_d(x[1]), d[2] * gelu_d(x[2]), d[3] * gelu_d(x[3])};
  }
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// work-groups (channel c, part q of gridDim.y): each sums a strided share of
// the channel's n_outer x S values and adds it to db[c] (zeroed before)
__global__ __launch_bounds__(256) void k_channel_sum(int64_t n_outer, int64_t C, int64_t S, const float* dz,
                                                     float* db) {
  __shared__ float red[256];
  const int64_t c = blockIdx.x;
  const int64_t n = n_outer * S, stride = (int64_t)gridDim.y * 256;
  float s = 0.0f;
  for (int64_t i = (int64_t)blockIdx.y * 256 + threadIdx.x; i < n; i += stride) {
    const int64_t o = i / S, j = i - o * S;
    s += dz[(o * C + c) * S + j];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(db + c, red[0]);
}

__global__ void k_zero(int64_t n, float* x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.0f;
}

__global__ void k_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// one work-group per sample: |yhat - y|^2 and |y|^2, then the gradient
__global__ __launch_bounds__(256) void k_rel_l2(int64_t n, const float* yhat, const float* y, float* per,
                                                float* grad, float inv_batch) {
  __shared__ float r0[256], r1[256];
  const int64_t b = blockIdx.x;
  const float* yh = yhat + b * n;
  const float* yy = y + b * n;
  float se = 0.0f, sy = 0.0f;
  for (int64_t j = threadIdx.x; j < n; j += 256) {
    const float d = yh[j] - yy[j];
    se += d * d;
    sy += yy[j] * yy[j];
  }
  r0[threadIdx.x] = se;
  r1[threadIdx.x] = sy;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      r0[threadIdx.x] += r0[threadIdx.x + k];
      r1[threadIdx.x] += r1[threadIdx.x + k];
    }
    __syncthreads();
  }
  const float ne = sqrtf(r0[0]), ny = sqrtf(r1[0]);
  if (threadIdx.x == 0) per[b] = ne / ny;
  if (grad) {
    const float s = (ne > 0.0f ? inv_batch / (ne * ny) : 0.0f);
    for (int64_t j = threadIdx.x; j < n; j += 256) grad[b * n + j] = s * (yh[j] - yy[j]);
  }
}

__global__ void k_mean(int64_t n, const float* per, float* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.0f;
    for (int64_t i = 0; i < n; ++i) s += per[i];
    out[0] = s / float(n);
  }
}

__global__ void k_scale(int64_t n, float* x, float s) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] *= s;
}

unsigned grid_for(int64_t n, int per_block = 256) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

int status(hipError_t st) { return st == hipSuccess ? 0 : -3; }

}  // namespace

extern "C" {

int fno_gemm(int64_t batch, int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t sAb, int64_t sAm,
             int64_t sAk, const float* B, int64_t sBb, int64_t sBk, int64_t sBn, float beta, float* C, int64_t sCb,
             int64_t sCm, int64_t sCn, int split_k, void* stream) {
  if (batch < 0 || M < 0 || N < 0 || K < 0 || split_k < 1) return -1;
  if (batch == 0 || M == 0 || N == 0) return 0;
  if (!A || !B || !C) return -1;
  hipStream_t s = (hipStream_t)stream;
  const int64_t tiles_n = (N + BN - 1) / BN, tiles_m = (M + BM - 1) / BM;
  if (batch * tiles_n * tiles_m > (int64_t(1) << 31) - 1) return -1;
  int64_t kchunk = K > 0 ? (K + split_k - 1) / split_k : BK;
  kchunk = (kchunk + BK - 1) / BK * BK;
  const int64_t splits = K > 0 ? (K + kchunk - 1) / kchunk : 1;
  if (splits > 65535) return -1;
  // beta goes into the product's own write, except with split K (the splits
  // add atomically into C scaled beforehand) or without a product (K = 0)
  if (K == 0 || (splits > 1 && beta != 1.0f)) {
    hipLaunchKernelGGL(k_scale_c, dim3(grid_for(batch * M * N)), dim3(256), 0, s, batch, M, N, C, sCb, sCm, sCn, beta);
    if (hipGetLastError() != hipSuccess) return -3;
  }
  if (K == 0) return 0;
  GemmArgs g{M, N, K, alpha, A, sAb, sAm, sAk, B, sBb, sBk, sBn, C, sCb, sCm, sCn, tiles_n, tiles_m, kchunk,
             splits > 1 ? 1 : 0, beta};
  hipLaunchKernelGGL(k_gemm, dim3((unsigned)(batch * tiles_n * tiles_m), 1, (unsigned)splits), dim3(256), 0, s, g);
  return status(hipGetLastError());
}

int fno_bias_act(int64_t n_outer, int64_t C, int64_t S, float* z, const float* bias, float* a, int act,
                 void* stream) {
  if (n_outer < 0 || C <= 0 || S <= 0 || !z || !a) return -1;
  if (S % 4 == 0 && aligned16(z) && aligned16(a)) {
    const int64_t rows = n_outer * C;
    if (rows == 0) return 0;
    const dim3 grid(std::min<unsigned>(grid_for(S / 4), 2048u), (unsigned)std::min<int64_t>(rows, 65535));
    hipLaunchKernelGGL(k_bias_act4, grid, dim3(256), 0, (hipStream_t)stream, rows, C, S / 4, reinterpret_cast<f4*>(z),
                       bias, reinterpret_cast<f4*>(a), act);
    return status(hipGetLastError());
  }
  hipLaunchKernelGGL(k_bias_act, dim3(grid_for(n_outer * C * S)), dim3(256), 0, (hipStream_t)stream, n_outer, C, S,
                     z, bias, a, act);
  return status(hipGetLastError());
}

int fno_gelu_backward(int64_t n, const float* z, const float* da, float* dz, void* stream) {
  if (n < 0 || !z || !da || !dz) return -1;
  if (n % 4 == 0 && aligned16(z) && aligned16(da) && aligned16(dz)) {
    if (n == 0) return 0;
    hipLaunchKernelGGL(k_gelu_bwd4, dim3(grid_for(n / 4)), dim3(256), 0, (hipStream_t)stream, n / 4,
                       reinterpret_cast<const f4*>(z), reinterpret_cast<const f4*>(da), reinterpret_cast<f4*>(dz));
    return status(hipGetLastError());
  }
  hipLaunchKernelGGL(k_gelu_bwd, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, n, z, da, dz);
  return status(hipGetLastError());
}

int fno_channel_sum(int64_t n_outer, int64_t C, int64_t S, const float* dz, float* db, void* stream) {
  if (n_outer < 0 || C <= 0 || S <= 0 || !dz || !db) return -1;
  if (C > 65535) return -1;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero, dim3(grid_for(C)), dim3(256), 0, s, C, db);
  if (hipGetLastError() != hipSuccess) return -3;
  // enough parts per channel to fill the chip, each summing >= 16 values per thread
  const int64_t n = n_outer * S;
  const int64_t parts = std::max<int64_t>(1, std::min<int64_t>((2048 + C - 1) / C, (n + 4095) / 4096));
  hipLaunchKernelGGL(k_channel_sum, dim3((unsigned)C, (unsigned)parts), dim3(256), 0, s, n_outer, C, S, dz, db);
  return status(hipGetLastError());
}

int fno_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps, int t,
             void* stream) {
  if (n < 0 || t < 1 || !p || !g || !m || !v) return -1;
  const float c1 = 1.0f - std::pow(b1, (float)t), c2 = 1.0f - std::pow(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, n, p, g, m, v, lr, b1, b2, eps,
                     c1, c2);
  return status(hipGetLastError());
}

int fno_rel_l2(int64_t n_batch, int64_t n, const float* yhat, const float* y, float* loss, float* grad,
               void* stream) {
  if (n_batch <= 0 || n <= 0 || !yhat || !y || !loss) return -1;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_rel_l2, dim3((unsigned)n_batch), dim3(256), 0, s, n, yhat, y, loss + 1, grad,
                     1.0f / float(n_batch));
  if (hipGetLastError() != hipSuccess) return -3;
  hipLaunchKernelGGL(k_mean, dim3(1), dim3(64), 0, s, n_batch, loss + 1, loss);
  return status(hipGetLastError());
}

int fno_scale(int64_t n, float* x, float s, void* stream) {
  if (n < 0 || !x) return -1;
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, n, x, s);
  return status(hipGetLastError());
}

}  // extern "C"
