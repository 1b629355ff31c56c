/*
 * fno.h -- C ABI of the spectral neural-operator kernels (BF16 operands on the
 * CDNA4 matrix cores, FP32 accumulation and FP32 storage).
 *
 * The learned surrogate maps a seafloor uplift field to the sea-surface
 * height eta(x, y, t) that the solver of seis.h computes. The paper motivates the map, not the network:
 * one-way linked tsunami models take the seafloor uplift as their input
 * (Sec. 2), and its benchmark's linked reference is driven by the recorded
 * seafloor displacement (Sec. 6.1). The network is a Fourier neural operator: pointwise
 * lift, spectral layers v <- GELU(K v + W v + b) whose K is a truncated 3-D
 * Fourier transform, a per-mode complex channel mixing and the inverse
 * transform, then a pointwise projection. Every transform and mixing step is
 * a (batched) matrix product, so the library exports one general strided
 * batched product plus the elementwise kernels; the network code composes
 * them (paper_2107_06640_amd/fno.py).
 *
 * All pointers are device pointers (FP32 unless stated), owned by the
 * caller; the stream is a hipStream_t (NULL = default stream). Every call
 * returns 0 or a negative error code (-1 bad argument, -3 HIP error) and
 * launches asynchronously.
 */
#ifndef FNO_H
#define FNO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* C[b](m, n) = alpha * sum_k A[b](m, k) B[b](k, n) + beta * C[b](m, n) for
 * b < batch, m < M, n < N, k < K, with element (m, k) of A[b] at
 * A + b*sAb + m*sAm + k*sAk (strides in elements, any sign-free layout:
 * transposes are stride choices), likewise B and C. Operands are rounded to
 * BF16 (nearest even) on load; products accumulate in FP32. split_k > 1
 * divides K among work-groups whose partial sums are added atomically (the
 * result is then not bitwise reproducible; C is scaled by beta first);
 * otherwise beta is applied in the product's own write. With beta = 0, C is
 * not read. C must not alias A or B. */
int fno_gemm(int64_t batch, int64_t M, int64_t N, int64_t K, float alpha, const float *A, int64_t sAb,
             int64_t sAm, int64_t sAk, const float *B, int64_t sBb, int64_t sBk, int64_t sBn, float beta,
             float *C, int64_t sCb, int64_t sCm, int64_t sCn, int split_k, void *stream);

/* z[o][c][s] += bias[c] (bias may be NULL); a = gelu(z) if act else a = z
 * (a may equal z when act is 0). Layout [n_outer][C][S]. gelu is the exact
 * x/2 (1 + erf(x / sqrt 2)). */
int fno_bias_act(int64_t n_outer, int64_t C, int64_t S, float *z, const float *bias, float *a, int act,
                 void *stream);

/* dz = da * gelu'(z) elementwise over n values (dz may equal da). */
int fno_gelu_backward(int64_t n, const float *z, const float *da, float *dz, void *stream);

/* db[c] = sum over o < n_outer, s < S of dz[o][c][s] (overwrites db; partial
 * sums of work-groups are added atomically, so the summation order, and the
 * last bits, may vary from call to call). C <= 65535. */
int fno_channel_sum(int64_t n_outer, int64_t C, int64_t S, const float *dz, float *db, void *stream);

/* Adam step t >= 1 on n parameters: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps). */
int fno_adam(int64_t n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps,
             int t, void *stream);

/* Relative L2 loss over n_batch samples of n values each. loss is a device
 * array of n_batch + 1 floats: loss[1 + b] = |yhat_b - y_b| / |y_b| and
 * loss[0] their mean; grad (may be NULL) receives the gradient of loss[0]
 * with respect to yhat. */
int fno_rel_l2(int64_t n_batch, int64_t n, const float *yhat, const float *y, float *loss, float *grad,
               void *stream);

/* x *= s over n values. */
int fno_scale(int64_t n, float *x, float s, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FNO_H */
