// Matrix-core element kernels (device code and launch templates), included
// by the translation units that instantiate them: tuned_f32.hip (FP32
// operands), tuned_bf16.hip (BF16 operands) and tuned.hip (reference-matrix
// images, which need the layouts only).
//
// A wavefront updates 16 elements. Every contraction with a reference matrix
// shared by all elements (stiffness K^d, face traces E_f, lifts L_f) is a
// matrix-core product C[16 x 16] += A[16 x k] B[k x 16] with the reference
// matrix as A (staged in LDS once per work-group) and the 16 elements as the
// 16 columns of B, one product per quantity. The element data stays in the
// output-fragment layout of those products (lane el + 16 g holds rows
// 16t + 4v + g of element el), which is directly the B-operand layout of the
// next product once the K index of A is permuted the same way, so the chain
// of contractions needs no data shuffles. Per-element 9x9 work (scaled star
// matrices, Godunov flux at the face nodes) is lane-local VALU work in FP32.
//
// Operand precisions: FP32 (v_mfma_f32_16x16x4_f32, K step of 4 rows) and
// BF16 (v_mfma_f32_16x16x16_bf16, K step of 16 rows, or gfx950's
// v_mfma_f32_16x16x32_bf16 over two row tiles at once); accumulation and the
// element state are FP32 in both.
//
// Algorithm (Sec. 4.1 and 4.2), scaled derivatives Dk = dt^k/k! d^kQ/dt^k:
//   predictor  D(k+1) = -1/(k+1) sum_d (K^d)^T (Dk (dt A*_d)^T)
//              I~ = sum_k Dk/(k+1)
//              Q += sum_d K^d (I~ (dt A*_d)^T) - sum_f L_f flux(E_f I~, own trace)
//              traces E_f I~ handed to the neighbours
//   corrector  Q -= sum_f L_f flux(neighbour trace)
#pragma once

#include <hip/hip_runtime.h>

#include <sys/stat.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <type_traits>
#include <vector>

#include "elastic.hpp"
#include "layout.hpp"
#include "tuned.hpp"

#ifndef SEIS_SOURCE_HASH
#define SEIS_SOURCE_HASH "unhashed"
#endif

namespace seis {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

// Operand types of the predictor, the shapes the autotuner chooses among:
struct OpF32 {};    // FP32 operands, I~ parked in LDS as far as it fits
struct OpF32H {};   // FP32 operands, I~ parked in HBM only (the LDS keeps the reference block)
struct OpBF16 {};   // BF16 operands, 16x16x16 products (K = one row tile)
struct OpBF16W {};  // BF16 operands, 16x16x32 products (K = two row tiles)
struct OpBF16X3 {}; // split BF16 operands: x = hi + lo, three 16x16x16 products hi hi + hi lo + lo hi
template <class Op>
constexpr bool split3 = std::is_same<Op, OpBF16X3>::value;
template <class Op>
constexpr bool is_bf = std::is_same<Op, OpBF16>::value || std::is_same<Op, OpBF16W>::value || split3<Op>;
template <class Op>
constexpr bool wide_k = std::is_same<Op, OpBF16W>::value;
template <class Op>
constexpr bool hbm_park = std::is_same<Op, OpF32H>::value;


__host__ __device__ inline unsigned short f2bf(float x) {
  // round to nearest even
  unsigned int u;
  std::memcpy(&u, &x, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float fl2 __attribute__((ext_vector_type(2)));

// two floats to packed BF16, round to nearest even (one v_cvt_pk_bf16_f32)
__device__ __forceinline__ unsigned pack2(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(fl2{a, b}, bf2));
}

__device__ __forceinline__ unsigned short f2bf_dev(float x) { return (unsigned short)(pack2(x, 0.0f) & 0xffffu); }

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef short s8 __attribute__((ext_vector_type(8)));

// One 16x16x32 BF16 product over two row tiles: the lane's four K entries of
// the first tile, then its four of the second. A and B use the same (lane
// group, slot) -> row assignment, so the pairing of their K entries is right
// whatever K index the hardware gives each slot.
__device__ __forceinline__ f4 mfma_k32(s4 a0, s4 a1, s4 b0, s4 b1, f4 c) {
  const s8 a = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
  const s8 b = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

__device__ __forceinline__ s4 pack4(float a, float b, float c, float d) {
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(s4, u2{pack2(a, b), pack2(c, d)});
}

// Split BF16 operands (OpBF16X3): x = hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (x - hi is exact in FP32), so that a product of two split
// operands, hi hi + hi lo + lo hi, keeps about 16 significant bits of each
// (the lo lo term is below FP32 accumulation round-off).
__device__ __forceinline__ float bf_value(short h) { return __uint_as_float((unsigned)(unsigned short)h << 16); }

__device__ __forceinline__ void split4(float a, float b, float c, float d, s4& hi, s4& lo) {
  hi = pack4(a, b, c, d);
  lo = pack4(a - bf_value(hi[0]), b - bf_value(hi[1]), c - bf_value(hi[2]), d - bf_value(hi[3]));
}

// acc += A B on the BF16 matrix cores: one product, or three for split operands
template <class Op>
__device__ __forceinline__ f4 mfma_bf(s4 ah, s4 al, s4 bh, s4 bl, f4 acc) {
  if constexpr (split3<Op>) {
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
  }
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
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

// Quantities carried by a 16-element group in the 4-quantity form (AC), used
// when every element of the group is acoustic: with mu = 0 the stress is -p I
// (Sec. 4.1), so s_yy and s_zz equal s_xx and the shear components vanish;
// s_xx (= -p) and the velocity remain. The 9-quantity form carries all nine.
template <bool AC>
__host__ __device__ constexpr bool carried(int p) {
  return !AC || p == 0 || p >= 6;
}

// complete a state of the 4-quantity form to the nine quantities of the embedding
template <bool AC>
__device__ __forceinline__ void embed(float (&u)[9]) {
  if constexpr (AC) {
    u[1] = u[0];
    u[2] = u[0];
    u[3] = 0.0f;
    u[4] = 0.0f;
    u[5] = 0.0f;
  }
}

// apply_star for either form: with mu = 0 the three normal-stress rows
// coincide and the shear rows vanish, and the velocity rows see only s_xx.
// The terms kept are those of the 9-quantity form that are not products
// with a zero.
template <bool AC>
__device__ __forceinline__ void star_q(float cx, float cy, float cz, float lam, float mu, float rinv,
                                       const float (&v)[9], float (&out)[9]) {
  if constexpr (!AC) {
    apply_star(cx, cy, cz, lam, mu, rinv, v, out);
  } else {
    const float nlam = -lam, nr = -rinv;
    out[0] = nlam * cx * v[6] + nlam * cy * v[7] + nlam * cz * v[8];
    out[6] = nr * (cx * v[0]);
    out[7] = nr * (cy * v[0]);
    out[8] = nr * (cz * v[0]);
  }
}

// Minus the Godunov flux A-hat^-(n) q^b at one face node (Sec. 4.2), with the
// middle state a linear map of the given trace: c = n_x, n_y, n_z, then the
// eight scaled coefficients of (s_n^b, v_n^b) from (s_n, v_n) and
// (t_t^b, v_t^b) from (t_t, v_t).
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
  // out is minus the flux (the sign every caller applies), so no sign flips
  out[0] = lam * vnb + mu * (w * nx * nx + 2.0f * vbx * nx);
  out[1] = lam * vnb + mu * (w * ny * ny + 2.0f * vby * ny);
  out[2] = lam * vnb + mu * (w * nz * nz + 2.0f * vbz * nz);
  out[3] = mu * (w * nx * ny + vbx * ny + vby * nx);
  out[4] = mu * (w * ny * nz + vby * nz + vbz * ny);
  out[5] = mu * (w * nx * nz + vbx * nz + vbz * nx);
  out[6] = rinv * (snb * nx + tbx);
  out[7] = rinv * (snb * ny + tby);
  out[8] = rinv * (snb * nz + tbz);
}

// node_flux for the rows an element of the 4-quantity form carries (AC: s_xx,
// where mu = 0 leaves lam v_n^b, and the velocity), from a trace of that form
// (IN_AC: traction s_xx n) or a full trace (the neighbour's trace: elastic at
// the seafloor). The terms kept are those of node_flux that are not products
// with a zero.
template <bool AC, bool IN_AC>
__device__ __forceinline__ void node_flux_q(const float* c, float lam, float mu, float rinv, const float (&in)[9],
                                            float (&out)[9]) {
  static_assert(AC || !IN_AC, "a trace of the 4-quantity form belongs to an element of that form");
  if constexpr (!AC) {
    node_flux(c, lam, mu, rinv, in, out);
  } else {
    const float nx = c[0], ny = c[1], nz = c[2];
    float tx, ty, tz;
    if constexpr (IN_AC) {
      tx = in[0] * nx;
      ty = in[0] * ny;
      tz = in[0] * nz;
    } else {
      tx = in[0] * nx + in[3] * ny + in[5] * nz;
      ty = in[3] * nx + in[1] * ny + in[4] * nz;
      tz = in[5] * nx + in[4] * ny + in[2] * nz;
    }
    const float sn = tx * nx + ty * ny + tz * nz;
    const float ttx = tx - sn * nx, tty = ty - sn * ny, ttz = tz - sn * nz;
    const float vn = in[6] * nx + in[7] * ny + in[8] * nz;
    const float vtx = in[6] - vn * nx, vty = in[7] - vn * ny, vtz = in[8] - vn * nz;
    const float snb = c[3] * sn + c[4] * vn;
    const float vnb = c[5] * sn + c[6] * vn;
    const float tbx = c[7] * ttx + c[8] * vtx, tby = c[7] * tty + c[8] * vty, tbz = c[7] * ttz + c[8] * vtz;
    out[0] = lam * vnb;
    out[6] = rinv * (snb * nx + tbx);
    out[7] = rinv * (snb * ny + tby);
    out[8] = rinv * (snb * nz + tbz);
  }
}

// ---------------------------------------------------------------------------
// Reference block in LDS. Natural row-major layouts (FP32) or rows padded to a
// multiple of 4 entries (BF16, so that four consecutive K entries are one
// aligned 8-byte read), followed by a zero tail. Fragment reads use
// compile-time strides, so every read is a per-lane base plus an immediate
// offset. Reads may run past a matrix into the next one or into the tail:
// such entries are finite and only meet zero B values (K index beyond the
// input rows) or feed output rows that are discarded.
template <class Op>
using RefT = typename std::conditional<!is_bf<Op>, float, unsigned short>::type;

// Face node held in slot c = 16t + 4g + v of a node tile (lane group g,
// register v): node 16t + 4v + g. The 4 x 4 (g, v) grid of a tile is
// transposed so that the nodes of a partial last tile fill whole K slabs (v)
// of the FP32 products first. The map is its own inverse.
__host__ __device__ constexpr int node_of(int c) { return (c & ~15) + 4 * (c & 3) + ((c >> 2) & 3); }

// State row held in fragment row i of a 16-row tile (lane group i / 4, slot
// i % 4): row 4 (i % 4) + i / 4 of the tile (the state layout runs over the
// lane groups first, see layout.hpp).
__device__ __forceinline__ int frag_row(int i) { return tile_perm(i); }

// Rows of the state (the basis index) appear in the image either in their
// natural order (FP32: the kernels permute their fragment indices instead,
// see frag_row) or, for BF16, already in fragment order (tile_perm, with every
// row dimension padded to whole tiles), because a BF16 fragment reads four
// consecutive K entries at once.
template <class Op, int N>
struct Lay {
  static constexpr bool BF = is_bf<Op>;
  static constexpr int B = nbasis(N), Bf = nface(N), B1 = nbasis(N - 1);
  static constexpr int RT = row_tiles(B), FT = row_tiles(Bf), RT1 = row_tiles(B1);
  static constexpr int PB = BF ? 16 * RT : B;     // extent of a B-row dimension in the image
  static constexpr int PB1 = BF ? 16 * RT1 : B1;  // extent of a B1-row dimension
  // Leading dimensions. BF16: multiples of 4 entries (a fragment reads four
  // consecutive K entries as one 8-byte word) whose count of 8-byte words is
  // odd, so that the 16 rows of a fragment read start on 16 distinct bank
  // pairs (a row stride of 128 bytes put all 16 on one pair). FP32: padded so
  // that the 64 lanes of a fragment read (16 rows x 4 K entries) fall on
  // distinct LDS banks up to pairs; a multiple of 8 (or 16 x FT for the lifts,
  // 8- to 16-way conflicts) is avoided.
  static constexpr int r4(int x) {
    return BF ? ((x + 3) / 4 % 2 == 1 ? (x + 3) / 4 * 4 : (x + 3) / 4 * 4 + 4) : x + (x % 8 == 0 ? 1 : 0);
  }
  static constexpr int ldK = r4(PB1);  // K^d[l < B][m < B1]   (volume: A(k,l) = K[k][l]; FP32 CK: A(m,l) = K[l][m])
  static constexpr int ldT = r4(PB);   // BF16 CK: (K^d)^T[m < B1][l < B]
  // face nodes in slot order (see node_of): FT * 16 slots per face
  static constexpr int ldE = r4(PB);                   // E_f[slot < 16 FT][row < B]
  static constexpr int ldL = BF ? r4(16 * FT) : 16 * FT + 3;  // L_f[row < B][slot < 16 FT]
  static constexpr int nK = 3 * PB * ldK;
  static constexpr int nT = BF ? 3 * PB1 * ldT : 0;
  static constexpr int nE = 4 * 16 * FT * ldE;
  static constexpr int nL = 4 * PB * ldL;
  static constexpr int maxld = (ldK > ldE ? ldK : ldE) > ldL ? (ldK > ldE ? ldK : ldE) : ldL;
  static constexpr int tail = 16 * (maxld > ldT ? maxld : ldT) + 64;
  // the lift block starts on a 16-byte boundary (the corrector stages it alone)
  static constexpr int oK = 0, oT = nK, oE = nK + nT, oL = (oE + nE + 7) / 8 * 8;
  // one image (a multiple of 16 bytes); split BF16 keeps the hi image and
  // then the lo image
  static constexpr int esz = BF ? 2 : 4;
  static constexpr int images = split3<Op> ? 2 : 1;
  static constexpr int total = ((oL + nL + tail) * esz + 15) / 16 * 16 / esz;
  static constexpr int bytes = images * total * esz;
  // the corrector stages only the lifts and the tail, [oL, total), of each image
  static constexpr int lift_elems = ((nL + tail) * esz + 15) / 16 * 16 / esz;
  static constexpr int lift_bytes = images * lift_elems * esz;
};

// A zero the compiler cannot see through. Views built with it are re-read
// from LDS where they are used, instead of being hoisted into registers for
// the whole kernel (the reference block is loop-invariant).
__device__ __forceinline__ int opaque_zero() {
  int z = 0;
  asm volatile("" : "+s"(z));
  return z;
}

// One 16-element group block of a fragment-layout array (Q, J or a face
// inbox) as a raw buffer: register r of the wavefront is the 256-byte slab at
// byte offset 256 r, each lane reading its own dword. The per-register offset
// goes to the scalar offset, so no per-access vector address is needed.
struct GroupBuf {
  __amdgpu_buffer_rsrc_t r;
  int lane4;
  int o;
  __device__ __forceinline__ GroupBuf(const float* base, int bytes, int lane)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, bytes, 0x00020000)),
        lane4(lane * 4), o(opaque_zero()) {}
  __device__ __forceinline__ float ld(int reg) const {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, lane4, o + reg * 256, 0));
  }
  __device__ __forceinline__ void st(int reg, float x) const {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, lane4, o + reg * 256, 0);
  }
};

// A(i, k) = R[i * LD + k] (row-major) or R[k * LD + i] (transposed store);
// for split BF16 the lo part of the same entry sits lo entries further on
template <class R, int LD, bool TR>
struct View {
  const R* p;
  int o;
  int lo;
  __device__ __forceinline__ View(const R* base, int lo_off = 0) : p(base), o(opaque_zero()), lo(lo_off) {}
  __device__ __forceinline__ R at(int i, int k) const { return TR ? p[o + k * LD + i] : p[o + i * LD + k]; }
  // four consecutive K entries k0..k0+3 (BF16, row-major only), and their lo parts
  __device__ __forceinline__ s4 at4(int i, int k0) const {
    static_assert(!TR, "four-entry reads need the row-major store");
    return *reinterpret_cast<const s4*>(p + o + i * LD + k0);
  }
  __device__ __forceinline__ s4 at4_lo(int i, int k0) const {
    return *reinterpret_cast<const s4*>(p + o + lo + i * LD + k0);
  }
};

// rows requested ahead by the pipelined contractions
constexpr int kPrefetch = 2;

// acc[mt][p] += sum_k A(16 mt + el, k) X[k][p]; X rows produced by rowfn(t, v, b[9])
// for the input rows k < nrows (rows 16t + 4g + v of this lane). With PIPE the
// rows come from memory: the next row (FP32) or row tile (BF16) is requested
// before the products of the current one, and a scheduling barrier per row
// keeps the compiler from hoisting every load of the loop (which would need a
// register per load in flight).
// NODEK: the K index runs over face nodes in slot order (node 16t + 4v + g in
// slot (t, g, v)) and the output rows are state rows; otherwise the K index
// runs over state rows (row 16t + 4v + g in register v of lane group g) and
// the output rows are face nodes. Either way a slab (t, v) holds K entries
// 16t + 4v .. 16t + 4v + 3, so a partial last tile needs only its first slabs.
// AC: only the quantities of the 4-quantity form (the others of acc and of
// the rows are neither read nor written).
template <class Op, class V, int NT, int MT, bool PIPE = false, bool NODEK = false, bool AC = false, class RowFn>
__device__ __forceinline__ void contract_fn(f4 (&acc)[MT][9], const V& A, int nrows, int el, int g, RowFn rowfn) {
  if constexpr (!is_bf<Op>) {
    constexpr int D = PIPE ? kPrefetch : 0;  // rows requested ahead
    float b[D + 1][9];
    float an[2][MT];  // A fragments of this row and the next (read from LDS one row ahead)
    // slab (t, v) holds rows (or nodes) 16t + 4v .. 16t + 4v + 3
    auto valid = [&](int i) { return i < 4 * NT && 16 * (i >> 2) + 4 * (i & 3) < nrows; };
    // FP32 images keep state rows in natural order: a fragment row (M side)
    // that is a state row is frag_row(el), a K index that is a state row is
    // 16t + 4v + g; node slots are stored in fragment order already
    const int mrow = NODEK ? frag_row(el) : el;
    auto load_a = [&](int i, float(&dst)[MT]) {
      const int k = NODEK ? 16 * (i >> 2) + 4 * g + (i & 3) : 16 * (i >> 2) + 4 * (i & 3) + g;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) dst[mt] = A.at(16 * mt + mrow, k);
    };
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (valid(j)) rowfn(j >> 2, j & 3, b[j % (D + 1)]);
    if constexpr (PIPE) load_a(0, an[0]);
#pragma unroll
    for (int i = 0; i < 4 * NT; ++i) {
      const int t = i >> 2, v = i & 3;
      if (!valid(i)) continue;
      float(&cur)[9] = b[i % (D + 1)];
      if constexpr (PIPE) {
        if (valid(i + D)) rowfn((i + D) >> 2, (i + D) & 3, b[(i + D) % (D + 1)]);
        if (valid(i + 1)) load_a(i + 1, an[(i + 1) & 1]);
      } else {
        rowfn(t, v, cur);
        load_a(i, an[i & 1]);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const float a = an[i & 1][mt];
#pragma unroll
        for (int p = 0; p < 9; ++p)
          if (carried<AC>(p)) acc[mt][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, cur[p], acc[mt][p], 0, 0, 0);
      }
      if constexpr (PIPE) __builtin_amdgcn_sched_barrier(0);
    }
  } else if constexpr (wide_k<Op>) {
    // two row tiles per 16x16x32 product (a lone last tile: one 16x16x16);
    // the rows of a pair are requested together, without a look-ahead
#pragma unroll
    for (int t = 0; t < NT; t += 2) {
      if (16 * t >= nrows) continue;
      const bool two = t + 1 < NT && 16 * (t + 1) < nrows;
      float c0[4][9], c1[4][9];
#pragma unroll
      for (int v = 0; v < 4; ++v) rowfn(t, v, c0[v]);
      if (two) {
#pragma unroll
        for (int v = 0; v < 4; ++v) rowfn(t + 1, v, c1[v]);
      }
      s4 a0[MT], a1[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        a0[mt] = A.at4(16 * mt + el, 16 * t + 4 * g);
        a1[mt] = two ? A.at4(16 * mt + el, 16 * (t + 1) + 4 * g) : s4{0, 0, 0, 0};
      }
#pragma unroll
      for (int p = 0; p < 9; ++p) {
        if (!carried<AC>(p)) continue;
        const s4 b0 = pack4(c0[0][p], c0[1][p], c0[2][p], c0[3][p]);
        const s4 b1 = two ? pack4(c1[0][p], c1[1][p], c1[2][p], c1[3][p]) : s4{0, 0, 0, 0};
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          acc[mt][p] = two ? mfma_k32(a0[mt], a1[mt], b0, b1, acc[mt][p])
                           : __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0[mt], b0, acc[mt][p], 0, 0, 0);
      }
      if constexpr (PIPE) __builtin_amdgcn_sched_barrier(0);
    }
  } else {
    float bv[2][4][9];
    s4 an[2][MT];  // A fragments of this row tile and the next
    s4 al[2][MT];  // their lo parts (split BF16)
    auto load_a = [&](int t, s4(&dst)[MT]) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        dst[mt] = A.at4(16 * mt + el, 16 * t + 4 * g);
        if constexpr (split3<Op>) al[t & 1][mt] = A.at4_lo(16 * mt + el, 16 * t + 4 * g);
      }
    };
    if constexpr (PIPE) {
#pragma unroll
      for (int v = 0; v < 4; ++v) rowfn(0, v, bv[0][v]);
      load_a(0, an[0]);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (16 * t >= nrows) continue;
      float(&cur)[4][9] = bv[t & 1];
      if constexpr (PIPE) {
        if (t + 1 < NT && 16 * (t + 1) < nrows) {
#pragma unroll
          for (int v = 0; v < 4; ++v) rowfn(t + 1, v, bv[(t + 1) & 1][v]);
          load_a(t + 1, an[(t + 1) & 1]);
        }
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) rowfn(t, v, cur[v]);
        load_a(t, an[t & 1]);
      }
      s4 b[9], bl[9];
#pragma unroll
      for (int p = 0; p < 9; ++p) {
        if (!carried<AC>(p)) continue;
        if constexpr (split3<Op>)
          split4(cur[0][p], cur[1][p], cur[2][p], cur[3][p], b[p], bl[p]);
        else
          b[p] = pack4(cur[0][p], cur[1][p], cur[2][p], cur[3][p]);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const s4 a = an[t & 1][mt];
        const s4 alo = split3<Op> ? al[t & 1][mt] : a;
#pragma unroll
        for (int p = 0; p < 9; ++p)
          if (carried<AC>(p)) acc[mt][p] = mfma_bf<Op>(a, alo, b[p], split3<Op> ? bl[p] : b[p], acc[mt][p]);
      }
      if constexpr (PIPE) __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// accumulate J += w D
template <bool AC, int RT, int RTO>
__device__ __forceinline__ void accum(float (&I)[RT][4][9], const float (&d)[RTO][4][9], float w) {
#pragma unroll
  for (int t = 0; t < RTO; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int p = 0; p < 9; ++p)
        if (carried<AC>(p)) I[t][v][p] += w * d[t][v][p];
}

// store a derivative (rows held in x, zero beyond) for the gravity kernel,
// completed to nine quantities
template <int N, bool AC, int RTX>
__device__ __forceinline__ void store_deriv(float* dst, const float (&x)[RTX][4][9], int g) {
  constexpr int B = nbasis(N), RT = row_tiles(B);
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * t + 4 * v + g;
      if (row >= B) continue;
#pragma unroll
      for (int p = 0; p < 9; ++p) {
        const int pc = carried<AC>(p) ? p : (p < 3 ? 0 : -1);  // quantity the value comes from
        dst[row * 9 + p] = (t < RTX && pc >= 0) ? x[t < RTX ? t : 0][v][pc < 0 ? 0 : pc] : 0.0f;
      }
    }
}

// One Cauchy-Kowalevski step D(K+1) = fk sum_d (K^d)^T (D(K) (dt A*_d)^T) for the
// output quantities [P0, P1) (of those the form AC carries); the star product
// of each input row is formed lane-locally right before it enters the matrix
// cores.
template <class Op, int N, int K, int RTI, int RTO, bool AC, int P0 = 0, int P1 = 9>
__device__ __forceinline__ void ck_step(const float (&din)[RTI][4][9], float (&dout)[RTO][4][9],
                                        const RefT<Op>* lds, const float* G, float lam, float mu, float rinv,
                                        int el, int g, float fk) {
  using L = Lay<Op, N>;
  constexpr int nin = nbasis(N - K), nout = nbasis(N - K - 1);
  constexpr int NP = P1 - P0;
  f4 acc[RTO][NP];
#pragma unroll
  for (int mt = 0; mt < RTO; ++mt)
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[mt][p] = f4{0.f, 0.f, 0.f, 0.f};
  if constexpr (!is_bf<Op>) {
    // slabs (d, row) in order; the K^d fragments of the next slab are read from
    // LDS while the products of the current one run
    const View<float, L::ldK, true> A0(lds + L::oK), A1(lds + L::oK + L::PB * L::ldK),
        A2(lds + L::oK + 2 * L::PB * L::ldK);  // A(m, l) = K^d[l][m]
    constexpr int NV = (nin / 16) * 4 + ((nin % 16) + 3) / 4;  // slabs (t, v) with 16t + 4v < nin
    const int mrow = frag_row(el);
    float an[2][RTO];
    auto load_a = [&](int s, float(&dst)[RTO]) {
      const int d = s / NV, i = s % NV, k = 16 * (i >> 2) + 4 * (i & 3) + g;
#pragma unroll
      for (int mt = 0; mt < RTO; ++mt)
        dst[mt] = d == 0 ? A0.at(16 * mt + mrow, k) : (d == 1 ? A1.at(16 * mt + mrow, k) : A2.at(16 * mt + mrow, k));
    };
    if constexpr (N <= 5) {
      // software pipeline over the slabs: while the products of slab s run,
      // the K^d fragments of slab s+1 are read from LDS and its star product
      // is formed (one scheduling region per slab, so neither is sunk to its
      // use). At N = 6 the second star buffer spills; that order keeps the
      // plain loop.
      auto star_of = [&](int s, float(&z)[9]) {
        const int d = s / NV, i = s % NV;
        star_q<AC>(G[3 * d], G[3 * d + 1], G[3 * d + 2], lam, mu, rinv, din[i >> 2][i & 3], z);
      };
      float zb[2][9];
      load_a(0, an[0]);
      star_of(0, zb[0]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int s = 0; s < 3 * NV; ++s) {
        if (s + 1 < 3 * NV) load_a(s + 1, an[(s + 1) & 1]);
#pragma unroll
        for (int mt = 0; mt < RTO; ++mt) {
          const float af = an[s & 1][mt];
#pragma unroll
          for (int p = 0; p < NP; ++p)
            if (carried<AC>(P0 + p))
              acc[mt][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, zb[s & 1][P0 + p], acc[mt][p], 0, 0, 0);
        }
        if (s + 1 < 3 * NV) star_of(s + 1, zb[(s + 1) & 1]);
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      load_a(0, an[0]);
#pragma unroll
      for (int s = 0; s < 3 * NV; ++s) {
        const int d = s / NV, i = s % NV, t = i >> 2, v = i & 3;
        if (s + 1 < 3 * NV) load_a(s + 1, an[(s + 1) & 1]);
        float z[9];
        star_q<AC>(G[3 * d], G[3 * d + 1], G[3 * d + 2], lam, mu, rinv, din[t][v], z);
#pragma unroll
        for (int mt = 0; mt < RTO; ++mt) {
          const float af = an[s & 1][mt];
#pragma unroll
          for (int p = 0; p < NP; ++p)
            if (carried<AC>(P0 + p)) acc[mt][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, z[P0 + p], acc[mt][p], 0, 0, 0);
        }
      }
    }
  } else {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    {
      const View<unsigned short, L::ldT, false> A(lds + L::oT + d * L::PB1 * L::ldT, L::total);  // (K^d)^T[m][l]
      if constexpr (wide_k<Op>) {
        // two input row tiles per 16x16x32 product
#pragma unroll
        for (int t = 0; t < RTI; t += 2) {
          if (16 * t >= nin) continue;
          const bool two = t + 1 < RTI && 16 * (t + 1) < nin;
          float z0[4][9], z1[4][9];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            star_q<AC>(G[3 * d], G[3 * d + 1], G[3 * d + 2], lam, mu, rinv, din[t][v], z0[v]);
            if (two) star_q<AC>(G[3 * d], G[3 * d + 1], G[3 * d + 2], lam, mu, rinv, din[two ? t + 1 : t][v], z1[v]);
          }
          s4 b0[NP], b1[NP];
#pragma unroll
          for (int p = 0; p < NP; ++p) {
            if (!carried<AC>(P0 + p)) continue;
            b0[p] = pack4(z0[0][P0 + p], z0[1][P0 + p], z0[2][P0 + p], z0[3][P0 + p]);
            b1[p] = two ? pack4(z1[0][P0 + p], z1[1][P0 + p], z1[2][P0 + p], z1[3][P0 + p]) : s4{0, 0, 0, 0};
          }
#pragma unroll
          for (int mt = 0; mt < RTO; ++mt) {
            const s4 a0 = A.at4(16 * mt + el, 16 * t + 4 * g);
            const s4 a1 = two ? A.at4(16 * mt + el, 16 * (t + 1) + 4 * g) : s4{0, 0, 0, 0};
#pragma unroll
            for (int p = 0; p < NP; ++p)
              if (carried<AC>(P0 + p))
                acc[mt][p] = two ? mfma_k32(a0, a1, b0[p], b1[p], acc[mt][p])
                                 : __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b0[p], acc[mt][p], 0, 0, 0);
          }
        }
        continue;
      }
#pragma unroll
      for (int t = 0; t < RTI; ++t) {
        if (16 * t >= nin) continue;
        float z[4][9];
#pragma unroll
        for (int v = 0; v < 4; ++v) star_q<AC>(G[3 * d], G[3 * d + 1], G[3 * d + 2], lam, mu, rinv, din[t][v], z[v]);
        s4 bz[NP], bzl[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          if (!carried<AC>(P0 + p)) continue;
          if constexpr (split3<Op>)
            split4(z[0][P0 + p], z[1][P0 + p], z[2][P0 + p], z[3][P0 + p], bz[p], bzl[p]);
          else
            bz[p] = pack4(z[0][P0 + p], z[1][P0 + p], z[2][P0 + p], z[3][P0 + p]);
        }
        const int k0 = 16 * t + 4 * g;
#pragma unroll
        for (int mt = 0; mt < RTO; ++mt) {
          const s4 af = A.at4(16 * mt + el, k0);
          const s4 afl = split3<Op> ? A.at4_lo(16 * mt + el, k0) : af;
#pragma unroll
          for (int p = 0; p < NP; ++p)
            if (carried<AC>(P0 + p)) acc[mt][p] = mfma_bf<Op>(af, afl, bz[p], split3<Op> ? bzl[p] : bz[p], acc[mt][p]);
        }
      }
    }
  }
  }
#pragma unroll
  for (int mt = 0; mt < RTO; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * mt + 4 * v + g;
#pragma unroll
      for (int p = 0; p < NP; ++p)
        if (carried<AC>(P0 + p)) dout[mt][v][P0 + p] = row < nout ? fk * acc[mt][p][v] : 0.0f;
    }
}

// First CK step straight from Q in memory (group base Qg): the stress rows of
// D1 read only the velocity columns of D0 and the velocity rows only the
// stress columns, so D0 is brought in as two column sets, both requested
// before the first products.
template <int N, bool AC, int C0, int C1>
__device__ __forceinline__ void load_q_cols(float (&din)[row_tiles(nbasis(N))][4][9], const float* Qg, int lane) {
  constexpr int B = nbasis(N), RT = row_tiles(B);
  const GroupBuf qb(Qg, RT * 36 * 256, lane);
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      // a register whose four rows are all >= B (the zero padding of the
      // tiled layout) is not loaded; the others are loaded whole, so that no
      // load sits behind a lane-dependent branch
#pragma unroll
      for (int p = 0; p < 9; ++p)
        din[t][v][p] = (p >= C0 && p < C1 && carried<AC>(p) && 16 * t + 4 * v < B) ? qb.ld((t * 4 + v) * 9 + p) : 0.0f;
    }
}

template <class Op, int N, bool AC, int P0, int P1, int C0, int C1>
__device__ __forceinline__ void ck_first_half(float (&d1)[row_tiles(nbasis(N - 1))][4][9],
                                              const float (&din)[row_tiles(nbasis(N))][4][9], const RefT<Op>* lds,
                                              const float* G, float lam, float mu, float rinv, int el, int g,
                                              float* gd) {
  constexpr int B = nbasis(N), RT = row_tiles(B), RT1 = row_tiles(nbasis(N - 1));
  if (gd) {
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + 4 * v + g;
        if (row >= B) continue;
#pragma unroll
        for (int p = C0; p < C1; ++p) gd[row * 9 + p] = carried<AC>(p) ? din[t][v][p] : (p < 3 ? din[t][v][0] : 0.0f);
      }
  }
  ck_step<Op, N, 0, RT, RT1, AC, P0, P1>(din, d1, lds, G, lam, mu, rinv, el, g, -1.0f);
}

template <class Op, int N, bool AC>
struct CK {
  // J = sum_{k >= 1} Dk/(k+1) (rows below B1); I~ = Q + J.
  __device__ static __forceinline__ void run(float (&J)[row_tiles(nbasis(N - 1))][4][9], const float* Qg, int lane,
                             const RefT<Op>* lds, const float* G, float lam, float mu, float rinv, int el, int g,
                             float* gd) {
    constexpr int B = nbasis(N), RT = row_tiles(B);
    constexpr int R1 = row_tiles(nbasis(N - 1));
    {
      float dv[RT][4][9], ds[RT][4][9];
      load_q_cols<N, AC, 6, 9>(dv, Qg, lane);
      load_q_cols<N, AC, 0, 6>(ds, Qg, lane);
      ck_first_half<Op, N, AC, 0, 6, 6, 9>(J, dv, lds, G, lam, mu, rinv, el, g, gd);
      __builtin_amdgcn_sched_barrier(0);
      ck_first_half<Op, N, AC, 6, 9, 0, 6>(J, ds, lds, G, lam, mu, rinv, el, g, gd);
    }
    if (gd) store_deriv<N, AC>(gd + 1 * B * 9, J, g);
#pragma unroll
    for (int t = 0; t < R1; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int p = 0; p < 9; ++p)
          if (carried<AC>(p)) J[t][v][p] *= 0.5f;  // J = D1/2
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (N >= 2) {
      constexpr int R2 = row_tiles(nbasis(N - 2));
      float d2[R2][4][9];
      ck_step<Op, N, 1, R1, R2, AC>(J, d2, lds, G, lam, mu, rinv, el, g, -1.0f);  // input D1/2
      if (gd) store_deriv<N, AC>(gd + 2 * B * 9, d2, g);
      accum<AC>(J, d2, 1.0f / 3.0f);
      if constexpr (N >= 3) {
        constexpr int R3 = row_tiles(nbasis(N - 3));
        float d3[R3][4][9];
        ck_step<Op, N, 2, R2, R3, AC>(d2, d3, lds, G, lam, mu, rinv, el, g, -1.0f / 3.0f);
        if (gd) store_deriv<N, AC>(gd + 3 * B * 9, d3, g);
        accum<AC>(J, d3, 0.25f);
        if constexpr (N >= 4) {
          constexpr int R4 = row_tiles(nbasis(N - 4));
          float d4[R4][4][9];
          ck_step<Op, N, 3, R3, R4, AC>(d3, d4, lds, G, lam, mu, rinv, el, g, -0.25f);
          if (gd) store_deriv<N, AC>(gd + 4 * B * 9, d4, g);
          accum<AC>(J, d4, 0.2f);
          if constexpr (N >= 5) {
            constexpr int R5 = row_tiles(nbasis(N - 5));
            float d5[R5][4][9];
            ck_step<Op, N, 4, R4, R5, AC>(d4, d5, lds, G, lam, mu, rinv, el, g, -0.2f);
            if (gd) store_deriv<N, AC>(gd + 5 * B * 9, d5, g);
            accum<AC>(J, d5, 1.0f / 6.0f);
            if constexpr (N >= 6) {
              constexpr int R6 = row_tiles(nbasis(N - 6));
              float d6[R6][4][9];
              ck_step<Op, N, 5, R5, R6, AC>(d5, d6, lds, G, lam, mu, rinv, el, g, -1.0f / 6.0f);
              if (gd) store_deriv<N, AC>(gd + 6 * B * 9, d6, g);
              accum<AC>(J, d6, 1.0f / 7.0f);
            }
          }
        }
      }
    }
  }
};

// dq[mt][p] += sum_d sum_l K^d(16 mt + el, l) (I~_l (dt A*_d)^T)_p over the rows
// l < B1 of I~ (rows produced by rowfn from memory), each row read once for
// all three d; software-pipelined like contract_fn.
template <class Op, int N, bool AC, class RowFn>
__device__ __forceinline__ void volume(f4 (&dq)[row_tiles(nbasis(N))][9], const RefT<Op>* lds, RowFn rowfn,
                                       const float* G, float lam, float mu, float rinv, int el, int g) {
  using L = Lay<Op, N>;
  constexpr int B = L::B, B1 = L::B1, RT = L::RT, RT1 = L::RT1;
  using R = RefT<Op>;
  const View<R, L::ldK, false> A0(lds + L::oK, L::total), A1(lds + L::oK + L::PB * L::ldK, L::total),
      A2(lds + L::oK + 2 * L::PB * L::ldK, L::total);
  if constexpr (!is_bf<Op>) {
    constexpr int D = kPrefetch;
    float xb[D + 1][9];
    auto valid = [&](int i) { return i < 4 * RT1 && 16 * (i >> 2) + 4 * (i & 3) < B1; };
    const int mrow = frag_row(el);
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (valid(j)) rowfn(j >> 2, j & 3, xb[j % (D + 1)]);
    float an[2][3][RT];  // K^d fragments of this row and the next
    auto load_a = [&](int i, float(&dst)[3][RT]) {
      const int k = 16 * (i >> 2) + 4 * (i & 3) + g;
#pragma unroll
      for (int mt = 0; mt < RT; ++mt) {
        dst[0][mt] = A0.at(16 * mt + mrow, k);
        dst[1][mt] = A1.at(16 * mt + mrow, k);
        dst[2][mt] = A2.at(16 * mt + mrow, k);
      }
    };
    load_a(0, an[0]);
#pragma unroll
    for (int i = 0; i < 4 * RT1; ++i) {
      const int t = i >> 2, v = i & 3;
      if (!valid(i)) continue;
      if (valid(i + D)) rowfn((i + D) >> 2, (i + D) & 3, xb[(i + D) % (D + 1)]);
      if (valid(i + 1)) load_a(i + 1, an[(i + 1) & 1]);
      const float(&x)[9] = xb[i % (D + 1)];
      const bool ok = 16 * t + 4 * v + g < B1;
      float z[3][9];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        star_q<AC>(G[3 * d], G[3 * d + 1], G[3 * d + 2], lam, mu, rinv, x, z[d]);
#pragma unroll
        for (int p = 0; p < 9; ++p)
          if (carried<AC>(p)) z[d][p] = ok ? z[d][p] : 0.0f;
      }
#pragma unroll
      for (int mt = 0; mt < RT; ++mt) {
        const float a0 = an[i & 1][0][mt], a1 = an[i & 1][1][mt], a2 = an[i & 1][2][mt];
#pragma unroll
        for (int p = 0; p < 9; ++p) {
          if (!carried<AC>(p)) continue;
          dq[mt][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, z[0][p], dq[mt][p], 0, 0, 0);
          dq[mt][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, z[1][p], dq[mt][p], 0, 0, 0);
          dq[mt][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, z[2][p], dq[mt][p], 0, 0, 0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  } else if constexpr (wide_k<Op>) {
    // two row tiles of I~ per 16x16x32 product
#pragma unroll
    for (int t = 0; t < RT1; t += 2) {
      if (16 * t >= B1) continue;
      const bool two = t + 1 < RT1 && 16 * (t + 1) < B1;
      float x0[4][9], x1[4][9];
#pragma unroll
      for (int v = 0; v < 4; ++v) rowfn(t, v, x0[v]);
      if (two) {
#pragma unroll
        for (int v = 0; v < 4; ++v) rowfn(t + 1, v, x1[v]);
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        s4 b0[9], b1[9];
        {
          float z[4][9];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const bool ok = 16 * t + 4 * v + g < B1;
            star_q<AC>(G[3 * d], G[3 * d + 1], G[3 * d + 2], lam, mu, rinv, x0[v], z[v]);
#pragma unroll
            for (int p = 0; p < 9; ++p)
              if (carried<AC>(p)) z[v][p] = ok ? z[v][p] : 0.0f;
          }
#pragma unroll
          for (int p = 0; p < 9; ++p)
            if (carried<AC>(p)) b0[p] = pack4(z[0][p], z[1][p], z[2][p], z[3][p]);
        }
        if (two) {
          float z[4][9];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const bool ok = 16 * (t + 1) + 4 * v + g < B1;
            star_q<AC>(G[3 * d], G[3 * d + 1], G[3 * d + 2], lam, mu, rinv, x1[v], z[v]);
#pragma unroll
            for (int p = 0; p < 9; ++p)
              if (carried<AC>(p)) z[v][p] = ok ? z[v][p] : 0.0f;
          }
#pragma unroll
          for (int p = 0; p < 9; ++p)
            if (carried<AC>(p)) b1[p] = pack4(z[0][p], z[1][p], z[2][p], z[3][p]);
        }
        const View<R, L::ldK, false>& A = d == 0 ? A0 : (d == 1 ? A1 : A2);
#pragma unroll
        for (int mt = 0; mt < RT; ++mt) {
          const s4 a0 = A.at4(16 * mt + el, 16 * t + 4 * g);
          const s4 a1 = two ? A.at4(16 * mt + el, 16 * (t + 1) + 4 * g) : s4{0, 0, 0, 0};
#pragma unroll
          for (int p = 0; p < 9; ++p)
            if (carried<AC>(p))
              dq[mt][p] = two ? mfma_k32(a0, a1, b0[p], b1[p], dq[mt][p])
                              : __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b0[p], dq[mt][p], 0, 0, 0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
    float xb[2][4][9];
#pragma unroll
    for (int v = 0; v < 4; ++v) rowfn(0, v, xb[0][v]);
#pragma unroll
    for (int t = 0; t < RT1; ++t) {
      if (16 * t >= B1) continue;
      if (t + 1 < RT1 && 16 * (t + 1) < B1) {
#pragma unroll
        for (int v = 0; v < 4; ++v) rowfn(t + 1, v, xb[(t + 1) & 1][v]);
      }
      const int k0 = 16 * t + 4 * g;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        float z[4][9];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool ok = 16 * t + 4 * v + g < B1;
          star_q<AC>(G[3 * d], G[3 * d + 1], G[3 * d + 2], lam, mu, rinv, xb[t & 1][v], z[v]);
#pragma unroll
          for (int p = 0; p < 9; ++p)
            if (carried<AC>(p)) z[v][p] = ok ? z[v][p] : 0.0f;
        }
        s4 b[9], bl[9];
#pragma unroll
        for (int p = 0; p < 9; ++p) {
          if (!carried<AC>(p)) continue;
          if constexpr (split3<Op>)
            split4(z[0][p], z[1][p], z[2][p], z[3][p], b[p], bl[p]);
          else
            b[p] = pack4(z[0][p], z[1][p], z[2][p], z[3][p]);
        }
        const View<R, L::ldK, false>& A = d == 0 ? A0 : (d == 1 ? A1 : A2);
#pragma unroll
        for (int mt = 0; mt < RT; ++mt) {
          const s4 a = A.at4(16 * mt + el, k0);
          const s4 alo = split3<Op> ? A.at4_lo(16 * mt + el, k0) : a;
#pragma unroll
          for (int p = 0; p < 9; ++p)
            if (carried<AC>(p)) dq[mt][p] = mfma_bf<Op>(a, alo, b[p], split3<Op> ? bl[p] : b[p], dq[mt][p]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <class Op>
__device__ __forceinline__ void stage_ref(void* lds, const void* ref, int bytes, int nthreads) {
  const uint4* src = reinterpret_cast<const uint4*>(ref);
  uint4* dst = reinterpret_cast<uint4*>(lds);
  for (int i = threadIdx.x; i < bytes / 16; i += nthreads) dst[i] = src[i];
}

// Predictor: persistent work-groups of W wavefronts; wavefront w of block b
// handles the 16-element groups first + b*W + w, then strides by gridDim*W.
// Logical work-group index. Work-groups are dispatched round-robin over the
// 8 XCDs (each with its own L2); with remap, XCD x gets a contiguous range of
// logical indices, so neighbouring 16-element groups (which exchange face
// traces) are handled under the same L2.
__device__ __forceinline__ int64_t logical_block(int remap) {
  const int64_t b = blockIdx.x, nb = gridDim.x;
  if (!remap || nb < 8) return b;
  const int64_t q = nb >> 3, r = nb & 7, x = b & 7, j = b >> 3;
  return x < r ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
}

// The predictor keeps I~ in an LDS slice per wavefront: all of it, in BF16,
// when the operands are BF16 (the products round it to BF16 anyway) and the
// slices fit beside the reference block; in FP32, as many leading row tiles
// as fit (the rest is parked in HBM). The node permutation table (6 x Bf
// entries) follows.
template <class Op, int N, int W>
struct PredLds {
  using L = Lay<Op, N>;
  static constexpr int slice = L::RT * 36 * 64;  // BF16 values per wavefront
  static constexpr int perm_bytes = (6 * L::Bf * 4 + 15) / 16 * 16;
  static constexpr int budget = 160 * 1024 - L::bytes - perm_bytes;
  // split BF16 keeps I~ in FP32 (in HBM: its two images leave no room in LDS)
  static constexpr bool park_lds = L::BF && !split3<Op> && W * slice * 2 <= budget;
  static constexpr int f32_fit = budget / (W * 36 * 64 * 4);
  static constexpr int f32_tiles =
      (L::BF || hbm_park<Op>) ? 0 : (f32_fit < L::RT ? (f32_fit > 0 ? f32_fit : 0) : L::RT);
  static constexpr int perm_off = L::bytes + (park_lds ? W * slice * 2 : W * f32_tiles * 36 * 64 * 4);
  static constexpr int bytes = perm_off + perm_bytes;
};

template <class Op, int N, int W>
__global__ __launch_bounds__(64 * W) void k_predict_tuned(TArgs a, int64_t e0, int64_t e1, Sched sc, int remap) {
  using L = Lay<Op, N>;
  constexpr int B = L::B, Bf = L::Bf, B1 = L::B1, RT = L::RT, FT = L::FT, RT1 = L::RT1;
  using R = RefT<Op>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const R* lds = reinterpret_cast<const R*>(lds_raw);
  stage_ref<Op>(lds_raw, a.ref, L::bytes, 64 * W);
  int* perm = reinterpret_cast<int*>(lds_raw + PredLds<Op, N, W>::perm_off);
  for (int i = threadIdx.x; i < 6 * Bf; i += 64 * W) perm[i] = a.pinv[i];
  __syncthreads();
  // the wavefront index is uniform across the wavefront: keep it (and every
  // group base and buffer descriptor derived from it) in scalar registers
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int el = lane & 15, g = lane >> 4;
  const int64_t gfirst = e0 >> 4, glast = (e1 - 1) >> 4;
  for (int64_t grp = gfirst + logical_block(remap) * W + w; grp <= glast; grp += (int64_t)gridDim.x * W) {
    // one body per form: the 4-quantity form for a group of acoustic elements
    auto body = [&](auto form) {
      constexpr bool AC = decltype(form)::value;
      const int64_t e = grp * 16 + el;
      const bool live = e >= e0 && e < e1;
      const int64_t ec = live ? e : e0;
      // hand-over descriptors of the four faces: targets, and mode | orientation << 2 per byte
      typedef int i4 __attribute__((ext_vector_type(4)));
      const i4 tg4 = *reinterpret_cast<const i4*>(a.tgt + ec * 4);
      const int mh = a.mh4[ec];
      float G[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) G[i] = a.G[ec * 9 + i];
      const float lam = a.mat[ec * 3 + 0], mu = a.mat[ec * 3 + 1], rinv = a.mat[ec * 3 + 2];
      const float* Qg = a.Q + grp * (int64_t)(RT * 36 * 64);
      const int gs0 = a.dslot[ec];
      const int gs = live ? gs0 : -1;
      float* gd = gs >= 0 ? a.gD + (int64_t)gs * (N + 1) * B * 9 : nullptr;

      // I~ = Q + J (J = sum_{k>=1} Dk/(k+1)) is parked in memory in the same
      // fragment layout (one coalesced access per register) so that the CK
      // registers are free for the face and volume phases, which stream I~
      // back (mostly from L2).
      float* Ig = a.Ib + grp * (int64_t)(RT * 36 * 64);
      // I~ parked in this wavefront's LDS slice (BF16) or in HBM (see PredLds)
      constexpr bool LP = PredLds<Op, N, W>::park_lds;
      constexpr int TF = PredLds<Op, N, W>::f32_tiles;  // FP32: leading row tiles of I~ kept in LDS
      unsigned short* ilds = reinterpret_cast<unsigned short*>(lds_raw + L::bytes) + w * PredLds<Op, N, W>::slice;
      float* flds = reinterpret_cast<float*>(lds_raw + L::bytes) + w * (TF * 36 * 64);
      {
        float J[RT1][4][9];
        CK<Op, N, AC>::run(J, Qg, lane, lds, G, lam, mu, rinv, el, g, gd);
        // a row tile of Q is loaded before any of its stores: raw buffer
        // accesses may alias, so a store between two loads would serialise them
        const GroupBuf qb(Qg, RT * 36 * 256, lane), ib(Ig, RT * 36 * 256, lane);
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          float x[36];
#pragma unroll
          for (int r = 0; r < 36; ++r)
            x[r] = (carried<AC>(r % 9) && 16 * t + 4 * (r / 9) < B) ? qb.ld(t * 36 + r) : 0.0f;  // padding rows: 0
#pragma unroll
          for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int p = 0; p < 9; ++p) {
              if (!carried<AC>(p)) continue;
              float y = x[v * 9 + p];
              if (t < RT1) y += J[t < RT1 ? t : 0][v][p];
              if constexpr (LP)
                ilds[((t * 4 + v) * 9 + p) * 64 + lane] = f2bf_dev(y);
              else if (t < TF)
                flds[((t * 4 + v) * 9 + p) * 64 + lane] = y;
              else
                ib.st((t * 4 + v) * 9 + p, y);
            }
        }
      }
      __builtin_amdgcn_sched_barrier(0);

      f4 dq[RT][9];
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int p = 0; p < 9; ++p)
          if (carried<AC>(p)) dq[t][p] = f4{0.f, 0.f, 0.f, 0.f};

      // rows of I~, read through a laundered base (one per contraction, so the
      // reads are not merged across contractions and kept live)
      auto itil_at = [&](const float* ip) {
        const GroupBuf ib(ip, RT * 36 * 256, lane);
        const float* fl = flds + opaque_zero();
        return [=](int t, int v, float (&b)[9]) {
#pragma unroll
          for (int p = 0; p < 9; ++p) {
            if (!carried<AC>(p)) continue;
            if constexpr (LP)
              b[p] = __uint_as_float((unsigned)ilds[((t * 4 + v) * 9 + p) * 64 + lane] << 16);
            else if (t < TF)
              b[p] = fl[((t * 4 + v) * 9 + p) * 64 + lane];
            else
              b[p] = ib.ld((t * 4 + v) * 9 + p);
          }
        };
      };

      // faces: traces at the nodes, hand-over, own-trace flux, lift. A real
      // loop: unrolled, the four faces' live ranges overlap and spill.
#pragma unroll 1
      for (int f = 0; f < 4; ++f) {
        // this face's flux coefficients, requested before the trace products
        float c[11];
#pragma unroll
        for (int i = 0; i < 11; ++i) c[i] = a.RCm[(ec * 4 + f) * 12 + i];
        f4 va[FT][9];
#pragma unroll
        for (int t = 0; t < FT; ++t)
#pragma unroll
          for (int p = 0; p < 9; ++p)
            if (carried<AC>(p)) va[t][p] = f4{0.f, 0.f, 0.f, 0.f};
        const View<R, L::ldE, false> AE(lds + L::oE + f * 16 * FT * L::ldE, L::total);
        contract_fn<Op, View<R, L::ldE, false>, RT, FT, true, false, AC>(va, AE, B, el, g, itil_at(Ig));
        float V[FT][4][9];
#pragma unroll
        for (int t = 0; t < FT; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const bool ok = 16 * t + 4 * v + g < Bf;  // node in slot (t, g, v)
#pragma unroll
            for (int p = 0; p < 9; ++p)
              if (carried<AC>(p)) V[t][v][p] = ok ? va[t][p][v] : 0.0f;
            embed<AC>(V[t][v]);  // the neighbour reads nine quantities
          }
        // hand-over into the neighbour's inbox (its node numbering, its time
        // step): a neighbour in the same cluster gets the full-step trace; a
        // coarser one half of it, accumulated over this element's two steps
        // (the parity of the step is per element: a launch may span clusters);
        // a finer one gets the full-step
        // trace here, which the half-step fix-up turns into its two halves.
        // Loads are unconditional (valid indices for every lane); only the
        // stores are masked.
        {
          const int md0 = (mh >> (8 * f)) & 3;
          const int32_t tg0 = f == 0 ? tg4[0] : (f == 1 ? tg4[1] : (f == 2 ? tg4[2] : tg4[3]));
          const int h = (mh >> (8 * f + 2)) & 7;
          const bool send = live && md0 != 0;
          const bool half = md0 == 3;
          const int parity = sc.parity(ec);
          const int32_t tg = send ? tg0 : 0;
#pragma unroll
          for (int t = 0; t < FT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int node = 16 * t + 4 * v + g;
              const int mr = perm[h * Bf + (node < Bf ? node : Bf - 1)];
              if (!send || node >= Bf) continue;
              float* blk = a.In + in_block(tg >> 2, tg & 3, mr, FT) * 576;
              const int l = in_lane(tg >> 2, mr);
              if (half && parity) {
                // second step of the pair: add to the first half (one writer per
                // slot; a no-return atomic keeps the load out of this kernel)
#pragma unroll
                for (int p = 0; p < 8; ++p) atomicAdd(blk + 8 * l + p, 0.5f * V[t][v][p]);
                atomicAdd(blk + 512 + l, 0.5f * V[t][v][8]);
              } else {
                const float s = half ? 0.5f : 1.0f;
                f4* d8 = reinterpret_cast<f4*>(blk + 8 * l);
                d8[0] = f4{s * V[t][v][0], s * V[t][v][1], s * V[t][v][2], s * V[t][v][3]};
                d8[1] = f4{s * V[t][v][4], s * V[t][v][5], s * V[t][v][6], s * V[t][v][7]};
                blk[512 + l] = s * V[t][v][8];
              }
            }
        }
#pragma unroll
        for (int t = 0; t < FT; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            float out[9];
            node_flux_q<AC, AC>(c, lam, mu, rinv, V[t][v], out);
#pragma unroll
            for (int p = 0; p < 9; ++p)
              if (carried<AC>(p)) V[t][v][p] = out[p];
          }
        const View<R, L::ldL, false> AL(lds + L::oL + f * L::PB * L::ldL, L::total);
        contract_fn<Op, View<R, L::ldL, false>, FT, RT, false, true, AC>(dq, AL, Bf, el, g,
                                                            [&](int t, int v, float (&b)[9]) {
#pragma unroll
                                                              for (int p = 0; p < 9; ++p)
                                                                if (carried<AC>(p)) b[p] = V[t][v][p];
                                                            });
      }

      // volume: dq += sum_d K^d (I~ (dt A*_d)^T) over the rows of I~ below B1,
      // the three directions from one pass over I~
      volume<Op, N, AC>(dq, lds, itil_at(Ig), G, lam, mu, rinv, el, g);
      __builtin_amdgcn_sched_barrier(0);

      {
        // Q += dq for live elements and rows below B
        // QB row tiles are requested before the first of their stores (raw
        // buffer accesses may alias, so a store orders later loads behind it):
        // one memory latency per QB tiles. All four tiles at order 6 in BF16;
        // two where registers are tighter.
        constexpr int QB = (L::BF && RT <= 4) ? RT : 2;
        const GroupBuf qb(a.Q + grp * (int64_t)(RT * 36 * 64), RT * 36 * 256, lane);
#pragma unroll
        for (int t0 = 0; t0 < RT; t0 += QB) {
          float q[QB][36];
#pragma unroll
          for (int u = 0; u < QB; ++u)
#pragma unroll
            for (int r = 0; r < 36; ++r)
              if (carried<AC>(r % 9))
                q[u][r] = (t0 + u < RT && 16 * (t0 + u) + 4 * (r / 9) < B) ? qb.ld((t0 + u) * 36 + r) : 0.0f;
#pragma unroll
          for (int u = 0; u < QB; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int t = t0 + u;
              if (t >= RT || !live || 16 * t + 4 * v + g >= B) continue;
              float y[9];
#pragma unroll
              for (int p = 0; p < 9; ++p)
                if (carried<AC>(p)) y[p] = q[u][v * 9 + p] + dq[t < RT ? t : 0][p][v];
              embed<AC>(y);  // the 4-quantity form stores s_yy = s_zz = s_xx and zero shear
#pragma unroll
              for (int p = 0; p < 9; ++p) qb.st((t * 4 + v) * 9 + p, y[p]);
            }
        }
      }
    };
    if (__builtin_amdgcn_readfirstlane(a.gac[grp]))
      body(std::true_type{});
    else
      body(std::false_type{});
  }
}

// corrector: (face, node tile) steps whose inbox traces are requested ahead
constexpr int kCorrAhead = 1;

// Corrector: Q -= sum_f L_f flux(neighbour trace of face f). The output rows
// are produced in SPLIT passes (the face fluxes are recomputed per
// pass from the inbox, which is L2-resident by then) so that the accumulators
// of one pass leave room for two wavefronts per SIMD: the two-pass form is
// compiled for at most 256 registers up to order 6 (at order 7 that would
// spill, and it keeps one wavefront per SIMD).
template <class Op, int N, int W, int SPLIT>
__global__ __launch_bounds__(64 * W, (SPLIT >= 2 && N <= 5) ? 2 : 1) void k_correct_tuned(TArgs a, int64_t e0, int64_t e1,
                                                                               int remap) {
  using L = Lay<Op, N>;
  constexpr int B = L::B, Bf = L::Bf, RT = L::RT, FT = L::FT;
  constexpr int NS = (SPLIT > RT) ? RT : SPLIT;
  constexpr int MH = (RT + NS - 1) / NS;  // row tiles per pass
  constexpr int CD = kCorrAhead;  // inbox steps requested ahead
  using R = RefT<Op>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  // only the lifts (and the tail their reads may run into) are staged: ldsL
  // holds the block from offset oL on
  const R* ldsL = reinterpret_cast<const R*>(lds_raw);
  stage_ref<Op>(lds_raw, reinterpret_cast<const R*>(a.ref) + L::oL, L::lift_elems * L::esz, 64 * W);
  if constexpr (split3<Op>)  // the lo image's lifts after the hi image's
    stage_ref<Op>(lds_raw + L::lift_elems * L::esz, reinterpret_cast<const R*>(a.ref) + L::total + L::oL,
                  L::lift_elems * L::esz, 64 * W);
  __syncthreads();
  // the wavefront index is uniform across the wavefront: keep it (and every
  // group base and buffer descriptor derived from it) in scalar registers
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int el = lane & 15, g = lane >> 4;
  const int64_t gfirst = e0 >> 4, glast = (e1 - 1) >> 4;
  for (int64_t grp = gfirst + logical_block(remap) * W + w; grp <= glast; grp += (int64_t)gridDim.x * W) {
    auto body = [&](auto form) {
      constexpr bool AC = decltype(form)::value;
      const int64_t e = grp * 16 + el;
      const bool live = e >= e0 && e < e1;
      const int64_t ec = live ? e : e0;
      const float lam = a.mat[ec * 3 + 0], mu = a.mat[ec * 3 + 1], rinv = a.mat[ec * 3 + 2];
#pragma unroll
      for (int h = 0; h < NS; ++h) {
        const int t0 = h * MH;
        f4 dq[MH][9];
#pragma unroll
        for (int t = 0; t < MH; ++t)
#pragma unroll
          for (int p = 0; p < 9; ++p)
            if (carried<AC>(p)) dq[t][p] = f4{0.f, 0.f, 0.f, 0.f};
        // the (face, node tile) steps are software-pipelined: the inbox traces
        // of step s + CD are requested while step s computes its Riemann fluxes
        // and its rows of the lift (one scheduling region per step, so the
        // requests are not sunk to their use)
        constexpr int NSTEP = 4 * FT;
        const float* inb = a.In + grp * 4 * (int64_t)(FT * 4 * 576);
        auto load_step = [&](int s, float(&dst)[4][9]) {
          const float* blk0 = inb + s * (4 * 576);  // face s / FT, tile s % FT
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if (16 * (s % FT) + 4 * v >= Bf) {  // all four nodes of the register are padding
#pragma unroll
              for (int p = 0; p < 9; ++p) dst[v][p] = 0.0f;
              continue;
            }
            const float* blk = blk0 + v * 576;
            const f4 i0 = reinterpret_cast<const f4*>(blk + 8 * lane)[0];
            const f4 i1 = reinterpret_cast<const f4*>(blk + 8 * lane)[1];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
              dst[v][p] = i0[p];
              dst[v][4 + p] = i1[p];
            }
            dst[v][8] = blk[512 + lane];
          }
        };
        // flux coefficients of the current face and the next (requested one
        // step before the next face starts)
        float c[2][11];
#pragma unroll
        for (int i = 0; i < 11; ++i) c[0][i] = a.RCp[(ec * 4) * 12 + i];
        float tb[CD + 1][4][9];
#pragma unroll
        for (int s = 0; s < CD; ++s) load_step(s, tb[s]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < NSTEP; ++s) {
          const int f = s / FT, t = s % FT;
          if (s + CD < NSTEP) load_step(s + CD, tb[(s + CD) % (CD + 1)]);
          if (t == FT - 1 && f + 1 < 4) {
#pragma unroll
            for (int i = 0; i < 11; ++i) c[(f + 1) & 1][i] = a.RCp[(ec * 4 + f + 1) * 12 + i];
          }
          float(&cur)[4][9] = tb[s % (CD + 1)];
          float V[4][9];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            float out[9];
            node_flux_q<AC, false>(c[f & 1], lam, mu, rinv, cur[v], out);  // the neighbour's trace has nine quantities
            const bool ok = 16 * t + 4 * v + g < Bf;  // node in slot (t, g, v)
#pragma unroll
            for (int p = 0; p < 9; ++p)
              if (carried<AC>(p)) V[v][p] = ok ? out[p] : 0.0f;
          }
          const View<R, L::ldL, false> AL(ldsL + f * L::PB * L::ldL + t0 * 16 * L::ldL + 16 * t, L::lift_elems);
          contract_fn<Op, View<R, L::ldL, false>, 1, MH, false, true, AC>(dq, AL, Bf - 16 * t < 16 ? Bf - 16 * t : 16, el,
                                                                      g, [&](int, int v, float (&b)[9]) {
#pragma unroll
                                                                        for (int p = 0; p < 9; ++p)
                                                                          if (carried<AC>(p)) b[p] = V[v][p];
                                                                      });
          __builtin_amdgcn_sched_barrier(0);
        }
        // up to four of the pass's row tiles are requested before their stores
        // (raw buffer accesses may alias): one memory latency per batch; one
        // tile at a time in the two-pass form, whose registers must leave room
        // for two wavefronts per SIMD
        constexpr int QB = SPLIT >= 2 ? 1 : (MH < 4 ? MH : 4);
        const GroupBuf qb(a.Q + grp * (int64_t)(RT * 36 * 64), RT * 36 * 256, lane);
#pragma unroll
        for (int u0 = 0; u0 < MH; u0 += QB) {
          float q[QB][36];
#pragma unroll
          for (int u = 0; u < QB; ++u)
#pragma unroll
            for (int r = 0; r < 36; ++r)
              if (carried<AC>(r % 9))
                q[u][r] = (u0 + u < MH && t0 + u0 + u < RT && 16 * (t0 + u0 + u) + 4 * (r / 9) < B)
                              ? qb.ld((t0 + u0 + u) * 36 + r)
                              : 0.0f;
#pragma unroll
          for (int u = 0; u < QB; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int uu = u0 + u, t = t0 + uu;
              if (uu >= MH || t >= RT || !live || 16 * t + 4 * v + g >= B) continue;
              float y[9];
#pragma unroll
              for (int p = 0; p < 9; ++p)
                if (carried<AC>(p)) y[p] = q[u][v * 9 + p] + dq[uu < MH ? uu : 0][p][v];
              embed<AC>(y);
#pragma unroll
              for (int p = 0; p < 9; ++p) qb.st((t * 4 + v) * 9 + p, y[p]);
            }
        }
      }
    };
    if (__builtin_amdgcn_readfirstlane(a.gac[grp]))
      body(std::true_type{});
    else
      body(std::false_type{});
  }
}

int g_num_cus = 0;

int num_cus() {
  if (g_num_cus == 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      g_num_cus = prop.multiProcessorCount;
    if (g_num_cus <= 0) g_num_cus = 256;
  }
  return g_num_cus;
}

// Work-groups per launch: one per W 16-element groups (cap 0), or at most cap
// per compute unit, persistent work-groups striding over the groups.
unsigned grid_size(int64_t ngroups, int W, int cap) {
  const int64_t full = (ngroups + W - 1) / W;
  if (cap <= 0) return (unsigned)full;
  return (unsigned)std::min<int64_t>(full, (int64_t)num_cus() * cap);
}

template <class KernelPtr>
hipError_t prep(KernelPtr k, int lds) {
  return hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}


template <class Op, int N, int W>
hipError_t launch_pred(const TArgs& a, int64_t e0, int64_t e1, const Sched& sc, const LaunchCfg& c, hipStream_t s) {
  if (e1 <= e0) return hipSuccess;
  using L = Lay<Op, N>;
  const int64_t ng = ((e1 - 1) >> 4) - (e0 >> 4) + 1;
  const unsigned grid = grid_size(ng, W, c.cap);
  constexpr int lds = PredLds<Op, N, W>::bytes;
  static_assert(lds <= 160 * 1024, "predictor LDS exceeds the 160 KB of a CU");
  static hipError_t attr = prep(k_predict_tuned<Op, N, W>, lds);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL((k_predict_tuned<Op, N, W>), dim3(grid), dim3(64 * W), lds, s, a, e0, e1, sc, c.remap);
  return hipGetLastError();
}

template <class Op, int N, int W, int SPLIT>
hipError_t launch_corr(const TArgs& a, int64_t e0, int64_t e1, const LaunchCfg& c, hipStream_t s) {
  if (e1 <= e0) return hipSuccess;
  using L = Lay<Op, N>;
  const int64_t ng = ((e1 - 1) >> 4) - (e0 >> 4) + 1;
  const unsigned grid = grid_size(ng, W, c.cap);
  static hipError_t attr = prep(k_correct_tuned<Op, N, W, SPLIT>, L::lift_bytes);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL((k_correct_tuned<Op, N, W, SPLIT>), dim3(grid), dim3(64 * W), L::lift_bytes, s, a, e0, e1,
                     c.remap);
  return hipGetLastError();
}

template <class Op>
hipError_t pred_dispatch(int N, const LaunchCfg& c, const TArgs& a, int64_t e0, int64_t e1, const Sched& sc,
                         hipStream_t s) {
  // the variant picks the sibling operand type of the same precision
  if constexpr (std::is_same<Op, OpF32>::value)
    if (c.variant == 1) return pred_dispatch<OpF32H>(N, c, a, e0, e1, sc, s);
  if constexpr (std::is_same<Op, OpBF16>::value)
    if (c.variant == 1) return pred_dispatch<OpBF16W>(N, c, a, e0, e1, sc, s);
  const int W = c.waves;
  // a shape whose LDS block does not fit a CU (split BF16 at order 7: two
  // images) is not compiled; the set-up rejects that combination
#define SEIS_P(NN, WW)                                                          \
  if (N == NN && W == WW) {                                                     \
    if constexpr (PredLds<Op, NN, WW>::bytes <= 160 * 1024)                     \
      return launch_pred<Op, NN, WW>(a, e0, e1, sc, c, s);                      \
    else                                                                        \
      return hipErrorInvalidValue;                                              \
  }
  SEIS_P(2, 2) SEIS_P(2, 4)
  SEIS_P(3, 2) SEIS_P(3, 4)
  SEIS_P(4, 2) SEIS_P(4, 4)
  SEIS_P(5, 2) SEIS_P(5, 4)
  SEIS_P(6, 2) SEIS_P(6, 4)
#undef SEIS_P
  return hipErrorInvalidValue;
}

template <class Op>
hipError_t corr_dispatch(int N, const LaunchCfg& c, const TArgs& a, int64_t e0, int64_t e1, hipStream_t s) {
  const int W = c.waves;
#define SEIS_C(NN, WW)                                                                   \
  if (N == NN && W == WW)                                                                \
    return c.split == 1 ? launch_corr<Op, NN, WW, 1>(a, e0, e1, c, s) : launch_corr<Op, NN, WW, 2>(a, e0, e1, c, s);
  SEIS_C(2, 2) SEIS_C(2, 4)
  SEIS_C(3, 2) SEIS_C(3, 4)
  SEIS_C(4, 2) SEIS_C(4, 4)
  SEIS_C(5, 2) SEIS_C(5, 4)
  SEIS_C(6, 2) SEIS_C(6, 4)
#undef SEIS_C
  return hipErrorInvalidValue;
}

}  // namespace

}  // namespace seis
