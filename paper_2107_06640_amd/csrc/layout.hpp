// Device layouts of the element state and of the face inboxes.
//
// Elements are processed by 64-lane wavefronts in groups of 16. Inside a
// group the data is stored in the order in which a wavefront holds it in the
// output fragments of a 16x16 matrix-core product: for row tile t (rows
// 16t..16t+15), value slot v (0..3) and quantity p, 64 consecutive values in
// lane order, lane = el + 16 g holding element el of the group at row
// 16t + 4v + g. One register of the wavefront is then one coalesced
// 256-byte load or store, and the plain kernels reach any (element, row,
// quantity) through the same index function.
//
// Inside a tile the rows run over the lane groups first (row 16t + 4v + g,
// not 16t + 4g + v): a register v then holds four consecutive rows, one per
// lane group, which is one K slab of an FP32 16x16x4 product. A tile that is
// only partly filled (the CK derivatives have 35, 20, 10, 4 and 1 rows at
// degree 5) then needs ceil(rows / 4) slabs instead of up to four.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace seis {

__host__ __device__ constexpr int row_tiles(int rows) { return (rows + 15) / 16; }

// Q[e][r][p] with RT row tiles per element.
__host__ __device__ inline int64_t qidx(int64_t e, int r, int p, int RT) {
  const int64_t grp = e >> 4;
  const int el = int(e & 15);
  const int t = r >> 4, v = (r >> 2) & 3, g = r & 3;
  return (((grp * RT + t) * 4 + v) * 9 + p) * 64 + el + 16 * g;
}

// In[e][f][m][p] with FT node tiles per face. Node m of a face sits in tile
// m >> 4, register v = (m >> 2) & 3 and lane group g = m & 3 (the transpose of
// the row order of Q inside a tile, so that a partial last tile fills whole
// register slots first). The nine quantities of one node sit together: per
// (group, face, tile, v) a block of 576 values, the quantities 0..7 of lane l
// at 8l..8l+7 (two aligned 16-byte vectors) and quantity 8 at 512 + l. A
// writer then hands over one node with three stores instead of nine, and a
// reader gets it with three loads.
__host__ __device__ inline int64_t in_block(int64_t e, int f, int m, int FT) {
  const int t = m >> 4, v = (m >> 2) & 3;
  return (((e >> 4) * 4 + f) * FT + t) * 4 + v;
}
__host__ __device__ inline int in_lane(int64_t e, int m) { return int(e & 15) + 16 * (m & 3); }
__host__ __device__ inline int64_t inidx(int64_t e, int f, int m, int p, int FT) {
  const int l = in_lane(e, m);
  return in_block(e, f, m, FT) * 576 + (p < 8 ? 8 * l + p : 512 + l);
}

// Position of row r inside its 16-row tile under the layout above when the
// tile is read as a 16 x 16 matrix-core fragment (lane group g, slot v ->
// fragment row 4g + v): the transposition of the 4 x 4 (g, v) grid, its own
// inverse.
__host__ __device__ constexpr int tile_perm(int r) { return (r & ~15) | ((r & 3) << 2) | ((r >> 2) & 3); }

// Sizes (values) of the padded arrays for E elements.
__host__ __device__ inline int64_t q_size(int64_t E, int RT) { return ((E + 15) >> 4) * RT * 4 * 9 * 64; }
__host__ __device__ inline int64_t in_size(int64_t E, int FT) { return ((E + 15) >> 4) * 4 * FT * 4 * 9 * 64; }

}  // namespace seis
