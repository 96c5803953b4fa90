// Sets of dense Hermitian blocks applied as y = sum_b R_b^T A_b R_b x: the
// macro-grid operator (one block per coarse element, Sec. 3 "Prolongation"),
// the additive Schwarz smoother (one inverse per vertex patch, Sec. 3
// "V-cycle and smoother") and the coarsest-level inverse.
//
// Storage: only the upper triangle of 32x32 tiles of each block, tiles of
// block b ordered by tile column J then tile row I <= J.  Inside a tile,
// entry (r, c) sits at [k][lane] with lane = 8 (r/4) + c/4 and
// k = 4 (r%4) + c%4, so that one wave reads a tile with 16 fully coalesced
// 64-lane loads and every lane holds a 4x4 sub-block.  A diagonal tile keeps
// only the sub-blocks on and above its diagonal (36 of 64, the diagonal 4x4
// sub-blocks whole): [k][slot] with 36 slots, 576 entries instead of 1024.
//
// Apply (four kernels, deterministic):
//  1. gather:  x_loc[b] = R_b x, zero-padded to 32 nt_b entries;
//  2. columns: FP64: one wave per (block, tile column J, segment of two tile
//     rows) loads both tiles before any arithmetic, writes A_IJ x_J (row
//     sums, one 32-vector per tile, laid out tile row by tile row) and
//     sum_{I<J} A_IJ^H x_I over the segment (one 32-vector per segment);
//     FP32: one wave per (block, pair of tile columns J0, J1, chunk of tile
//     rows) writes A_I,J0 x_J0 + A_I,J1 x_J1 per row I (one 32-vector per
//     two tiles) and the column sums of both columns over the chunk;
//  3. rows:    half a wave per (block, tile row I) adds the column partials
//     of column I and the row partials of row I (contiguous) into y_loc[b];
//  4. scatter: one thread per vector entry adds y_loc of every block holding
//     it, in a fixed order, and applies the epilogue; it can also write the
//     result into the local vector of the set applied next (the smoother
//     after a residual, the residual after a smoother), whose gather is
//     then left out.
#pragma once
#include "common.hpp"

namespace dpg {

enum { RED_SET = 0, RED_RESID = 1, RED_AXPY = 2, RED_SET_SCALED = 3 };

constexpr int kTileFull = 1024, kTileDiag = 576, kDiagSlots = 36;

// Entry offset of tile (I, J), I <= J, inside its block: the tile columns
// before J hold J (J - 1) / 2 full tiles and J diagonal tiles, and the tiles
// of column J come in order I = 0..J.
__host__ __device__ __forceinline__ int64_t tile_entry(int I, int J) {
  return (int64_t)kTileFull * ((int64_t)J * (J - 1) / 2 + I) + (int64_t)kTileDiag * J;
}

// Slot of sub-block (ra, cb), ra <= cb, in a diagonal tile: row-major order
// of the upper triangle of the 8 x 8 sub-block grid.
__host__ __device__ __forceinline__ int diag_slot(int ra, int cb) {
  return ra * 8 - ra * (ra - 1) / 2 + (cb - ra);
}

struct HermSet {
  int nblk = 0;
  int64_t nvec = 0;          // length of the target vector
  int64_t ntiles = 0, npart = 0, nunits = 0, nrows = 0, nloc = 0, packed = 0;
  int64_t nent = 0;          // stored tile entries
  int64_t full = 0;          // sum of n_b^2 (entries of the full blocks)
  std::vector<int32_t> n_h;  // block sizes (host)
  std::vector<int64_t> tile_off_h, ent_off_h;   // per block: first tile index, first entry
  std::vector<int64_t> loc_off_h;                // per block: first row of its local vectors
  DevBuf<int32_t> bn;
  DevBuf<int64_t> ent_off, cp_off, rp_off, loc_off;
  DevBuf<int32_t> gidx;      // [nloc] vector index of each padded local row, -1 = padding
  DevBuf<int4> units;        // two int4 descriptors per (block, J, tile-row pair), block order
  DevBuf<int2> rows;         // (block, I)
  DevBuf<int4> rowd;         // per (block, I): column-partial base, row-partial base,
                             // segment count | (row-partial count << 16), local offset
  // the same for the FP32 apply by column pairs (strips); partials in p32
  DevBuf<int4> sunits, srowd;
  int64_t snunits = 0, snpart = 0;
  DevBuf<int4> tdesc;        // (block, I, J, 0) per stored tile (packing)
  DevBuf<int32_t> red_ptr;   // CSR over vector entries
  DevBuf<int32_t> red_ent;   // offsets into the local vectors
  DevBuf<double2> t64;       // tiles, FP64
  DevBuf<float2> t32;        // tiles, FP32 (mixed precision)
  DevBuf<double2> p64, xl64, yl64;   // partials and local vectors
  DevBuf<float2> p32, xl32, yl32;
  Prof *prof = nullptr;      // kernel timing of the owning context
  int64_t bytes_fp64() const { return nent * 16; }
  int64_t bytes_fp32() const { return nent * 8; }
  // algorithmic entries: packed Hermitian n(n+1)/2 per block
  int64_t packed_entries() const { return packed; }

  // idx: per block the vector index of each local row (concatenated).
  void build(const std::vector<int32_t> &sizes, const std::vector<int32_t> &idx_concat,
             int64_t nvec_, bool fp64, bool fp32, Budget *bud, hipStream_t s);
  // Fill the tiles from dense column-major sources: block b reads
  // src[src_off[b] + map(i) + map(j) * ld[b]] where map is the identity when
  // map_off[b] < 0, else map[map_off[b] + i].
  void pack(const double2 *src, const int64_t *src_off_dev, const int32_t *ld_dev,
            const int64_t *map_off_dev, const int32_t *map_dev, hipStream_t s, int64_t tile0 = 0,
            int64_t ntile_count = -1);
};

// y <- epilogue(sum_b R_b^T A_b R_b x): RED_SET y = Ax; RED_RESID y = r - Ax;
// RED_AXPY y += theta Ax; RED_SET_SCALED y = theta Ax.
// gathered: the local vector of H already holds R_b x (a previous
// application forwarded x to H), so x is not read.  fwd: a block set on the
// same vector whose local vector receives the new y (its padding rows stay
// zero: they are zeroed at build and never written by a forward), for an
// application of fwd to y that follows with gathered = true.
template <typename T>
void herm_apply(HermSet &H, const cplx_t<T> *x, cplx_t<T> *y, const cplx_t<T> *r, int mode,
                T theta, hipStream_t s, bool gathered = false, HermSet *fwd = nullptr);

}  // namespace dpg
