// Sets of dense Hermitian blocks applied as y = sum_b R_b^T A_b R_b x: the
// macro-grid operator (one block per coarse element, Sec. 3 "Prolongation"),
// the additive Schwarz smoother (one inverse per vertex patch, Sec. 3
// "V-cycle and smoother") and the coarsest-level inverse.
//
// Storage: only the upper triangle of 32x32 tiles of each block, tiles of
// block b ordered by tile column J then tile row I <= J; diagonal tiles are
// stored whole.  Inside a tile, entry (r, c) sits at [k][lane] with
// lane = 8 (r/4) + c/4 and k = 4 (r%4) + c%4, so that one wave reads a tile
// with 16 fully coalesced 64-lane loads and every lane holds a 4x4 sub-block.
//
// Apply (two kernels, deterministic): one wave per (block, tile column J)
// streams the tiles of that column once, producing A_IJ x_J (row sums, per
// tile) and sum_{I<J} A_IJ^H x_I (column sums, per column) into a partial
// buffer; then one thread per vector entry adds the partials of every block
// holding it, in a fixed order, and applies the epilogue.
#pragma once
#include "common.hpp"

namespace dpg {

enum { RED_SET = 0, RED_RESID = 1, RED_AXPY = 2, RED_SET_SCALED = 3 };

struct HermSet {
  int nblk = 0;
  int64_t nvec = 0;          // length of the target vector
  int64_t ntiles = 0, npart = 0, nunits = 0;
  std::vector<int32_t> n_h;  // block sizes (host)
  std::vector<int64_t> tile_off_h;
  DevBuf<int32_t> bn;
  DevBuf<int64_t> tile_off, part_off, idx_off;
  DevBuf<int32_t> idx;       // concatenated vector indices of every block
  DevBuf<int2> units;        // (block, J), largest columns first
  DevBuf<int4> tdesc;        // (block, I, J, 0) per stored tile (packing)
  DevBuf<int32_t> red_ptr;   // CSR over vector entries
  DevBuf<int2> red_ent;      // (block, local row)
  DevBuf<double2> t64;       // tiles, FP64
  DevBuf<float2> t32;        // tiles, FP32 (mixed precision)
  DevBuf<double2> p64;       // partials
  DevBuf<float2> p32;
  Prof *prof = nullptr;      // kernel timing of the owning context
  int64_t bytes_fp64() const { return ntiles * 1024 * 16; }
  int64_t bytes_fp32() const { return ntiles * 1024 * 8; }
  // algorithmic bytes: packed Hermitian n(n+1)/2 entries per block
  int64_t packed_entries() const;

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
template <typename T>
void herm_apply(HermSet &H, const cplx_t<T> *x, cplx_t<T> *y, const cplx_t<T> *r, int mode,
                T theta, hipStream_t s);

}  // namespace dpg
