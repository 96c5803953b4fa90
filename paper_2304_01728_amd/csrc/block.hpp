// Multi-right-hand-side forms of the solve phase (nr columns at once).
//
// Block vectors hold nr columns interleaved: entry (d, k) of an n x nr block
// sits at d * nr + k, so the gathers and scatters of the single-column path
// move nr contiguous values per index.  The operators are the same objects as
// in the single-column path (Hermitian block sets, transfer CSR matrices,
// condensation blocks); each stored block is streamed once per application
// for all nr columns, which turns the matrix-vector products into products
// with 32 x nr panels.
#pragma once
#include "common.hpp"
#include "hblocks.hpp"

namespace dpg {

constexpr int kMaxCols = 32;   // columns per block solve

// Work vectors of one Hermitian block set for nr columns.
struct HermBlockBufs {
  int cap = 0;
  DevBuf<double2> xl64, yl64;
  DevBuf<float2> xl32, yl32;
  // local vectors zeroed when allocated: a forward (below) writes only the
  // rows a vector entry maps to
  void ensure(const HermSet &H, int nr, bool fp64, bool fp32, Budget *bud, hipStream_t s);
};

// Y <- epilogue(sum_b R_b^T A_b R_b X) for nr columns (modes as herm_apply).
// gathered: W already holds the local rows of X (a previous application
// forwarded them).  fwd, fwd_bufs: a block set on the same vector and its
// buffers, whose local vectors receive the new Y for an application of fwd
// to Y that follows with gathered = true.  Rows of a block past its size
// may hold stale finite values from another width; they meet only the zero
// padding of the tiles.  One column goes through herm_apply (the single-
// vector local vectors of the sets).
template <typename T>
void herm_apply_blk(HermSet &H, HermBlockBufs &W, const cplx_t<T> *X, cplx_t<T> *Y,
                    const cplx_t<T> *R, int mode, T theta, int nr, hipStream_t s,
                    bool gathered = false, HermSet *fwd = nullptr,
                    HermBlockBufs *fwd_bufs = nullptr);

// The local vectors of a block set for nr columns stored column by column
// ([nr][nloc]: column k at k * nloc), so that the slice of one block is an
// n x nr column-major panel with leading dimension nloc (the smoother with
// recomputed patch inverses multiplies it with dense GEMMs).  FP64.
// xl <- R X (gather from the interleaved block vector X);
void herm_gather_cols(const HermSet &H, const double2 *X, double2 *xl, int nr, hipStream_t s);
// Y <- epilogue(sum_b R_b^T yl_b) into the interleaved block vector Y (modes
// as herm_apply).
void herm_scatter_cols(const HermSet &H, const double2 *yl, double2 *Y, const double2 *R,
                       int mode, double theta, int nr, hipStream_t s);

// y[i, k] (+)= sum_j val[j] x[col[j], k] over CSR rows.
template <typename T>
void launch_csr_blk(int64_t nrows, const int64_t *ptr, const int32_t *col, const T *val,
                    const cplx_t<T> *x, cplx_t<T> *y, int add, int nr, hipStream_t s);

// Macro condensation and expansion of nr columns (see launch_condense_local,
// launch_condense_reduce, launch_expand).
template <typename T>
void launch_condense_blk(const cplx_t<T> *WH, int nI, int nBf, const int32_t *blkI, int nblk,
                         int64_t nM, const int64_t *macro_B, const int32_t *red_ptr,
                         const int32_t *red_ent, const cplx_t<T> *rc, cplx_t<T> *c,
                         cplx_t<T> *rB, int nr, hipStream_t s);
template <typename T>
void launch_expand_blk(const cplx_t<T> *WH, const cplx_t<T> *Tinv, int nI, int nBf,
                       const int32_t *blkI, const int32_t *blkBm, int nblk, const cplx_t<T> *rc,
                       const cplx_t<T> *eB, int64_t nM, const int64_t *macro_B, cplx_t<T> *ec,
                       int nr, hipStream_t s);

// Column-major [nr][n] <-> interleaved [n][nr] (FP64).
void launch_interleave(int64_t n, int nr, const double2 *cols, double2 *blk, hipStream_t s);
void launch_deinterleave(int64_t n, int nr, const double2 *blk, double2 *cols, hipStream_t s);

// Column k of an interleaved block of width w: blk[:, k] = src (zero when src
// is null), or dst = blk[:, k].
void launch_set_col(int64_t n, int w, int k, const double2 *src, double2 *blk, hipStream_t s);
void launch_get_col(int64_t n, int w, int k, const double2 *blk, double2 *dst, hipStream_t s);
// dst (n x w_new) <- src (n x w_old), columns beyond w_old zero (dst != src).
void launch_rewidth(int64_t n, int w_old, int w_new, const double2 *src, double2 *dst,
                    hipStream_t s);

// ---- per-column CG on interleaved FP64 blocks ----------------------------------------
// Device scalars sc[q * kMaxCols + k] for column k: q = 0 rz, 1 pq, 2 alpha,
// 3 beta, 4 ||r||^2, 5 ||b||^2, 6 breakdown flag, 7 r^H z_old.  act[k] != 0
// marks a column that still iterates; a frozen column takes alpha = beta = 0,
// so its x, r and p stay as they are.
constexpr int kColDotBlocks = 256;
void cgb_dot(int64_t n, int nr, const double2 *a, const double2 *b, double *partial, double *sc,
             int q, hipStream_t s);                                  // sc[q] = Re(a^H b)
void cgb_alpha(int64_t n, int nr, const double2 *p, const double2 *qv, double *partial,
               double *sc, const int *act, hipStream_t s);
void cgb_update_xr(int64_t n, int nr, double2 *x, double2 *r, const double2 *p, const double2 *qv,
                   double *partial, double *sc, hipStream_t s);
void cgb_beta(int64_t n, int nr, const double2 *r, const double2 *z, const double2 *zold,
              double *partial, double *sc, const int *act, hipStream_t s);
void cgb_update_p(int64_t n, int nr, double2 *p, const double2 *z, const double *sc,
                  hipStream_t s);
// Scalars of a column that joins a running block solve (its x, p, z and z_old
// columns zero, r = b): rz = 1, the others 0, so that its first beta step
// sets p = z and rz = r^H z.
void cgb_reset_col(double *sc, int k, hipStream_t s);

}  // namespace dpg
