// Batched dense complex-FP64 linear algebra on gfx950: Cholesky (lower),
// forward triangular solve with many right-hand sides, and GEMM with
// normal / transposed / conjugate-transposed operands.  Every item of a batch
// has its own sizes and leading dimensions; matrices are column-major and
// addressed as base pointer + per-item element offset.
//
// The factorisations proceed by 64-wide panels grouped in 128-wide blocks: a
// small kernel factors the 64x64 diagonal block of every item and inverts it
// in LDS, the panel is then a product with that inverse, and the updates are
// spread over (64x64 tiles x items), so that large blocks use the whole GPU
// instead of one compute unit each.  The diagonal-block inverses go to a
// caller-provided work area (dense_work_size elements), where a following
// triangular solve with the same factor can take them.
#pragma once
#include "common.hpp"

namespace dpg {

struct PotrfItem { int64_t a; int n, lda; };
struct TrsmItem { int64_t l, b; int n, ncols, ldl, ldb; };
struct GemmItem { int64_t a, b, c; int m, n, k, lda, ldb, ldc; };

enum { OP_N = 0, OP_T = 1, OP_C = 2 };
enum { GEMM_FULL = 0, GEMM_UPPER_LOWTRI = 1, GEMM_HERM = 2, GEMM_HERM_LOWTRI = 3 };

// Work-area size (double2 elements) for nitems items of order <= nmax.
int64_t dense_work_size(int nitems, int nmax);

// Optional per-kernel timing of one routine call: with prof on, every launch
// is timed with HIP events under its kernel's class (DPG_K_POTRF_DIAG ...
// DPG_K_TRSM_UPDATE) together with its share of the routine's algorithmic
// flops, the LAPACK count split by the steps of the blocked algorithm
// (diagonal block 4/3 kb^3, panel 4 m kb^2, updates 8 per complex
// multiply-add of the lower triangle; forward solves 4 kb^2 per column and
// 8 m kw per column of the updates, restricted to the lower triangle of the
// result for an identity right-hand side).  The item sizes come from the
// host: n (order per item) or n_all for every item, ncols likewise.
struct DenseProf {
  Prof *prof = nullptr;
  const int32_t *n = nullptr;
  int n_all = 0;
  const int32_t *ncols = nullptr;
  int ncols_all = 0;
  int order(int i) const { return n ? n[i] : n_all; }
  int cols(int i) const { return ncols ? ncols[i] : ncols_all; }
  bool on() const { return prof && prof->on; }
};

// In-place lower Cholesky A = L L^H of every item (upper triangle untouched).
// info[item] = 0 on success, j+1 if pivot j was not positive.  nmax = largest n.
// On return the work area holds the inverse of every diagonal block.
void potrf_batched(double2 *base, const PotrfItem *items_dev, int nitems, int *info_dev, int nmax,
                   double2 *work, hipStream_t s, const DenseProf *dp = nullptr);

// B <- L^-1 B for every item (L lower, from a Cholesky factor).  With
// identity_rhs, B must hold the identity and only the lower-triangular part
// of the result is formed (the rest stays zero).  inverses_ready: the work
// area already holds the diagonal-block inverses of L (left there by
// potrf_batched with the same items and max_n).
void trsm_batched(const double2 *lbase, double2 *bbase, const TrsmItem *items_dev, int nitems,
                  int max_n, int max_cols, bool identity_rhs, double2 *work, bool inverses_ready,
                  hipStream_t s, const DenseProf *dp = nullptr);

// C <- alpha op(A) op(B) + beta C for every item.  mode GEMM_UPPER_LOWTRI
// computes only the upper 64x64 tiles (tile row <= tile column) of a product
// whose operands are lower triangular in the inner index (X^H X with X lower
// triangular), starting the inner sum at the tile's diagonal.  GEMM_HERM and
// GEMM_HERM_LOWTRI are for Hermitian results (m = n, and C Hermitian on entry
// when beta != 0): they compute the upper tiles, as GEMM_FULL and
// GEMM_UPPER_LOWTRI do, and also store the conjugate transpose of each
// off-diagonal tile in the lower triangle.
void gemm_batched(int opa, int opb, double2 alpha, const double2 *abase, const double2 *bbase,
                  double2 beta, double2 *cbase, const GemmItem *items_dev, int nitems, int max_m,
                  int max_n, hipStream_t s, int mode = GEMM_FULL);

}  // namespace dpg
