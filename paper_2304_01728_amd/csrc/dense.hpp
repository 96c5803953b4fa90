// Batched dense complex-FP64 linear algebra on gfx950: Cholesky (lower),
// forward triangular solve with many right-hand sides, and GEMM with
// normal / transposed / conjugate-transposed operands.  Every item of a batch
// has its own sizes and leading dimensions; matrices are column-major and
// addressed as base pointer + per-item element offset.
#pragma once
#include "common.hpp"

namespace dpg {

struct PotrfItem { int64_t a; int n, lda; };
struct TrsmItem { int64_t l, b; int n, ncols, ldl, ldb; };
struct GemmItem { int64_t a, b, c; int m, n, k, lda, ldb, ldc; };

enum { OP_N = 0, OP_T = 1, OP_C = 2 };

// In-place lower Cholesky A = L L^H of every item (upper triangle untouched).
// info[item] = 0 on success, j+1 if pivot j was not positive.
void potrf_batched(double2 *base, const PotrfItem *items_dev, int nitems, int *info_dev,
                   hipStream_t s);

// B <- L^-1 B for every item (L lower, from a Cholesky factor).  max_cols is
// the largest ncols of the batch.
void trsm_batched(const double2 *lbase, double2 *bbase, const TrsmItem *items_dev, int nitems,
                  int max_cols, hipStream_t s);

// C <- alpha op(A) op(B) + beta C for every item.  max_m / max_n bound the
// tile grid.
void gemm_batched(int opa, int opb, double2 alpha, const double2 *abase, const double2 *bbase,
                  double2 beta, double2 *cbase, const GemmItem *items_dev, int nitems, int max_m,
                  int max_n, hipStream_t s);

}  // namespace dpg
