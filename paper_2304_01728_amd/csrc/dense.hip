// Batched dense complex-FP64 kernels: Cholesky, forward solve, GEMM.
//
// The rank-k updates share one tile routine: a workgroup of 256 threads
// stages 64x16 slices of op(A) and 16x64 slices of op(B) in LDS and its four
// waves accumulate the 64x64 complex output tile on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64).  The FP64 matrix and vector peaks of MI355X are
// equal (78.6 TFLOP/s); the matrix cores win because they reuse each operand
// sixteen times inside the instruction, where vector FMAs would need one LDS
// read per two complex multiply-adds.
//
// Factorisations are blocked twice: 128-wide blocks, each processed in
// 32-wide panel steps (one launch for the panel -- one workgroup per item or
// per 64 rows -- and one for the rank-32 update, which stays inside the
// 128-wide block), then one rank-128 update of the trailing matrix spread
// over (64x64 tiles x items).  The trailing matrix is thus read and written
// once per 128 columns.
#include <cmath>

#include "dense.hpp"

namespace dpg {
namespace {

constexpr int TM = 64, TN = 64, TK = 16, NT = 256, NB = 32, NBO = 128;
typedef double v4d __attribute__((ext_vector_type(4)));

struct GemmSmem {
  double2 As[TM][TK + 1];
  double2 Bs[TK][TN + 1];
};

template <int OP> __device__ inline double2 ld_op(const double2 *X, int ldx, int r, int c) {
  // element (r, c) of op(X)
  if (OP == OP_N) return X[r + (int64_t)c * ldx];
  double2 v = X[c + (int64_t)r * ldx];
  if (OP == OP_C) v.y = -v.y;
  return v;
}

// C[r0:r0+64, c0:c0+64] (clipped to m x n) <- alpha op(A) op(B) + beta C with
// inner indices k_begin..k-1.  lower_only leaves entries above the diagonal
// alone.  Must be called by all 256 threads of the workgroup.
template <int OPA, int OPB>
__device__ __forceinline__ void gemm_tile(int m, int n, int k, int k_begin, int r0, int c0, double2 alpha,
                          const double2 *A, int lda, const double2 *B, int ldb, double2 beta,
                          double2 *C, int ldc, bool lower_only, GemmSmem &sm) {
  const int tid = threadIdx.x;
  // FP64 matrix cores: v_mfma_f64_16x16x4f64 computes D(16x16) += A(16x4) B(4x16)
  // with A[i][k] in lane i + 16k, B[k][j] in lane j + 16k and D[i][j] in
  // lane j + 16 (i % 4), element i / 4.  Wave w owns the 32x32 sub-tile at
  // (32 (w / 2), 32 (w % 2)) as 2x2 blocks; a complex product takes four real
  // MFMAs (re*re - im*im, re*im + im*re).
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = 32 * (wave >> 1), wc = 32 * (wave & 1);
  const int li = lane & 15, lk = lane >> 4;
  v4d acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc_re[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
      acc_im[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    }
#pragma unroll 1
  for (int k0 = k_begin; k0 < k; k0 += TK) {
    for (int e = tid; e < TM * TK; e += NT) {
      int rr, kk;
      if (OPA == OP_N) { rr = e % TM; kk = e / TM; } else { kk = e % TK; rr = e / TK; }
      const int r = r0 + rr, kg = k0 + kk;
      sm.As[rr][kk] = (r < m && kg < k) ? ld_op<OPA>(A, lda, r, kg) : mk(0.0, 0.0);
    }
    for (int e = tid; e < TK * TN; e += NT) {
      int kk, cc;
      if (OPB == OP_N) { kk = e % TK; cc = e / TK; } else { cc = e % TN; kk = e / TN; }
      const int c = c0 + cc, kg = k0 + kk;
      sm.Bs[kk][cc] = (c < n && kg < k) ? ld_op<OPB>(B, ldb, kg, c) : mk(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      double2 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = sm.As[wr + 16 * i + li][ks + lk];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = sm.Bs[ks + lk][wc + 16 * j + li];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, acc_re[i][j], 0, 0, 0);
          acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[i].y, b[j].y, acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].y, acc_im[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].x, acc_im[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  const bool use_beta = beta.x != 0.0 || beta.y != 0.0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = r0 + wr + 16 * i + lk + 4 * e, c = c0 + wc + 16 * j + li;
        if (r < m && c < n && (!lower_only || c <= r)) {
          double2 *p = &C[r + (int64_t)c * ldc];
          double2 v = cmul(alpha, mk(acc_re[i][j][e], acc_im[i][j][e]));
          if (use_beta) v = cfma(beta, *p, v);
          *p = v;
        }
      }
}

// ---- Cholesky -------------------------------------------------------------------

// Factor the diagonal block [k0, k0+32) of every item in LDS.
__global__ __launch_bounds__(NT) void k_potrf_diag(double2 *base, const PotrfItem *items,
                                                   int *info, int k0) {
  __shared__ double2 D[NB][NB + 1];
  __shared__ int fail;
  const PotrfItem it = items[blockIdx.x];
  const int n = it.n, lda = it.lda, tid = threadIdx.x;
  if (k0 >= n || info[blockIdx.x] != 0) return;
  double2 *A = base + it.a;
  const int kb = min(NB, n - k0);
  if (tid == 0) fail = 0;
  for (int e = tid; e < kb * kb; e += NT) {
    const int i = e % kb, j = e / kb;
    if (j <= i) D[i][j] = A[(k0 + i) + (int64_t)(k0 + j) * lda];
  }
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    if (tid == 0) {
      double d = D[j][j].x;
      if (!(d > 0.0)) {
        if (!fail) fail = k0 + j + 1;
        d = 1.0;
      }
      D[j][j] = mk(sqrt(d), 0.0);
    }
    __syncthreads();
    const double inv = 1.0 / D[j][j].x;
    for (int i = j + 1 + tid; i < kb; i += NT) D[i][j] = cscale(D[i][j], inv);
    __syncthreads();
    const int rem = kb - j - 1;
    for (int e = tid; e < rem * rem; e += NT) {
      const int i = j + 1 + e % rem, jj = j + 1 + e / rem;
      if (jj <= i) D[i][jj] = csub(D[i][jj], cmul(D[i][j], cconj(D[jj][j])));
    }
    __syncthreads();
  }
  if (fail) {
    if (tid == 0) info[blockIdx.x] = fail;
    return;
  }
  for (int e = tid; e < kb * kb; e += NT) {
    const int i = e % kb, j = e / kb;
    if (j <= i) A[(k0 + i) + (int64_t)(k0 + j) * lda] = D[i][j];
  }
}

// Panel below the diagonal block: X = A_panel L_kk^-H, one row per thread.
__global__ __launch_bounds__(64) void k_potrf_panel(double2 *base, const PotrfItem *items,
                                                    const int *info, int k0) {
  __shared__ double2 D[NB][NB + 1];
  const PotrfItem it = items[blockIdx.y];
  const int n = it.n, lda = it.lda, tid = threadIdx.x;
  if (k0 + NB >= n || info[blockIdx.y] != 0) return;
  const int r0 = k0 + NB + blockIdx.x * 64;
  if (r0 >= n) return;
  double2 *A = base + it.a;
  for (int e = tid; e < NB * NB; e += 64) {
    const int i = e % NB, j = e / NB;
    if (j <= i) D[i][j] = A[(k0 + i) + (int64_t)(k0 + j) * lda];
  }
  __syncthreads();
  const int r = r0 + tid;
  if (r >= n) return;
  double2 x[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) x[t] = A[r + (int64_t)(k0 + t) * lda];
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    double2 v = x[t];
#pragma unroll
    for (int u = 0; u < t; ++u) v = csub(v, cmul(x[u], cconj(D[t][u])));
    x[t] = cscale(v, 1.0 / D[t][t].x);
  }
#pragma unroll
  for (int t = 0; t < NB; ++t) A[r + (int64_t)(k0 + t) * lda] = x[t];
}

// Update C[r, c] -= sum_{k in [k_lo, k_hi)} A[r, k] conj(A[c, k]) for
// c in [c_lo, c_hi), r >= c (lower triangle only).
__global__ __launch_bounds__(NT) void k_potrf_update(double2 *base, const PotrfItem *items,
                                                     const int *info, int k_lo, int k_hi,
                                                     int c_lo, int c_hi, int tiles_c) {
  __shared__ GemmSmem sm;
  const PotrfItem it = items[blockIdx.y];
  const int n = it.n, lda = it.lda;
  const int m = n - c_lo, nc = min(c_hi, n) - c_lo, kw = min(k_hi, n) - k_lo;
  if (m <= 0 || nc <= 0 || kw <= 0 || info[blockIdx.y] != 0) return;
  const int ti = blockIdx.x / tiles_c, tj = blockIdx.x % tiles_c;
  if (ti * TM >= m || tj * TN >= nc || ti < tj) return;
  double2 *A = base + it.a;
  const double2 *P = A + c_lo + (int64_t)k_lo * lda;
  double2 *C = A + c_lo + (int64_t)c_lo * lda;
  gemm_tile<OP_N, OP_C>(m, nc, kw, 0, ti * TM, tj * TN, mk(-1.0, 0.0), P, lda, P, lda,
                        mk(1.0, 0.0), C, lda, ti == tj, sm);
}

// ---- triangular solve -------------------------------------------------------------

// Rows [k0, k0+32) of B: solve L_kk X = B_k, one column per thread.
__global__ __launch_bounds__(64) void k_trsm_diag(const double2 *lbase, double2 *bbase,
                                                  const TrsmItem *items, int k0, int tri) {
  __shared__ double2 D[NB][NB + 1];
  const TrsmItem it = items[blockIdx.y];
  const int n = it.n, tid = threadIdx.x;
  if (k0 >= n) return;
  const int kb = min(NB, n - k0);
  const int ncols = tri ? min(it.ncols, k0 + kb) : it.ncols;
  const int c = blockIdx.x * 64 + tid;
  if (blockIdx.x * 64 >= ncols) return;
  const double2 *L = lbase + it.l;
  double2 *B = bbase + it.b;
  for (int e = tid; e < kb * kb; e += 64) {
    const int i = e % kb, j = e / kb;
    if (j <= i) D[i][j] = L[(k0 + i) + (int64_t)(k0 + j) * it.ldl];
  }
  __syncthreads();
  if (c >= ncols) return;
  double2 x[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t)
    if (t < kb) x[t] = B[(k0 + t) + (int64_t)c * it.ldb];
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    if (t < kb) {
      double2 v = x[t];
#pragma unroll
      for (int u = 0; u < NB; ++u)
        if (u < t) v = csub(v, cmul(D[t][u], x[u]));
      x[t] = cscale(v, 1.0 / D[t][t].x);
    }
  }
#pragma unroll
  for (int t = 0; t < NB; ++t)
    if (t < kb) B[(k0 + t) + (int64_t)c * it.ldb] = x[t];
}

// B[r, c] -= sum_{k in [k_lo, k_hi)} L[r, k] X[k, c] for r in [r_lo, r_hi),
// one 64x64 tile per workgroup.
__global__ __launch_bounds__(NT) void k_trsm_update(const double2 *lbase, double2 *bbase,
                                                    const TrsmItem *items, int k_lo, int k_hi,
                                                    int r_lo, int r_hi, int tri, int tiles_c) {
  __shared__ GemmSmem sm;
  const TrsmItem it = items[blockIdx.y];
  const int n = it.n;
  const int m = min(r_hi, n) - r_lo, kw = min(k_hi, n) - k_lo;
  if (m <= 0 || kw <= 0) return;
  const int ncols = tri ? min(it.ncols, k_hi) : it.ncols;
  const int ti = blockIdx.x / tiles_c, tj = blockIdx.x % tiles_c;
  if (ti * TM >= m || tj * TN >= ncols) return;
  const double2 *L = lbase + it.l;
  double2 *B = bbase + it.b;
  gemm_tile<OP_N, OP_N>(m, ncols, kw, 0, ti * TM, tj * TN, mk(-1.0, 0.0),
                        L + r_lo + (int64_t)k_lo * it.ldl, it.ldl, B + k_lo, it.ldb,
                        mk(1.0, 0.0), B + r_lo, it.ldb, false, sm);
}

// ---- GEMM ----------------------------------------------------------------------------

template <int OPA, int OPB>
__global__ __launch_bounds__(NT) void k_gemm(double2 alpha, const double2 *abase,
                                             const double2 *bbase, double2 beta, double2 *cbase,
                                             const GemmItem *items, int tiles_n, int mode) {
  __shared__ GemmSmem sm;
  const GemmItem it = items[blockIdx.y];
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  const int r0 = tm * TM, c0 = tn * TN;
  if (r0 >= it.m || c0 >= it.n) return;
  int kb = 0;
  if (mode == GEMM_UPPER_LOWTRI) {
    if (tm > tn) return;
    kb = c0;   // X lower triangular: rows below max(r0, c0) = c0 only
  }
  gemm_tile<OPA, OPB>(it.m, it.n, it.k, kb, r0, c0, alpha, abase + it.a, it.lda, bbase + it.b,
                      it.ldb, beta, cbase + it.c, it.ldc, false, sm);
}

template <int OPA>
void gemm_dispatch_b(int opb, dim3 g, hipStream_t s, double2 alpha, const double2 *a,
                     const double2 *b, double2 beta, double2 *c, const GemmItem *it, int tn,
                     int mode) {
  if (opb == OP_N) hipLaunchKernelGGL((k_gemm<OPA, OP_N>), g, dim3(NT), 0, s, alpha, a, b, beta, c, it, tn, mode);
  else if (opb == OP_T) hipLaunchKernelGGL((k_gemm<OPA, OP_T>), g, dim3(NT), 0, s, alpha, a, b, beta, c, it, tn, mode);
  else hipLaunchKernelGGL((k_gemm<OPA, OP_C>), g, dim3(NT), 0, s, alpha, a, b, beta, c, it, tn, mode);
}

}  // namespace

void potrf_batched(double2 *base, const PotrfItem *items_dev, int nitems, int *info_dev, int nmax,
                   hipStream_t s) {
  if (nitems <= 0 || nmax <= 0) return;
  HIP_OK(hipMemsetAsync(info_dev, 0, nitems * sizeof(int), s));
  for (int K0 = 0; K0 < nmax; K0 += NBO) {
    const int K1 = std::min(K0 + NBO, nmax);
    for (int k0 = K0; k0 < K1; k0 += NB) {
      hipLaunchKernelGGL(k_potrf_diag, dim3(nitems), dim3(NT), 0, s, base, items_dev, info_dev, k0);
      const int rows = nmax - k0 - NB;
      if (rows <= 0) continue;
      hipLaunchKernelGGL(k_potrf_panel, dim3(cdiv(rows, 64), nitems), dim3(64), 0, s, base,
                         items_dev, info_dev, k0);
      // rank-32 update of the rest of this block column only
      const int c_lo = k0 + NB, c_hi = K1;
      if (c_lo < c_hi) {
        const int tr = (int)cdiv(nmax - c_lo, TM), tc = (int)cdiv(c_hi - c_lo, TN);
        hipLaunchKernelGGL(k_potrf_update, dim3(tr * tc, nitems), dim3(NT), 0, s, base,
                           items_dev, info_dev, k0, k0 + NB, c_lo, c_hi, tc);
      }
    }
    // rank-128 update of the trailing matrix
    if (K1 < nmax) {
      const int t = (int)cdiv(nmax - K1, TM);
      hipLaunchKernelGGL(k_potrf_update, dim3(t * t, nitems), dim3(NT), 0, s, base, items_dev,
                         info_dev, K0, K1, K1, nmax, t);
    }
  }
  LAUNCH_OK();
}

void trsm_batched(const double2 *lbase, double2 *bbase, const TrsmItem *items_dev, int nitems,
                  int max_n, int max_cols, bool identity_rhs, hipStream_t s) {
  if (nitems <= 0 || max_cols <= 0 || max_n <= 0) return;
  const int tri = identity_rhs ? 1 : 0;
  for (int K0 = 0; K0 < max_n; K0 += NBO) {
    const int K1 = std::min(K0 + NBO, max_n);
    for (int k0 = K0; k0 < K1; k0 += NB) {
      const int cols = tri ? std::min(max_cols, k0 + NB) : max_cols;
      hipLaunchKernelGGL(k_trsm_diag, dim3(cdiv(cols, 64), nitems), dim3(64), 0, s, lbase, bbase,
                         items_dev, k0, tri);
      // rows of this block row below the solved 32
      const int r_lo = k0 + NB, r_hi = K1;
      if (r_lo < r_hi) {
        const int tc = (int)cdiv(cols, TN);
        hipLaunchKernelGGL(k_trsm_update, dim3(cdiv(r_hi - r_lo, TM) * tc, nitems), dim3(NT), 0,
                           s, lbase, bbase, items_dev, k0, k0 + NB, r_lo, r_hi, tri, tc);
      }
    }
    if (K1 < max_n) {
      const int cols = tri ? std::min(max_cols, K1) : max_cols;
      const int tc = (int)cdiv(cols, TN);
      hipLaunchKernelGGL(k_trsm_update, dim3(cdiv(max_n - K1, TM) * tc, nitems), dim3(NT), 0, s,
                         lbase, bbase, items_dev, K0, K1, K1, max_n, tri, tc);
    }
  }
  LAUNCH_OK();
}

void gemm_batched(int opa, int opb, double2 alpha, const double2 *abase, const double2 *bbase,
                  double2 beta, double2 *cbase, const GemmItem *items_dev, int nitems, int max_m,
                  int max_n, hipStream_t s, int mode) {
  if (nitems <= 0 || max_m <= 0 || max_n <= 0) return;
  const int tm = (int)cdiv(max_m, TM), tn = (int)cdiv(max_n, TN);
  dim3 g(tm * tn, nitems);
  if (opa == OP_N) gemm_dispatch_b<OP_N>(opb, g, s, alpha, abase, bbase, beta, cbase, items_dev, tn, mode);
  else if (opa == OP_T) gemm_dispatch_b<OP_T>(opb, g, s, alpha, abase, bbase, beta, cbase, items_dev, tn, mode);
  else gemm_dispatch_b<OP_C>(opb, g, s, alpha, abase, bbase, beta, cbase, items_dev, tn, mode);
  LAUNCH_OK();
}

}  // namespace dpg
