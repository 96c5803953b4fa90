// Batched dense complex-FP64 kernels: Cholesky, forward solve, GEMM.
//
// One workgroup of 256 threads (4 waves) works on one item (Cholesky), one
// 64-column panel of one item (triangular solve) or one 64x64 output tile of
// one item (GEMM).  The rank-k updates share one register-blocked tile
// routine: the workgroup stages 64x16 slices of op(A) and 16x64 slices of
// op(B) in LDS and every thread accumulates a 4x4 block of the tile.  On
// MI355X the FP64 vector and matrix-core peaks are equal (78.6 TFLOP/s), so
// FP64 FMAs on the vector units are the plain choice here.
#include "dense.hpp"

namespace dpg {
namespace {

constexpr int TM = 64, TN = 64, TK = 16, NT = 256, NB = 32;

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
// inner dimension k.  lower_only leaves entries above the diagonal alone.
// Must be called by all 256 threads of the workgroup.
template <int OPA, int OPB>
__device__ void gemm_tile(int m, int n, int k, int r0, int c0, double2 alpha, const double2 *A,
                          int lda, const double2 *B, int ldb, double2 beta, double2 *C, int ldc,
                          bool lower_only, GemmSmem &sm) {
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  double2 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = mk(0.0, 0.0);
  for (int k0 = 0; k0 < k; k0 += TK) {
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
#pragma unroll 4
    for (int kk = 0; kk < TK; ++kk) {
      double2 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sm.As[ty + 16 * i][kk];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = sm.Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = cfma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  const bool use_beta = beta.x != 0.0 || beta.y != 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = r0 + ty + 16 * i, c = c0 + tx + 16 * j;
      if (r < m && c < n && (!lower_only || c <= r)) {
        double2 *p = &C[r + (int64_t)c * ldc];
        double2 v = cmul(alpha, acc[i][j]);
        if (use_beta) v = cfma(beta, *p, v);
        *p = v;
      }
    }
}

__global__ __launch_bounds__(NT) void k_potrf(double2 *base, const PotrfItem *items, int *info) {
  __shared__ GemmSmem sm;
  __shared__ double2 D[NB][NB + 1];
  __shared__ int fail;
  const PotrfItem it = items[blockIdx.x];
  double2 *A = base + it.a;
  const int n = it.n, lda = it.lda, tid = threadIdx.x;
  if (tid == 0) fail = 0;
  __syncthreads();
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int kb = min(NB, n - k0);
    for (int e = tid; e < kb * kb; e += NT) {
      const int i = e % kb, j = e / kb;
      if (j <= i) D[i][j] = A[(k0 + i) + (int64_t)(k0 + j) * lda];
    }
    __syncthreads();
    // unblocked factorisation of the diagonal block in LDS
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
    // panel below: X = A_panel L_kk^-H, one row per thread
    for (int r = k0 + kb + tid; r < n; r += NT) {
      double2 x[NB];
#pragma unroll
      for (int t = 0; t < NB; ++t)
        if (t < kb) x[t] = A[r + (int64_t)(k0 + t) * lda];
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        if (t < kb) {
          double2 v = x[t];
#pragma unroll
          for (int u = 0; u < NB; ++u)
            if (u < t) v = csub(v, cmul(x[u], cconj(D[t][u])));
          x[t] = cscale(v, 1.0 / D[t][t].x);
        }
      }
#pragma unroll
      for (int t = 0; t < NB; ++t)
        if (t < kb) A[r + (int64_t)(k0 + t) * lda] = x[t];
    }
    __syncthreads();
    const int nt = n - k0 - kb;
    if (nt > 0) {
      const double2 *P = A + (k0 + kb) + (int64_t)k0 * lda;
      double2 *Ct = A + (k0 + kb) + (int64_t)(k0 + kb) * lda;
      const int tiles = (nt + TM - 1) / TM;
      for (int ti = 0; ti < tiles; ++ti)
        for (int tj = 0; tj <= ti; ++tj)
          gemm_tile<OP_N, OP_C>(nt, nt, kb, ti * TM, tj * TN, mk(-1.0, 0.0), P, lda, P, lda,
                                mk(1.0, 0.0), Ct, lda, ti == tj, sm);
    }
    __syncthreads();
  }
  if (tid == 0) info[blockIdx.x] = 0;
}

__global__ __launch_bounds__(NT) void k_trsm(const double2 *lbase, double2 *bbase,
                                             const TrsmItem *items) {
  __shared__ GemmSmem sm;
  __shared__ double2 D[NB][NB + 1];
  const TrsmItem it = items[blockIdx.y];
  const int c0 = blockIdx.x * TN;
  if (c0 >= it.ncols) return;
  const int nc = min(TN, it.ncols - c0);
  const double2 *L = lbase + it.l;
  double2 *B = bbase + it.b + (int64_t)c0 * it.ldb;
  const int n = it.n, ldl = it.ldl, ldb = it.ldb, tid = threadIdx.x;
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int kb = min(NB, n - k0);
    for (int e = tid; e < kb * kb; e += NT) {
      const int i = e % kb, j = e / kb;
      if (j <= i) D[i][j] = L[(k0 + i) + (int64_t)(k0 + j) * ldl];
    }
    __syncthreads();
    if (tid < nc) {
      double2 x[NB];
#pragma unroll
      for (int t = 0; t < NB; ++t)
        if (t < kb) x[t] = B[(k0 + t) + (int64_t)tid * ldb];
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
        if (t < kb) B[(k0 + t) + (int64_t)tid * ldb] = x[t];
    }
    __syncthreads();
    const int nr = n - k0 - kb;
    if (nr > 0) {
      const int tiles = (nr + TM - 1) / TM;
      for (int ti = 0; ti < tiles; ++ti)
        gemm_tile<OP_N, OP_N>(nr, nc, kb, ti * TM, 0, mk(-1.0, 0.0),
                              L + (k0 + kb) + (int64_t)k0 * ldl, ldl, B + k0, ldb, mk(1.0, 0.0),
                              B + k0 + kb, ldb, false, sm);
    }
    __syncthreads();
  }
}

template <int OPA, int OPB>
__global__ __launch_bounds__(NT) void k_gemm(double2 alpha, const double2 *abase,
                                             const double2 *bbase, double2 beta, double2 *cbase,
                                             const GemmItem *items, int tiles_n) {
  __shared__ GemmSmem sm;
  const GemmItem it = items[blockIdx.y];
  const int r0 = (blockIdx.x / tiles_n) * TM, c0 = (blockIdx.x % tiles_n) * TN;
  if (r0 >= it.m || c0 >= it.n) return;
  gemm_tile<OPA, OPB>(it.m, it.n, it.k, r0, c0, alpha, abase + it.a, it.lda, bbase + it.b,
                      it.ldb, beta, cbase + it.c, it.ldc, false, sm);
}

template <int OPA>
void gemm_dispatch_b(int opb, dim3 g, hipStream_t s, double2 alpha, const double2 *a,
                     const double2 *b, double2 beta, double2 *c, const GemmItem *it, int tn) {
  if (opb == OP_N) hipLaunchKernelGGL((k_gemm<OPA, OP_N>), g, dim3(NT), 0, s, alpha, a, b, beta, c, it, tn);
  else if (opb == OP_T) hipLaunchKernelGGL((k_gemm<OPA, OP_T>), g, dim3(NT), 0, s, alpha, a, b, beta, c, it, tn);
  else hipLaunchKernelGGL((k_gemm<OPA, OP_C>), g, dim3(NT), 0, s, alpha, a, b, beta, c, it, tn);
}

}  // namespace

void potrf_batched(double2 *base, const PotrfItem *items_dev, int nitems, int *info_dev,
                   hipStream_t s) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_potrf, dim3(nitems), dim3(NT), 0, s, base, items_dev, info_dev);
  LAUNCH_OK();
}

void trsm_batched(const double2 *lbase, double2 *bbase, const TrsmItem *items_dev, int nitems,
                  int max_cols, hipStream_t s) {
  if (nitems <= 0 || max_cols <= 0) return;
  hipLaunchKernelGGL(k_trsm, dim3(cdiv(max_cols, TN), nitems), dim3(NT), 0, s, lbase, bbase,
                     items_dev);
  LAUNCH_OK();
}

void gemm_batched(int opa, int opb, double2 alpha, const double2 *abase, const double2 *bbase,
                  double2 beta, double2 *cbase, const GemmItem *items_dev, int nitems, int max_m,
                  int max_n, hipStream_t s) {
  if (nitems <= 0 || max_m <= 0 || max_n <= 0) return;
  const int tm = (int)cdiv(max_m, TM), tn = (int)cdiv(max_n, TN);
  dim3 g(tm * tn, nitems);
  if (opa == OP_N) gemm_dispatch_b<OP_N>(opb, g, s, alpha, abase, bbase, beta, cbase, items_dev, tn);
  else if (opa == OP_T) gemm_dispatch_b<OP_T>(opb, g, s, alpha, abase, bbase, beta, cbase, items_dev, tn);
  else gemm_dispatch_b<OP_C>(opb, g, s, alpha, abase, bbase, beta, cbase, items_dev, tn);
  LAUNCH_OK();
}

}  // namespace dpg
