// Batched dense complex-FP64 kernels: Cholesky, forward solve, GEMM.
//
// The rank-k updates share one tile routine: a workgroup of 256 threads
// stages 64x16 slices of op(A) and 16x64 slices of op(B) in LDS and its four
// waves accumulate the 64x64 complex output tile on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64), three real products per complex one.  The tile
// kernels run two waves per SIMD: the three accumulator sets and the
// prefetched slice take 184-192 registers, which at three waves (168) spilled.  The FP64 matrix and vector peaks of MI355X are
// equal (78.6 TFLOP/s); the matrix cores win because they reuse each operand
// sixteen times inside the instruction, where vector FMAs would need one LDS
// read per two complex multiply-adds.
//
// Factorisations are blocked twice: 128-wide blocks, each processed in
// 64-wide panel steps, then one rank-128 update of the trailing matrix spread
// over (64x64 tiles x items), so the trailing matrix is read and written once
// per 128 columns.  A panel step factors (or, for the triangular solve, takes)
// the 64x64 diagonal block and its inverse in LDS; the panel itself is then a
// small product with that inverse on the matrix cores, and the update inside
// the 128-wide block a rank-64 product.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "dense.hpp"

namespace dpg {
namespace {

constexpr int TM = 64, TN = 64, TK = 16, NT = 256, NB = 64, NBO = 128;
// entries of a k-slice of op(A) (and of op(B)) per thread
constexpr int QS = TM * TK / NT;
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

// Position (lo, hi), lo <= hi, of index t in the column-major enumeration of
// a triangle: (0,0) (0,1) (1,1) (0,2) (1,2) (2,2) ...  Triangular tile sets
// are launched as exactly these tiles: workgroups that exit at once still
// cost dispatch time.
__device__ __forceinline__ void tri_index(int t, int &lo, int &hi) {
  // single-precision estimate (t < 2^21 here), corrected by the two loops
  int h = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((h + 1) * (h + 2) / 2 <= t) ++h;
  while (h * (h + 1) / 2 > t) --h;
  hi = h;
  lo = t - h * (h + 1) / 2;
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Tiled kernels (grid: tiles x items) remap the hardware id so that all
// tiles of item 8 g + x run on XCD x, which keeps the operand panels an item's
// tiles share in one L2 while items stay interleaved over the XCDs.  Items of
// a last incomplete group of 8 keep the plain order.
// 32-bit unsigned arithmetic: the tiled launches here have gridDim.x *
// gridDim.y < 2^32 (at most a few thousand tiles times 65535 items).
__device__ __forceinline__ void xcd_remap(int &bx, int &by) {
  const uint32_t gx = gridDim.x;
  const uint32_t L = blockIdx.x + blockIdx.y * gx;
  const uint32_t grp = 8u * gx, full = (gridDim.y / 8u) * grp;
  if (L < full) {
    const uint32_t g = L / grp, w = L - g * grp;
    bx = (int)(w / 8u);
    by = (int)(8u * g + (w & 7u));
  } else {
    bx = (int)(L % gx);
    by = (int)(L / gx);
  }
}

// One k-slice of op(A) (64 x 16) and op(B) (16 x 64), QS = 4 entries of each per
// thread.  Every load is issued (entries outside m x k and k x n read the
// nearest entry inside, which exists because the tile is not empty), and the
// returned mask marks the entries inside; store_slice writes zeros for the
// others and conjugates an OP_C operand.  Loads guarded by a branch, or
// conjugated as they arrive, made the compiler wait for each load of the
// prefetch before issuing the next.
template <int OPA, int OPB>
__device__ __forceinline__ unsigned load_slice(int m, int n, int k, int k0, int r0, int c0,
                                               const double2 *A, int lda, const double2 *B,
                                               int ldb, double2 ra[QS], double2 rb[QS]) {
  const int tid = threadIdx.x;
  unsigned ok = 0;
#pragma unroll
  for (int q = 0; q < QS; ++q) {
    const int e = tid + NT * q;
    int rr, kk;
    if (OPA == OP_N) { rr = e % TM; kk = e / TM; } else { kk = e % TK; rr = e / TK; }
    const int r = r0 + rr, kg = k0 + kk;
    ok |= (unsigned)(r < m && kg < k) << q;
    ra[q] = ld_op<OPA == OP_C ? OP_T : OPA>(A, lda, min(r, m - 1), min(kg, k - 1));
  }
#pragma unroll
  for (int q = 0; q < QS; ++q) {
    const int e = tid + NT * q;
    int kk, cc;
    if (OPB == OP_N) { kk = e % TK; cc = e / TK; } else { cc = e % TN; kk = e / TN; }
    const int c = c0 + cc, kg = k0 + kk;
    ok |= (unsigned)(c < n && kg < k) << (QS + q);
    rb[q] = ld_op<OPB == OP_C ? OP_T : OPB>(B, ldb, min(kg, k - 1), min(c, n - 1));
  }
  return ok;
}

template <int OPA, int OPB>
__device__ __forceinline__ void store_slice(const double2 ra[QS], const double2 rb[QS], unsigned ok,
                                            GemmSmem &sm) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < QS; ++q) {
    const int e = tid + NT * q;
    int rr, kk;
    if (OPA == OP_N) { rr = e % TM; kk = e / TM; } else { kk = e % TK; rr = e / TK; }
    const double2 v = OPA == OP_C ? cconj(ra[q]) : ra[q];
    sm.As[rr][kk] = ((ok >> q) & 1) ? v : mk(0.0, 0.0);
  }
#pragma unroll
  for (int q = 0; q < QS; ++q) {
    const int e = tid + NT * q;
    int kk, cc;
    if (OPB == OP_N) { kk = e % TK; cc = e / TK; } else { cc = e % TN; kk = e / TN; }
    const double2 v = OPB == OP_C ? cconj(rb[q]) : rb[q];
    sm.Bs[kk][cc] = ((ok >> (QS + q)) & 1) ? v : mk(0.0, 0.0);
  }
}

// C[r0:r0+64, c0:c0+64] (clipped to m x n) <- alpha op(A) op(B) + beta C with
// inner indices k_begin..k-1.  lower_only leaves entries above the diagonal
// alone; mirror also stores the conjugate of each result at the transposed
// position.  Must be called by all 256 threads of the workgroup.  C may alias A or B when the tile's output covers
// exactly the operand rows / columns it reads (all reads precede the writes).
template <int OPA, int OPB>
__device__ __forceinline__ void gemm_tile(int m, int n, int k, int k_begin, int r0, int c0, double2 alpha,
                          const double2 *A, int lda, const double2 *B, int ldb, double2 beta,
                          double2 *C, int ldc, bool lower_only, GemmSmem &sm,
                          bool mirror = false) {
  const int tid = threadIdx.x;
  // FP64 matrix cores: v_mfma_f64_16x16x4f64 computes D(16x16) += A(16x4) B(4x16)
  // with A[i][k] in lane i + 16k, B[k][j] in lane j + 16k and D[i][j] in
  // lane j + 16 (i % 4), element i / 4.  Wave w owns the 32x32 sub-tile at
  // (32 (w / 2), 32 (w % 2)) as 2x2 blocks.  A complex product takes three
  // real MFMAs (the three-multiplication form): P1 = sum a_re b_re,
  // P2 = sum a_im b_im, P3 = sum (a_re + a_im)(b_re + b_im); then
  // re = P1 - P2 and im = P3 - P1 - P2.  The real part is as accurate as with
  // four products; the imaginary part's error bound grows from
  // 2 u sum |a||b| to about 4 u sum |a||b|, still a normwise bound of the same
  // order, which is what the factorisations and products here need.  The
  // three products are issued term by term so that two updates of one
  // accumulator are never adjacent.
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = 32 * (wave >> 1), wc = 32 * (wave & 1);
  const int li = lane & 15, lk = lane >> 4;
  v4d acc_p1[2][2], acc_p2[2][2], acc_p3[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc_p1[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
      acc_p2[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
      acc_p3[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    }
  // 16x16 blocks whose results are never stored take no matrix-core work:
  // those outside m x n (the ragged last tile row or column of sizes such as
  // 451 = 7 x 64 + 3) and, with lower_only, those strictly above the
  // diagonal.  The mask is uniform over the wave; a wave with every block
  // active runs the unguarded loop.
  unsigned act = 0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int br = r0 + wr + 16 * i, bc = c0 + wc + 16 * j;
      const bool on = br < m && bc < n && !(lower_only && bc > br + 15);
      act |= (unsigned)on << (2 * i + j);
    }
  act = __builtin_amdgcn_readfirstlane(act);
  // The next k-slice is fetched into registers while the current one is
  // multiplied from LDS, so global latency hides behind the matrix cores.
  auto mma_slice = [&](auto guarded) {
    constexpr bool G = decltype(guarded)::value;
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      double2 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = sm.As[wr + 16 * i + li][ks + lk];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = sm.Bs[ks + lk][wc + 16 * j + li];
      double sa[2], sb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) sa[i] = a[i].x + a[i].y;
#pragma unroll
      for (int j = 0; j < 2; ++j) sb[j] = b[j].x + b[j].y;
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          if (!G || (act >> (2 * i + j) & 1))
            acc_p1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, acc_p1[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          if (!G || (act >> (2 * i + j) & 1))
            acc_p2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].y, acc_p2[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          if (!G || (act >> (2 * i + j) & 1))
            acc_p3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[i], sb[j], acc_p3[i][j], 0, 0, 0);
    }
  };
  double2 ra[QS], rb[QS];
  unsigned ok = 0;
  if (k_begin < k) ok = load_slice<OPA, OPB>(m, n, k, k_begin, r0, c0, A, lda, B, ldb, ra, rb);
#pragma unroll 1
  for (int k0 = k_begin; k0 < k; k0 += TK) {
    store_slice<OPA, OPB>(ra, rb, ok, sm);
    __syncthreads();
    if (k0 + TK < k) ok = load_slice<OPA, OPB>(m, n, k, k0 + TK, r0, c0, A, lda, B, ldb, ra, rb);
    if (act) mma_slice(std::true_type{});
    __syncthreads();
  }
  // The C entries of a row block (eight per lane) are loaded together, from
  // the nearest entry inside m x n where outside (the value is then unused),
  // before any is combined and stored.
  const bool use_beta = beta.x != 0.0 || beta.y != 0.0;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    double2 cv[2][4];
    if (use_beta) {
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = r0 + wr + 16 * i + lk + 4 * e, c = c0 + wc + 16 * j + li;
          cv[j][e] = C[min(r, m - 1) + (int64_t)min(c, n - 1) * ldc];
        }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = r0 + wr + 16 * i + lk + 4 * e, c = c0 + wc + 16 * j + li;
        if (r < m && c < n && (!lower_only || c <= r)) {
          const double p1 = acc_p1[i][j][e], p2 = acc_p2[i][j][e];
          double2 v = cmul(alpha, mk(p1 - p2, acc_p3[i][j][e] - p1 - p2));
          if (use_beta) v = cfma(beta, cv[j][e], v);
          C[r + (int64_t)c * ldc] = v;
          if (mirror) C[c + (int64_t)r * ldc] = cconj(v);
        }
      }
  }
}

// ---- diagonal blocks -------------------------------------------------------------

// A 64x64 lower triangle in registers of 512 threads.  Rows i and 63 - i form
// a pair with 65 entries, numbered (i, 0..i) then (63 - i, 0..63 - i); the 16
// threads of pair p = t / 16 own entries t % 16 + 16 m, m < kQ.
constexpr int NTD = 512, kQ = 5;

struct Slot { int i, c; bool on; };

__device__ __forceinline__ Slot slot_of(int m, int kb) {
  const int p = threadIdx.x >> 4, e = (threadIdx.x & 15) + 16 * m;
  Slot s;
  if (e <= p) { s.i = p; s.c = e; }
  else { s.i = NB - 1 - p; s.c = e - p - 1; }
  s.on = e <= NB && s.i < kb;   // e < 65 entries; c <= i < kb then holds
  return s;
}

// Elimination of a kb x kb diagonal block held in registers, applied at the
// same time to an identity block so that it also yields the inverse factor.
// Step j broadcasts column j of the current Schur complement and row j of the
// transformed identity through LDS (double buffered, one barrier per step);
// the multiplier of row i is a_ij / a_jj.  The update reads every operand and
// masks with zero multipliers instead of branching.
// FACTOR: a holds the block of A; it is eliminated (square-root free, the
//   pivots d_j stay on the diagonal) and L = a_ic / sqrt(d_c), L^-1 = x / sqrt(d_i).
// otherwise: a holds a lower triangular factor L (left unchanged) and the
//   identity becomes L~^-1 with L~ = L diag(L)^-1, so L^-1 = x / l_ii.
// scale[i] receives sqrt(d_i) or l_ii; the return value is 1 + the first
// pivot that was not positive, or 0.  All NTD threads must call it.
template <bool FACTOR>
__device__ int eliminate(double2 a[kQ], double2 x[kQ], int kb, double2 (*cb)[NB],
                         double2 (*rb)[NB], double *scale) {
  const int tid = threadIdx.x, p = tid >> 4;
  __shared__ int fail;
  if (tid == 0) fail = 0;
  for (int e = tid; e < 2 * NB; e += NTD) {
    cb[e / NB][e % NB] = mk(0.0, 0.0);
    rb[e / NB][e % NB] = mk(0.0, 0.0);
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < kQ; ++m) {
    const Slot sl = slot_of(m, kb);
    if (!sl.on) continue;
    if (sl.c == 0) cb[0][sl.i] = a[m];
    if (sl.i == 0) rb[0][0] = x[m];
    if (!FACTOR && sl.i == sl.c) scale[sl.i] = a[m].x;
  }
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    const int u = j & 1;
    const double d = cb[u][j].x;
    const double inv = d > 0.0 ? 1.0 / d : 0.0;
    if (FACTOR && tid == 0) {
      scale[j] = d > 0.0 ? sqrt(d) : 1.0;
      if (!(d > 0.0) && !fail) fail = j + 1;
    }
    const double2 m_lo = cscale(cb[u][p], inv), m_hi = cscale(cb[u][NB - 1 - p], inv);
    double2 cv[kQ], rv[kQ];
#pragma unroll
    for (int m = 0; m < kQ; ++m) {
      const Slot sl = slot_of(m, kb);
      cv[m] = cb[u][sl.c & (NB - 1)];
      rv[m] = rb[u][sl.c & (NB - 1)];
    }
#pragma unroll
    for (int m = 0; m < kQ; ++m) {
      const Slot sl = slot_of(m, kb);
      const bool live = sl.on && sl.i > j;
      const double2 mi = live ? (sl.i == p ? m_lo : m_hi) : mk(0.0, 0.0);
      const double2 v = sl.c > j ? cconj(cv[m]) : rv[m];
      const double2 pr = cmul(mi, v);
      if (FACTOR) a[m] = csub(a[m], sl.c > j ? pr : mk(0.0, 0.0));
      x[m] = csub(x[m], sl.c <= j ? pr : mk(0.0, 0.0));
    }
    if (j + 1 < kb) {
#pragma unroll
      for (int m = 0; m < kQ; ++m) {
        const Slot sl = slot_of(m, kb);
        if (!sl.on) continue;
        if (sl.c == j + 1) cb[u ^ 1][sl.i] = a[m];
        if (sl.i == j + 1) rb[u ^ 1][sl.c] = x[m];
      }
    }
    __syncthreads();
  }
  return fail;
}

// Write L^-1 (x / scale[i]) zero-padded to 64 x 64, column-major, to w.
__device__ void store_inverse(const double2 x[kQ], int kb, const double *scale, double2 *w) {
#pragma unroll
  for (int m = 0; m < kQ; ++m) {
    const Slot sl = slot_of(m, kb);
    if (!sl.on) continue;
    w[sl.i + sl.c * NB] = cscale(x[m], 1.0 / scale[sl.i]);
    if (sl.c < sl.i) w[sl.c + sl.i * NB] = mk(0.0, 0.0);
  }
  for (int e = threadIdx.x; e < NB * NB; e += NTD) {
    const int i = e % NB, c = e / NB;
    if (i >= kb || c >= kb) w[e] = mk(0.0, 0.0);
  }
}

// Owned entries of a kb x kb lower triangle from column-major X (ld ldx);
// x becomes the identity's share.
__device__ __forceinline__ void load_block(const double2 *X, int ldx, int kb, double2 a[kQ],
                                           double2 x[kQ]) {
#pragma unroll
  for (int m = 0; m < kQ; ++m) {
    const Slot sl = slot_of(m, kb);
    a[m] = sl.on ? X[sl.i + (int64_t)sl.c * ldx] : mk(0.0, 0.0);
    x[m] = mk(sl.on && sl.c == sl.i ? 1.0 : 0.0, 0.0);
  }
}

// ---- Cholesky -------------------------------------------------------------------

// Diagonal blocks in 16 x 16 sub-blocks.  The 64 x 64 block (padded beyond
// kb with the identity) and its inverse live in LDS as packed lower
// triangles (67 KB, two workgroups per compute unit).  For each sub-block
// column s: one wave factors the diagonal sub-block by elimination, applying
// the same row operations to an identity, which also yields the sub-block's
// inverse X_ss; the sub-blocks below become products with X_ss and the
// trailing lower triangle is updated, both by the whole workgroup, in the
// same two phases as the block forward elimination of the identity that
// gives the rest of L^-1 (X_st = X_ss Y_st, then Y_rt -= L_rs X_st).
constexpr int DB = 16, NTB = 256, NPK = NB * (NB + 1) / 2;

// packed column-major lower triangle: entry (i, j), i >= j
__device__ __forceinline__ int pk(int i, int j) { return j * NB - (j * (j - 1)) / 2 + (i - j); }

struct DiagSmem {
  double2 L[NPK];
  double2 X[NPK];   // L^-1
  double2 row_a[DB], row_x[DB];
  int fail;         // 1 + first pivot (in the block) that was not positive
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 1 / d for d > 0: hardware reciprocal estimate and two Newton steps
// r <- r (2 - d r), each of which squares the relative error.
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}

// Wave 0: sub-block (o, o) -> L_oo in place, L_oo^-1 into X.  Lane (i, g)
// holds row i, columns 4g..4g+3 of the full Hermitian sub-block and of the
// identity.  Step k subtracts m_i times the pivot row from every row i > k,
// m_i = a_ik / a_kk (a_ik = conj(a_ki)), in all columns of both: the
// sub-block becomes U = D Lu^H (Lu unit lower, zeros below the diagonal) and
// the identity Lu^-1 (row k of the identity part is zero right of column k,
// so those columns take no change).  Updating every column keeps the step
// free of per-column selects.  The only exchange per step is the pivot row,
// through LDS.
// a - m r as four fused multiply-adds
__device__ __forceinline__ double2 cfms(double2 m, double2 r, double2 a) {
  return mk(fma(-m.x, r.x, fma(m.y, r.y, a.x)), fma(-m.x, r.y, fma(-m.y, r.x, a.y)));
}

__device__ void factor_sub(DiagSmem &sm, int o) {
  const int lane = threadIdx.x, i = lane & 15, g = lane >> 4;
  double2 a[4], x[4];
  double di = 1.0;
  int fail = 0;
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
    const int j = 4 * g + jj;
    const double2 v = sm.L[pk(o + max(i, j), o + min(i, j))];
    a[jj] = mk(v.x, i >= j ? v.y : -v.y);
    x[jj] = mk(i == j ? 1.0 : 0.0, 0.0);
  }
#pragma unroll 1
  for (int k = 0; k < DB; ++k) {
    if (i == k) {
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        sm.row_a[4 * g + jj] = a[jj];
        sm.row_x[4 * g + jj] = x[jj];
      }
    }
    wave_sync();
    const double d = sm.row_a[k].x;
    const double2 ri = sm.row_a[i];
    double2 ra[4], rx[4];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      ra[jj] = sm.row_a[4 * g + jj];
      rx[jj] = sm.row_x[4 * g + jj];
    }
    const bool ok = d > 0.0;
    if (!ok && fail == 0) fail = k + 1;
    const double r = recip(d);
    const double inv = ok && i > k ? r : 0.0;
    if (i == k) di = d;
    const double2 m = cscale(cconj(ri), inv);
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      a[jj] = cfms(m, ra[jj], a[jj]);
      x[jj] = cfms(m, rx[jj], x[jj]);
    }
    wave_sync();
  }
  if (fail) {
    if (lane == 0 && sm.fail == 0) sm.fail = o + fail;
    return;
  }
  // with d_i = U_ii: L = Lu D^(1/2), so L_ji = conj(U_ij) / sqrt(d_i) below
  // the diagonal, L_ii = sqrt(d_i), and (L^-1)_ij = (Lu^-1)_ij / sqrt(d_i)
  const double si = sqrt(di), rsi = 1.0 / si;
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
    const int j = 4 * g + jj;
    if (j > i) sm.L[pk(o + j, o + i)] = cscale(cconj(a[jj]), rsi);
    else if (j == i) sm.L[pk(o + i, o + i)] = mk(si, 0.0);
    if (i >= j) sm.X[pk(o + i, o + j)] = cscale(x[jj], rsi);
  }
}

// Factor the diagonal block [k0, k0+kb) of every item, write L_kk back and
// L_kk^-1 (zero-padded to 64 x 64) to the work area (slot k0 / 64 of the
// item).  A pivot that is not positive marks the item as failed.
__global__ __launch_bounds__(NTB, 2) void k_potrf_diag(double2 *base, const PotrfItem *items,
                                                    int *info, int k0, int kend, double2 *work,
                                                    int wslots) {
  __shared__ DiagSmem sm;
  const PotrfItem it = items[blockIdx.x];
  const int n = it.n, lda = it.lda;
  const int kb = min(NB, min(kend, n) - k0);
  if (kb <= 0 || info[blockIdx.x] != 0) return;
  double2 *A = base + it.a + k0 + (int64_t)k0 * lda;
  const int tid = threadIdx.x;
  // all sixteen loads of a thread are issued before the LDS stores (entries
  // outside the kb x kb block read the nearest one inside and are replaced
  // by the identity padding; entries above the diagonal, which are not used,
  // read the diagonal entry of their column, so that only the lines of the
  // lower triangle are fetched)
  constexpr int kLd = NB * NB / NTB;
  double2 v[kLd];
#pragma unroll
  for (int q = 0; q < kLd; ++q) {
    const int e = tid + NTB * q, i = e % NB, j = e / NB;
    v[q] = A[min(max(i, j), kb - 1) + (int64_t)min(j, kb - 1) * lda];
  }
#pragma unroll
  for (int q = 0; q < kLd; ++q) {
    const int e = tid + NTB * q, i = e % NB, j = e / NB;
    if (i < j) continue;
    sm.L[pk(i, j)] = (i < kb && j < kb) ? v[q] : mk(i == j ? 1.0 : 0.0, 0.0);
    sm.X[pk(i, j)] = mk(0.0, 0.0);
  }
  if (tid == 0) sm.fail = 0;
  __syncthreads();
  // Block forward elimination of the identity runs along (X = L^-1): the
  // (r, t) slots of X (r > t) accumulate Y_rt = -sum_u L_ru X_ut over the
  // steps u < r, and step r turns them into X_rt = X_rr Y_rt.
  for (int s = 0; s < NB / DB; ++s) {
    const int o = s * DB, r0 = o + DB, prow = NB - r0;
    if (tid < 64) factor_sub(sm, o);
    __syncthreads();
    if (sm.fail) break;
    // (a) sub-blocks below: L_rs = A_rs L_ss^-H (X_ss lower: terms t <= j);
    // (b) X_st = X_ss Y_st for t < s (X_ss lower: terms k <= i).  One 16 x 16
    // tile per wave on the FP64 matrix cores; a wave reads and then overwrites
    // only its own tile (and reads X_ss), so the tiles need no barrier between.
    {
      const int wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
      const int nb = prow / DB;
      for (int tt = wave; tt < nb + s; tt += NTB / 64) {
        v4d cre = {0.0, 0.0, 0.0, 0.0}, cim = {0.0, 0.0, 0.0, 0.0};
        if (tt < nb) {
          const int ri = r0 + DB * tt;
#pragma unroll
          for (int ks = 0; ks < DB; ks += 4) {
            const int k = ks + lk;
            const double2 av = sm.L[pk(ri + li, o + k)];
            const double2 xv = sm.X[pk(o + li, o + min(k, li))];
            const double2 bv = k <= li ? xv : mk(0.0, 0.0);
            cre = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.x, cre, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv.x, cim, 0, 0, 0);
            cre = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv.y, cre, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.x, bv.y, cim, 0, 0, 0);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) sm.L[pk(ri + 4 * v + lk, o + li)] = mk(cre[v], cim[v]);
        } else {
          const int tc = DB * (tt - nb);
#pragma unroll
          for (int ks = 0; ks < DB; ks += 4) {
            const int k = ks + lk;
            const double2 xv = sm.X[pk(o + li, o + min(k, li))];
            const double2 av = k <= li ? xv : mk(0.0, 0.0);
            const double2 bv = sm.X[pk(o + k, tc + li)];
            cre = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.x, cre, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.y, cim, 0, 0, 0);
            cre = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.y, bv.y, cre, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv.x, cim, 0, 0, 0);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) sm.X[pk(o + 4 * v + lk, tc + li)] = mk(cre[v], cim[v]);
        }
      }
    }
    __syncthreads();
    if (prow == 0) break;
    // (c) trailing lower triangle: A_ij -= sum_t L_it conj(L_jt); (d) Y_rt -=
    // L_rs X_st for r > s, t <= s (X_ss lower: terms k >= j).  Both as 16 x 16
    // tiles on the FP64 matrix cores (k = 16 in four steps of 4, four real
    // products per complex one), one wave per tile; neither reads what the
    // other writes.
    {
      const int wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
      const int nb = prow / DB, ntc = nb * (nb + 1) / 2, ntd = nb * (s + 1);
      for (int tt = wave; tt < ntc + ntd; tt += NTB / 64) {
        v4d cre = {0.0, 0.0, 0.0, 0.0}, cim = {0.0, 0.0, 0.0, 0.0};
        if (tt < ntc) {
          int bi = 0, bj = tt;   // lower tile number tt, row by row
          while (bj > bi) {
            bj -= bi + 1;
            ++bi;
          }
          const int ri = r0 + DB * bi, rj = r0 + DB * bj;
#pragma unroll
          for (int ks = 0; ks < DB; ks += 4) {
            const int c = o + ks + lk;
            const double2 av = sm.L[pk(ri + li, c)], bv = sm.L[pk(rj + li, c)];
            cre = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.x, cre, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv.x, cim, 0, 0, 0);
            cre = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv.y, cre, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.x, bv.y, cim, 0, 0, 0);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int R = ri + 4 * v + lk, Cc = rj + li;
            if (bi != bj || R >= Cc) {
              const int q = pk(R, Cc);
              sm.L[q] = csub(sm.L[q], mk(cre[v], cim[v]));
            }
          }
        } else {
          const int u = tt - ntc, rr = r0 + DB * (u / (s + 1)), tc = DB * (u % (s + 1));
#pragma unroll
          for (int ks = 0; ks < DB; ks += 4) {
            const int kr = o + ks + lk, cc = tc + li;
            const double2 av = sm.L[pk(rr + li, kr)];
            const double2 xv = sm.X[pk(max(kr, cc), cc)];
            const double2 bv = kr >= cc ? xv : mk(0.0, 0.0);
            cre = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.x, cre, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.y, cim, 0, 0, 0);
            cre = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.y, bv.y, cre, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv.x, cim, 0, 0, 0);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int q = pk(rr + 4 * v + lk, tc + li);
            sm.X[q] = csub(sm.X[q], mk(cre[v], cim[v]));
          }
        }
      }
    }
    __syncthreads();
  }
  if (sm.fail) {
    if (tid == 0) info[blockIdx.x] = k0 + sm.fail;
    return;
  }
  for (int e = tid; e < NB * NB; e += NTB) {
    const int i = e % NB, j = e / NB;
    if (i >= j && i < kb) A[i + (int64_t)j * lda] = sm.L[pk(i, j)];
  }
  double2 *w = work + ((int64_t)blockIdx.x * wslots + k0 / NB) * NB * NB;
  for (int e = tid; e < NB * NB; e += NTB) {
    const int i = e % NB, j = e / NB;
    w[e] = (i >= j && i < kb && j < kb) ? sm.X[pk(i, j)] : mk(0.0, 0.0);
  }
}

// Panel below the diagonal block: X = A_panel L_kk^-H as a product with the
// stored inverse, one 64-row tile per workgroup, in place.
__global__ __launch_bounds__(NT, 2) void k_potrf_panel(double2 *base, const PotrfItem *items,
                                                    const int *info, int k0, int kend,
                                                    const double2 *work, int wslots) {
  __shared__ GemmSmem sm;
  int bx, by;
  xcd_remap(bx, by);
  const PotrfItem it = items[by];
  const int n = it.n, lda = it.lda;
  const int kb = min(NB, min(kend, n) - k0);
  if (kb <= 0 || info[by] != 0) return;
  const int m = n - (k0 + kb), r0 = bx * TM;
  if (r0 >= m) return;
  double2 *P = base + it.a + (k0 + kb) + (int64_t)k0 * lda;
  const double2 *W = work + ((int64_t)by * wslots + k0 / NB) * NB * NB;
  gemm_tile<OP_N, OP_C>(m, kb, kb, 0, r0, 0, mk(1.0, 0.0), P, lda, W, NB, mk(0.0, 0.0), P, lda,
                        false, sm);
}

// Update C[r, c] -= sum_{k in [k_lo, k_hi)} A[r, k] conj(A[c, k]) for
// c in [c_lo, c_hi), r >= c (lower triangle only).
__global__ __launch_bounds__(NT, 2) void k_potrf_update(double2 *base, const PotrfItem *items,
                                                     const int *info, int k_lo, int k_hi,
                                                     int c_lo, int c_hi, int tiles_c) {
  // tiles_c > 0: grid of tiles_c tile columns; tiles_c = 0: the lower
  // triangle of tiles (ti >= tj) enumerated by tri_index
  __shared__ GemmSmem sm;
  int bx, by;
  xcd_remap(bx, by);
  const PotrfItem it = items[by];
  const int n = it.n, lda = it.lda;
  const int m = n - c_lo, nc = min(c_hi, n) - c_lo, kw = min(k_hi, n) - k_lo;
  if (m <= 0 || nc <= 0 || kw <= 0 || info[by] != 0) return;
  int ti, tj;
  if (tiles_c > 0) {
    ti = bx / tiles_c;
    tj = bx % tiles_c;
  } else {
    tri_index(bx, tj, ti);
  }
  if (ti * TM >= m || tj * TN >= nc || ti < tj) return;
  double2 *A = base + it.a;
  const double2 *P = A + c_lo + (int64_t)k_lo * lda;
  double2 *C = A + c_lo + (int64_t)c_lo * lda;
  gemm_tile<OP_N, OP_C>(m, nc, kw, 0, ti * TM, tj * TN, mk(-1.0, 0.0), P, lda, P, lda,
                        mk(1.0, 0.0), C, lda, ti == tj, sm);
}

// ---- triangular solve -------------------------------------------------------------

// Inverse of every diagonal block of L (all blocks at once: L is final).
__global__ __launch_bounds__(NTD) void k_trsm_inv(const double2 *lbase, const TrsmItem *items,
                                                 double2 *work, int wslots) {
  __shared__ double2 cb[2][NB], rb[2][NB];
  __shared__ double scale[NB];
  const TrsmItem it = items[blockIdx.y];
  const int k0 = blockIdx.x * NB;
  const int kb = min(NB, it.n - k0);
  if (kb <= 0) return;
  double2 a[kQ], x[kQ];
  load_block(lbase + it.l + k0 + (int64_t)k0 * it.ldl, it.ldl, kb, a, x);
  eliminate<false>(a, x, kb, cb, rb, scale);
  store_inverse(x, kb, scale, work + ((int64_t)blockIdx.y * wslots + blockIdx.x) * NB * NB);
}

// Rows [k0, k0+kb) of B: X_k = L_kk^-1 B_k, one 64-column tile per workgroup,
// in place.
__global__ __launch_bounds__(NT, 2) void k_trsm_solve(double2 *bbase, const TrsmItem *items, int k0,
                                                   int kend, int tri, const double2 *work,
                                                   int wslots) {
  __shared__ GemmSmem sm;
  int bx, by;
  xcd_remap(bx, by);
  const TrsmItem it = items[by];
  const int kb = min(NB, min(kend, it.n) - k0);
  if (kb <= 0) return;
  const int ncols = tri ? min(it.ncols, k0 + kb) : it.ncols;
  const int c0 = bx * TN;
  if (c0 >= ncols) return;
  double2 *Bk = bbase + it.b + k0;
  const double2 *W = work + ((int64_t)by * wslots + k0 / NB) * NB * NB;
  gemm_tile<OP_N, OP_N>(kb, ncols, kb, 0, 0, c0, mk(1.0, 0.0), W, NB, Bk, it.ldb, mk(0.0, 0.0),
                        Bk, it.ldb, false, sm);
}

// B[r, c] -= sum_{k in [k_lo, k_hi)} L[r, k] X[k, c] for r in [r_lo, r_hi),
// one 64x64 tile per workgroup.
__global__ __launch_bounds__(NT, 2) void k_trsm_update(const double2 *lbase, double2 *bbase,
                                                    const TrsmItem *items, int k_lo, int k_hi,
                                                    int r_lo, int r_hi, int tri, int tiles_c) {
  __shared__ GemmSmem sm;
  int bx, by;
  xcd_remap(bx, by);
  const TrsmItem it = items[by];
  const int n = it.n;
  const int m = min(r_hi, n) - r_lo, kw = min(k_hi, n) - k_lo;
  if (m <= 0 || kw <= 0) return;
  const int ncols = tri ? min(it.ncols, k_hi) : it.ncols;
  const int ti = bx / tiles_c, tj = bx % tiles_c;
  if (ti * TM >= m || tj * TN >= ncols) return;
  const double2 *L = lbase + it.l;
  double2 *B = bbase + it.b;
  gemm_tile<OP_N, OP_N>(m, ncols, kw, 0, ti * TM, tj * TN, mk(-1.0, 0.0),
                        L + r_lo + (int64_t)k_lo * it.ldl, it.ldl, B + k_lo, it.ldb,
                        mk(1.0, 0.0), B + r_lo, it.ldb, false, sm);
}

// ---- GEMM ----------------------------------------------------------------------------

template <int OPA, int OPB>
__global__ __launch_bounds__(NT, 2) void k_gemm(double2 alpha, const double2 *abase,
                                             const double2 *bbase, double2 beta, double2 *cbase,
                                             const GemmItem *items, int tiles_n, int mode) {
  __shared__ GemmSmem sm;
  int bx, by;
  xcd_remap(bx, by);
  const GemmItem it = items[by];
  // GEMM_FULL: tiles_n tile columns; otherwise the upper tiles by tri_index
  int tm, tn;
  if (mode == GEMM_FULL) {
    tm = bx / tiles_n;
    tn = bx % tiles_n;
  } else {
    tri_index(bx, tm, tn);
  }
  const int r0 = tm * TM, c0 = tn * TN;
  if (r0 >= it.m || c0 >= it.n) return;
  int kb = 0;
  if (mode == GEMM_UPPER_LOWTRI || mode == GEMM_HERM_LOWTRI)
    kb = c0;   // X lower triangular: rows below max(r0, c0) = c0 only
  const bool mirror = (mode == GEMM_HERM || mode == GEMM_HERM_LOWTRI) && tm < tn;
  gemm_tile<OPA, OPB>(it.m, it.n, it.k, kb, r0, c0, alpha, abase + it.a, it.lda, bbase + it.b,
                      it.ldb, beta, cbase + it.c, it.ldc, false, sm, mirror);
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

int64_t dense_work_size(int nitems, int nmax) {
  return (int64_t)std::max(nitems, 0) * cdiv(std::max(nmax, 1), NB) * NB * NB;
}

// info <- 0 for every item: a kernel rather than a memset node, since the
// Cholesky may run inside a captured HIP graph (the smoother with recomputed
// patch inverses).
__global__ __launch_bounds__(256) void k_zero_info(int *info, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) info[i] = 0;
}

// Algorithmic flops of the launches of one routine call (DenseProf): sums
// over the items of the blocked algorithm's step counts.
namespace {
template <typename F> double over_items(const DenseProf *dp, int nitems, F f) {
  double t = 0.0;
  for (int i = 0; i < nitems; ++i) t += f(dp->order(i), dp->cols(i));
  return t;
}
const DenseProf *prof_on(const DenseProf *dp) { return dp && dp->on() ? dp : nullptr; }
Prof *prof_of(const DenseProf *dp) { return dp ? dp->prof : nullptr; }
}  // namespace

void potrf_batched(double2 *base, const PotrfItem *items_dev, int nitems, int *info_dev, int nmax,
                   double2 *work, hipStream_t s, const DenseProf *dp) {
  if (nitems <= 0 || nmax <= 0) return;
  const int kmax = nmax;
  const int wslots = (int)cdiv(nmax, NB);
  const DenseProf *pf = prof_on(dp);
  hipLaunchKernelGGL(k_zero_info, dim3(cdiv(nitems, 256)), dim3(256), 0, s, info_dev, nitems);
  for (int K0 = 0; K0 < kmax; K0 += NBO) {
    const int K1 = std::min(K0 + NBO, kmax);
    for (int k0 = K0; k0 < K1; k0 += NB) {
      const int kb = std::min(NB, K1 - k0);
      {
        const double w = pf ? over_items(pf, nitems, [&](int n, int) {
          const double b = std::max(0, std::min(NB, std::min(K1, n) - k0));
          return 4.0 / 3.0 * b * b * b;
        }) : 0.0;
        ProfScope ps(prof_of(dp), DPG_K_POTRF_DIAG, w, s);
        hipLaunchKernelGGL(k_potrf_diag, dim3(nitems), dim3(NTB), 0, s, base, items_dev, info_dev,
                           k0, K1, work, wslots);
      }
      const int rows = nmax - k0 - kb;
      if (rows <= 0) continue;
      {
        const double w = pf ? over_items(pf, nitems, [&](int n, int) {
          const int b = std::max(0, std::min(NB, std::min(K1, n) - k0));
          const double m = b > 0 ? std::max(0, n - (k0 + b)) : 0;
          return 4.0 * m * b * b;
        }) : 0.0;
        ProfScope ps(prof_of(dp), DPG_K_POTRF_PANEL, w, s);
        hipLaunchKernelGGL(k_potrf_panel, dim3(cdiv(rows, TM), nitems), dim3(NT), 0, s, base,
                           items_dev, info_dev, k0, K1, (const double2 *)work, wslots);
      }
      // update of the rest of this block column only
      const int c_lo = k0 + kb, c_hi = K1;
      if (c_lo < c_hi) {
        const double w = pf ? over_items(pf, nitems, [&](int n, int) {
          const double kw = std::max(0, std::min(k0 + kb, n) - k0);
          double macs = 0.0;
          for (int c = c_lo; c < std::min(c_hi, n); ++c) macs += kw * (n - c);
          return 8.0 * macs;
        }) : 0.0;
        ProfScope ps(prof_of(dp), DPG_K_POTRF_UPDATE, w, s);
        const int tr = (int)cdiv(nmax - c_lo, TM), tc = (int)cdiv(c_hi - c_lo, TN);
        hipLaunchKernelGGL(k_potrf_update, dim3(tr * tc, nitems), dim3(NT), 0, s, base,
                           items_dev, info_dev, k0, k0 + kb, c_lo, c_hi, tc);
      }
    }
    // block update of the trailing matrix
    if (K1 < nmax) {
      const double w = pf ? over_items(pf, nitems, [&](int n, int) {
        const double kw = std::max(0, std::min(K1, n) - K0), t = std::max(0, n - K1);
        return 8.0 * kw * t * (t + 1) / 2;
      }) : 0.0;
      ProfScope ps(prof_of(dp), DPG_K_POTRF_UPDATE, w, s);
      const int t = (int)cdiv(nmax - K1, TM);
      hipLaunchKernelGGL(k_potrf_update, dim3(t * (t + 1) / 2, nitems), dim3(NT), 0, s, base,
                         items_dev, info_dev, K0, K1, K1, nmax, 0);
    }
  }
  LAUNCH_OK();
}

void trsm_batched(const double2 *lbase, double2 *bbase, const TrsmItem *items_dev, int nitems,
                  int max_n, int max_cols, bool identity_rhs, double2 *work, bool inverses_ready,
                  hipStream_t s, const DenseProf *dp) {
  if (nitems <= 0 || max_cols <= 0 || max_n <= 0) return;
  const int tri = identity_rhs ? 1 : 0;
  const int wslots = (int)cdiv(max_n, NB);
  const DenseProf *pf = prof_on(dp);
  if (!inverses_ready) {
    ProfScope ps(prof_of(dp), DPG_K_TRSM_INV, 0.0, s);   // no algorithmic flops of its own
    hipLaunchKernelGGL(k_trsm_inv, dim3(wslots, nitems), dim3(NTD), 0, s, lbase, items_dev, work,
                       wslots);
  }
  // multiply-adds of an update of rows [r_lo, r_hi) by inner indices
  // [k_lo, k_hi) for an item of order n with nc columns (identity right-hand
  // side: column c has nonzeros in rows >= c only)
  auto upd = [&](int n, int nc, int k_lo, int k_hi, int r_lo, int r_hi) {
    const double m = std::max(0, std::min(r_hi, n) - r_lo);
    const int ke = std::min(k_hi, n);
    const double kw = std::max(0, ke - k_lo);
    if (m <= 0 || kw <= 0) return 0.0;
    if (!tri) return 8.0 * m * kw * nc;
    return 8.0 * m * ((double)k_lo * kw + kw * (kw + 1) / 2);
  };
  for (int K0 = 0; K0 < max_n; K0 += NBO) {
    const int K1 = std::min(K0 + NBO, max_n);
    for (int k0 = K0; k0 < K1; k0 += NB) {
      const int kb = std::min(NB, K1 - k0);
      const int cols = tri ? std::min(max_cols, k0 + kb) : max_cols;
      {
        const double w = pf ? over_items(pf, nitems, [&](int n, int nc) {
          const double b = std::max(0, std::min(NB, std::min(K1, n) - k0));
          if (b <= 0) return 0.0;
          // identity right-hand side: full solves for the columns left of the
          // block, triangular ones inside it
          return tri ? 4.0 * k0 * b * b + 4.0 / 3.0 * b * b * b : 4.0 * b * b * nc;
        }) : 0.0;
        ProfScope ps(prof_of(dp), DPG_K_TRSM_SOLVE, w, s);
        hipLaunchKernelGGL(k_trsm_solve, dim3(cdiv(cols, TN), nitems), dim3(NT), 0, s, bbase,
                           items_dev, k0, K1, tri, (const double2 *)work, wslots);
      }
      // rows of this block row below the solved ones
      const int r_lo = k0 + kb, r_hi = K1;
      if (r_lo < r_hi) {
        const double w = pf ? over_items(pf, nitems, [&](int n, int nc) {
          return upd(n, nc, k0, k0 + kb, r_lo, r_hi);
        }) : 0.0;
        ProfScope ps(prof_of(dp), DPG_K_TRSM_UPDATE, w, s);
        const int tc = (int)cdiv(cols, TN);
        hipLaunchKernelGGL(k_trsm_update, dim3(cdiv(r_hi - r_lo, TM) * tc, nitems), dim3(NT), 0,
                           s, lbase, bbase, items_dev, k0, k0 + kb, r_lo, r_hi, tri, tc);
      }
    }
    if (K1 < max_n) {
      const double w = pf ? over_items(pf, nitems, [&](int n, int nc) {
        return upd(n, nc, K0, K1, K1, max_n);
      }) : 0.0;
      ProfScope ps(prof_of(dp), DPG_K_TRSM_UPDATE, w, s);
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
  const int tm = (int)cdiv(max_m, TM), tn = (int)cdiv(max_n, TN), t = std::max(tm, tn);
  dim3 g(mode == GEMM_FULL ? tm * tn : t * (t + 1) / 2, nitems);
  if (opa == OP_N) gemm_dispatch_b<OP_N>(opb, g, s, alpha, abase, bbase, beta, cbase, items_dev, tn, mode);
  else if (opa == OP_T) gemm_dispatch_b<OP_T>(opb, g, s, alpha, abase, bbase, beta, cbase, items_dev, tn, mode);
  else gemm_dispatch_b<OP_C>(opb, g, s, alpha, abase, bbase, beta, cbase, items_dev, tn, mode);
  LAUNCH_OK();
}

}  // namespace dpg
