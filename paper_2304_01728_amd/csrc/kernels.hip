// Hierarchy-setup and solve-phase kernels (see kernels.hpp).
#include "kernels.hpp"

#include "hblocks.hpp"

namespace dpg {
namespace {

constexpr int kMaxB = 2048, kMaxI = 1024;

// ---- setup -----------------------------------------------------------------------

// Gather form: a thread forms one entry (r, c) of T[b] as the sum, in child
// order, of the entries of the children that hold both r and c; a workgroup
// covers 256 rows of one column, so the column's child indices are uniform.
// Every entry is written once and the grid spreads over (rows, columns,
// blocks), so a level with few blocks still fills the GPU.
// One workgroup per (block, kAsmCols columns); the threads take the rows.
// Whether child ch holds column c is the same for the whole column, so the
// children without it are skipped by a uniform branch and each entry loads
// only from the children that hold its column (about 1.5 on average); the
// child slots of the thread's rows are loaded once for all its columns.
// The children are summed in order.
// ROWS rows per thread: nT <= 256 ROWS (instances for 4, 8 and 12).
constexpr int kAsmCols = 32;
template <int ROWS>
__global__ __launch_bounds__(256) void k_macro_assemble(const double2 *__restrict__ E, int n_tr,
                                                        const int32_t *__restrict__ child_inv,
                                                        int N, int b0, int nT,
                                                        double2 *__restrict__ T) {
  const int c0 = blockIdx.x * kAsmCols, b = b0 + blockIdx.y;
  const int Nc = N / 2;
  const int ci = b % Nc, cj = (b / Nc) % Nc, ck = b / (Nc * Nc);
  const int64_t n2 = (int64_t)n_tr * n_tr;
  const double2 *Ech[8];
#pragma unroll
  for (int ch = 0; ch < 8; ++ch) {
    const int e = (2 * ci + (ch & 1)) + N * ((2 * cj + ((ch >> 1) & 1)) + N * (2 * ck + (ch >> 2)));
    Ech[ch] = E + (int64_t)e * n2;
  }
  int lr[ROWS][8];
#pragma unroll
  for (int q = 0; q < ROWS; ++q) {
    const int r = threadIdx.x + 256 * q;
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) lr[q][ch] = r < nT ? child_inv[ch * nT + r] : -1;
  }
  double2 *Tb = T + (int64_t)blockIdx.y * nT * nT;
  const int cend = min(c0 + kAsmCols, nT);
  for (int c = c0; c < cend; ++c) {
    int lc[8];
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) lc[ch] = child_inv[ch * nT + c];
#pragma unroll
    for (int q = 0; q < ROWS; ++q) {
      const int r = threadIdx.x + 256 * q;
      if (256 * q >= nT) break;
      double2 v[8];
#pragma unroll
      for (int ch = 0; ch < 8; ++ch) {
        v[ch] = mk(0.0, 0.0);
        if (lc[ch] >= 0) v[ch] = Ech[ch][max(lr[q][ch], 0) + (int64_t)lc[ch] * n_tr];
      }
      double2 acc = mk(0.0, 0.0);
#pragma unroll
      for (int ch = 0; ch < 8; ++ch)
        if (lc[ch] >= 0 && lr[q][ch] >= 0) acc = cadd(acc, v[ch]);
      if (r < nT) Tb[r + (int64_t)c * nT] = acc;
    }
  }
}

__global__ __launch_bounds__(256) void k_copy_sub(const double2 *__restrict__ src,
                                                  int64_t src_stride, int lds, int r0, int c0,
                                                  int rows, int cols, double2 *__restrict__ dst,
                                                  int64_t dst_stride, int ldd,
                                                  const int32_t *__restrict__ dlist) {
  // one wave per column, its lanes over the rows
  const int j = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (j >= cols) return;
  const int64_t db = dlist ? dlist[blockIdx.y] : blockIdx.y;
  double2 *dc = dst + db * dst_stride + (int64_t)j * ldd;
  if (!src) {
    for (int i = threadIdx.x & 63; i < rows; i += 64) dc[i] = mk(0.0, 0.0);
    return;
  }
  const double2 *sc = src + blockIdx.y * src_stride + r0 + (int64_t)(c0 + j) * lds;
  for (int i = threadIdx.x & 63; i < rows; i += 64) dc[i] = sc[i];
}

// Entry (i, j) of a Hermitian block stored as packed upper 32x32 tiles (the
// layout of a HermSet: tile (I, J <= I) at tile_entry, entry (r, c) of a full
// tile at [4 (r % 4) + c % 4][8 (r / 4) + c / 4], a diagonal tile by its upper
// 4x4 sub-blocks); the lower triangle by conjugate transposition.
__device__ __forceinline__ double2 herm_tile_entry(const double2 *__restrict__ blk, int i, int j) {
  const bool low = i > j;
  const int a = low ? j : i, b = low ? i : j;
  const int I = a >> 5, J = b >> 5, r = a & 31, c = b & 31;
  const int k = 4 * (r & 3) + (c & 3);
  const double2 v = I < J ? blk[tile_entry(I, J) + k * 64 + 8 * (r >> 2) + (c >> 2)]
                          : blk[tile_entry(I, I) + k * kDiagSlots + diag_slot(r >> 2, c >> 2)];
  return low ? cconj(v) : v;
}

// The patch gather below with the macro blocks read from their packed tiles
// (tiles + ent_off[b] per block b) instead of full squares: pidx[b nBf + s]
// is the packed position of the block's local slot s.
__global__ __launch_bounds__(256) void k_patch_gather_tiles(
    const double2 *__restrict__ tiles, const int64_t *__restrict__ ent_off,
    const int32_t *__restrict__ pidx, int nBf, int Nc, const int64_t *__restrict__ pptr,
    const int32_t *__restrict__ pslot, int v0, const int64_t *__restrict__ dst_off,
    double2 *__restrict__ S) {
  const int v = v0 + blockIdx.x;
  const int64_t p0 = pptr[v];
  const int n = (int)(pptr[v + 1] - p0);
  const int jb = blockIdx.y * 8;
  if (jb >= n) return;
  const int vx = v % (Nc + 1), vy = (v / (Nc + 1)) % (Nc + 1), vz = v / ((Nc + 1) * (Nc + 1));
  int blk[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int ci = vx - 1 + (c & 1), cj = vy - 1 + ((c >> 1) & 1), ck = vz - 1 + (c >> 2);
    blk[c] = (ci >= 0 && cj >= 0 && ck >= 0 && ci < Nc && cj < Nc && ck < Nc)
                 ? ci + Nc * (cj + Nc * ck) : -1;
  }
  const int32_t *sl = pslot + p0 * 8;
  double2 *Sv = S + dst_off[blockIdx.x];
  const int jend = min(jb + 8, n);
  for (int j = jb; j < jend; ++j) {
    int pj[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int sj = blk[c] >= 0 ? sl[j * 8 + c] : -1;
      pj[c] = sj >= 0 ? pidx[(int64_t)blk[c] * nBf + sj] : -1;
    }
    for (int i = j + threadIdx.x; i < n; i += 256) {
      double2 acc = mk(0.0, 0.0);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        if (pj[c] < 0) continue;
        const int si = sl[(int64_t)i * 8 + c];
        if (si < 0) continue;
        const int pi = pidx[(int64_t)blk[c] * nBf + si];
        acc = cadd(acc, herm_tile_entry(tiles + ent_off[blk[c]], pi, pj[c]));
      }
      Sv[i + (int64_t)j * n] = acc;
    }
  }
}

// One workgroup per (patch, kGatCols columns j); the threads take the rows
// i >= j (the Cholesky that follows reads the lower triangle only).  Whether
// cell c holds column j is the same for the whole column, so the cells
// without it are skipped by a uniform branch and each entry loads only from
// the cells that hold its column.  Cells are summed in order.
constexpr int kGatCols = 8;
__global__ __launch_bounds__(256) void k_patch_gather(const double2 *__restrict__ Mfull, int nBf,
                                                      int Nc, const int64_t *__restrict__ pptr,
                                                      const int32_t *__restrict__ pslot, int v0,
                                                      const int64_t *__restrict__ dst_off,
                                                      double2 *__restrict__ S) {
  const int v = v0 + blockIdx.x;
  const int64_t p0 = pptr[v];
  const int n = (int)(pptr[v + 1] - p0);
  const int jb = blockIdx.y * kGatCols;
  if (jb >= n) return;
  const int vx = v % (Nc + 1), vy = (v / (Nc + 1)) % (Nc + 1), vz = v / ((Nc + 1) * (Nc + 1));
  int blk[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int ci = vx - 1 + (c & 1), cj = vy - 1 + ((c >> 1) & 1), ck = vz - 1 + (c >> 2);
    blk[c] = (ci >= 0 && cj >= 0 && ck >= 0 && ci < Nc && cj < Nc && ck < Nc)
                 ? ci + Nc * (cj + Nc * ck) : -1;
  }
  const int32_t *sl = pslot + p0 * 8;
  double2 *Sv = S + dst_off[blockIdx.x];
  const int64_t nb2 = (int64_t)nBf * nBf;
  const int jend = min(jb + kGatCols, n);
  for (int j = jb; j < jend; ++j) {
    int sj[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) sj[c] = blk[c] >= 0 ? sl[j * 8 + c] : -1;
    for (int i = j + threadIdx.x; i < n; i += 256) {
      const int4 s0 = *reinterpret_cast<const int4 *>(sl + (int64_t)i * 8);
      const int4 s1 = *reinterpret_cast<const int4 *>(sl + (int64_t)i * 8 + 4);
      const int si[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
      double2 w[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        w[c] = mk(0.0, 0.0);
        if (sj[c] >= 0) w[c] = Mfull[blk[c] * nb2 + max(si[c], 0) + (int64_t)sj[c] * nBf];
      }
      double2 acc = mk(0.0, 0.0);
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (sj[c] >= 0 && si[c] >= 0) acc = cadd(acc, w[c]);
      Sv[i + (int64_t)j * n] = acc;
    }
  }
}

__global__ __launch_bounds__(256) void k_identity(const int64_t *__restrict__ off,
                                                  const int32_t *__restrict__ nn,
                                                  double2 *__restrict__ X) {
  // one wave per column, its lanes over the rows
  const int n = nn[blockIdx.y];
  const int j = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (j >= n) return;
  double2 *xc = X + off[blockIdx.y] + (int64_t)j * n;
  for (int i = threadIdx.x & 63; i < n; i += 64) xc[i] = mk(i == j ? 1.0 : 0.0, 0.0);
}

__global__ __launch_bounds__(256) void k_assemble_dense(const double2 *__restrict__ E, int n_tr,
                                                        const int32_t *__restrict__ edofs,
                                                        int nel, int n0,
                                                        double2 *__restrict__ T0) {
  for (int64_t k = threadIdx.x; k < (int64_t)n0 * n0; k += 256) T0[k] = mk(0.0, 0.0);
  __syncthreads();
  const int n2 = n_tr * n_tr;
  for (int e = 0; e < nel; ++e) {
    const int32_t *d = edofs + (int64_t)e * n_tr;
    for (int k = threadIdx.x; k < n2; k += 256) {
      const int gi = d[k % n_tr], gj = d[k / n_tr];
      if (gi >= 0 && gj >= 0) {
        double2 *dst = &T0[gi + (int64_t)gj * n0];
        *dst = cadd(*dst, E[(int64_t)e * n2 + k]);
      }
    }
    __syncthreads();
  }
}

// ---- solve phase --------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_csr(int64_t nrows, const int64_t *__restrict__ ptr,
                                             const int32_t *__restrict__ col,
                                             const T *__restrict__ val,
                                             const cplx_t<T> *__restrict__ x,
                                             cplx_t<T> *__restrict__ y, int add) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nrows) return;
  cplx_t<T> acc;
  acc.x = 0;
  acc.y = 0;
  for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) acc = cadd(acc, cscale(x[col[k]], val[k]));
  y[i] = add ? cadd(y[i], acc) : acc;
}

// One workgroup per (block, 64 boundary slots): wave w sums the interior
// unknowns i = w, w + 4, ... for its 64 slots (coalesced reads of one column
// of W^H per step), and the four partial sums are added in a fixed order.
// Seven or more workgroups per block keep the GPU busy on the coarse levels,
// which have few blocks.
template <typename T>
__global__ __launch_bounds__(256) void k_condense_local(const cplx_t<T> *__restrict__ WH, int nI,
                                                        int nBf, const int32_t *__restrict__ blkI,
                                                        const cplx_t<T> *__restrict__ rc,
                                                        cplx_t<T> *__restrict__ c) {
  using C = cplx_t<T>;
  __shared__ C rI[kMaxI];
  __shared__ C part[4][64];
  const int b = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sl = blockIdx.y * 64 + lane;
  for (int i = threadIdx.x; i < nI; i += 256) rI[i] = rc[blkI[(int64_t)b * nI + i]];
  __syncthreads();
  const C *W = WH + (int64_t)b * nBf * nI;
  C a0, a1;
  a0.x = a0.y = 0;
  a1.x = a1.y = 0;
  if (sl < nBf) {
    int i = wave;
    for (; i + 4 < nI; i += 8) {
      a0 = cfma(W[sl + (int64_t)i * nBf], rI[i], a0);
      a1 = cfma(W[sl + (int64_t)(i + 4) * nBf], rI[i + 4], a1);
    }
    if (i < nI) a0 = cfma(W[sl + (int64_t)i * nBf], rI[i], a0);
  }
  part[wave][lane] = cadd(a0, a1);
  __syncthreads();
  if (wave == 0 && sl < nBf)
    c[(int64_t)b * nBf + sl] = cadd(cadd(part[0][lane], part[1][lane]),
                                    cadd(part[2][lane], part[3][lane]));
}

template <typename T>
__global__ __launch_bounds__(256) void k_condense_reduce(int64_t nM,
                                                         const int64_t *__restrict__ macro_B,
                                                         const int32_t *__restrict__ red_ptr,
                                                         const int32_t *__restrict__ red_ent,
                                                         const cplx_t<T> *__restrict__ rc,
                                                         const cplx_t<T> *__restrict__ c,
                                                         cplx_t<T> *__restrict__ rB) {
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= nM) return;
  cplx_t<T> acc = rc[macro_B[m]];
  for (int32_t k = red_ptr[m]; k < red_ptr[m + 1]; ++k) acc = csub(acc, c[red_ent[k]]);
  rB[m] = acc;
}

template <typename C> __device__ inline C wave_sum(C v) {
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o, 64);
    v.y += __shfl_xor(v.y, o, 64);
  }
  return v;
}

// One workgroup per (block, group of kExpRows interior unknowns), one wave
// per unknown at a time: many short workgroups instead of one long one per
// block keep the GPU busy when a level has few blocks.
constexpr int kExpRows = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_expand(const cplx_t<T> *__restrict__ WH,
                                                const cplx_t<T> *__restrict__ Tinv, int nI,
                                                int nBf, const int32_t *__restrict__ blkI,
                                                const int32_t *__restrict__ blkBm,
                                                const cplx_t<T> *__restrict__ rc,
                                                const cplx_t<T> *__restrict__ eB,
                                                cplx_t<T> *__restrict__ ec) {
  using C = cplx_t<T>;
  __shared__ C eBs[kMaxB];
  __shared__ C rI[kMaxI];
  const int b = blockIdx.x, i0 = blockIdx.y * kExpRows, i1 = min(nI, i0 + kExpRows);
  for (int sl = threadIdx.x; sl < nBf; sl += 256) {
    const int m = blkBm[(int64_t)b * nBf + sl];
    C v;
    v.x = 0;
    v.y = 0;
    if (m >= 0) v = eB[m];
    eBs[sl] = v;
  }
  for (int i = threadIdx.x; i < nI; i += 256) rI[i] = rc[blkI[(int64_t)b * nI + i]];
  __syncthreads();
  const C *W = WH + (int64_t)b * nBf * nI;
  const C *Ti = Tinv + (int64_t)b * nI * nI;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = i0 + wave; i < i1; i += 4) {
    C u, v;
    u.x = u.y = 0;
    v.x = v.y = 0;
    // u = (WH^H eB)_i = sum_sl conj(WH[sl, i]) eB[sl]; v = (Tinv rI)_i = sum_j conj(Tinv[j, i]) rI[j]
    for (int sl = lane; sl < nBf; sl += 64) u = cfmaconj(W[sl + (int64_t)i * nBf], eBs[sl], u);
    for (int j = lane; j < nI; j += 64) v = cfmaconj(Ti[j + (int64_t)i * nI], rI[j], v);
    u = wave_sum(u);
    v = wave_sum(v);
    if (lane == 0) ec[blkI[(int64_t)b * nI + i]] = csub(v, u);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_scatter_macro(int64_t nM, const int64_t *__restrict__ macro_B,
                                                       const cplx_t<T> *__restrict__ eB,
                                                       cplx_t<T> *__restrict__ ec) {
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m < nM) ec[macro_B[m]] = eB[m];
}

__global__ __launch_bounds__(256) void k_assemble_vec(int64_t n, const int32_t *__restrict__ ptr,
                                                      const int32_t *__restrict__ ent,
                                                      const double2 *__restrict__ se,
                                                      int64_t se_stride,
                                                      double2 *__restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  double2 acc = mk(0.0, 0.0);
  for (int32_t k = ptr[t]; k < ptr[t + 1]; ++k) acc = cadd(acc, se[ent[k]]);
  out[t] = acc;
  (void)se_stride;
}

__global__ __launch_bounds__(256) void k_fields(const double2 *__restrict__ recL,
                                                const double2 *__restrict__ recY,
                                                const double2 *__restrict__ recYb, int nf,
                                                int ntr, int nrhs, int col,
                                                const int32_t *__restrict__ edofs,
                                                const double2 *__restrict__ x,
                                                double2 *__restrict__ out) {
  __shared__ double2 v[kMaxI];
  __shared__ double2 xt[kMaxB];
  const int e = blockIdx.x;
  for (int j = threadIdx.x; j < ntr; j += 256) {
    const int32_t t = edofs[(int64_t)e * ntr + j];
    xt[j] = t >= 0 ? x[t] : mk(0.0, 0.0);
  }
  __syncthreads();
  const double2 *Y = recY + (int64_t)e * nf * ntr;
  const double2 *Yb = recYb + ((int64_t)e * nrhs + col) * nf;
  const double2 *L = recL + (int64_t)e * nf * nf;
  for (int i = threadIdx.x; i < nf; i += 256) {
    double2 acc = Yb[i];
    for (int j = 0; j < ntr; ++j) acc = csub(acc, cmul(Y[i + (int64_t)j * nf], xt[j]));
    v[i] = acc;
  }
  __syncthreads();
  // L^H u = v, column by column from the last unknown
  for (int i = nf - 1; i >= 0; --i) {
    if (threadIdx.x == 0) v[i] = cscale(v[i], 1.0 / L[i + (int64_t)i * nf].x);
    __syncthreads();
    for (int k = threadIdx.x; k < i; k += 256)
      v[k] = csub(v[k], cmul(cconj(L[i + (int64_t)k * nf]), v[i]));
    __syncthreads();
  }
  for (int i = threadIdx.x; i < nf; i += 256) out[(int64_t)e * nf + i] = v[i];
}

// Error indicator, step 1: the unknowns [x_f; x_t] of element e0 + blockIdx.x
// for load column blockIdx.y.  K holds, per element (stride ks, leading
// dimension ld), the factor L of K_ff in its first nf columns and
// Y = L^-1 [K_ft | b] in the columns after: x_f = L^-H (Y_b - Y_t x_t).
// X[i] is m x nr (leading dimension m = nf + ntr), x_t gathered from x
// (column r at x + r nvec) through the element map (-1: absent, zero).
__global__ __launch_bounds__(256) void k_indicator_x(const double2 *__restrict__ K, int64_t ks,
                                                     int ld, int nf, int ntr, int nr,
                                                     const int32_t *__restrict__ edofs,
                                                     const double2 *__restrict__ x, int64_t nvec,
                                                     double2 *__restrict__ X) {
  __shared__ double2 v[kMaxI];
  __shared__ double2 xt[kMaxB];
  const int e = blockIdx.x, r = blockIdx.y, m = nf + ntr;
  const double2 *xr = x + (int64_t)r * nvec;
  double2 *Xe = X + ((int64_t)e * nr + r) * m;
  for (int j = threadIdx.x; j < ntr; j += 256) {
    const int32_t t = edofs[(int64_t)e * ntr + j];
    xt[j] = t >= 0 ? xr[t] : mk(0.0, 0.0);
    Xe[nf + j] = xt[j];
  }
  __syncthreads();
  const double2 *Ke = K + (int64_t)e * ks;
  for (int i = threadIdx.x; i < nf; i += 256) {
    double2 acc = Ke[i + (int64_t)(m + r) * ld];
    for (int j = 0; j < ntr; ++j) acc = csub(acc, cmul(Ke[i + (int64_t)(nf + j) * ld], xt[j]));
    v[i] = acc;
  }
  __syncthreads();
  for (int i = nf - 1; i >= 0; --i) {   // L^H u = v from the last unknown
    if (threadIdx.x == 0) v[i] = cscale(v[i], 1.0 / Ke[i + (int64_t)i * ld].x);
    __syncthreads();
    for (int k = threadIdx.x; k < i; k += 256)
      v[k] = csub(v[k], cmul(cconj(Ke[i + (int64_t)k * ld]), v[i]));
    __syncthreads();
  }
  for (int i = threadIdx.x; i < nf; i += 256) Xe[i] = v[i];
}

// Error indicator, step 3: out[r * nel_out + e0 + e] = || W[e](:, c0 + r) ||^2
// over n rows (W per element at stride ws, leading dimension ld).
__global__ __launch_bounds__(256) void k_colnorm2(const double2 *__restrict__ W, int64_t ws,
                                                  int ld, int n, int c0, int e0, int64_t nel_out,
                                                  double *__restrict__ out) {
  __shared__ double red[256];
  const int e = blockIdx.x, r = blockIdx.y;
  const double2 *w = W + (int64_t)e * ws + (int64_t)(c0 + r) * ld;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += w[i].x * w[i].x + w[i].y * w[i].y;
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(int64_t)r * nel_out + e0 + e] = red[0];
}

template <typename C> __global__ void k_zero(int64_t n, C *a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    a[i].x = 0;
    a[i].y = 0;
  }
}

__global__ void k_to32(int64_t n, const double2 *a, float2 *b) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) b[i] = mkf((float)a[i].x, (float)a[i].y);
}
__global__ void k_to64(int64_t n, const float2 *a, double2 *b) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) b[i] = mk((double)a[i].x, (double)a[i].y);
}

// ---- CG ---------------------------------------------------------------------------------

__device__ inline double block_sum(double v) {
  __shared__ double sh[4];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

// partial[blockIdx] = sum over a grid-stride slice of Re(conj(a) b)
__global__ __launch_bounds__(256) void k_dot_partial(int64_t n, const double2 *__restrict__ a,
                                                     const double2 *__restrict__ b,
                                                     double *__restrict__ partial) {
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    s += a[i].x * b[i].x + a[i].y * b[i].y;
  s = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_dot2_partial(int64_t n, const double2 *__restrict__ r,
                                                      const double2 *__restrict__ z,
                                                      const double2 *__restrict__ zo,
                                                      double *__restrict__ partial) {
  double s = 0.0, t = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    s += r[i].x * z[i].x + r[i].y * z[i].y;
    t += r[i].x * zo[i].x + r[i].y * zo[i].y;
  }
  s = block_sum(s);
  t = block_sum(t);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s;
    partial[kDotBlocks + blockIdx.x] = t;
  }
}

__device__ inline double sum_partials(const double *partial) {
  double s = 0.0;
  for (int i = threadIdx.x; i < kDotBlocks; i += 256) s += partial[i];
  return block_sum(s);
}

// mode 0: dst = sum; 1: pq / alpha; 2: ||r||^2; 3: beta
__global__ __launch_bounds__(256) void k_final(const double *__restrict__ partial, double *dst,
                                               double *sc, int mode) {
  const double s = sum_partials(partial);
  double t = 0.0;
  if (mode == 3) t = sum_partials(partial + kDotBlocks);
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    *dst = s;
  } else if (mode == 1) {
    sc[1] = s;
    if (!(s > 0.0) || !isfinite(s)) sc[6] = 1.0;
    sc[2] = sc[0] / s;
  } else if (mode == 2) {
    sc[4] = s;
  } else {
    // flexible (Polak-Ribiere) beta = Re(r^H (z - z_old)) / Re(r_old^H z_old)
    sc[3] = (s - t) / sc[0];
    sc[7] = t;
    sc[0] = s;
    if (!isfinite(sc[3])) sc[6] = 1.0;
  }
}

__global__ __launch_bounds__(256) void k_update_xr(int64_t n, double2 *__restrict__ x,
                                                   double2 *__restrict__ r,
                                                   const double2 *__restrict__ p,
                                                   const double2 *__restrict__ q,
                                                   double *__restrict__ partial,
                                                   const double *__restrict__ sc) {
  const double a = sc[2];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    x[i] = mk(x[i].x + a * p[i].x, x[i].y + a * p[i].y);
    const double2 ri = mk(r[i].x - a * q[i].x, r[i].y - a * q[i].y);
    r[i] = ri;
    s += ri.x * ri.x + ri.y * ri.y;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_update_p(int64_t n, double2 *__restrict__ p,
                                                  const double2 *__restrict__ z,
                                                  const double *__restrict__ sc) {
  const double b = sc[3];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = mk(z[i].x + b * p[i].x, z[i].y + b * p[i].y);
}

}  // namespace

// ---- launchers --------------------------------------------------------------------------

void launch_macro_assemble(const double2 *E, int n_tr, const int32_t *child_inv, int N, int b0,
                           int count, int nT, double2 *T, hipStream_t s) {
  if (count <= 0) return;
  if (count > 65535 || nT > 256 * 12) throw DpgError(-1, "macro assembly grid too large");
  const dim3 g(cdiv(nT, kAsmCols), count);
  if (nT <= 256 * 4)
    hipLaunchKernelGGL(k_macro_assemble<4>, g, dim3(256), 0, s, E, n_tr, child_inv, N, b0, nT, T);
  else if (nT <= 256 * 8)
    hipLaunchKernelGGL(k_macro_assemble<8>, g, dim3(256), 0, s, E, n_tr, child_inv, N, b0, nT, T);
  else
    hipLaunchKernelGGL(k_macro_assemble<12>, g, dim3(256), 0, s, E, n_tr, child_inv, N, b0, nT, T);
  LAUNCH_OK();
}

void launch_copy_sub(const double2 *src, int64_t src_stride, int lds, int r0, int c0, int rows,
                     int cols, double2 *dst, int64_t dst_stride, int ldd, int count,
                     hipStream_t s, const int32_t *dlist) {
  if (count <= 0 || rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(k_copy_sub, dim3(cdiv(cols, 4), count), dim3(256), 0, s,
                     src, src_stride, lds, r0, c0, rows, cols, dst, dst_stride, ldd, dlist);
  LAUNCH_OK();
}

void launch_patch_gather_tiles(const double2 *tiles, const int64_t *ent_off, const int32_t *pidx,
                               int nBf, int Nc, const int64_t *patch_ptr,
                               const int32_t *patch_slot, int v0, int count, int nmax,
                               const int64_t *dst_off, double2 *S, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_patch_gather_tiles, dim3(count, cdiv(nmax, kGatCols)), dim3(256), 0, s,
                     tiles, ent_off, pidx, nBf, Nc, patch_ptr, patch_slot, v0, dst_off, S);
  LAUNCH_OK();
}

void launch_patch_gather(const double2 *Mfull, int nBf, int Nc, const int64_t *patch_ptr,
                         const int32_t *patch_slot, int v0, int count, int nmax,
                         const int64_t *dst_off, double2 *S, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_patch_gather, dim3(count, cdiv(nmax, kGatCols)), dim3(256), 0, s, Mfull,
                     nBf, Nc, patch_ptr, patch_slot, v0, dst_off, S);
  LAUNCH_OK();
}

void launch_identity(const int64_t *off, const int32_t *n, int count, int nmax, double2 *X,
                     hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_identity, dim3(cdiv(nmax, 4), count), dim3(256), 0, s,
                     off, n, X);
  LAUNCH_OK();
}

void launch_assemble_dense(const double2 *E, int n_tr, const int32_t *edofs, int nel, int n0,
                           double2 *T0, hipStream_t s) {
  hipLaunchKernelGGL(k_assemble_dense, dim3(1), dim3(256), 0, s, E, n_tr, edofs, nel, n0, T0);
  LAUNCH_OK();
}

template <typename T>
void launch_csr(int64_t nrows, const int64_t *ptr, const int32_t *col, const T *val,
                const cplx_t<T> *x, cplx_t<T> *y, int add, hipStream_t s) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL((k_csr<T>), dim3(cdiv(nrows, 256)), dim3(256), 0, s, nrows, ptr, col, val, x,
                     y, add);
  LAUNCH_OK();
}

template <typename T>
void launch_condense_local(const cplx_t<T> *WH, int nI, int nBf, const int32_t *blkI, int nblk,
                           const cplx_t<T> *rc, cplx_t<T> *c, hipStream_t s) {
  if (nI > kMaxI || nBf > kMaxB) throw DpgError(-1, "macro block too large");
  hipLaunchKernelGGL((k_condense_local<T>), dim3(nblk, cdiv(nBf, 64)), dim3(256), 0, s, WH, nI,
                     nBf, blkI, rc, c);
  LAUNCH_OK();
}

template <typename T>
void launch_condense_reduce(int64_t nM, const int64_t *macro_B, const int32_t *red_ptr,
                            const int32_t *red_ent, const cplx_t<T> *rc, const cplx_t<T> *c,
                            cplx_t<T> *rB, hipStream_t s) {
  hipLaunchKernelGGL((k_condense_reduce<T>), dim3(cdiv(nM, 256)), dim3(256), 0, s, nM, macro_B,
                     red_ptr, red_ent, rc, c, rB);
  LAUNCH_OK();
}

template <typename T>
void launch_expand(const cplx_t<T> *WH, const cplx_t<T> *Tinv, int nI, int nBf,
                   const int32_t *blkI, const int32_t *blkBm, int nblk, const cplx_t<T> *rc,
                   const cplx_t<T> *eB, int64_t nM, const int64_t *macro_B, cplx_t<T> *ec,
                   hipStream_t s) {
  if (nI > kMaxI || nBf > kMaxB) throw DpgError(-1, "macro block too large");
  hipLaunchKernelGGL((k_scatter_macro<T>), dim3(cdiv(nM, 256)), dim3(256), 0, s, nM, macro_B, eB,
                     ec);
  LAUNCH_OK();
  hipLaunchKernelGGL((k_expand<T>), dim3(nblk, cdiv(nI, kExpRows)), dim3(256), 0, s, WH, Tinv, nI,
                     nBf, blkI, blkBm, rc, eB, ec);
  LAUNCH_OK();
}

void launch_assemble_vec(int64_t n, const int32_t *ptr, const int32_t *ent, const double2 *se,
                         int64_t se_stride, double2 *out, hipStream_t s) {
  hipLaunchKernelGGL(k_assemble_vec, dim3(cdiv(n, 256)), dim3(256), 0, s, n, ptr, ent, se,
                     se_stride, out);
  LAUNCH_OK();
}

void launch_fields(const double2 *recL, const double2 *recY, const double2 *recYb, int nf,
                   int ntr, int nrhs, int col, const int32_t *edofs, int nel, const double2 *x,
                   double2 *out, hipStream_t s) {
  if (nf > kMaxI || ntr > kMaxB) throw DpgError(-1, "element too large for field recovery");
  hipLaunchKernelGGL(k_fields, dim3(nel), dim3(256), 0, s, recL, recY, recYb, nf, ntr, nrhs, col,
                     edofs, x, out);
  LAUNCH_OK();
}

void launch_indicator_x(const double2 *K, int64_t ks, int ld, int nf, int ntr, int nr,
                        const int32_t *edofs, int count, const double2 *x, int64_t nvec,
                        double2 *X, hipStream_t s) {
  if (nf > kMaxI || ntr > kMaxB) throw DpgError(-1, "element too large for the error indicator");
  if (count <= 0 || nr <= 0) return;
  hipLaunchKernelGGL(k_indicator_x, dim3(count, nr), dim3(256), 0, s, K, ks, ld, nf, ntr, nr,
                     edofs, x, nvec, X);
  LAUNCH_OK();
}

void launch_colnorm2(const double2 *W, int64_t ws, int ld, int n, int c0, int ncols, int e0,
                     int count, int64_t nel_out, double *out, hipStream_t s) {
  if (count <= 0 || ncols <= 0) return;
  hipLaunchKernelGGL(k_colnorm2, dim3(count, ncols), dim3(256), 0, s, W, ws, ld, n, c0, e0,
                     nel_out, out);
  LAUNCH_OK();
}

template <typename C> void launch_zero(int64_t n, C *a, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_zero<C>), dim3(cdiv(n, 256)), dim3(256), 0, s, n, a);
  LAUNCH_OK();
}
template void launch_zero<double2>(int64_t, double2 *, hipStream_t);
template void launch_zero<float2>(int64_t, float2 *, hipStream_t);

void launch_to32(int64_t n, const double2 *a, float2 *b, hipStream_t s) {
  hipLaunchKernelGGL(k_to32, dim3(cdiv(n, 256)), dim3(256), 0, s, n, a, b);
  LAUNCH_OK();
}
void launch_to64(int64_t n, const float2 *a, double2 *b, hipStream_t s) {
  hipLaunchKernelGGL(k_to64, dim3(cdiv(n, 256)), dim3(256), 0, s, n, a, b);
  LAUNCH_OK();
}

void dot_re(int64_t n, const double2 *a, const double2 *b, double *partial, double *dst,
            hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(256), 0, s, n, a, b, partial);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, s, partial, dst, (double *)nullptr, 0);
  LAUNCH_OK();
}

void cg_alpha(int64_t n, const double2 *p, const double2 *q, double *partial, double *sc,
              hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(256), 0, s, n, p, q, partial);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, s, partial, (double *)nullptr, sc, 1);
  LAUNCH_OK();
}

void cg_update_xr(int64_t n, double2 *x, double2 *r, const double2 *p, const double2 *q,
                  double *partial, double *sc, hipStream_t s) {
  hipLaunchKernelGGL(k_update_xr, dim3(kDotBlocks), dim3(256), 0, s, n, x, r, p, q, partial, sc);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, s, partial, (double *)nullptr, sc, 2);
  LAUNCH_OK();
}

void cg_beta(int64_t n, const double2 *r, const double2 *z, const double2 *zold, double *partial,
             double *sc, hipStream_t s) {
  hipLaunchKernelGGL(k_dot2_partial, dim3(kDotBlocks), dim3(256), 0, s, n, r, z, zold, partial);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, s, partial, (double *)nullptr, sc, 3);
  LAUNCH_OK();
}

void cg_update_p(int64_t n, double2 *p, const double2 *z, const double *sc, hipStream_t s) {
  hipLaunchKernelGGL(k_update_p, dim3(cdiv(n, 256)), dim3(256), 0, s, n, p, z, sc);
  LAUNCH_OK();
}

template void launch_csr<double>(int64_t, const int64_t *, const int32_t *, const double *,
                                 const double2 *, double2 *, int, hipStream_t);
template void launch_csr<float>(int64_t, const int64_t *, const int32_t *, const float *,
                                const float2 *, float2 *, int, hipStream_t);
template void launch_condense_local<double>(const double2 *, int, int, const int32_t *, int,
                                            const double2 *, double2 *, hipStream_t);
template void launch_condense_local<float>(const float2 *, int, int, const int32_t *, int,
                                           const float2 *, float2 *, hipStream_t);
template void launch_condense_reduce<double>(int64_t, const int64_t *, const int32_t *,
                                             const int32_t *, const double2 *, const double2 *,
                                             double2 *, hipStream_t);
template void launch_condense_reduce<float>(int64_t, const int64_t *, const int32_t *,
                                            const int32_t *, const float2 *, const float2 *,
                                            float2 *, hipStream_t);
template void launch_expand<double>(const double2 *, const double2 *, int, int, const int32_t *,
                                    const int32_t *, int, const double2 *, const double2 *,
                                    int64_t, const int64_t *, double2 *, hipStream_t);
template void launch_expand<float>(const float2 *, const float2 *, int, int, const int32_t *,
                                   const int32_t *, int, const float2 *, const float2 *, int64_t,
                                   const int64_t *, float2 *, hipStream_t);

}  // namespace dpg
