// Multi-right-hand-side kernels (see block.hpp).
#include <algorithm>

#include "block.hpp"
#include "kernels.hpp"

namespace dpg {
namespace {

constexpr int kBMaxI = 1024;   // interior unknowns per macro block (as the single path)
constexpr int KC = 4;          // columns per workgroup in the condensation kernels

template <typename C> __device__ inline C czero() {
  C r;
  r.x = 0;
  r.y = 0;
  return r;
}

// ---- Hermitian block sets ------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_gather_blk(int64_t nloc, int nr,
                                                    const int32_t *__restrict__ gidx,
                                                    const cplx_t<T> *__restrict__ x,
                                                    cplx_t<T> *__restrict__ xl) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nloc * nr) return;
  const int64_t i = e / nr;
  const int k = (int)(e % nr);
  const int32_t g = gidx[i];
  xl[e] = g >= 0 ? x[(int64_t)g * nr + k] : czero<cplx_t<T>>();
}

// One wave per (block b, tile row I): Y_I (32 x nr) = sum_J A_IJ X_J over the
// stored upper tiles of row I (J >= I) and the conjugate transposes of the
// stored tiles of column I (J < I), so no partial sums leave the wave.
//
// FP32, on the matrix cores.  Y_I (32 x 32, columns past
// nr are padding) accumulates three real 32x32x32 products per tile (the
// three-multiplication complex product: a quarter fewer matrix-core
// operations, and an imaginary part formed as p3 - p1 - p2, which in FP32
// can lose digits when it is small against |A||X|; this path is the
// mixed-precision preconditioner, corrected by the FP64 outer iteration),
// with v_mfma_f32_32x32x2f32: lane l supplies A[l%32][k] and B[k][l%32] for
// k = l/32 of each two-column slice, and receives result row
// 8(v/4) + 4(l/32) + v%4, column l%32 in register v.  The tile A_IJ is
// staged in LDS column by column (double-buffered, rows XOR-swizzled per
// group of four columns); X_J goes straight from global memory into the
// B operands, which for nr = 32 are contiguous 512-byte rows.  The next
// tile and X_J are loaded while the current ones are multiplied.
// Workgroup g runs on XCD g % 8, so each XCD is given a contiguous range of
// tile rows: the rows of one block then share its tiles and X in one L2.
typedef float v16f __attribute__((ext_vector_type(16)));
typedef double v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(64, 2) void k_rows_mfma(const float2 *__restrict__ tiles,
                                                  const int2 *__restrict__ rows, int64_t nrows,
                                                  const int32_t *__restrict__ bn,
                                                  const int64_t *__restrict__ ent_off,
                                                  const int64_t *__restrict__ loc_off,
                                                  const float2 *__restrict__ xl,
                                                  float2 *__restrict__ yl, int nr) {
  __shared__ float2 As[2][32 * 32];
  const int64_t per = (nrows + 7) / 8;
  const int64_t w = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (w >= nrows) return;
  const int lane = threadIdx.x, a = lane >> 3, q = lane & 7;
  const int kk = lane >> 5, n = lane & 31;
  // columns past nr read column nr - 1: B column n only feeds result column
  // n, and those results are not stored
  const int ncl = n < nr ? n : nr - 1;
  const int2 bi = rows[w];
  const int b = bi.x, I = bi.y;
  const int nt = (bn[b] + 31) >> 5;
  const int64_t e0 = ent_off[b];
  // a diagonal tile stores the sub-blocks a <= q only (slot diag_slot(a, q))
  const bool dup = a <= q;
  const int dsl = dup ? diag_slot(a, q) : 0;
  const float2 *xb = xl + loc_off[b] * nr + ncl;
  auto load = [&](int J, float2 *tt, float2 *xx) {
    // (wave-uniform branch, constant strides: immediate load offsets); lanes
    // below the diagonal of a diagonal tile read slot 0 (in range), their
    // values are not staged
    if (J != I) {
      const float2 *tp = tiles + e0 + (J > I ? tile_entry(I, J) : tile_entry(J, I)) + lane;
#pragma unroll
      for (int k = 0; k < 16; ++k) tt[k] = tp[k * 64];
    } else {
      const float2 *tp = tiles + e0 + tile_entry(I, I) + dsl;
#pragma unroll
      for (int k = 0; k < 16; ++k) tt[k] = tp[k * kDiagSlots];
    }
    const float2 *xp = xb + (int64_t)(32 * J + kk) * nr;
#pragma unroll
    for (int s = 0; s < 16; ++s) xx[s] = xp[(int64_t)2 * s * nr];
  };
  // three real products (Gauss): p1 = Re A Re X, p2 = Im A Im X,
  // p3 = (Re A + Im A)(Re X + Im X); Re Y = p1 - p2, Im Y = p3 - p1 - p2
  v16f p1, p2, p3;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    p1[v] = 0.f;
    p2[v] = 0.f;
    p3[v] = 0.f;
  }
  // one tile: start loading tile Jn into tn/xn, stage t as A_IJ in LDS,
  // multiply; the scheduling barriers keep the loads ahead of the products
  auto step = [&](int J, int Jn, const float2 *t, const float2 *x, float2 *tn, float2 *xn) {
    load(Jn, tn, xn);
    __builtin_amdgcn_sched_barrier(0);
    const bool up = J >= I;
    float2 *buf = As[J & 1];
    // the lane holds stored entries (4a + i, 4q + j) at 4i + j; A_IJ is the
    // stored tile (J >= I) or the conjugate transpose of tile (J, I)
    if (J != I) {
      const float sg = up ? 1.f : -1.f;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = up ? 4 * q + j : 4 * a + i;
          const int m = up ? 4 * a + i : 4 * q + j;
          const float2 v = t[4 * i + j];
          buf[c * 32 + (m ^ (2 * ((c >> 2) & 7)))] = make_float2(v.x, sg * v.y);
        }
    } else {
      // diagonal tile: lanes a <= q write their sub-block, lanes a < q also
      // its conjugate transpose below the diagonal
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = 4 * q + j, m = 4 * a + i;
          const float2 v = t[4 * i + j];
          if (dup) buf[c * 32 + (m ^ (2 * ((c >> 2) & 7)))] = v;
          if (a < q) buf[m * 32 + (c ^ (2 * ((m >> 2) & 7)))] = make_float2(v.x, -v.y);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const float2 av = buf[(2 * s + kk) * 32 + (n ^ (2 * (s >> 1)))];
      p1 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, x[s].x, p1, 0, 0, 0);
      p2 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, x[s].y, p2, 0, 0, 0);
      p3 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x + av.y, x[s].x + x[s].y, p3, 0, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  // two register sets in turn; the load after the last tile repeats it
  float2 tA[16], xA[16], tB[16], xB[16];
  load(0, tA, xA);
  int J = 0;
  for (; J + 1 < nt; J += 2) {
    step(J, J + 1, tA, xA, tB, xB);
    step(J + 1, J + 2 < nt ? J + 2 : J + 1, tB, xB, tA, xA);
  }
  if (J < nt) step(J, J, tA, xA, tB, xB);
  if (n >= nr) return;
  float2 *yb = yl + (loc_off[b] + 32 * I) * nr + n;
#pragma unroll
  for (int v = 0; v < 16; ++v)
    yb[(int64_t)(8 * (v >> 2) + 4 * kk + (v & 3)) * nr] =
        make_float2(p1[v] - p2[v], p3[v] - p1[v] - p2[v]);
}

// FP64 form on the matrix cores (v_mfma_f64_16x16x4f64: lane l supplies
// A[l%16][k] and B[k][l%16] for k = l/16 of each four-column step, and
// receives result row 4v + l/16, column l%16 in element v).  A wave forms
// Y_I as 2 x 2 blocks of 16 x 16, each complex product as four real ones
// (the outer-iteration operator keeps full FP64 accuracy).  The tile A_IJ is
// staged in LDS column by column (stride 33, double-buffered); X_J goes from
// global memory straight into the B operands; the next tile and X_J are
// loaded into a second register set while the current ones are multiplied
// (one wave per SIMD, eight independent accumulators).
__global__ __launch_bounds__(64) void k_rows_mfma64(const double2 *__restrict__ tiles,
                                                    const int2 *__restrict__ rows, int64_t nrows,
                                                    const int32_t *__restrict__ bn,
                                                    const int64_t *__restrict__ ent_off,
                                                    const int64_t *__restrict__ loc_off,
                                                    const double2 *__restrict__ xl,
                                                    double2 *__restrict__ yl, int nr) {
  __shared__ double2 As[2][32 * 33];
  const int64_t per = (nrows + 7) / 8;
  const int64_t w = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (w >= nrows) return;
  const int lane = threadIdx.x, a = lane >> 3, q = lane & 7;
  const int li = lane & 15, lk = lane >> 4;
  // columns past nr read column nr - 1; their results are not stored
  const int c0 = li < nr ? li : nr - 1, c1 = 16 + li < nr ? 16 + li : nr - 1;
  const int2 bi = rows[w];
  const int b = bi.x, I = bi.y;
  const int nt = (bn[b] + 31) >> 5;
  const int64_t e0 = ent_off[b];
  // a diagonal tile stores the sub-blocks a <= q only (slot diag_slot(a, q))
  const bool dup = a <= q;
  const int dsl = dup ? diag_slot(a, q) : 0;
  const double2 *xb = xl + loc_off[b] * nr;
  auto load = [&](int J, double2 *tt, double2 *xx) {
    // (wave-uniform branch, constant strides: immediate load offsets); lanes
    // below the diagonal of a diagonal tile read slot 0 (in range), their
    // values are not staged
    if (J != I) {
      const double2 *tp = tiles + e0 + (J > I ? tile_entry(I, J) : tile_entry(J, I)) + lane;
#pragma unroll
      for (int k = 0; k < 16; ++k) tt[k] = tp[k * 64];
    } else {
      const double2 *tp = tiles + e0 + tile_entry(I, I) + dsl;
#pragma unroll
      for (int k = 0; k < 16; ++k) tt[k] = tp[k * kDiagSlots];
    }
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const double2 *xr = xb + (int64_t)(32 * J + 4 * ks + lk) * nr;
      xx[2 * ks] = xr[c0];
      xx[2 * ks + 1] = xr[c1];
    }
  };
  v4d are[2][2], aim[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      are[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
      aim[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    }
  auto step = [&](int J, int Jn, const double2 *t, const double2 *x, double2 *tn, double2 *xn) {
    load(Jn, tn, xn);
    __builtin_amdgcn_sched_barrier(0);
    const bool up = J >= I;
    double2 *buf = As[J & 1];
    // the lane holds stored entries (4a + i, 4q + j) at 4i + j; A_IJ is the
    // stored tile (J >= I) or the conjugate transpose of tile (J, I)
    if (J != I) {
      const double sg = up ? 1.0 : -1.0;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = up ? 4 * q + j : 4 * a + i;
          const int m = up ? 4 * a + i : 4 * q + j;
          const double2 v = t[4 * i + j];
          buf[c * 33 + m] = make_double2(v.x, sg * v.y);
        }
    } else {
      // diagonal tile: lanes a <= q write their sub-block, lanes a < q also
      // its conjugate transpose below the diagonal
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = 4 * q + j, m = 4 * a + i;
          const double2 v = t[4 * i + j];
          if (dup) buf[c * 33 + m] = v;
          if (a < q) buf[m * 33 + c] = make_double2(v.x, -v.y);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int c = 4 * ks + lk;
      const double2 ar[2] = {buf[c * 33 + li], buf[c * 33 + 16 + li]};
      const double2 xv[2] = {x[2 * ks], x[2 * ks + 1]};
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          are[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i].x, xv[j].x, are[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          aim[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i].x, xv[j].y, aim[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          are[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ar[i].y, xv[j].y, are[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          aim[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i].y, xv[j].x, aim[i][j], 0, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  double2 tA[16], xA[16], tB[16], xB[16];
  load(0, tA, xA);
  int J = 0;
  for (; J + 1 < nt; J += 2) {
    step(J, J + 1, tA, xA, tB, xB);
    step(J + 1, J + 2 < nt ? J + 2 : J + 1, tB, xB, tA, xA);
  }
  if (J < nt) step(J, J, tA, xA, tB, xB);
  double2 *yb = yl + (loc_off[b] + 32 * I) * nr;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = 16 * j + li;
      if (col >= nr) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        yb[(int64_t)(16 * i + 4 * v + lk) * nr + col] = make_double2(are[i][j][v], aim[i][j][v]);
    }
}

// With FWD the result (d, k) also goes to the local rows of the next block
// set that hold d (its reduction lists), in that set's block buffers.
template <typename T, int MODE, bool FWD>
__global__ __launch_bounds__(256) void k_scatter_blk(int64_t nvec, int nr,
                                                     const int32_t *__restrict__ red_ptr,
                                                     const int32_t *__restrict__ red_ent,
                                                     const cplx_t<T> *__restrict__ yl,
                                                     const cplx_t<T> *__restrict__ r,
                                                     cplx_t<T> *__restrict__ y, T theta,
                                                     const int32_t *__restrict__ fwd_ptr,
                                                     const int32_t *__restrict__ fwd_ent,
                                                     cplx_t<T> *__restrict__ fwd_xl) {
  using C = cplx_t<T>;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nvec * nr) return;
  const int64_t d = e / nr;
  const int k = (int)(e % nr);
  C acc = czero<C>();
  for (int32_t j = red_ptr[d]; j < red_ptr[d + 1]; ++j)
    acc = cadd(acc, yl[(int64_t)red_ent[j] * nr + k]);
  C out;
  if (MODE == RED_SET) out = acc;
  else if (MODE == RED_RESID) out = csub(r[e], acc);
  else if (MODE == RED_AXPY) out = cadd(y[e], cscale(acc, theta));
  else out = cscale(acc, theta);
  y[e] = out;
  if (FWD)
    for (int32_t j = fwd_ptr[d]; j < fwd_ptr[d + 1]; ++j)
      fwd_xl[(int64_t)fwd_ent[j] * nr + k] = out;
}

// Local vectors column by column ([nr][nloc]).
__global__ __launch_bounds__(256) void k_gather_cols(int64_t nloc, int nr,
                                                     const int32_t *__restrict__ gidx,
                                                     const double2 *__restrict__ x,
                                                     double2 *__restrict__ xl) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nloc * nr) return;
  const int64_t i = e % nloc;
  const int k = (int)(e / nloc);
  const int32_t g = gidx[i];
  xl[e] = g >= 0 ? x[(int64_t)g * nr + k] : czero<double2>();
}

template <int MODE>
__global__ __launch_bounds__(256) void k_scatter_cols(int64_t nvec, int64_t nloc, int nr,
                                                      const int32_t *__restrict__ red_ptr,
                                                      const int32_t *__restrict__ red_ent,
                                                      const double2 *__restrict__ yl,
                                                      const double2 *__restrict__ r,
                                                      double2 *__restrict__ y, double theta) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nvec * nr) return;
  const int64_t d = e / nr;
  const int k = (int)(e % nr);
  double2 acc = czero<double2>();
  for (int32_t j = red_ptr[d]; j < red_ptr[d + 1]; ++j)
    acc = cadd(acc, yl[(int64_t)k * nloc + red_ent[j]]);
  if (MODE == RED_SET) y[e] = acc;
  else if (MODE == RED_RESID) y[e] = csub(r[e], acc);
  else if (MODE == RED_AXPY) y[e] = cadd(y[e], cscale(acc, theta));
  else y[e] = cscale(acc, theta);
}

// ---- transfers and condensation ----------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_csr_blk(int64_t nrows, int nr,
                                                 const int64_t *__restrict__ ptr,
                                                 const int32_t *__restrict__ col,
                                                 const T *__restrict__ val,
                                                 const cplx_t<T> *__restrict__ x,
                                                 cplx_t<T> *__restrict__ y, int add) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nrows * nr) return;
  const int64_t i = e / nr;
  const int k = (int)(e % nr);
  cplx_t<T> acc = czero<cplx_t<T>>();
  for (int64_t j = ptr[i]; j < ptr[i + 1]; ++j)
    acc = cadd(acc, cscale(x[(int64_t)col[j] * nr + k], val[j]));
  y[e] = add ? cadd(y[e], acc) : acc;
}

// c_b[sl, k] = sum_i WH_b[sl, i] rc[I_b(i), k] for the KC columns of blockIdx.y.
template <typename T>
__global__ __launch_bounds__(256) void k_condense_local_blk(const cplx_t<T> *__restrict__ WH,
                                                            int nI, int nBf,
                                                            const int32_t *__restrict__ blkI,
                                                            const cplx_t<T> *__restrict__ rc,
                                                            cplx_t<T> *__restrict__ c, int nr) {
  using C = cplx_t<T>;
  __shared__ C rI[kBMaxI][KC];
  const int b = blockIdx.x, k0 = blockIdx.y * KC, kc = min(KC, nr - k0);
  for (int e = threadIdx.x; e < nI * KC; e += 256) {
    const int i = e / KC, k = e % KC;
    rI[i][k] = k < kc ? rc[(int64_t)blkI[(int64_t)b * nI + i] * nr + k0 + k] : czero<C>();
  }
  __syncthreads();
  const C *W = WH + (int64_t)b * nBf * nI;
  for (int sl = threadIdx.x; sl < nBf; sl += 256) {
    C acc[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) acc[k] = czero<C>();
    for (int i = 0; i < nI; ++i) {
      const C wv = W[sl + (int64_t)i * nBf];
#pragma unroll
      for (int k = 0; k < KC; ++k) acc[k] = cfma(wv, rI[i][k], acc[k]);
    }
    for (int k = 0; k < kc; ++k) c[((int64_t)b * nBf + sl) * nr + k0 + k] = acc[k];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_condense_reduce_blk(int64_t nM, int nr,
                                                             const int64_t *__restrict__ macro_B,
                                                             const int32_t *__restrict__ red_ptr,
                                                             const int32_t *__restrict__ red_ent,
                                                             const cplx_t<T> *__restrict__ rc,
                                                             const cplx_t<T> *__restrict__ c,
                                                             cplx_t<T> *__restrict__ rB) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nM * nr) return;
  const int64_t m = e / nr;
  const int k = (int)(e % nr);
  cplx_t<T> acc = rc[macro_B[m] * nr + k];
  for (int32_t j = red_ptr[m]; j < red_ptr[m + 1]; ++j)
    acc = csub(acc, c[(int64_t)red_ent[j] * nr + k]);
  rB[e] = acc;
}

template <typename C> __device__ inline C wave_sum_c(C v) {
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o, 64);
    v.y += __shfl_xor(v.y, o, 64);
  }
  return v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_scatter_macro_blk(int64_t nM, int nr,
                                                           const int64_t *__restrict__ macro_B,
                                                           const cplx_t<T> *__restrict__ eB,
                                                           cplx_t<T> *__restrict__ ec) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < nM * nr) ec[macro_B[e / nr] * nr + e % nr] = eB[e];
}

// ec[I_b(i), k] = sum_j conj(Tinv[j, i]) rc[I_b(j), k] - sum_sl conj(WH[sl, i]) eB_b[sl, k],
// one wave per interior unknown i, KC columns per workgroup.
template <typename T>
__global__ __launch_bounds__(256) void k_expand_blk(const cplx_t<T> *__restrict__ WH,
                                                    const cplx_t<T> *__restrict__ Tinv, int nI,
                                                    int nBf, const int32_t *__restrict__ blkI,
                                                    const int32_t *__restrict__ blkBm,
                                                    const cplx_t<T> *__restrict__ rc,
                                                    const cplx_t<T> *__restrict__ eB,
                                                    cplx_t<T> *__restrict__ ec, int nr) {
  using C = cplx_t<T>;
  extern __shared__ __align__(16) char smem[];
  C(*eBs)[KC] = reinterpret_cast<C(*)[KC]>(smem);
  C(*rIs)[KC] = reinterpret_cast<C(*)[KC]>(smem + sizeof(C) * KC * nBf);
  const int b = blockIdx.x, k0 = blockIdx.y * KC, kc = min(KC, nr - k0);
  for (int e = threadIdx.x; e < nBf * KC; e += 256) {
    const int sl = e / KC, k = e % KC;
    const int m = blkBm[(int64_t)b * nBf + sl];
    eBs[sl][k] = (m >= 0 && k < kc) ? eB[(int64_t)m * nr + k0 + k] : czero<C>();
  }
  for (int e = threadIdx.x; e < nI * KC; e += 256) {
    const int i = e / KC, k = e % KC;
    rIs[i][k] = k < kc ? rc[(int64_t)blkI[(int64_t)b * nI + i] * nr + k0 + k] : czero<C>();
  }
  __syncthreads();
  const C *W = WH + (int64_t)b * nBf * nI;
  const C *Ti = Tinv + (int64_t)b * nI * nI;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = wave; i < nI; i += 4) {
    C acc[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) acc[k] = czero<C>();
    for (int j = lane; j < nI; j += 64) {
      const C tv = cconj(Ti[j + (int64_t)i * nI]);
#pragma unroll
      for (int k = 0; k < KC; ++k) acc[k] = cfma(tv, rIs[j][k], acc[k]);
    }
    for (int sl = lane; sl < nBf; sl += 64) {
      const C wv = cconj(W[sl + (int64_t)i * nBf]);
#pragma unroll
      for (int k = 0; k < KC; ++k) acc[k] = csub(acc[k], cmul(wv, eBs[sl][k]));
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) acc[k] = wave_sum_c(acc[k]);
    if (lane < kc) {
      C v = acc[0];
#pragma unroll
      for (int k = 1; k < KC; ++k)
        if (lane == k) v = acc[k];
      ec[(int64_t)blkI[(int64_t)b * nI + i] * nr + k0 + lane] = v;
    }
  }
}

__global__ __launch_bounds__(256) void k_interleave(int64_t n, int nr, const double2 *__restrict__ cols,
                                                    double2 *__restrict__ blk, int dir) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * nr) return;
  const int64_t d = e / nr;
  const int k = (int)(e % nr);
  if (dir == 0) blk[e] = cols[(int64_t)k * n + d];
  else blk[(int64_t)k * n + d] = cols[e];
}

// Column k of an interleaved block of width w: set from a plain vector (or
// zero), or copied out.
__global__ __launch_bounds__(256) void k_col(int64_t n, int w, int k, const double2 *__restrict__ src,
                                             double2 *__restrict__ dst, int dir) {
  const int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (d >= n) return;
  if (dir == 0) dst[d * w + k] = src ? src[d] : mk(0.0, 0.0);
  else dst[d] = src[d * w + k];
}

// dst (width w_new) <- src (width w_old): columns k < min(w_old, w_new) kept,
// new columns zero.
__global__ __launch_bounds__(256) void k_rewidth(int64_t n, int w_old, int w_new,
                                                 const double2 *__restrict__ src,
                                                 double2 *__restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * w_new) return;
  const int64_t d = e / w_new;
  const int k = (int)(e % w_new);
  dst[e] = k < w_old ? src[d * w_old + k] : mk(0.0, 0.0);
}

// A column joining a block solve: rz = 1 (so that its first flexible beta is
// finite; it multiplies a zero search direction), every other scalar 0.
__global__ void k_col_reset(double *sc, int k) {
  const int q = threadIdx.x;
  if (q < 8) sc[q * kMaxCols + k] = q == 0 ? 1.0 : 0.0;
}

// ---- per-column CG --------------------------------------------------------------------

// Per workgroup and column: sums of Re(a^H b) (and Re(a^H c) when c).
__global__ __launch_bounds__(256) void k_coldot(int64_t n, int nr, const double2 *__restrict__ a,
                                                const double2 *__restrict__ bv,
                                                const double2 *__restrict__ cv,
                                                double *__restrict__ partial) {
  __shared__ double sh[2][256];
  const int t = threadIdx.x, rpb = 256 / nr, k = t % nr;
  const bool on = t < rpb * nr;
  double s = 0.0, u = 0.0;
  if (on)
    for (int64_t i = (int64_t)blockIdx.x * rpb + t / nr; i < n; i += (int64_t)gridDim.x * rpb) {
      const double2 x = a[i * nr + k], y = bv[i * nr + k];
      s += x.x * y.x + x.y * y.y;
      if (cv) {
        const double2 z = cv[i * nr + k];
        u += x.x * z.x + x.y * z.y;
      }
    }
  sh[0][t] = s;
  sh[1][t] = u;
  __syncthreads();
  if (t < nr) {
    double ss = 0.0, uu = 0.0;
    for (int j = 0; j < rpb; ++j) {
      ss += sh[0][t + j * nr];
      uu += sh[1][t + j * nr];
    }
    partial[(int64_t)blockIdx.x * kMaxCols + t] = ss;
    partial[(int64_t)(kColDotBlocks + blockIdx.x) * kMaxCols + t] = uu;
  }
}

// Column reductions and the scalar updates of the CG step (mode: 0 store the
// dot in slot q, 1 alpha, 2 ||r||^2, 3 flexible beta).
__global__ __launch_bounds__(64) void k_colfinal(const double *__restrict__ partial, int nr,
                                                 double *__restrict__ sc,
                                                 const int *__restrict__ act, int mode, int q) {
  const int k = threadIdx.x;
  if (k >= nr) return;
  double s = 0.0, u = 0.0;
  for (int j = 0; j < kColDotBlocks; ++j) {
    s += partial[(int64_t)j * kMaxCols + k];
    u += partial[(int64_t)(kColDotBlocks + j) * kMaxCols + k];
  }
  double *S = sc;
  const bool on = act ? act[k] != 0 : true;
  if (mode == 0) {
    S[q * kMaxCols + k] = s;
  } else if (mode == 1) {
    S[1 * kMaxCols + k] = s;
    if (on && (!(s > 0.0) || !isfinite(s))) S[6 * kMaxCols + k] = 1.0;
    S[2 * kMaxCols + k] = on ? S[0 * kMaxCols + k] / s : 0.0;
  } else if (mode == 2) {
    S[4 * kMaxCols + k] = s;
  } else {
    // flexible (Polak-Ribiere) beta = Re(r^H (z - z_old)) / Re(r_old^H z_old)
    const double beta = on ? (s - u) / S[0 * kMaxCols + k] : 0.0;
    S[3 * kMaxCols + k] = beta;
    S[7 * kMaxCols + k] = u;
    S[0 * kMaxCols + k] = s;
    if (on && !isfinite(beta)) S[6 * kMaxCols + k] = 1.0;
  }
}

__global__ __launch_bounds__(256) void k_update_xr_blk(int64_t n, int nr, double2 *__restrict__ x,
                                                       double2 *__restrict__ r,
                                                       const double2 *__restrict__ p,
                                                       const double2 *__restrict__ qv,
                                                       double *__restrict__ partial,
                                                       const double *__restrict__ sc) {
  __shared__ double sh[256];
  const int t = threadIdx.x, rpb = 256 / nr, k = t % nr;
  const bool on = t < rpb * nr;
  const double al = on ? sc[2 * kMaxCols + k] : 0.0;
  double s = 0.0;
  if (on)
    for (int64_t i = (int64_t)blockIdx.x * rpb + t / nr; i < n; i += (int64_t)gridDim.x * rpb) {
      const int64_t e = i * nr + k;
      x[e] = mk(x[e].x + al * p[e].x, x[e].y + al * p[e].y);
      const double2 ri = mk(r[e].x - al * qv[e].x, r[e].y - al * qv[e].y);
      r[e] = ri;
      s += ri.x * ri.x + ri.y * ri.y;
    }
  sh[t] = s;
  __syncthreads();
  if (t < nr) {
    double ss = 0.0;
    for (int j = 0; j < rpb; ++j) ss += sh[t + j * nr];
    partial[(int64_t)blockIdx.x * kMaxCols + t] = ss;
    partial[(int64_t)(kColDotBlocks + blockIdx.x) * kMaxCols + t] = 0.0;
  }
}

__global__ __launch_bounds__(256) void k_update_p_blk(int64_t n, int nr, double2 *__restrict__ p,
                                                      const double2 *__restrict__ z,
                                                      const double *__restrict__ sc) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * nr) return;
  const double be = sc[3 * kMaxCols + (int)(e % nr)];
  p[e] = mk(z[e].x + be * p[e].x, z[e].y + be * p[e].y);
}

}  // namespace

void HermBlockBufs::ensure(const HermSet &H, int nr, bool fp64, bool fp32, Budget *bud,
                           hipStream_t s) {
  if (nr <= cap) return;
  if (fp64) {
    xl64.alloc(H.nloc * nr, bud);
    yl64.alloc(H.nloc * nr, bud);
    launch_zero(H.nloc * nr, xl64.p, s);
  }
  if (fp32) {
    xl32.alloc(H.nloc * nr, bud);
    yl32.alloc(H.nloc * nr, bud);
    launch_zero(H.nloc * nr, xl32.p, s);
  }
  cap = nr;
}

template <typename T, int MODE>
void launch_scatter_blk(const HermSet &H, int nr, const cplx_t<T> *yl, const cplx_t<T> *R,
                        cplx_t<T> *Y, T theta, const HermSet *fwd, cplx_t<T> *fxl,
                        hipStream_t s) {
  const dim3 g(cdiv(H.nvec * nr, 256));
  if (fwd)
    hipLaunchKernelGGL((k_scatter_blk<T, MODE, true>), g, dim3(256), 0, s, H.nvec, nr,
                       H.red_ptr.p, H.red_ent.p, yl, R, Y, theta, fwd->red_ptr.p,
                       fwd->red_ent.p, fxl);
  else
    hipLaunchKernelGGL((k_scatter_blk<T, MODE, false>), g, dim3(256), 0, s, H.nvec, nr,
                       H.red_ptr.p, H.red_ent.p, yl, R, Y, theta, nullptr, nullptr, nullptr);
}

template <typename T>
void herm_apply_blk(HermSet &H, HermBlockBufs &W, const cplx_t<T> *X, cplx_t<T> *Y,
                    const cplx_t<T> *R, int mode, T theta, int nr, hipStream_t s, bool gathered,
                    HermSet *fwd, HermBlockBufs *fwd_bufs) {
  if (nr < 1 || nr > kMaxCols || nr > W.cap) throw DpgError(-1, "block apply: bad column count");
  if (nr == 1) {   // one column: the HBM-bound single-vector apply (same layout)
    herm_apply<T>(H, X, Y, R, mode, theta, s, gathered, fwd);
    return;
  }
  cplx_t<T> *fxl = nullptr;
  if (fwd) {
    if (!fwd_bufs || fwd->nvec != H.nvec || nr > fwd_bufs->cap)
      throw DpgError(-1, "forwarded block set does not match this one");
    if constexpr (sizeof(T) == 8) fxl = fwd_bufs->xl64.p;
    else fxl = fwd_bufs->xl32.p;
    if (!fxl) throw DpgError(-1, "forwarded block set has no local vectors of this precision");
  }
  const cplx_t<T> *tiles;
  cplx_t<T> *xl, *yl;
  if constexpr (sizeof(T) == 8) {
    tiles = H.t64.p;
    xl = W.xl64.p;
    yl = W.yl64.p;
  } else {
    tiles = H.t32.p;
    xl = W.xl32.p;
    yl = W.yl32.p;
  }
  if (!tiles || !xl) throw DpgError(-6, "block set has no tiles of this precision");
  if (!gathered) {
    ProfScope ps(H.prof, DPG_K_REDUCE, 0.0, s);
    hipLaunchKernelGGL((k_gather_blk<T>), dim3(cdiv(H.nloc * nr, 256)), dim3(256), 0, s, H.nloc,
                       nr, H.gidx.p, X, xl);
    LAUNCH_OK();
  }
  {
    ProfScope ps(H.prof, sizeof(T) == 8 ? DPG_K_APPLYB64 : DPG_K_APPLYB32,
                 8.0 * (double)H.full * nr, s);
    if constexpr (sizeof(T) == 4) {
      const int64_t per = (H.nrows + 7) / 8;
      if (8 * per > INT32_MAX) throw DpgError(-1, "block apply: too many tile rows");
      hipLaunchKernelGGL(k_rows_mfma, dim3((unsigned)(8 * per)), dim3(64), 0, s, tiles, H.rows.p,
                         H.nrows, H.bn.p, H.ent_off.p, H.loc_off.p, xl, yl, nr);
    } else {
      const int64_t per = (H.nrows + 7) / 8;
      if (8 * per > INT32_MAX) throw DpgError(-1, "block apply: too many tile rows");
      hipLaunchKernelGGL(k_rows_mfma64, dim3((unsigned)(8 * per)), dim3(64), 0, s, tiles,
                         H.rows.p, H.nrows, H.bn.p, H.ent_off.p, H.loc_off.p, xl, yl, nr);
    }
    LAUNCH_OK();
  }
  ProfScope ps(H.prof, DPG_K_REDUCE, 0.0, s);
  switch (mode) {
    case RED_SET: launch_scatter_blk<T, RED_SET>(H, nr, yl, R, Y, theta, fwd, fxl, s); break;
    case RED_RESID: launch_scatter_blk<T, RED_RESID>(H, nr, yl, R, Y, theta, fwd, fxl, s); break;
    case RED_AXPY: launch_scatter_blk<T, RED_AXPY>(H, nr, yl, R, Y, theta, fwd, fxl, s); break;
    default: launch_scatter_blk<T, RED_SET_SCALED>(H, nr, yl, R, Y, theta, fwd, fxl, s);
  }
  LAUNCH_OK();
}

void herm_gather_cols(const HermSet &H, const double2 *X, double2 *xl, int nr, hipStream_t s) {
  if (nr < 1 || nr > kMaxCols) throw DpgError(-1, "column gather: bad column count");
  ProfScope ps(H.prof, DPG_K_REDUCE, 0.0, s);
  hipLaunchKernelGGL(k_gather_cols, dim3(cdiv(H.nloc * nr, 256)), dim3(256), 0, s, H.nloc, nr,
                     H.gidx.p, X, xl);
  LAUNCH_OK();
}

void herm_scatter_cols(const HermSet &H, const double2 *yl, double2 *Y, const double2 *R,
                       int mode, double theta, int nr, hipStream_t s) {
  if (nr < 1 || nr > kMaxCols) throw DpgError(-1, "column scatter: bad column count");
  ProfScope ps(H.prof, DPG_K_REDUCE, 0.0, s);
  const dim3 g(cdiv(H.nvec * nr, 256));
  switch (mode) {
    case RED_SET:
      hipLaunchKernelGGL((k_scatter_cols<RED_SET>), g, dim3(256), 0, s, H.nvec, H.nloc, nr, H.red_ptr.p, H.red_ent.p, yl, R, Y, theta);
      break;
    case RED_RESID:
      hipLaunchKernelGGL((k_scatter_cols<RED_RESID>), g, dim3(256), 0, s, H.nvec, H.nloc, nr, H.red_ptr.p, H.red_ent.p, yl, R, Y, theta);
      break;
    case RED_AXPY:
      hipLaunchKernelGGL((k_scatter_cols<RED_AXPY>), g, dim3(256), 0, s, H.nvec, H.nloc, nr, H.red_ptr.p, H.red_ent.p, yl, R, Y, theta);
      break;
    default:
      hipLaunchKernelGGL((k_scatter_cols<RED_SET_SCALED>), g, dim3(256), 0, s, H.nvec, H.nloc, nr, H.red_ptr.p, H.red_ent.p, yl, R, Y, theta);
  }
  LAUNCH_OK();
}

template <typename T>
void launch_csr_blk(int64_t nrows, const int64_t *ptr, const int32_t *col, const T *val,
                    const cplx_t<T> *x, cplx_t<T> *y, int add, int nr, hipStream_t s) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL((k_csr_blk<T>), dim3(cdiv(nrows * nr, 256)), dim3(256), 0, s, nrows, nr, ptr,
                     col, val, x, y, add);
  LAUNCH_OK();
}

template <typename T>
void launch_condense_blk(const cplx_t<T> *WH, int nI, int nBf, const int32_t *blkI, int nblk,
                         int64_t nM, const int64_t *macro_B, const int32_t *red_ptr,
                         const int32_t *red_ent, const cplx_t<T> *rc, cplx_t<T> *c,
                         cplx_t<T> *rB, int nr, hipStream_t s) {
  if (nI > kBMaxI) throw DpgError(-1, "macro block too large");
  hipLaunchKernelGGL((k_condense_local_blk<T>), dim3(nblk, cdiv(nr, KC)), dim3(256), 0, s, WH, nI,
                     nBf, blkI, rc, c, nr);
  LAUNCH_OK();
  hipLaunchKernelGGL((k_condense_reduce_blk<T>), dim3(cdiv(nM * nr, 256)), dim3(256), 0, s, nM, nr,
                     macro_B, red_ptr, red_ent, rc, c, rB);
  LAUNCH_OK();
}

template <typename T>
void launch_expand_blk(const cplx_t<T> *WH, const cplx_t<T> *Tinv, int nI, int nBf,
                       const int32_t *blkI, const int32_t *blkBm, int nblk, const cplx_t<T> *rc,
                       const cplx_t<T> *eB, int64_t nM, const int64_t *macro_B, cplx_t<T> *ec,
                       int nr, hipStream_t s) {
  // the boundary and interior values of KC columns of one macro block stay in
  // LDS; beyond 64 KB (order 4 in FP64) the kernel asks for more, up to the
  // 160 KB a gfx950 workgroup can hold
  const size_t lds = sizeof(cplx_t<T>) * KC * ((size_t)nBf + nI);
  if (lds > 160 * 1024) throw DpgError(-1, "macro block too large for the block expansion");
  if (lds > 64 * 1024)
    HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_expand_blk<T>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((k_scatter_macro_blk<T>), dim3(cdiv(nM * nr, 256)), dim3(256), 0, s, nM, nr,
                     macro_B, eB, ec);
  LAUNCH_OK();
  hipLaunchKernelGGL((k_expand_blk<T>), dim3(nblk, cdiv(nr, KC)), dim3(256), lds, s, WH, Tinv, nI,
                     nBf, blkI, blkBm, rc, eB, ec, nr);
  LAUNCH_OK();
}

void launch_interleave(int64_t n, int nr, const double2 *cols, double2 *blk, hipStream_t s) {
  hipLaunchKernelGGL(k_interleave, dim3(cdiv(n * nr, 256)), dim3(256), 0, s, n, nr, cols, blk, 0);
  LAUNCH_OK();
}
void launch_deinterleave(int64_t n, int nr, const double2 *blk, double2 *cols, hipStream_t s) {
  hipLaunchKernelGGL(k_interleave, dim3(cdiv(n * nr, 256)), dim3(256), 0, s, n, nr, blk, cols, 1);
  LAUNCH_OK();
}

void launch_set_col(int64_t n, int w, int k, const double2 *src, double2 *blk, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_col, dim3(cdiv(n, 256)), dim3(256), 0, s, n, w, k, src, blk, 0);
  LAUNCH_OK();
}
void launch_get_col(int64_t n, int w, int k, const double2 *blk, double2 *dst, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_col, dim3(cdiv(n, 256)), dim3(256), 0, s, n, w, k, blk, dst, 1);
  LAUNCH_OK();
}
void launch_rewidth(int64_t n, int w_old, int w_new, const double2 *src, double2 *dst,
                    hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_rewidth, dim3(cdiv(n * w_new, 256)), dim3(256), 0, s, n, w_old, w_new,
                     src, dst);
  LAUNCH_OK();
}
void cgb_reset_col(double *sc, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_col_reset, dim3(1), dim3(64), 0, s, sc, k);
  LAUNCH_OK();
}

void cgb_dot(int64_t n, int nr, const double2 *a, const double2 *b, double *partial, double *sc,
             int q, hipStream_t s) {
  hipLaunchKernelGGL(k_coldot, dim3(kColDotBlocks), dim3(256), 0, s, n, nr, a, b,
                     (const double2 *)nullptr, partial);
  hipLaunchKernelGGL(k_colfinal, dim3(1), dim3(64), 0, s, partial, nr, sc, (const int *)nullptr, 0,
                     q);
  LAUNCH_OK();
}

void cgb_alpha(int64_t n, int nr, const double2 *p, const double2 *qv, double *partial,
               double *sc, const int *act, hipStream_t s) {
  hipLaunchKernelGGL(k_coldot, dim3(kColDotBlocks), dim3(256), 0, s, n, nr, p, qv,
                     (const double2 *)nullptr, partial);
  hipLaunchKernelGGL(k_colfinal, dim3(1), dim3(64), 0, s, partial, nr, sc, act, 1, 0);
  LAUNCH_OK();
}

void cgb_update_xr(int64_t n, int nr, double2 *x, double2 *r, const double2 *p, const double2 *qv,
                   double *partial, double *sc, hipStream_t s) {
  hipLaunchKernelGGL(k_update_xr_blk, dim3(kColDotBlocks), dim3(256), 0, s, n, nr, x, r, p, qv,
                     partial, sc);
  hipLaunchKernelGGL(k_colfinal, dim3(1), dim3(64), 0, s, partial, nr, sc, (const int *)nullptr, 2,
                     0);
  LAUNCH_OK();
}

void cgb_beta(int64_t n, int nr, const double2 *r, const double2 *z, const double2 *zold,
              double *partial, double *sc, const int *act, hipStream_t s) {
  hipLaunchKernelGGL(k_coldot, dim3(kColDotBlocks), dim3(256), 0, s, n, nr, r, z, zold, partial);
  hipLaunchKernelGGL(k_colfinal, dim3(1), dim3(64), 0, s, partial, nr, sc, act, 3, 0);
  LAUNCH_OK();
}

void cgb_update_p(int64_t n, int nr, double2 *p, const double2 *z, const double *sc,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_update_p_blk, dim3(cdiv(n * nr, 256)), dim3(256), 0, s, n, nr, p, z, sc);
  LAUNCH_OK();
}

template void herm_apply_blk<double>(HermSet &, HermBlockBufs &, const double2 *, double2 *,
                                     const double2 *, int, double, int, hipStream_t, bool,
                                     HermSet *, HermBlockBufs *);
template void herm_apply_blk<float>(HermSet &, HermBlockBufs &, const float2 *, float2 *,
                                    const float2 *, int, float, int, hipStream_t, bool,
                                    HermSet *, HermBlockBufs *);
template void launch_csr_blk<double>(int64_t, const int64_t *, const int32_t *, const double *,
                                     const double2 *, double2 *, int, int, hipStream_t);
template void launch_csr_blk<float>(int64_t, const int64_t *, const int32_t *, const float *,
                                    const float2 *, float2 *, int, int, hipStream_t);
template void launch_condense_blk<double>(const double2 *, int, int, const int32_t *, int, int64_t,
                                          const int64_t *, const int32_t *, const int32_t *,
                                          const double2 *, double2 *, double2 *, int, hipStream_t);
template void launch_condense_blk<float>(const float2 *, int, int, const int32_t *, int, int64_t,
                                         const int64_t *, const int32_t *, const int32_t *,
                                         const float2 *, float2 *, float2 *, int, hipStream_t);
template void launch_expand_blk<double>(const double2 *, const double2 *, int, int,
                                        const int32_t *, const int32_t *, int, const double2 *,
                                        const double2 *, int64_t, const int64_t *, double2 *, int,
                                        hipStream_t);
template void launch_expand_blk<float>(const float2 *, const float2 *, int, int, const int32_t *,
                                       const int32_t *, int, const float2 *, const float2 *,
                                       int64_t, const int64_t *, float2 *, int, hipStream_t);

}  // namespace dpg
