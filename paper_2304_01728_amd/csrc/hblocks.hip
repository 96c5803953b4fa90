// Hermitian block sets: packing and apply kernels (see hblocks.hpp).
#include <algorithm>
#include <numeric>

#include "hblocks.hpp"
#include "kernels.hpp"

namespace dpg {
namespace {

template <typename C> __device__ __forceinline__ C czero() {
  C r;
  r.x = 0;
  r.y = 0;
  return r;
}

template <typename C> __device__ inline C shfl_xor_c(C v, int m) {
  C r;
  r.x = __shfl_xor(v.x, m, 64);
  r.y = __shfl_xor(v.y, m, 64);
  return r;
}

template <typename C> __device__ inline C sel4(C v0, C v1, C v2, C v3, int i) {
  C r;
  r.x = i == 0 ? v0.x : i == 1 ? v1.x : i == 2 ? v2.x : v3.x;
  r.y = i == 0 ? v0.y : i == 1 ? v1.y : i == 2 ? v2.y : v3.y;
  return r;
}

// Cross-lane moves inside rows of 16 lanes (DPP): quad_perm [1,0,3,2],
// quad_perm [2,3,0,1] and the mirror inside each group of 8 lanes.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141;

template <int CTRL> __device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                               CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double dpp(double v) {
  int2 i = __builtin_bit_cast(int2, v);
  i.x = __builtin_amdgcn_update_dpp(0, i.x, CTRL, 0xF, 0xF, false);
  i.y = __builtin_amdgcn_update_dpp(0, i.y, CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, i);
}
template <int CTRL, typename C> __device__ __forceinline__ C dpp_c(C v) {
  C r;
  r.x = dpp<CTRL>(v.x);
  r.y = dpp<CTRL>(v.y);
  return r;
}
template <typename C> __device__ __forceinline__ C csel(bool c, C a, C b) {
  C r;
  r.x = c ? a.x : b.x;
  r.y = c ? a.y : b.y;
  return r;
}

// Reduce-scatter of four row values over the 8 lanes cb = 0..7 of a group:
// lanes cb and cb^1 return the full sum of row cb/2.  Three exchange rounds
// (partners 7-cb, cb^2, cb^1), each moving one value per lane after the
// first, which moves two.
template <typename C> __device__ __forceinline__ C rowsum_scatter(const C rs[4], int cb) {
  const bool lo = cb < 4;
  C k0 = csel(lo, rs[0], rs[2]), k1 = csel(lo, rs[1], rs[3]);
  const C s0 = csel(lo, rs[2], rs[0]), s1 = csel(lo, rs[3], rs[1]);
  k0 = cadd(k0, dpp_c<kDppHalfMirror>(s0));
  k1 = cadd(k1, dpp_c<kDppHalfMirror>(s1));
  const bool b1 = cb & 2;
  C k = csel(b1, k1, k0);
  k = cadd(k, dpp_c<kDppXor2>(csel(b1, k0, k1)));
  return cadd(k, dpp_c<kDppXor1>(k));
}

// Tile entries are read once per application: non-temporal loads keep them
// from displacing the x entries and partials in the caches.
__device__ __forceinline__ double2 ld_nt(const double2 *p) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 ld_nt(const float2 *p) {
  typedef float v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
  return make_float2(v.x, v.y);
}

template <typename C> __device__ __forceinline__ void load_tile(const C *__restrict__ tp, C t[16]) {
#pragma unroll
  for (int k = 0; k < 16; ++k) t[k] = ld_nt(tp + k * 64);
}

// A tile by its lane's first entry and the stride between its 16 entries: 64
// for a full tile, 36 for a diagonal one, whose lanes below the diagonal
// read slot 0 (in range) and are zeroed by mask_lower once the data is
// needed.  One code path for both kinds: behind a branch, the compiler made
// the loads of either kind wait for those of the other.
template <typename C>
__device__ __forceinline__ void load_strided(const C *__restrict__ tp, int st, C t[16]) {
#pragma unroll
  for (int k = 0; k < 16; ++k) t[k] = ld_nt(tp + k * st);
}
template <typename C> __device__ __forceinline__ void mask_lower(bool keep, C t[16]) {
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    t[k].x = keep ? t[k].x : 0;
    t[k].y = keep ? t[k].y : 0;
  }
}

// Row sums of one tile into its partial slot; column sums accumulated where
// off holds: every sub-block of an off-diagonal tile, the sub-blocks strictly
// above the diagonal of a diagonal tile (their conjugate transposes are the
// sub-blocks below it, which are not stored).
template <typename C>
__device__ __forceinline__ void do_tile(const C t[16], const C xJ[4], const C *xr, bool off,
                                        int ra, int cb, C cacc[4], C *__restrict__ slot) {
  C rs[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    C a;
    a.x = 0;
    a.y = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) a = cfma(t[4 * i + j], xJ[j], a);
    rs[i] = a;
  }
  if (off) {
    C xI[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) xI[i] = xr[4 * ra + i];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) cacc[j] = cfmaconj(t[4 * i + j], xI[i], cacc[j]);
  }
  const C v = rowsum_scatter(rs, cb);
  if (!(cb & 1)) slot[4 * ra + (cb >> 1)] = v;
}

// Tile columns are cut into segments of at most kSeg tiles, one wave each.
// Two tiles, both loaded before any arithmetic, stream fastest: longer
// segments leave only one tile in flight while the other is being used.
constexpr int kSeg = 2;

// Column-sum slots of a block: column J has ceil((J+1)/kSeg) segment slots;
// colbase(J) = 32 sum_{j=1..J} ceil(j/kSeg).
__host__ __device__ __forceinline__ int64_t colbase(int J) {
  const int64_t q = J / kSeg, r = J % kSeg;
  return 32 * (kSeg * q * (q + 1) / 2 + r * (q + 1));
}

// offset of the row-sum slot (I, J), I <= J, inside the row partials of a block
__host__ __device__ __forceinline__ int64_t row_slot(int nt, int I, int J) {
  return ((int64_t)I * nt - (int64_t)I * (I - 1) / 2 + (J - I)) * 32;
}

// The FP32 apply (k_strips) takes tile columns in pairs, "strips" (J0 = 2 s,
// J1 = 2 s + 1; the last strip of a block with an odd tile count has one
// column), whose tile rows 0..J1 are cut into chunks of at most kChunk rows,
// one wave each.  Per row I the wave loads tiles (I, J0) and (I, J1) and
// writes their row sums as one 32-vector (slot (I, s)); the column sums of
// both columns accumulate in registers over the chunk (one slot per column
// and chunk).  Partials per 1024-entry tile: 16 + 8 entries instead of the
// 32 + 16 of the segments above (and the x entries of a row once per two
// tiles), which pays in FP32, where they weigh twice as much against the
// tiles; FP64 streams its 16 KB tiles faster as segments.
constexpr int kChunk = 4;

// Row-sum slots of a block with nt tile columns (ns = ceil(nt / 2) strips):
// row I is covered by the strips s >= I / 2, its slots are contiguous, and
// rows come in order: slot(I, s) = I ns - floor((I - 1)^2 / 4) + s - I / 2.
__host__ __device__ __forceinline__ int64_t strip_row_slot(int ns, int I, int s) {
  return (int64_t)I * ns - (int64_t)(I - 1) * (I - 1) / 4 + s - I / 2;
}
__host__ __forceinline__ int64_t strip_row_slots(int nt) {
  return (int64_t)nt * ((nt + 1) / 2) - (int64_t)(nt - 1) * (nt - 1) / 4;
}
__host__ __forceinline__ int strip_rows(int nt, int s) { return std::min(2 * s + 2, nt); }
__host__ __forceinline__ int strip_chunks(int nt, int s) {
  return (strip_rows(nt, s) + kChunk - 1) / kChunk;
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather_x(int64_t nloc, const int32_t *__restrict__ gidx,
                                                  const cplx_t<T> *__restrict__ x,
                                                  cplx_t<T> *__restrict__ xl) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nloc) return;
  const int32_t g = gidx[i];
  cplx_t<T> v;
  v.x = 0;
  v.y = 0;
  if (g >= 0) v = x[g];
  xl[i] = v;
}

// One wave per (block, tile column J, pair of tile rows I0, I0 + 1 <= J).  The
// unit's descriptor (two int4, see HermSet::build) holds every address the
// wave needs and is read with scalar loads (the wave index is made uniform),
// so the tile loads follow it at once and the x loads come after them (with
// x first, the compiler waited for x, and a vector-loaded descriptor, before
// issuing the tiles).  The x entries of the two tile rows are staged in LDS
// (wave-private), which keeps registers for the tiles and the vector memory
// queue for tile data.
template <typename T>
__global__ __launch_bounds__(256) void k_units(const cplx_t<T> *__restrict__ tiles,
                                               const int4 *__restrict__ units, int64_t nunits,
                                               const cplx_t<T> *__restrict__ xloc,
                                               cplx_t<T> *__restrict__ part) {
  static_assert(kSeg == 2, "k_units handles segments of two tile rows");
  using C = cplx_t<T>;
  __shared__ C xs[4][kSeg * 32];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // workgroup g runs on XCD g % 8: each XCD takes a contiguous range of
  // units (the grid is a multiple of 8; workgroups past the end exit)
  const int64_t per = gridDim.x / 8, wg = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  const int64_t wv = wg * 4 + wave;
  if (wv >= nunits) return;
  const int lane = threadIdx.x & 63, ra = lane >> 3, cb = lane & 7;
  const int4 d0 = units[2 * wv], d1 = units[2 * wv + 1];
  const int64_t ent = (int64_t)(uint32_t)d0.x | ((int64_t)d0.y << 32);
  // a one-tile segment is a diagonal tile; of two, the first is off-diagonal
  const bool two = d1.w & 1, off0 = d1.w & 2, off1 = d1.w & 4;
  const bool upper = ra <= cb, strict = ra < cb;
  const C *tp = tiles + ent;
  C t0[16], t1[16], xJ[4], cacc[4];
  // tiles first, then x (lanes past the unit's rows read its last row); all
  // of them arrive before any arithmetic
  const int ds = upper ? diag_slot(ra, cb) : 0;
  load_strided(tp + (off0 ? lane : ds), off0 ? 64 : kDiagSlots, t0);
  if (two) load_strided(tp + kTileFull + (off1 ? lane : ds), off1 ? 64 : kDiagSlots, t1);
  const int nx = 32 * (1 + two);
  const C v = xloc[d0.z + min(lane, nx - 1)];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    xJ[j] = xloc[d0.w + 4 * cb + j];
    cacc[j].x = 0;
    cacc[j].y = 0;
  }
  C *xw = xs[wave];
  C w;
  w.x = lane < nx ? v.x : 0;
  w.y = lane < nx ? v.y : 0;
  xw[lane] = w;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (!off0) mask_lower(upper, t0);
  if (two && !off1) mask_lower(upper, t1);
  do_tile(t0, xJ, xw, off0 || strict, ra, cb, cacc, part + d1.x);
  if (two) do_tile(t1, xJ, xw + 32, off1 || strict, ra, cb, cacc, part + d1.x + d1.y);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    cacc[j] = cadd(cacc[j], shfl_xor_c(cacc[j], 8));
    cacc[j] = cadd(cacc[j], shfl_xor_c(cacc[j], 16));
    cacc[j] = cadd(cacc[j], shfl_xor_c(cacc[j], 32));
  }
  if (ra < 4) part[d1.z + 4 * cb + ra] = sel4(cacc[0], cacc[1], cacc[2], cacc[3], ra);
}

// One wave per (block, strip s, chunk of tile rows [Ia, Ib)).  The unit's
// descriptor (two int4, see HermSet::build) is read with scalar loads (the
// wave index is made uniform).  Each row step issues the loads of both tiles,
// then the x entries of the row, before any arithmetic.  A diagonal tile and
// an absent one (row J1 of column J0, the second column of a one-column
// strip) are read through the diagonal tile's 36-slot layout at an address
// inside it, and masked: one load path for every kind (behind branches the
// compiler made the loads of one kind wait for the other's).
template <typename T>
__global__ __launch_bounds__(256) void k_strips(const cplx_t<T> *__restrict__ tiles,
                                               const int4 *__restrict__ units, int64_t nunits,
                                               const cplx_t<T> *__restrict__ xloc,
                                               cplx_t<T> *__restrict__ part) {
  using C = cplx_t<T>;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // workgroup g runs on XCD g % 8: each XCD takes a contiguous range of
  // units (the grid is a multiple of 8; workgroups past the end exit)
  const int64_t per = gridDim.x / 8, wg = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  const int64_t wv = wg * 4 + wave;
  if (wv >= nunits) return;
  const int lane = threadIdx.x & 63, ra = lane >> 3, cb = lane & 7;
  const int4 d0 = units[2 * wv], d1 = units[2 * wv + 1];
  const int64_t ent = (int64_t)(uint32_t)d0.x | ((int64_t)d0.y << 32);
  const int J0 = d1.x & 0xffff, nt = d1.x >> 16, J1 = J0 + 1;
  const int Ia = d1.y & 0xffff, Ib = d1.y >> 16;
  const bool two = J1 < nt;
  const int ns = (nt + 1) >> 1, s = J0 >> 1;
  const bool upper = ra <= cb, strict = ra < cb;
  const int ds = upper ? diag_slot(ra, cb) : 0;
  const C *t0 = tiles + ent;                                   // tile (0, J0)
  const C *t1 = two ? t0 + (int64_t)kTileFull * J0 + kTileDiag : t0;   // tile (0, J1)
  const C *xb = xloc + d0.z;
  C *rp = part + d0.w;
  C xJ0[4], xJ1[4], c0[4], c1[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    xJ0[j] = xb[32 * J0 + 4 * cb + j];
    xJ1[j] = xb[32 * (two ? J1 : J0) + 4 * cb + j];
    c0[j].x = 0;
    c0[j].y = 0;
    c1[j].x = 0;
    c1[j].y = 0;
  }
#pragma unroll 1
  for (int I = Ia; I < Ib; ++I) {
    // (I, J0): full for I < J0, diagonal for I == J0, absent for I == J1;
    // (I, J1): full for I < J1, diagonal for I == J1, absent without J1
    const bool fa = I < J0, fb = two && I < J1;
    const bool ka = fa || (I == J0 && upper), kb = fb || (two && I == J1 && upper);
    const C *pa = fa ? t0 + (int64_t)kTileFull * I + lane : t0 + (int64_t)kTileFull * J0 + ds;
    const C *pb = fb ? t1 + (int64_t)kTileFull * I + lane
                     : two ? t1 + (int64_t)kTileFull * J1 + ds : t0 + (int64_t)kTileFull * J0 + ds;
    C ta[16], tb[16], xI[4];
    load_strided(pa, fa ? 64 : kDiagSlots, ta);
    load_strided(pb, fb ? 64 : kDiagSlots, tb);
#pragma unroll
    for (int i = 0; i < 4; ++i) xI[i] = xb[32 * I + 4 * ra + i];
    mask_lower(ka, ta);
    mask_lower(kb, tb);
    C rs[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      C a;
      a.x = 0;
      a.y = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) a = cfma(ta[4 * i + j], xJ0[j], a);
#pragma unroll
      for (int j = 0; j < 4; ++j) a = cfma(tb[4 * i + j], xJ1[j], a);
      rs[i] = a;
    }
    // column sums: every sub-block of a full tile, the sub-blocks strictly
    // above the diagonal of a diagonal one (masked entries are zero)
    C xa[4], xbb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      xa[i] = csel(fa || strict, xI[i], czero<C>());
      xbb[i] = csel(fb || strict, xI[i], czero<C>());
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        c0[j] = cfmaconj(ta[4 * i + j], xa[i], c0[j]);
        c1[j] = cfmaconj(tb[4 * i + j], xbb[i], c1[j]);
      }
    const C v = rowsum_scatter(rs, cb);
    if (!(cb & 1)) rp[32 * strip_row_slot(ns, I, s) + 4 * ra + (cb >> 1)] = v;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    c0[j] = cadd(c0[j], shfl_xor_c(c0[j], 8));
    c0[j] = cadd(c0[j], shfl_xor_c(c0[j], 16));
    c0[j] = cadd(c0[j], shfl_xor_c(c0[j], 32));
    c1[j] = cadd(c1[j], shfl_xor_c(c1[j], 8));
    c1[j] = cadd(c1[j], shfl_xor_c(c1[j], 16));
    c1[j] = cadd(c1[j], shfl_xor_c(c1[j], 32));
  }
  if (ra < 4) {
    part[d1.z + 4 * cb + ra] = sel4(c0[0], c0[1], c0[2], c0[3], ra);
    if (two) part[d1.w + 4 * cb + ra] = sel4(c1[0], c1[1], c1[2], c1[3], ra);
  }
}

// Half a wave per (block, tile row I): y_loc rows of I = column sums of the
// segments of tile column I + row sums of tiles (I, J >= I).  The row's
// descriptor (rowd, see HermSet::build) gives both partial bases and counts
// with one load.  The slots are independent loads: eight are in flight per
// lane (a row of a 24-tile block sums 25 slots), summed in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void k_rows(const int4 *__restrict__ rowd, int64_t nrows,
                                              const cplx_t<T> *__restrict__ part,
                                              cplx_t<T> *__restrict__ yl) {
  using C = cplx_t<T>;
  constexpr int U = 8;
  const int64_t hw = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 5;
  if (hw >= nrows) return;
  const int r = threadIdx.x & 31;
  const int4 d = rowd[hw];
  const C *cp = part + d.x + r;
  const C *rp = part + d.y + r;
  const int nseg = d.z & 0xffff, tot = nseg + (d.z >> 16);
  C acc[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    acc[u].x = 0;
    acc[u].y = 0;
  }
  for (int q0 = 0; q0 < tot; q0 += U) {
    C v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0 + u;
      v[u].x = 0;
      v[u].y = 0;
      if (q < tot) v[u] = q < nseg ? cp[q * 32] : rp[(q - nseg) * 32];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = cadd(acc[u], v[u]);
  }
#pragma unroll
  for (int w = U / 2; w >= 1; w /= 2)
#pragma unroll
    for (int u = 0; u < w; ++u) acc[u] = cadd(acc[u], acc[u + w]);
  yl[d.w + r] = acc[0];
}

// With FWD the result of entry d is also written to every local row of the
// next block set that holds d (its reduction list), which is then applied
// without its own gather: the same values the gather would read.
template <typename T, int MODE, bool FWD>
__global__ __launch_bounds__(256) void k_scatter(int64_t nvec, const int32_t *__restrict__ red_ptr,
                                                 const int32_t *__restrict__ red_ent,
                                                 const cplx_t<T> *__restrict__ yl,
                                                 const cplx_t<T> *__restrict__ r,
                                                 cplx_t<T> *__restrict__ y, T theta,
                                                 const int32_t *__restrict__ fwd_ptr,
                                                 const int32_t *__restrict__ fwd_ent,
                                                 cplx_t<T> *__restrict__ fwd_xl) {
  using C = cplx_t<T>;
  const int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (d >= nvec) return;
  C acc;
  acc.x = 0;
  acc.y = 0;
  for (int32_t k = red_ptr[d]; k < red_ptr[d + 1]; ++k) acc = cadd(acc, yl[red_ent[k]]);
  C out;
  if (MODE == RED_SET) out = acc;
  else if (MODE == RED_RESID) out = csub(r[d], acc);
  else if (MODE == RED_AXPY) out = cadd(y[d], cscale(acc, theta));
  else out = cscale(acc, theta);
  y[d] = out;
  if (FWD)
    for (int32_t k = fwd_ptr[d]; k < fwd_ptr[d + 1]; ++k) fwd_xl[fwd_ent[k]] = out;
}

__global__ __launch_bounds__(256) void k_pack(const int4 *__restrict__ tdesc, int64_t tile0,
                                              const int32_t *__restrict__ bn,
                                              const int64_t *__restrict__ ent_off,
                                              const double2 *__restrict__ src,
                                              const int64_t *__restrict__ src_off,
                                              const int32_t *__restrict__ ld,
                                              const int64_t *__restrict__ map_off,
                                              const int32_t *__restrict__ map,
                                              double2 *__restrict__ t64, float2 *__restrict__ t32) {
  const int64_t t = tile0 + blockIdx.x;
  const int4 td = tdesc[t];
  const int b = td.x, I = td.y, J = td.z, n = bn[b];
  const int64_t mo = map_off ? map_off[b] : -1;
  const int64_t t0 = ent_off[b] + tile_entry(I, J);
  for (int e = threadIdx.x; e < kTileFull; e += 256) {
    const int k = e >> 6, lane = e & 63, ra = lane >> 3, cb = lane & 7;
    if (I == J && ra > cb) continue;   // below the diagonal of a diagonal tile
    const int64_t dst = t0 + (I == J ? k * kDiagSlots + diag_slot(ra, cb) : e);
    const int ri = 4 * ra + (k >> 2), cj = 4 * cb + (k & 3);
    const int row = 32 * I + ri, col = 32 * J + cj;
    double2 v = mk(0.0, 0.0);
    if (row < n && col < n) {
      const int64_t mr = mo >= 0 ? map[mo + row] : row, mc = mo >= 0 ? map[mo + col] : col;
      v = src[src_off[b] + mr + mc * (int64_t)ld[b]];
    }
    if (t64) t64[dst] = v;
    if (t32) t32[dst] = mkf((float)v.x, (float)v.y);
  }
}

}  // namespace

void HermSet::build(const std::vector<int32_t> &sizes, const std::vector<int32_t> &idx_concat,
                    int64_t nvec_, bool fp64, bool fp32, Budget *bud, hipStream_t s) {
  nblk = (int)sizes.size();
  nvec = nvec_;
  n_h = sizes;
  std::vector<int64_t> toff(nblk), eoff(nblk), cpo(nblk), rpo(nblk), loff(nblk);
  int64_t t = 0, p = 0, lo = 0, ii = 0;
  nent = 0;
  packed = 0;
  full = 0;
  std::vector<int4> un;
  std::vector<int2> rw;
  std::vector<int4> td;
  std::vector<int32_t> gi;
  for (int b = 0; b < nblk; ++b) {
    const int n = sizes[b], nt = (n + 31) / 32;
    toff[b] = t;
    eoff[b] = nent;
    nent += tile_entry(0, nt);
    cpo[b] = p;
    p += colbase(nt);
    rpo[b] = p;
    p += (int64_t)nt * (nt + 1) / 2 * 32;
    loff[b] = lo;
    t += (int64_t)nt * (nt + 1) / 2;
    lo += (int64_t)nt * 32;
    packed += (int64_t)n * (n + 1) / 2;
    full += (int64_t)n * n;
    for (int i = 0; i < 32 * nt; ++i) gi.push_back(i < n ? idx_concat[ii + i] : -1);
    ii += n;
    for (int J = 0; J < nt; ++J) {
      for (int seg = 0; seg * kSeg <= J; ++seg) un.push_back(make_int4(b, J, seg * kSeg, seg));
      rw.push_back(make_int2(b, J));
      for (int I = 0; I <= J; ++I) td.push_back(make_int4(b, I, J, 0));
    }
  }
  if (ii != (int64_t)idx_concat.size()) throw DpgError(-1, "HermSet: index list size mismatch");
  // units in block order (block, tile column, segment): the waves of
  // neighbouring workgroups stream neighbouring tiles (longest first, the
  // blocks mixed, was 1.3 % slower at 16^3, shuffled slower still)
  ntiles = t;
  npart = p;
  nloc = lo;
  nunits = (int64_t)un.size();
  if (npart >= (1LL << 31) || nloc >= (1LL << 31))
    throw DpgError(-1, "HermSet: partial or local vectors beyond 32-bit offsets");
  // unit descriptors: {entry offset of tile (I0, J) lo, hi, x offset of tile
  // row I0, of tile column J}, {row-partial slot of (I0, J), step to the slot of (I0 + 1, J),
  // column-partial slot, flags: 1 two tiles, 2 first tile off-diagonal, 4
  // second tile off-diagonal}
  std::vector<int4> ud(2 * un.size());
  for (size_t k = 0; k < un.size(); ++k) {
    const int b = un[k].x, J = un[k].y, I0 = un[k].z, seg = un[k].w;
    const int nt = (sizes[b] + 31) / 32;
    const int64_t tile = eoff[b] + tile_entry(I0, J);
    const int64_t r0 = rpo[b] + row_slot(nt, I0, J);
    const int64_t rd = I0 + 1 <= J ? row_slot(nt, I0 + 1, J) - row_slot(nt, I0, J) : 0;
    const int64_t cs = cpo[b] + colbase(J) + seg * 32;
    const int flags = (I0 + 1 <= J ? 1 : 0) | (I0 < J ? 2 : 0) | (I0 + 1 < J ? 4 : 0);
    ud[2 * k] = make_int4((int)(uint32_t)(tile & 0xffffffff), (int)(tile >> 32),
                          (int)(loff[b] + 32 * I0), (int)(loff[b] + 32 * J));
    ud[2 * k + 1] = make_int4((int)r0, (int)rd, (int)cs, flags);
  }
  nrows = (int64_t)rw.size();
  std::vector<int4> rd(rw.size());
  for (size_t k = 0; k < rw.size(); ++k) {
    const int b = rw[k].x, I = rw[k].y, nt = (sizes[b] + 31) / 32;
    const int nseg = (I + kSeg) / kSeg, nrw = nt - I;
    if (nseg > 0xffff || nrw > 0x7fff) throw DpgError(-1, "HermSet: block too large for row descriptors");
    rd[k] = make_int4((int)(cpo[b] + colbase(I)), (int)(rpo[b] + row_slot(nt, I, I)),
                      nseg | (nrw << 16), (int)(loff[b] + 32 * I));
  }
  // FP32: units (block, strip, chunk), in that order: {entry offset of
  // tile (0, J0) lo, hi, x offset of the block, row-sum base of the block},
  // {J0 | nt << 16, Ia | Ib << 16, column-sum slot of J0, of J1 (0 without
  // J1)}; rows: the column sums of tile column I (one slot per chunk of its
  // strip) and the row sums of tile row I (one slot per strip s >= I / 2)
  std::vector<int4> sud, srd;
  if (fp32) {
    struct Unit { int4 d0, d1; };
    std::vector<Unit> su;
    std::vector<int64_t> scpo(nblk), srpo(nblk);
    std::vector<std::vector<int32_t>> cbase(nblk);
    int64_t sp = 0;
    for (int b = 0; b < nblk; ++b) {
      const int nt = (sizes[b] + 31) / 32;
      if (nt > 0x7fff) throw DpgError(-1, "HermSet: block too large for strip descriptors");
      std::vector<int32_t> &cbv = cbase[b];
      cbv.assign(nt + 1, 0);
      for (int J = 0; J < nt; ++J) cbv[J + 1] = cbv[J] + strip_chunks(nt, J / 2);
      scpo[b] = sp;
      sp += 32LL * cbv[nt];
      srpo[b] = sp;
      sp += 32 * strip_row_slots(nt);
    }
    snpart = sp;
    if (snpart >= (1LL << 31)) throw DpgError(-1, "HermSet: partials beyond 32-bit offsets");
    for (int b = 0; b < nblk; ++b) {
      const int nt = (sizes[b] + 31) / 32;
      for (int st = 0; 2 * st < nt; ++st) {
        const int J0 = 2 * st, J1 = J0 + 1, rws = strip_rows(nt, st);
        const bool two = J1 < nt;
        const int64_t tile = eoff[b] + tile_entry(0, J0);
        for (int c = 0; c * kChunk < rws; ++c) {
          const int Ia = c * kChunk, Ib = std::min(rws, Ia + kChunk);
          Unit u;
          u.d0 = make_int4((int)(uint32_t)(tile & 0xffffffff), (int)(tile >> 32), (int)loff[b],
                           (int)srpo[b]);
          u.d1 = make_int4(J0 | (nt << 16), Ia | (Ib << 16),
                           (int)(scpo[b] + 32LL * (cbase[b][J0] + c)),
                           two ? (int)(scpo[b] + 32LL * (cbase[b][J1] + c)) : 0);
          su.push_back(u);
        }
      }
    }
    snunits = (int64_t)su.size();
    sud.resize(2 * su.size());
    for (size_t k = 0; k < su.size(); ++k) {
      sud[2 * k] = su[k].d0;
      sud[2 * k + 1] = su[k].d1;
    }
    srd.resize(rw.size());
    for (size_t k = 0; k < rw.size(); ++k) {
      const int b = rw[k].x, I = rw[k].y, nt = (sizes[b] + 31) / 32, ns = (nt + 1) / 2;
      const int nseg = strip_chunks(nt, I / 2), nrw = ns - I / 2;
      srd[k] = make_int4((int)(scpo[b] + 32LL * cbase[b][I]),
                         (int)(srpo[b] + 32 * strip_row_slot(ns, I, I / 2)), nseg | (nrw << 16),
                         (int)(loff[b] + 32 * I));
    }
  }
  tile_off_h = toff;
  ent_off_h = eoff;
  loc_off_h = loff;
  // reduction lists: for every vector entry, the local rows holding it
  std::vector<int32_t> cnt(nvec + 1, 0);
  for (int32_t v : gi) {
    if (v >= nvec) throw DpgError(-1, "HermSet: index out of range");
    if (v >= 0) cnt[v + 1]++;
  }
  for (int64_t d = 0; d < nvec; ++d) cnt[d + 1] += cnt[d];
  std::vector<int32_t> ent(cnt[nvec]);
  std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t k = 0; k < (int64_t)gi.size(); ++k)
    if (gi[k] >= 0) ent[fill[gi[k]]++] = (int32_t)k;
  bn.upload(sizes, bud, s);
  ent_off.upload(eoff, bud, s);
  cp_off.upload(cpo, bud, s);
  rp_off.upload(rpo, bud, s);
  loc_off.upload(loff, bud, s);
  gidx.upload(gi, bud, s);
  units.upload(ud, bud, s);
  rows.upload(rw, bud, s);
  rowd.upload(rd, bud, s);
  tdesc.upload(td, bud, s);
  red_ptr.upload(cnt, bud, s);
  red_ent.upload(ent, bud, s);
  if (fp64) {
    t64.alloc(nent, bud);
    p64.alloc(npart, bud);
    xl64.alloc(nloc, bud);
    yl64.alloc(nloc, bud);
    launch_zero(nloc, xl64.p, s);
  }
  if (fp32) {
    sunits.upload(sud, bud, s);
    srowd.upload(srd, bud, s);
    t32.alloc(nent, bud);
    p32.alloc(snpart, bud);
    xl32.alloc(nloc, bud);
    yl32.alloc(nloc, bud);
    launch_zero(nloc, xl32.p, s);
  }
  HIP_OK(hipStreamSynchronize(s));
}

void HermSet::pack(const double2 *src, const int64_t *src_off_dev, const int32_t *ld_dev,
                   const int64_t *map_off_dev, const int32_t *map_dev, hipStream_t s,
                   int64_t tile0, int64_t count) {
  if (count < 0) count = ntiles - tile0;
  if (count <= 0) return;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)count), dim3(256), 0, s, tdesc.p, tile0, bn.p,
                     ent_off.p, src,
                     src_off_dev, ld_dev, map_off_dev, map_dev, t64.p, t32.p);
  LAUNCH_OK();
}

template <typename T, int MODE>
void launch_scatter(const HermSet &H, const cplx_t<T> *yl, const cplx_t<T> *r, cplx_t<T> *y,
                    T theta, HermSet *fwd, cplx_t<T> *fxl, hipStream_t s) {
  const dim3 g(cdiv(H.nvec, 256));
  if (fwd)
    hipLaunchKernelGGL((k_scatter<T, MODE, true>), g, dim3(256), 0, s, H.nvec, H.red_ptr.p,
                       H.red_ent.p, yl, r, y, theta, fwd->red_ptr.p, fwd->red_ent.p, fxl);
  else
    hipLaunchKernelGGL((k_scatter<T, MODE, false>), g, dim3(256), 0, s, H.nvec, H.red_ptr.p,
                       H.red_ent.p, yl, r, y, theta, nullptr, nullptr, nullptr);
}

template <typename T> cplx_t<T> *local_x(HermSet &H) {
  if constexpr (sizeof(T) == 8) return H.xl64.p;
  else return H.xl32.p;
}

template <typename T>
void herm_apply(HermSet &H, const cplx_t<T> *x, cplx_t<T> *y, const cplx_t<T> *r, int mode,
                T theta, hipStream_t s, bool gathered, HermSet *fwd) {
  const cplx_t<T> *tiles;
  cplx_t<T> *part, *xl, *yl;
  if constexpr (sizeof(T) == 8) {
    tiles = H.t64.p;
    part = H.p64.p;
    yl = H.yl64.p;
  } else {
    tiles = H.t32.p;
    part = H.p32.p;
    yl = H.yl32.p;
  }
  xl = local_x<T>(H);
  if (!tiles || !part) throw DpgError(-6, "block set has no tiles of this precision");
  cplx_t<T> *fxl = fwd ? local_x<T>(*fwd) : nullptr;
  if (fwd && (!fxl || fwd->nvec != H.nvec))
    throw DpgError(-1, "forwarded block set does not match this one");
  if (!gathered) {
    ProfScope ps(H.prof, DPG_K_REDUCE, 0.0, s);
    hipLaunchKernelGGL((k_gather_x<T>), dim3(cdiv(H.nloc, 256)), dim3(256), 0, s, H.nloc,
                       H.gidx.p, x, xl);
    LAUNCH_OK();
  }
  {
    ProfScope ps(H.prof, sizeof(T) == 8 ? DPG_K_APPLY64 : DPG_K_APPLY32,
                 (double)H.packed_entries() * sizeof(cplx_t<T>), s);
    if constexpr (sizeof(T) == 8)
      hipLaunchKernelGGL((k_units<T>), dim3(8 * cdiv(cdiv(H.nunits, 4), 8)), dim3(256), 0, s,
                         tiles, H.units.p, H.nunits, xl, part);
    else
      hipLaunchKernelGGL((k_strips<T>), dim3(8 * cdiv(cdiv(H.snunits, 4), 8)), dim3(256), 0, s,
                         tiles, H.sunits.p, H.snunits, xl, part);
    LAUNCH_OK();
  }
  ProfScope ps(H.prof, DPG_K_REDUCE, 0.0, s);
  hipLaunchKernelGGL((k_rows<T>), dim3(cdiv(H.nrows, 8)), dim3(256), 0, s,
                     sizeof(T) == 8 ? H.rowd.p : H.srowd.p, H.nrows, part, yl);
  LAUNCH_OK();
  switch (mode) {
    case RED_SET: launch_scatter<T, RED_SET>(H, yl, r, y, theta, fwd, fxl, s); break;
    case RED_RESID: launch_scatter<T, RED_RESID>(H, yl, r, y, theta, fwd, fxl, s); break;
    case RED_AXPY: launch_scatter<T, RED_AXPY>(H, yl, r, y, theta, fwd, fxl, s); break;
    default: launch_scatter<T, RED_SET_SCALED>(H, yl, r, y, theta, fwd, fxl, s);
  }
  LAUNCH_OK();
}

template void herm_apply<double>(HermSet &, const double2 *, double2 *, const double2 *, int,
                                 double, hipStream_t, bool, HermSet *);
template void herm_apply<float>(HermSet &, const float2 *, float2 *, const float2 *, int, float,
                                hipStream_t, bool, HermSet *);

}  // namespace dpg
