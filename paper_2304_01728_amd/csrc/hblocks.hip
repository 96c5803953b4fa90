// Hermitian block sets: packing and apply kernels (see hblocks.hpp).
#include <algorithm>
#include <numeric>

#include "hblocks.hpp"

namespace dpg {
namespace {

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

// One wave per (block, tile column J).
template <typename T>
__global__ __launch_bounds__(256) void k_units(const cplx_t<T> *__restrict__ tiles,
                                               const int2 *__restrict__ units, int64_t nunits,
                                               const int32_t *__restrict__ bn,
                                               const int64_t *__restrict__ tile_off,
                                               const int64_t *__restrict__ part_off,
                                               const int64_t *__restrict__ idx_off,
                                               const int32_t *__restrict__ idx,
                                               const cplx_t<T> *__restrict__ x,
                                               cplx_t<T> *__restrict__ part) {
  using C = cplx_t<T>;
  const int64_t wv = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wv >= nunits) return;
  const int lane = threadIdx.x & 63, ra = lane >> 3, cb = lane & 7;
  const int2 u = units[wv];
  const int b = u.x, J = u.y;
  const int n = bn[b], nt = (n + 31) >> 5;
  const int32_t *ix = idx + idx_off[b];
  C zero;
  zero.x = 0;
  zero.y = 0;
  C xJ[4], cacc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = 32 * J + 4 * cb + j;
    xJ[j] = c < n ? x[ix[c]] : zero;
    cacc[j] = zero;
  }
  const C *tp = tiles + (tile_off[b] + (int64_t)J * (J + 1) / 2) * 1024 + lane;
  C *pb = part + part_off[b];
  C *rp = pb + (int64_t)nt * 32 + (int64_t)J * (J + 1) / 2 * 32;
  for (int I = 0; I <= J; ++I, tp += 1024) {
    C t[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) t[k] = tp[k * 64];
    C xI[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 32 * I + 4 * ra + i;
      xI[i] = r < n ? x[ix[r]] : zero;
    }
    C rs[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      C a = zero;
#pragma unroll
      for (int j = 0; j < 4; ++j) a = cfma(t[4 * i + j], xJ[j], a);
      rs[i] = a;
    }
    if (I < J) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) cacc[j] = cfmaconj(t[4 * i + j], xI[i], cacc[j]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      rs[i] = cadd(rs[i], shfl_xor_c(rs[i], 1));
      rs[i] = cadd(rs[i], shfl_xor_c(rs[i], 2));
      rs[i] = cadd(rs[i], shfl_xor_c(rs[i], 4));
    }
    if (cb < 4) rp[I * 32 + 4 * ra + cb] = sel4(rs[0], rs[1], rs[2], rs[3], cb);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    cacc[j] = cadd(cacc[j], shfl_xor_c(cacc[j], 8));
    cacc[j] = cadd(cacc[j], shfl_xor_c(cacc[j], 16));
    cacc[j] = cadd(cacc[j], shfl_xor_c(cacc[j], 32));
  }
  if (ra < 4) pb[J * 32 + 4 * cb + ra] = sel4(cacc[0], cacc[1], cacc[2], cacc[3], ra);
}

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_reduce(int64_t nvec, const int32_t *__restrict__ red_ptr,
                                                const int2 *__restrict__ red_ent,
                                                const int32_t *__restrict__ bn,
                                                const int64_t *__restrict__ part_off,
                                                const cplx_t<T> *__restrict__ part,
                                                const cplx_t<T> *__restrict__ r,
                                                cplx_t<T> *__restrict__ y, T theta) {
  using C = cplx_t<T>;
  const int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (d >= nvec) return;
  C acc;
  acc.x = 0;
  acc.y = 0;
  for (int32_t k = red_ptr[d]; k < red_ptr[d + 1]; ++k) {
    const int2 be = red_ent[k];
    const int nt = (bn[be.x] + 31) >> 5, I = be.y >> 5, rr = be.y & 31;
    const C *pb = part + part_off[be.x];
    acc = cadd(acc, pb[I * 32 + rr]);
    const C *rp = pb + (int64_t)nt * 32 + rr;
    for (int J = I; J < nt; ++J) acc = cadd(acc, rp[((int64_t)J * (J + 1) / 2 + I) * 32]);
  }
  if (MODE == RED_SET) y[d] = acc;
  else if (MODE == RED_RESID) y[d] = csub(r[d], acc);
  else if (MODE == RED_AXPY) y[d] = cadd(y[d], cscale(acc, theta));
  else y[d] = cscale(acc, theta);
}

__global__ __launch_bounds__(256) void k_pack(const int4 *__restrict__ tdesc, int64_t tile0,
                                              const int32_t *__restrict__ bn,
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
  for (int e = threadIdx.x; e < 1024; e += 256) {
    const int k = e >> 6, lane = e & 63;
    const int ri = 4 * (lane >> 3) + (k >> 2), cj = 4 * (lane & 7) + (k & 3);
    const int row = 32 * I + ri, col = 32 * J + cj;
    double2 v = mk(0.0, 0.0);
    if (row < n && col < n) {
      const int64_t mr = mo >= 0 ? map[mo + row] : row, mc = mo >= 0 ? map[mo + col] : col;
      v = src[src_off[b] + mr + mc * (int64_t)ld[b]];
    }
    if (t64) t64[t * 1024 + e] = v;
    if (t32) t32[t * 1024 + e] = mkf((float)v.x, (float)v.y);
  }
}

}  // namespace

int64_t HermSet::packed_entries() const {
  int64_t s = 0;
  for (int32_t n : n_h) s += (int64_t)n * (n + 1) / 2;
  return s;
}

void HermSet::build(const std::vector<int32_t> &sizes, const std::vector<int32_t> &idx_concat,
                    int64_t nvec_, bool fp64, bool fp32, Budget *bud, hipStream_t s) {
  nblk = (int)sizes.size();
  nvec = nvec_;
  n_h = sizes;
  std::vector<int64_t> toff(nblk), poff(nblk), ioff(nblk);
  int64_t t = 0, p = 0, ii = 0;
  std::vector<int2> un;
  std::vector<int4> td;
  for (int b = 0; b < nblk; ++b) {
    const int nt = (sizes[b] + 31) / 32;
    toff[b] = t;
    poff[b] = p;
    ioff[b] = ii;
    t += (int64_t)nt * (nt + 1) / 2;
    p += (int64_t)nt * 32 + (int64_t)nt * (nt + 1) / 2 * 32;
    ii += sizes[b];
    for (int J = 0; J < nt; ++J) {
      un.push_back(make_int2(b, J));
      for (int I = 0; I <= J; ++I) td.push_back(make_int4(b, I, J, 0));
    }
  }
  if (ii != (int64_t)idx_concat.size()) throw DpgError(-1, "HermSet: index list size mismatch");
  std::stable_sort(un.begin(), un.end(), [](int2 a, int2 b) { return a.y > b.y; });
  ntiles = t;
  npart = p;
  nunits = (int64_t)un.size();
  tile_off_h = toff;
  // reduction lists: for every vector entry, the (block, row) pairs holding it
  std::vector<int32_t> cnt(nvec + 1, 0);
  for (int32_t v : idx_concat) {
    if (v < 0 || v >= nvec) throw DpgError(-1, "HermSet: index out of range");
    cnt[v + 1]++;
  }
  for (int64_t d = 0; d < nvec; ++d) cnt[d + 1] += cnt[d];
  std::vector<int2> ent(idx_concat.size());
  std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
  for (int b = 0; b < nblk; ++b)
    for (int i = 0; i < sizes[b]; ++i) ent[fill[idx_concat[ioff[b] + i]]++] = make_int2(b, i);
  bn.upload(sizes, bud, s);
  tile_off.upload(toff, bud, s);
  part_off.upload(poff, bud, s);
  idx_off.upload(ioff, bud, s);
  idx.upload(idx_concat, bud, s);
  units.upload(un, bud, s);
  tdesc.upload(td, bud, s);
  red_ptr.upload(cnt, bud, s);
  red_ent.upload(ent, bud, s);
  if (fp64) {
    t64.alloc(ntiles * 1024, bud);
    p64.alloc(npart, bud);
  }
  if (fp32) {
    t32.alloc(ntiles * 1024, bud);
    p32.alloc(npart, bud);
  }
  HIP_OK(hipStreamSynchronize(s));
}

void HermSet::pack(const double2 *src, const int64_t *src_off_dev, const int32_t *ld_dev,
                   const int64_t *map_off_dev, const int32_t *map_dev, hipStream_t s,
                   int64_t tile0, int64_t count) {
  if (count < 0) count = ntiles - tile0;
  if (count <= 0) return;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)count), dim3(256), 0, s, tdesc.p, tile0, bn.p, src,
                     src_off_dev, ld_dev, map_off_dev, map_dev, t64.p, t32.p);
  LAUNCH_OK();
}

template <typename T>
void herm_apply(HermSet &H, const cplx_t<T> *x, cplx_t<T> *y, const cplx_t<T> *r, int mode,
                T theta, hipStream_t s) {
  const cplx_t<T> *tiles;
  cplx_t<T> *part;
  if constexpr (sizeof(T) == 8) {
    tiles = H.t64.p;
    part = H.p64.p;
  } else {
    tiles = H.t32.p;
    part = H.p32.p;
  }
  if (!tiles || !part) throw DpgError(-6, "block set has no tiles of this precision");
  {
    ProfScope ps(H.prof, sizeof(T) == 8 ? DPG_K_APPLY64 : DPG_K_APPLY32,
                 (double)H.packed_entries() * sizeof(cplx_t<T>), s);
    hipLaunchKernelGGL((k_units<T>), dim3(cdiv(H.nunits, 4)), dim3(256), 0, s, tiles, H.units.p,
                       H.nunits, H.bn.p, H.tile_off.p, H.part_off.p, H.idx_off.p, H.idx.p, x, part);
    LAUNCH_OK();
  }
  ProfScope ps(H.prof, DPG_K_REDUCE, 0.0, s);
  const dim3 g(cdiv(H.nvec, 256));
  switch (mode) {
    case RED_SET:
      hipLaunchKernelGGL((k_reduce<T, RED_SET>), g, dim3(256), 0, s, H.nvec, H.red_ptr.p, H.red_ent.p, H.bn.p, H.part_off.p, part, r, y, theta);
      break;
    case RED_RESID:
      hipLaunchKernelGGL((k_reduce<T, RED_RESID>), g, dim3(256), 0, s, H.nvec, H.red_ptr.p, H.red_ent.p, H.bn.p, H.part_off.p, part, r, y, theta);
      break;
    case RED_AXPY:
      hipLaunchKernelGGL((k_reduce<T, RED_AXPY>), g, dim3(256), 0, s, H.nvec, H.red_ptr.p, H.red_ent.p, H.bn.p, H.part_off.p, part, r, y, theta);
      break;
    default:
      hipLaunchKernelGGL((k_reduce<T, RED_SET_SCALED>), g, dim3(256), 0, s, H.nvec, H.red_ptr.p, H.red_ent.p, H.bn.p, H.part_off.p, part, r, y, theta);
  }
  LAUNCH_OK();
}

template void herm_apply<double>(HermSet &, const double2 *, double2 *, const double2 *, int,
                                 double, hipStream_t);
template void herm_apply<float>(HermSet &, const float2 *, float2 *, const float2 *, int, float,
                                hipStream_t);

}  // namespace dpg
