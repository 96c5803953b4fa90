// Element DPG matrices: Gram matrix, ultraweak form B and loads (Sec. 2).
//
// On an axis-aligned box every integral of the matrices is a product of 1-D
// integrals, so each entry of G and B is a short sum of table products
// (exact; no quadrature at run time).  The test basis is orthonormal, which
// turns every 1-D mass factor into a Kronecker delta.  Loads are integrated
// with p+dp+5 Gauss points per direction by sum factorisation in LDS.
#include <cmath>

#include "element.hpp"
#include "topology.hpp"

namespace dpg {

void build_elem_tables(int p, int dp, ElemTables &t) {
  const int P1 = p + dp + 1;
  if (P1 > 8 || p + dp + 5 > 12) throw DpgError(-1, "order too high (p + dp <= 7 supported)");
  t = ElemTables{};
  t.P1 = P1;
  t.p = p;
  t.nql = p + dp + 5;
  std::vector<double> x, w;
  gauss_legendre(P1 + 2, x, w);
  auto Lt = [](int a, double s) { return std::sqrt((2 * a + 1) / 2.0) * legendre(a, s); };
  auto Ltd = [](int a, double s) { return std::sqrt((2 * a + 1) / 2.0) * legendre_d(a, s); };
  for (int a = 0; a < P1; ++a) {
    for (int b = 0; b < P1; ++b) {
      double kk = 0, dm = 0;
      for (size_t q = 0; q < x.size(); ++q) {
        kk += w[q] * Ltd(a, x[q]) * Ltd(b, x[q]);
        dm += w[q] * Ltd(a, x[q]) * Lt(b, x[q]);
      }
      t.KK[a * kMX + b] = kk;
      t.DM[a * kMX + b] = dm;
    }
    for (int n = 0; n < p; ++n) {
      double fm = 0, fd = 0;
      for (size_t q = 0; q < x.size(); ++q) {
        fm += w[q] * Lt(a, x[q]) * legendre(n, x[q]);
        fd += w[q] * Ltd(a, x[q]) * legendre(n, x[q]);
      }
      t.fM[a * kMX + n] = fm;
      t.fD[a * kMX + n] = fd;
    }
    for (int c = 0; c <= p; ++c) {
      double hm = 0;
      for (size_t q = 0; q < x.size(); ++q) hm += w[q] * Lt(a, x[q]) * h1_fun(p, c, x[q]);
      t.hM[a * kMX + c] = hm;
    }
    t.tEnd[a * 2 + 0] = Lt(a, -1.0);
    t.tEnd[a * 2 + 1] = Lt(a, 1.0);
  }
  for (int c = 0; c <= p; ++c) {
    t.hEnd[c * 2 + 0] = h1_fun(p, c, -1.0);
    t.hEnd[c * 2 + 1] = h1_fun(p, c, 1.0);
  }
  std::vector<double> xl, wl;
  gauss_legendre(t.nql, xl, wl);
  for (int q = 0; q < t.nql; ++q) {
    t.xq[q] = xl[q];
    t.wq[q] = wl[q];
    for (int a = 0; a < P1; ++a) t.Lq[a * kMQ + q] = Lt(a, xl[q]);
  }
}

void build_descriptors(int p, int dp, std::vector<int4> &test, std::vector<int4> &trial) {
  const int P = p + dp;
  test.clear();
  trial.clear();
  for (int c = 0; c <= P; ++c)
    for (int b = 0; b <= P; ++b)
      for (int a = 0; a <= P; ++a) test.push_back(make_int4(0, a, b, c));
  for (int d = 0; d < 3; ++d) {
    int lim[3] = {P, P, P};
    lim[d] = P + 1;
    for (int c = 0; c < lim[2]; ++c)
      for (int b = 0; b < lim[1]; ++b)
        for (int a = 0; a < lim[0]; ++a) test.push_back(make_int4(1 + d, a, b, c));
  }
  for (int f = 0; f < 4; ++f)
    for (int c = 0; c < p; ++c)
      for (int b = 0; b < p; ++b)
        for (int a = 0; a < p; ++a) trial.push_back(make_int4(f, a, b, c));
  for (int c = 0; c <= p; ++c)
    for (int b = 0; b <= p; ++b)
      for (int a = 0; a <= p; ++a)
        if (a == 0 || a == p || b == 0 || b == p || c == 0 || c == p)
          trial.push_back(make_int4(4, a, b, c));
  for (int f = 0; f < 6; ++f)
    for (int n = 0; n < p; ++n)
      for (int m = 0; m < p; ++m) trial.push_back(make_int4(5 + f, m, n, 0));
}

namespace {

__device__ inline void elem_cell(int e, int N, int c[3]) {
  c[0] = e % N;
  c[1] = (e / N) % N;
  c[2] = e / (N * N);
}

__global__ __launch_bounds__(256) void k_gram(const ElemTables *__restrict__ tb,
                                              const int4 *__restrict__ test, int nt, ElemGeom g,
                                              const double *__restrict__ kappa, int e0,
                                              double2 *__restrict__ G) {
  // one wave per column j, its lanes over the rows i >= j (Hermitian: the
  // Cholesky that follows reads the lower triangle only)
  const int j = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (j >= nt) return;
  const int e = g.elist ? g.elist[e0 + blockIdx.y] : e0 + blockIdx.y;
  const int4 tj = test[j];
  const double hh = 0.5 * g.h, w = g.omega, kap = kappa ? kappa[e] : 1.0;
  const int b[3] = {tj.y, tj.z, tj.w};
  double2 *Gc = G + (int64_t)blockIdx.y * nt * nt + (int64_t)j * nt;
  for (int i = j + (threadIdx.x & 63); i < nt; i += 64) {
  const int4 ti = test[i];
  const int a[3] = {ti.y, ti.z, ti.w};
  const bool dl[3] = {a[0] == b[0], a[1] == b[1], a[2] == b[2]};
  double re = 0.0, im = 0.0;
  if (ti.x == 0 && tj.x == 0) {
    if (dl[0] && dl[1] && dl[2]) re += (w * w * kap * kap + g.alpha) * hh * hh * hh;
    for (int d = 0; d < 3; ++d)
      if (dl[(d + 1) % 3] && dl[(d + 2) % 3]) re += hh * tb->KK[a[d] * kMX + b[d]];
  } else if (ti.x == 0) {
    // (A* v_j, A* q_i): -i w kappa int (d_d v_j) q_i + i w int v_j d_d q_i
    const int d = tj.x - 1;
    if (dl[(d + 1) % 3] && dl[(d + 2) % 3])
      im = w * hh * hh * (tb->DM[a[d] * kMX + b[d]] - kap * tb->DM[b[d] * kMX + a[d]]);
  } else if (tj.x == 0) {
    const int d = ti.x - 1;
    if (dl[(d + 1) % 3] && dl[(d + 2) % 3])
      im = -w * hh * hh * (tb->DM[b[d] * kMX + a[d]] - kap * tb->DM[a[d] * kMX + b[d]]);
  } else {
    const int ei = ti.x - 1, d = tj.x - 1;
    if (d == ei) {
      if (dl[(d + 1) % 3] && dl[(d + 2) % 3]) re += hh * tb->KK[a[d] * kMX + b[d]];
      if (dl[0] && dl[1] && dl[2]) re += (w * w + g.alpha) * hh * hh * hh;
    } else {
      // int (d_d v_j)(d_e v_i): derivative on v_j along d, on v_i along e
      const int f = 3 - d - ei;
      if (dl[f]) re = hh * tb->DM[b[d] * kMX + a[d]] * tb->DM[a[ei] * kMX + b[ei]];
    }
  }
  Gc[i] = mk(re, im);
  }
}

__global__ __launch_bounds__(256) void k_bmat(const ElemTables *__restrict__ tb,
                                              const int4 *__restrict__ test,
                                              const int4 *__restrict__ trial, int nt, int m,
                                              ElemGeom g, const double *__restrict__ kappa,
                                              const double *__restrict__ Zel, int e0,
                                              double2 *__restrict__ BL, int64_t strideBL) {
  // one wave per trial function j, its lanes over the test functions i
  const int j = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (j >= m) return;
  const int e = g.elist ? g.elist[e0 + blockIdx.y] : e0 + blockIdx.y;
  const int4 tr = trial[j];
  const double hh = 0.5 * g.h, w = g.omega, kap = kappa ? kappa[e] : 1.0;
  const double Z = Zel ? Zel[e] : 1.0;
  int cell[3];
  elem_cell(e, g.N, cell);
  double2 *Bc = BL + (int64_t)blockIdx.y * strideBL + (int64_t)j * nt;
  for (int i = threadIdx.x & 63; i < nt; i += 64) {
  const int4 ti = test[i];
  const int a[3] = {ti.y, ti.z, ti.w};
  const int isq = ti.x == 0, ev = ti.x - 1;   // ev = component of v (if not q)
  double re = 0.0, im = 0.0;
  if (tr.x <= 3) {
    const int n[3] = {tr.y, tr.z, tr.w};
    double fm[3], fd[3];
    for (int d = 0; d < 3; ++d) {
      fm[d] = tb->fM[a[d] * kMX + n[d]];
      fd[d] = tb->fD[a[d] * kMX + n[d]];
    }
    if (tr.x == 0) {            // pressure field
      if (isq) im = w * kap * hh * hh * hh * fm[0] * fm[1] * fm[2];
      else re = -hh * hh * fd[ev] * fm[(ev + 1) % 3] * fm[(ev + 2) % 3];
    } else {                    // velocity field component d
      const int d = tr.x - 1;
      if (isq) re = -hh * hh * fd[d] * fm[(d + 1) % 3] * fm[(d + 2) % 3];
      else if (ev == d) im = w * hh * hh * hh * fm[0] * fm[1] * fm[2];
    }
  } else if (tr.x == 4) {       // pressure trace, H1 lattice point l
    const int l[3] = {tr.y, tr.z, tr.w};
    if (!isq) {
      // <phat, v.n> over the two faces normal to the component of v
      const double ip = hh * hh * tb->hM[a[(ev + 1) % 3] * kMX + l[(ev + 1) % 3]] *
                        tb->hM[a[(ev + 2) % 3] * kMX + l[(ev + 2) % 3]];
      for (int s = 0; s < 2; ++s)
        re += (s ? 1.0 : -1.0) * tb->tEnd[a[ev] * 2 + s] * tb->hEnd[l[ev] * 2 + s] * ip;
    } else {
      // <Z^-1 phat, q> on Gamma faces
      for (int d = 0; d < 3; ++d)
        for (int s = 0; s < 2; ++s) {
          const bool gam = (s == 0 && cell[d] == 0) || (s == 1 && cell[d] == g.N - 1);
          if (!gam) continue;
          re += tb->tEnd[a[d] * 2 + s] * tb->hEnd[l[d] * 2 + s] * hh * hh *
                tb->hM[a[(d + 1) % 3] * kMX + l[(d + 1) % 3]] *
                tb->hM[a[(d + 2) % 3] * kMX + l[(d + 2) % 3]] / Z;
        }
    }
  } else {                      // flux on face f = 2 d + s, in-plane degrees (m, n)
    const int f = tr.x - 5, d = f >> 1, s = f & 1;
    const bool gam = (s == 0 && cell[d] == 0) || (s == 1 && cell[d] == g.N - 1);
    if (isq && !gam) {
      const int f1 = d == 0 ? 1 : 0, f2 = d == 2 ? 1 : 2;
      re = (s ? 1.0 : -1.0) * tb->tEnd[a[d] * 2 + s] * hh * hh * tb->fM[a[f1] * kMX + tr.y] *
           tb->fM[a[f2] * kMX + tr.z];
    }
  }
  Bc[i] = mk(re, im);
  }
}

constexpr int LX = 8, LQ = 12;

__global__ __launch_bounds__(256) void k_load(const ElemTables *__restrict__ tb, int nt, int m,
                                              ElemGeom g, const double *__restrict__ Zel,
                                              const LoadDesc *__restrict__ ld,
                                              const double *__restrict__ src,
                                              const double2 *__restrict__ u0q, int e0,
                                              double2 *__restrict__ BL, int64_t strideBL) {
  __shared__ double2 buf1[LQ * LQ * LQ];   // point values, then second contraction
  __shared__ double2 buf2[LX * LQ * LQ];   // first contraction
  __shared__ double2 lq[LX * LX * LX];     // q-part of the load
  const int tid = threadIdx.x;
  const int e = g.elist ? g.elist[e0 + blockIdx.x] : e0 + blockIdx.x, r = blockIdx.y;
  const LoadDesc L = ld[r];
  const int P1 = tb->P1, nq = tb->nql;
  const double hh = 0.5 * g.h;
  int cell[3];
  elem_cell(e, g.N, cell);
  double x0[3];
  for (int d = 0; d < 3; ++d) x0[d] = g.org[d] + g.h * cell[d];
  for (int k = tid; k < P1 * P1 * P1; k += 256) lq[k] = mk(0.0, 0.0);
  __syncthreads();
  if (L.nsrc > 0) {
    for (int k = tid; k < nq * nq * nq; k += 256) {
      const int ix = k % nq, iy = (k / nq) % nq, iz = k / (nq * nq);
      const double X = x0[0] + (tb->xq[ix] + 1.0) * hh, Y = x0[1] + (tb->xq[iy] + 1.0) * hh,
                   Zc = x0[2] + (tb->xq[iz] + 1.0) * hh;
      double fr = 0.0, fi = 0.0;
      for (int s = 0; s < L.nsrc; ++s) {
        const double *S = src + 6 * (L.src0 + s);
        const double sg = S[3];
        const double r2 = (X - S[0]) * (X - S[0]) + (Y - S[1]) * (Y - S[1]) + (Zc - S[2]) * (Zc - S[2]);
        const double v = exp(-r2 / (2.0 * sg * sg)) / (2.0 * M_PI * sg * sg * sqrt(2.0 * M_PI * sg * sg));
        fr += S[4] * v;
        fi += S[5] * v;
      }
      const double wt = tb->wq[ix] * tb->wq[iy] * tb->wq[iz];
      buf1[k] = mk(fr * wt, fi * wt);
    }
    __syncthreads();
    // T1[a][z][y] = sum_x Lq[a][x] F[z][y][x]
    for (int k = tid; k < P1 * nq * nq; k += 256) {
      const int yz = k % (nq * nq), aa = k / (nq * nq);
      double2 acc = mk(0.0, 0.0);
      for (int ix = 0; ix < nq; ++ix) acc = cadd(acc, cscale(buf1[yz * nq + ix], tb->Lq[aa * kMQ + ix]));
      buf2[k] = acc;
    }
    __syncthreads();
    // T2[a][b][z] = sum_y Lq[b][y] T1[a][z][y]
    for (int k = tid; k < P1 * P1 * nq; k += 256) {
      const int iz = k % nq, bb = (k / nq) % P1, aa = k / (nq * P1);
      double2 acc = mk(0.0, 0.0);
      for (int iy = 0; iy < nq; ++iy)
        acc = cadd(acc, cscale(buf2[(aa * nq + iz) * nq + iy], tb->Lq[bb * kMQ + iy]));
      buf1[k] = acc;
    }
    __syncthreads();
    for (int k = tid; k < P1 * P1 * P1; k += 256) {
      const int aa = k % P1, bb = (k / P1) % P1, cc = k / (P1 * P1);
      double2 acc = mk(0.0, 0.0);
      for (int iz = 0; iz < nq; ++iz)
        acc = cadd(acc, cscale(buf1[(aa * P1 + bb) * nq + iz], tb->Lq[cc * kMQ + iz]));
      lq[k] = cadd(lq[k], cscale(acc, hh * hh * hh));
    }
    __syncthreads();
  }
  const bool pw = L.amp[0] != 0.0 || L.amp[1] != 0.0;
  if (pw || L.u0_off >= 0) {
    const double Z = Zel ? Zel[e] : 1.0;
    for (int d = 0; d < 3; ++d)
      for (int s = 0; s < 2; ++s) {
        const bool gam = (s == 0 && cell[d] == 0) || (s == 1 && cell[d] == g.N - 1);
        if (!gam) continue;
        const int f1 = d == 0 ? 1 : 0, f2 = d == 2 ? 1 : 2;
        const double nd = s ? 1.0 : -1.0;          // outward normal = nd e_d
        const double fac = 1.0 / Z - L.dir[d] * nd;
        const double2 *uq =
            L.u0_off >= 0
                ? u0q + L.u0_off + boundary_face(d, s, cell[f1], cell[f2], g.N) * nq * nq
                : nullptr;
        for (int k = tid; k < nq * nq; k += 256) {
          const int p1 = k % nq, p2 = k / nq;
          double2 u = mk(0.0, 0.0);
          if (pw) {   // plane wave: u0 = (Z^-1 - d.n) A exp(-i w d.x)
            double X[3];
            X[d] = x0[d] + (s ? g.h : 0.0);
            X[f1] = x0[f1] + (tb->xq[p1] + 1.0) * hh;
            X[f2] = x0[f2] + (tb->xq[p2] + 1.0) * hh;
            const double th = -g.omega * (L.dir[0] * X[0] + L.dir[1] * X[1] + L.dir[2] * X[2]);
            double sn, cs;
            sincos(th, &sn, &cs);
            u = mk(fac * (L.amp[0] * cs - L.amp[1] * sn), fac * (L.amp[0] * sn + L.amp[1] * cs));
          }
          if (uq) u = cadd(u, uq[k]);
          const double wt = tb->wq[p1] * tb->wq[p2];
          buf1[k] = mk(wt * u.x, wt * u.y);
        }
        __syncthreads();
        // C1[a1][p2] = sum_p1 Lq[a1][p1] F[p2][p1]
        for (int k = tid; k < P1 * nq; k += 256) {
          const int p2 = k % nq, a1 = k / nq;
          double2 acc = mk(0.0, 0.0);
          for (int p1 = 0; p1 < nq; ++p1) acc = cadd(acc, cscale(buf1[p2 * nq + p1], tb->Lq[a1 * kMQ + p1]));
          buf2[k] = acc;
        }
        __syncthreads();
        for (int k = tid; k < P1 * P1 * P1; k += 256) {
          const int deg[3] = {k % P1, (k / P1) % P1, k / (P1 * P1)};
          double2 acc = mk(0.0, 0.0);
          for (int p2 = 0; p2 < nq; ++p2)
            acc = cadd(acc, cscale(buf2[deg[f1] * nq + p2], tb->Lq[deg[f2] * kMQ + p2]));
          lq[k] = cadd(lq[k], cscale(acc, hh * hh * tb->tEnd[deg[d] * 2 + s]));
        }
        __syncthreads();
      }
  }
  double2 *col = BL + (int64_t)blockIdx.x * strideBL + (int64_t)(m + r) * nt;
  for (int k = tid; k < nt; k += 256) col[k] = k < P1 * P1 * P1 ? lq[k] : mk(0.0, 0.0);
}

}  // namespace

void launch_gram(const ElemTables *tb, const int4 *test, int nt, ElemGeom g, const double *kappa,
                 int e0, int count, double2 *G, hipStream_t s) {
  hipLaunchKernelGGL(k_gram, dim3(cdiv(nt, 4), count), dim3(256), 0, s, tb, test,
                     nt, g, kappa, e0, G);
  LAUNCH_OK();
}

void launch_bmat(const ElemTables *tb, const int4 *test, const int4 *trial, int nt, int m,
                 ElemGeom g, const double *kappa, const double *Zel, int e0, int count,
                 double2 *BL, int64_t strideBL, hipStream_t s) {
  hipLaunchKernelGGL(k_bmat, dim3(cdiv(m, 4), count), dim3(256), 0, s, tb, test,
                     trial, nt, m, g, kappa, Zel, e0, BL, strideBL);
  LAUNCH_OK();
}

void launch_load(const ElemTables *tb, int nt, int m, ElemGeom g, const double *Zel,
                 const LoadDesc *ld, const double *src, const double2 *u0q, int nrhs, int e0,
                 int count, double2 *BL, int64_t strideBL, hipStream_t s) {
  if (nrhs <= 0) return;
  hipLaunchKernelGGL(k_load, dim3(count, nrhs), dim3(256), 0, s, tb, nt, m, g, Zel, ld, src, u0q,
                     e0, BL, strideBL);
  LAUNCH_OK();
}

}  // namespace dpg
