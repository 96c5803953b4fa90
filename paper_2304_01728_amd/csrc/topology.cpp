// Host-side topology and 1-D tables; see topology.hpp.
#include "topology.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace dpg {

static const double kPi = 3.14159265358979323846;

double legendre(int n, double x) {
  if (n == 0) return 1.0;
  double p0 = 1.0, p1 = x;
  for (int k = 1; k < n; ++k) {
    double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

double legendre_d(int n, double x) {
  // P'_{k+1} = P'_{k-1} + (2k+1) P_k
  if (n == 0) return 0.0;
  double dm1 = 0.0, d = 1.0;  // P'_0, P'_1
  for (int k = 1; k < n; ++k) {
    double dn = dm1 + (2 * k + 1) * legendre(k, x);
    dm1 = d;
    d = dn;
  }
  return d;
}

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  // Newton iteration on P_n from the Chebyshev-like initial guess; nodes
  // returned ascending.
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double t = std::cos(kPi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double dt = legendre(n, t) / legendre_d(n, t);
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double d = legendre_d(n, t);
    x[n - 1 - i] = t;
    w[n - 1 - i] = 2.0 / ((1.0 - t * t) * d * d);
  }
}

double h1_fun(int r, int a, double x) {
  if (a == 0) return 0.5 * (1.0 - x);
  if (a == r) return 0.5 * (1.0 + x);
  int k = a + 1;
  return (legendre(k, x) - legendre(k - 2, x)) / std::sqrt(2.0 * (2 * k - 1));
}

double h1_fun_d(int r, int a, double x) {
  if (a == 0) return -0.5;
  if (a == r) return 0.5;
  int k = a + 1;
  return std::sqrt((2 * k - 1) / 2.0) * legendre(k - 1, x);
}

static double clean(double v) { return std::fabs(v) < 1e-13 ? 0.0 : v; }

std::vector<double> twoscale_leg(int r) {
  // coefficient of fine P_n on half h in coarse P_m: (2n+1)/2 int P_m(xi(eta)) P_n(eta)
  std::vector<double> gx, gw;
  gauss_legendre(r + 2, gx, gw);
  std::vector<double> R(2 * r * r, 0.0);
  for (int h = 0; h < 2; ++h)
    for (int n = 0; n < r; ++n)
      for (int m = 0; m < r; ++m) {
        double s = 0.0;
        for (size_t q = 0; q < gx.size(); ++q) {
          double xi = h == 0 ? 0.5 * (gx[q] - 1.0) : 0.5 * (gx[q] + 1.0);
          s += gw[q] * legendre(m, xi) * legendre(n, gx[q]);
        }
        R[(h * r + n) * r + m] = clean(s * (2 * n + 1) / 2.0);
      }
  return R;
}

std::vector<double> twoscale_h1(int r) {
  // Hierarchical expansion on each half: vertex coefficients are the end
  // values; bubble coefficients are int f' phi_k' (the phi_k' are
  // orthonormal and orthogonal to constants, so the linear part drops out).
  std::vector<double> gx, gw;
  gauss_legendre(r + 2, gx, gw);
  std::vector<double> R((2 * r + 1) * (r + 1), 0.0);
  for (int h = 0; h < 2; ++h) {
    double sh = h == 0 ? -0.5 : 0.5;  // xi = eta/2 + sh
    for (int a = 0; a <= r; ++a) {
      int base = h * r;
      R[(base + 0) * (r + 1) + a] = clean(h1_fun(r, a, -0.5 + sh));
      R[(base + r) * (r + 1) + a] = clean(h1_fun(r, a, 0.5 + sh));
      for (int b = 1; b < r; ++b) {
        double s = 0.0;
        for (size_t q = 0; q < gx.size(); ++q)
          s += gw[q] * 0.5 * h1_fun_d(r, a, 0.5 * gx[q] + sh) * h1_fun_d(r, b, gx[q]);
        R[(base + b) * (r + 1) + a] = clean(s);
      }
    }
  }
  return R;
}

void Numbering::build(int N_, int p_) {
  N = N_;
  p = p_;
  M = N * p;
  int64_t L = M + 1;
  h1_index.assign(L * L * L, -1);
  int64_t k = 0;
  h1_lat.clear();
  for (int Z = 0; Z <= M; ++Z)
    for (int Y = 0; Y <= M; ++Y)
      for (int X = 0; X <= M; ++X)
        if (X % p == 0 || Y % p == 0 || Z % p == 0) {
          h1_index[(Z * L + Y) * L + X] = (int32_t)k++;
          h1_lat.push_back((Z * L + Y) * L + X);
        }
  n_h1 = k;
  n_fam = (int64_t)(N - 1) * M * M;
  n = n_h1 + 3 * n_fam;
  if (n != n_trace(N, p)) throw std::runtime_error("trace count mismatch");
}

void Numbering::describe(int64_t idx, int &kind, int c[3]) const {
  if (idx < n_h1) {
    int64_t L = M + 1, id = h1_lat[idx];
    kind = 0;
    c[0] = (int)(id % L);
    c[1] = (int)((id / L) % L);
    c[2] = (int)(id / (L * L));
    return;
  }
  int64_t r = idx - n_h1;
  int d = (int)(r / n_fam);
  r -= (int64_t)d * n_fam;
  kind = d + 1;
  c[1] = (int)(r % M);
  r /= M;
  c[2] = (int)(r % M);
  c[0] = (int)(r / M) + 1;
}

void ElementLayout::build(int p_) {
  p = p_;
  lat.clear();
  for (int c = 0; c <= p; ++c)
    for (int b = 0; b <= p; ++b)
      for (int a = 0; a <= p; ++a)
        if (a == 0 || a == p || b == 0 || b == p || c == 0 || c == p) {
          lat.push_back(a);
          lat.push_back(b);
          lat.push_back(c);
        }
  n_h1 = (int)lat.size() / 3;
  n_tr = n_h1 + 6 * p * p;
}

std::vector<int32_t> element_dofs(const Numbering &num, const ElementLayout &el) {
  const int N = num.N, p = num.p;
  std::vector<int32_t> out((int64_t)N * N * N * el.n_tr, -1);
  for (int k = 0; k < N; ++k)
    for (int j = 0; j < N; ++j)
      for (int i = 0; i < N; ++i) {
        int64_t e = i + (int64_t)N * (j + (int64_t)N * k);
        int32_t *row = &out[e * el.n_tr];
        for (int q = 0; q < el.n_h1; ++q)
          row[q] = (int32_t)num.h1(i * p + el.lat[3 * q], j * p + el.lat[3 * q + 1],
                                   k * p + el.lat[3 * q + 2]);
        const int cell[3] = {i, j, k};
        int o = el.n_h1;
        for (int d = 0; d < 3; ++d) {
          const int a1 = d == 0 ? 1 : 0, a2 = d == 2 ? 1 : 2;
          for (int s = 0; s < 2; ++s) {
            int plane = cell[d] + s;
            for (int n = 0; n < p; ++n)
              for (int m = 0; m < p; ++m, ++o)
                row[o] = (plane > 0 && plane < N)
                             ? (int32_t)num.flux(d, plane, cell[a1] * p + m, cell[a2] * p + n)
                             : -1;
          }
        }
      }
  return out;
}

// ---------------------------------------------------------------------------
// macro level

static inline bool on_block_boundary(int a, int b, int c, int q) {
  return a == 0 || a == q || b == 0 || b == q || c == 0 || c == q;
}

int MacroLevel::slot_in_block(const Numbering &fine, int64_t t, int ci, int cj, int ck) const {
  const int q = 2 * p;
  int kind, c[3];
  fine.describe(t, kind, c);
  const int cell[3] = {ci, cj, ck};
  if (kind == 0) {
    int a = c[0] - q * ci, b = c[1] - q * cj, cc = c[2] - q * ck;
    if (a < 0 || a > q || b < 0 || b > q || cc < 0 || cc > q) return -1;
    return bslot_tab[(cc * (q + 1) + b) * (q + 1) + a];
  }
  int d = kind - 1, s = c[0];
  const int a1 = d == 0 ? 1 : 0, a2 = d == 2 ? 1 : 2;
  int side;
  if (s == 2 * cell[d]) side = 0;
  else if (s == 2 * cell[d] + 2) side = 1;
  else return -1;
  int t1 = c[1] - q * cell[a1], t2 = c[2] - q * cell[a2];
  if (t1 < 0 || t1 >= q || t2 < 0 || t2 >= q) return -1;
  int nlat = (q + 1) * (q + 1) * (q + 1) - (q - 1) * (q - 1) * (q - 1);
  return nlat + (2 * d + side) * q * q + t2 * q + t1;
}

void MacroLevel::build(const Numbering &fine, const ElementLayout &el) {
  N = fine.N;
  p = fine.p;
  if (N % 2) throw std::runtime_error("macro level needs an even mesh");
  Nc = N / 2;
  const int q = 2 * p;
  const int nlat = (q + 1) * (q + 1) * (q + 1) - (q - 1) * (q - 1) * (q - 1);
  nBf = nlat + 6 * q * q;
  nI = (q - 1) * (q - 1) * (q - 1) - 8 * (p - 1) * (p - 1) * (p - 1) + 3 * q * q;

  // macro set: on the coarse skeleton
  macro_of.assign(fine.n, -1);
  macro_B.clear();
  {
    const int64_t L = fine.M + 1;
    for (int Z = 0; Z <= fine.M; ++Z)
      for (int Y = 0; Y <= fine.M; ++Y)
        for (int X = 0; X <= fine.M; ++X) {
          int32_t t = fine.h1_index[((int64_t)Z * L + Y) * L + X];
          if (t >= 0 && (X % q == 0 || Y % q == 0 || Z % q == 0)) macro_of[t] = 1;
        }
    for (int d = 0; d < 3; ++d)
      for (int s = 2; s < N; s += 2)
        for (int T2 = 0; T2 < fine.M; ++T2)
          for (int T1 = 0; T1 < fine.M; ++T1) macro_of[fine.flux(d, s, T1, T2)] = 1;
    int64_t k = 0;
    for (int64_t t = 0; t < fine.n; ++t)
      if (macro_of[t] > 0) {
        macro_of[t] = (int32_t)k++;
        macro_B.push_back(t);
      } else {
        macro_of[t] = -1;
      }
    nM = k;
  }

  // local lattice tables of a block: boundary slots and interior ranks
  bslot_tab.assign((q + 1) * (q + 1) * (q + 1), -1);
  std::vector<int> &bslot = bslot_tab;
  std::vector<int> irank((q + 1) * (q + 1) * (q + 1), -1);
  {
    int nb = 0, ni = 0;
    for (int z = 0; z <= q; ++z)
      for (int y = 0; y <= q; ++y)
        for (int x = 0; x <= q; ++x) {
          int id = (z * (q + 1) + y) * (q + 1) + x;
          if (on_block_boundary(x, y, z, q)) bslot[id] = nb++;
          else if (x == p || y == p || z == p) irank[id] = ni++;
        }
  }
  const int nIlat = nI - 3 * q * q;

  const int64_t nblk = (int64_t)Nc * Nc * Nc;
  blkB.assign(nblk * nBf, -1);
  blkI.assign(nblk * nI, -1);
  for (int ck = 0; ck < Nc; ++ck)
    for (int cj = 0; cj < Nc; ++cj)
      for (int ci = 0; ci < Nc; ++ci) {
        int64_t b = ci + (int64_t)Nc * (cj + (int64_t)Nc * ck);
        int32_t *B = &blkB[b * nBf];
        int32_t *I = &blkI[b * nI];
        for (int z = 0; z <= q; ++z)
          for (int y = 0; y <= q; ++y)
            for (int x = 0; x <= q; ++x) {
              int id = (z * (q + 1) + y) * (q + 1) + x;
              int64_t t = fine.h1(q * ci + x, q * cj + y, q * ck + z);
              if (bslot[id] >= 0) B[bslot[id]] = (int32_t)t;
              else if (irank[id] >= 0) I[irank[id]] = (int32_t)t;
            }
        const int cell[3] = {ci, cj, ck};
        for (int d = 0; d < 3; ++d) {
          const int a1 = d == 0 ? 1 : 0, a2 = d == 2 ? 1 : 2;
          for (int side = 0; side < 2; ++side) {
            int s = 2 * cell[d] + 2 * side;
            for (int t2 = 0; t2 < q; ++t2)
              for (int t1 = 0; t1 < q; ++t1) {
                int slot = nlat + (2 * d + side) * q * q + t2 * q + t1;
                B[slot] = (s > 0 && s < N)
                              ? (int32_t)fine.flux(d, s, q * cell[a1] + t1, q * cell[a2] + t2)
                              : -1;
              }
          }
          int s = 2 * cell[d] + 1;
          for (int t2 = 0; t2 < q; ++t2)
            for (int t1 = 0; t1 < q; ++t1)
              I[nIlat + d * q * q + t2 * q + t1] =
                  (int32_t)fine.flux(d, s, q * cell[a1] + t1, q * cell[a2] + t2);
        }
      }
  blkB_ptr.assign(nblk + 1, 0);
  blkB_present.clear();
  for (int64_t b = 0; b < nblk; ++b) {
    for (int s = 0; s < nBf; ++s)
      if (blkB[b * nBf + s] >= 0) blkB_present.push_back(s);
    blkB_ptr[b + 1] = (int64_t)blkB_present.size();
  }

  // child local dof -> [B slots | I] position
  child_map.assign(8 * el.n_tr, -1);
  for (int c = 0; c < 8; ++c) {
    int ca = c & 1, cb = (c >> 1) & 1, cc = (c >> 2) & 1;
    int32_t *m = &child_map[c * el.n_tr];
    for (int k = 0; k < el.n_h1; ++k) {
      int x = ca * p + el.lat[3 * k], y = cb * p + el.lat[3 * k + 1], z = cc * p + el.lat[3 * k + 2];
      int id = (z * (q + 1) + y) * (q + 1) + x;
      m[k] = bslot[id] >= 0 ? bslot[id] : nBf + irank[id];
    }
    const int off[3] = {ca, cb, cc};
    int o = el.n_h1;
    for (int d = 0; d < 3; ++d) {
      const int a1 = d == 0 ? 1 : 0, a2 = d == 2 ? 1 : 2;
      for (int s = 0; s < 2; ++s) {
        int plane = off[d] + s;  // 0, 1 or 2 in child units
        for (int n = 0; n < p; ++n)
          for (int mm = 0; mm < p; ++mm, ++o) {
            int t1 = off[a1] * p + mm, t2 = off[a2] * p + n;
            if (plane == 1) m[o] = nBf + nIlat + d * q * q + t2 * q + t1;
            else m[o] = nlat + (2 * d + (plane == 2 ? 1 : 0)) * q * q + t2 * q + t1;
          }
      }
    }
  }

  // vertex patches: support interval [lo, hi] of coarse cells per axis
  const int64_t nv = (int64_t)(Nc + 1) * (Nc + 1) * (Nc + 1);
  std::vector<int64_t> cnt(nv + 1, 0);
  auto interval = [&](int64_t t, int lo[3], int hi[3]) {
    int kind, c[3];
    fine.describe(t, kind, c);
    if (kind == 0) {
      for (int a = 0; a < 3; ++a) {
        int X = c[a];
        if (X % q == 0) {
          lo[a] = std::max(X / q - 1, 0);
          hi[a] = std::min(X / q, Nc - 1);
        } else {
          lo[a] = hi[a] = X / q;
        }
      }
    } else {
      int d = kind - 1;
      const int a1 = d == 0 ? 1 : 0, a2 = d == 2 ? 1 : 2;
      lo[d] = c[0] / 2 - 1;
      hi[d] = c[0] / 2;
      lo[a1] = hi[a1] = c[1] / q;
      lo[a2] = hi[a2] = c[2] / q;
    }
  };
  std::vector<int> LO(3 * nM), HI(3 * nM);
  for (int64_t m = 0; m < nM; ++m) interval(macro_B[m], &LO[3 * m], &HI[3 * m]);
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int64_t> fill;
    if (pass == 1) {
      patch_ptr.assign(nv + 1, 0);
      for (int64_t v = 0; v < nv; ++v) patch_ptr[v + 1] = patch_ptr[v] + cnt[v];
      patch_idx.assign(patch_ptr[nv], -1);
      fill.assign(patch_ptr.begin(), patch_ptr.end() - 1);
    }
    for (int64_t m = 0; m < nM; ++m) {
      const int *lo = &LO[3 * m], *hi = &HI[3 * m];
      for (int vz = hi[2]; vz <= lo[2] + 1 && vz <= Nc; ++vz)
        for (int vy = hi[1]; vy <= lo[1] + 1 && vy <= Nc; ++vy)
          for (int vx = hi[0]; vx <= lo[0] + 1 && vx <= Nc; ++vx) {
            int64_t v = ((int64_t)vz * (Nc + 1) + vy) * (Nc + 1) + vx;
            if (pass == 0) cnt[v]++;
            else patch_idx[fill[v]++] = (int32_t)m;
          }
    }
  }
  patch_slot.assign(patch_idx.size() * 8, -1);
  for (int64_t v = 0; v < nv; ++v) {
    int vx = (int)(v % (Nc + 1)), vy = (int)((v / (Nc + 1)) % (Nc + 1)), vz = (int)(v / ((Nc + 1) * (Nc + 1)));
    for (int64_t k = patch_ptr[v]; k < patch_ptr[v + 1]; ++k) {
      int64_t t = macro_B[patch_idx[k]];
      for (int c = 0; c < 8; ++c) {
        int ci = vx - 1 + (c & 1), cj = vy - 1 + ((c >> 1) & 1), ck = vz - 1 + ((c >> 2) & 1);
        if (ci < 0 || cj < 0 || ck < 0 || ci >= Nc || cj >= Nc || ck >= Nc) continue;
        patch_slot[k * 8 + c] = slot_in_block(fine, t, ci, cj, ck);
      }
    }
  }
}

// Position of lattice point (a, b, c) of [0, p]^3 in an element's local layout.
static std::vector<int> lattice_positions(const ElementLayout &el) {
  const int p = el.p;
  std::vector<int> pos((p + 1) * (p + 1) * (p + 1), -1);
  for (int k = 0; k < el.n_h1; ++k)
    pos[(el.lat[3 * k + 2] * (p + 1) + el.lat[3 * k + 1]) * (p + 1) + el.lat[3 * k]] = k;
  return pos;
}

void MacroLevel::build_order(const Numbering &num, const ElementLayout &el) {
  N = num.N;
  p = num.p;
  Nc = N;
  nBf = el.n_tr;
  nI = 0;
  nM = num.n;
  macro_of.resize(num.n);
  macro_B.resize(num.n);
  for (int64_t t = 0; t < num.n; ++t) {
    macro_of[t] = (int32_t)t;
    macro_B[t] = t;
  }
  blkB = element_dofs(num, el);
  blkI.clear();
  child_map.clear();
  bslot_tab.clear();
  const int64_t nblk = (int64_t)N * N * N;
  blkB_ptr.assign(nblk + 1, 0);
  blkB_present.clear();
  for (int64_t b = 0; b < nblk; ++b) {
    std::vector<std::pair<int32_t, int32_t>> pres;   // (canonical index, local slot)
    for (int s = 0; s < nBf; ++s)
      if (blkB[b * nBf + s] >= 0) pres.push_back({blkB[b * nBf + s], s});
    std::sort(pres.begin(), pres.end());
    for (auto &e : pres) blkB_present.push_back(e.second);
    blkB_ptr[b + 1] = (int64_t)blkB_present.size();
  }
  // support intervals of every unknown, in elements per axis
  const std::vector<int> lpos = lattice_positions(el);
  const int64_t nv = (int64_t)(N + 1) * (N + 1) * (N + 1);
  std::vector<int> LO(3 * nM), HI(3 * nM);
  for (int64_t t = 0; t < nM; ++t) {
    int kind, c[3];
    num.describe(t, kind, c);
    int *lo = &LO[3 * t], *hi = &HI[3 * t];
    if (kind == 0) {
      for (int a = 0; a < 3; ++a) {
        if (c[a] % p == 0) {
          lo[a] = std::max(c[a] / p - 1, 0);
          hi[a] = std::min(c[a] / p, N - 1);
        } else {
          lo[a] = hi[a] = c[a] / p;
        }
      }
    } else {
      const int d = kind - 1, a1 = d == 0 ? 1 : 0, a2 = d == 2 ? 1 : 2;
      lo[d] = c[0] - 1;
      hi[d] = c[0];
      lo[a1] = hi[a1] = c[1] / p;
      lo[a2] = hi[a2] = c[2] / p;
    }
  }
  std::vector<int64_t> cnt(nv + 1, 0);
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int64_t> fill;
    if (pass == 1) {
      patch_ptr.assign(nv + 1, 0);
      for (int64_t v = 0; v < nv; ++v) patch_ptr[v + 1] = patch_ptr[v] + cnt[v];
      patch_idx.assign(patch_ptr[nv], -1);
      fill.assign(patch_ptr.begin(), patch_ptr.end() - 1);
    }
    for (int64_t m = 0; m < nM; ++m) {
      const int *lo = &LO[3 * m], *hi = &HI[3 * m];
      for (int vz = hi[2]; vz <= lo[2] + 1 && vz <= N; ++vz)
        for (int vy = hi[1]; vy <= lo[1] + 1 && vy <= N; ++vy)
          for (int vx = hi[0]; vx <= lo[0] + 1 && vx <= N; ++vx) {
            const int64_t v = ((int64_t)vz * (N + 1) + vy) * (N + 1) + vx;
            if (pass == 0) cnt[v]++;
            else patch_idx[fill[v]++] = (int32_t)m;
          }
    }
  }
  // local slot of unknown t in element (ci, cj, ck), or -1
  auto local_slot = [&](int64_t t, const int cell[3]) -> int {
    int kind, c[3];
    num.describe(t, kind, c);
    if (kind == 0) {
      int l[3];
      for (int a = 0; a < 3; ++a) {
        l[a] = c[a] - p * cell[a];
        if (l[a] < 0 || l[a] > p) return -1;
      }
      return lpos[(l[2] * (p + 1) + l[1]) * (p + 1) + l[0]];
    }
    const int d = kind - 1, a1 = d == 0 ? 1 : 0, a2 = d == 2 ? 1 : 2;
    int side;
    if (c[0] == cell[d]) side = 0;
    else if (c[0] == cell[d] + 1) side = 1;
    else return -1;
    const int t1 = c[1] - p * cell[a1], t2 = c[2] - p * cell[a2];
    if (t1 < 0 || t1 >= p || t2 < 0 || t2 >= p) return -1;
    return el.n_h1 + (2 * d + side) * p * p + t2 * p + t1;
  };
  patch_slot.assign(patch_idx.size() * 8, -1);
  for (int64_t v = 0; v < nv; ++v) {
    const int vx = (int)(v % (N + 1)), vy = (int)((v / (N + 1)) % (N + 1)),
              vz = (int)(v / ((int64_t)(N + 1) * (N + 1)));
    for (int64_t k = patch_ptr[v]; k < patch_ptr[v + 1]; ++k)
      for (int c = 0; c < 8; ++c) {
        const int cell[3] = {vx - 1 + (c & 1), vy - 1 + ((c >> 1) & 1), vz - 1 + ((c >> 2) & 1)};
        if (cell[0] < 0 || cell[1] < 0 || cell[2] < 0 || cell[0] >= N || cell[1] >= N ||
            cell[2] >= N)
          continue;
        patch_slot[k * 8 + c] = local_slot(patch_idx[k], cell);
      }
  }
}

// ---------------------------------------------------------------------------
// prolongation

void Prolongation::build_order(const MacroLevel &mc, const Numbering &fine,
                               const Numbering &coarse, const ElementLayout &el_fine,
                               const ElementLayout &el_coarse) {
  const int q = fine.p, qc = coarse.p;
  if (qc != q - 1 || coarse.N != fine.N) throw std::runtime_error("order level mismatch");
  // fine 1-D local index of a coarse one: a vertex stays a vertex, bubble a'
  // is the same function at index a' (the highest fine bubble has no source)
  auto up = [&](int Xc) { return q * (Xc / qc) + Xc % qc; };
  ptr.assign(mc.nM + 1, 0);
  std::vector<int32_t> src(fine.n, -1);   // coarse unknown injected into each fine one
  for (int64_t tc = 0; tc < coarse.n; ++tc) {
    int kind, c[3];
    coarse.describe(tc, kind, c);
    int64_t t;
    if (kind == 0) t = fine.h1(up(c[0]), up(c[1]), up(c[2]));
    else t = fine.flux(kind - 1, c[0], up(c[1]), up(c[2]));
    if (t < 0) throw std::runtime_error("order injection: no fine unknown");
    src[t] = (int32_t)tc;
  }
  col.clear();
  val.clear();
  for (int64_t m = 0; m < mc.nM; ++m) {
    if (src[m] >= 0) {
      col.push_back(src[m]);
      val.push_back(1.0);
    }
    ptr[m + 1] = (int64_t)col.size();
  }
  tptr.assign(coarse.n + 1, 0);
  for (int32_t cidx : col) tptr[cidx + 1]++;
  for (int64_t i = 0; i < coarse.n; ++i) tptr[i + 1] += tptr[i];
  tcol.assign(col.size(), 0);
  tval.assign(col.size(), 0.0);
  std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
  for (int64_t m = 0; m < mc.nM; ++m)
    for (int64_t k = ptr[m]; k < ptr[m + 1]; ++k) {
      const int64_t dst = fill[col[k]]++;
      tcol[dst] = (int32_t)m;
      tval[dst] = val[k];
    }
  // element-local injection, [n_tr(coarse)] columns of nBf = n_tr(fine) rows
  const std::vector<int> lpos = lattice_positions(el_fine);
  local.assign((int64_t)mc.nBf * el_coarse.n_tr, 0.0);
  auto upl = [&](int a) { return a == qc ? q : a; };
  for (int k = 0; k < el_coarse.n_h1; ++k) {
    const int kf = lpos[(upl(el_coarse.lat[3 * k + 2]) * (q + 1) + upl(el_coarse.lat[3 * k + 1])) *
                            (q + 1) +
                        upl(el_coarse.lat[3 * k])];
    local[(int64_t)k * mc.nBf + kf] = 1.0;
  }
  for (int f = 0; f < 6; ++f)
    for (int n = 0; n < qc; ++n)
      for (int m = 0; m < qc; ++m) {
        const int kc = el_coarse.n_h1 + f * qc * qc + n * qc + m;
        const int kf = el_fine.n_h1 + f * q * q + n * q + m;
        local[(int64_t)kc * mc.nBf + kf] = 1.0;
      }
}

void Prolongation::build(const MacroLevel &mc, const Numbering &fine, const Numbering &coarse,
                         const ElementLayout &el) {
  const int p = mc.p, q = 2 * p, Nc = mc.Nc;
  std::vector<double> R1 = twoscale_h1(p), R0 = twoscale_leg(p);
  auto r1 = [&](int row, int col) { return R1[row * (p + 1) + col]; };
  auto r0 = [&](int row, int col) { return R0[row * p + col]; };
  ptr.assign(mc.nM + 1, 0);
  col.clear();
  val.clear();
  for (int64_t m = 0; m < mc.nM; ++m) {
    int kind, c[3];
    fine.describe(mc.macro_B[m], kind, c);
    std::vector<std::pair<int32_t, double>> ent;
    if (kind == 0) {
      int cell[3], loc[3];
      for (int a = 0; a < 3; ++a) {
        cell[a] = std::min(c[a] / q, Nc - 1);
        loc[a] = c[a] - q * cell[a];
      }
      for (int cz = 0; cz <= p; ++cz) {
        double vz = r1(loc[2], cz);
        if (vz == 0.0) continue;
        for (int cy = 0; cy <= p; ++cy) {
          double vy = r1(loc[1], cy);
          if (vy == 0.0) continue;
          for (int cx = 0; cx <= p; ++cx) {
            double vx = r1(loc[0], cx);
            if (vx == 0.0) continue;
            int64_t ct = coarse.h1(p * cell[0] + cx, p * cell[1] + cy, p * cell[2] + cz);
            if (ct < 0) continue;  // coarse interior bubble: not a trace unknown
            ent.push_back({(int32_t)ct, vx * vy * vz});
          }
        }
      }
    } else {
      int d = kind - 1;
      int f1 = c[1] / p, f2 = c[2] / p;
      int row1 = (f1 % 2) * p + c[1] % p, row2 = (f2 % 2) * p + c[2] % p;
      for (int n = 0; n < p; ++n) {
        double v2 = r0(row2, n);
        if (v2 == 0.0) continue;
        for (int mm = 0; mm < p; ++mm) {
          double v1 = r0(row1, mm);
          if (v1 == 0.0) continue;
          ent.push_back({(int32_t)coarse.flux(d, c[0] / 2, (f1 / 2) * p + mm, (f2 / 2) * p + n),
                         v1 * v2});
        }
      }
    }
    std::sort(ent.begin(), ent.end());
    for (auto &e : ent) {
      col.push_back(e.first);
      val.push_back(e.second);
    }
    ptr[m + 1] = (int64_t)col.size();
  }
  // transpose
  tptr.assign(coarse.n + 1, 0);
  for (int32_t cidx : col) tptr[cidx + 1]++;
  for (int64_t i = 0; i < coarse.n; ++i) tptr[i + 1] += tptr[i];
  tcol.assign(col.size(), 0);
  tval.assign(col.size(), 0.0);
  std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
  for (int64_t m = 0; m < mc.nM; ++m)
    for (int64_t k = ptr[m]; k < ptr[m + 1]; ++k) {
      int64_t dst = fill[col[k]]++;
      tcol[dst] = (int32_t)m;
      tval[dst] = val[k];
    }
  // dense local P of one coarse element: [nBf x n_tr], column-major
  const int nlat = (q + 1) * (q + 1) * (q + 1) - (q - 1) * (q - 1) * (q - 1);
  local.assign((int64_t)mc.nBf * el.n_tr, 0.0);
  int slot = 0;
  for (int z = 0; z <= q; ++z)
    for (int y = 0; y <= q; ++y)
      for (int x = 0; x <= q; ++x) {
        if (!on_block_boundary(x, y, z, q)) continue;
        for (int k = 0; k < el.n_h1; ++k)
          local[(int64_t)k * mc.nBf + slot] =
              r1(x, el.lat[3 * k]) * r1(y, el.lat[3 * k + 1]) * r1(z, el.lat[3 * k + 2]);
        ++slot;
      }
  for (int f = 0; f < 6; ++f)
    for (int t2 = 0; t2 < q; ++t2)
      for (int t1 = 0; t1 < q; ++t1) {
        int s = nlat + f * q * q + t2 * q + t1;
        for (int n = 0; n < p; ++n)
          for (int mm = 0; mm < p; ++mm) {
            int k = el.n_h1 + f * p * p + n * p + mm;
            local[(int64_t)k * mc.nBf + s] = r0(t1, mm) * r0(t2, n);
          }
      }
}

}  // namespace dpg
