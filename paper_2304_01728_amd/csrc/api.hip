// C ABI of libdpgmg (include/dpgmg.h): setup, element stage, hierarchy,
// preconditioned CG with the DPG-MG V-cycle, exports.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "ctx.hpp"

using namespace dpg;

// Scratch of dpg_solve_noalloc: the reduction partials (2 kDotBlocks doubles)
// and the eight CG scalars of the column being solved.  Each GPU the library
// runs on holds one copy until the process ends.  Host code never uses this
// name as an address: dpg_setup looks up the device address once per device
// (scratch_device_ptr) and the kernels receive that pointer.
constexpr int kScratchDoubles = 2 * kDotBlocks + 8;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on device dev, which must be the current device
// on the first call for it.
double *scratch_device_ptr(int dev, bool resolve) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) throw DpgError(DPG_EDEVICE, "device index out of range");
  if (!g_scratch[dev] && resolve) {
    void *ptr = nullptr;
    HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw DpgError(DPG_EDEVICE, "no device address for the solve scratch");
    g_scratch[dev] = static_cast<double *>(ptr);
  }
  return g_scratch[dev];
}
}  // namespace

namespace {

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) {
  return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

// LAPACK-style flop counts of complex double routines
double f_potrf(double n) { return 4.0 / 3.0 * n * n * n; }
double f_trsm(double n, double k) { return 4.0 * n * n * k; }
double f_gemm(double m, double n, double k) { return 8.0 * m * n * k; }
double f_herk(double n, double k) { return 4.0 * n * n * k; }   // Hermitian product, one triangle

#define PROF(cls, work) ProfScope _prof_scope(&c->prof, (cls), (double)(work), c->stream)

template <class F> int guarded(dpg_ctx *c, F &&f) {
  try {
    return f();
  } catch (const DpgError &e) {
    if (c) c->err = e.what();
    return e.code;
  } catch (const std::exception &e) {
    if (c) c->err = e.what();
    return DPG_EINVAL;
  }
}

// Mesh sizes from finest to coarsest: halve while N is even and N > 2; a
// mesh with N = 2 is halved once.
std::vector<int> level_sizes(int N, int nlevels) {
  std::vector<int> s{N};
  while (N % 2 == 0 && (N > 2 || s.size() == 1)) {
    N /= 2;
    s.push_back(N);
  }
  if (nlevels > 0 && (int)s.size() > nlevels) s.resize(nlevels);
  return s;
}

// Boundary load points of the finest mesh: 6 N^2 faces of nql^2 points.
int64_t boundary_points(const dpg_ctx *c) {
  return 6LL * c->N * c->N * c->tables_h.nql * c->tables_h.nql;
}

// (mesh size, order) of every level, finest first: with 1 <= p_min < p the
// order is lowered on the finest mesh one step at a time down to p_min
// (order levels), then the mesh is halved (level_sizes).
std::vector<std::pair<int, int>> level_plan(int N, int p, int p_min, int nlevels) {
  std::vector<std::pair<int, int>> plan;
  const int pm = p_min > 0 ? p_min : p;
  for (int q = p; q > pm; --q) plan.push_back({N, q});
  for (int n : level_sizes(N, 0)) plan.push_back({n, pm});
  if (nlevels > 0 && (int)plan.size() > nlevels) plan.resize(nlevels);
  return plan;
}

void set_loads(dpg_ctx *c, const dpg_load *loads, int nrhs) {
  c->nrhs = nrhs;
  c->ld_h.assign(nrhs, LoadDesc{});
  c->src_h.clear();
  std::vector<double2> u0;
  const int64_t nbp = boundary_points(c);
  for (int r = 0; r < nrhs; ++r) {
    LoadDesc &d = c->ld_h[r];
    d.u0_off = -1;
    if (loads[r].u0_qp) {
      d.u0_off = (int64_t)u0.size();
      for (int64_t k = 0; k < nbp; ++k) {
        const double2 v = mk(loads[r].u0_qp[2 * k], loads[r].u0_qp[2 * k + 1]);
        if (!std::isfinite(v.x) || !std::isfinite(v.y))
          throw DpgError(DPG_EINVAL, "impedance data at the boundary points is not finite");
        u0.push_back(v);
      }
    }
    for (int k = 0; k < 3; ++k) d.dir[k] = loads[r].dir[k];
    d.amp[0] = loads[r].amp[0];
    d.amp[1] = loads[r].amp[1];
    d.src0 = (int)(c->src_h.size() / 6);
    d.nsrc = loads[r].nsrc;
    if (d.nsrc < 0 || (d.nsrc > 0 && !loads[r].src)) throw DpgError(DPG_EINVAL, "bad source list");
    for (int k = 0; k < 6 * d.nsrc; ++k) c->src_h.push_back(loads[r].src[k]);
    for (int k = 0; k < d.nsrc; ++k)
      if (!(loads[r].src[6 * k + 3] > 0.0)) throw DpgError(DPG_EINVAL, "source width must be > 0");
  }
  c->ld.upload(c->ld_h, &c->bud, c->stream);
  if (u0.empty()) c->u0q.release();
  else c->u0q.upload(u0, &c->bud, c->stream);
  if (c->src_h.empty()) c->src_h.push_back(0.0);
  c->src.upload(c->src_h, &c->bud, c->stream);
  HIP_OK(hipStreamSynchronize(c->stream));
}

// Elements that a new set of loads needs.  Returns true (all elements) unless
// every load consists of Gaussian point sources only; then list receives the
// elements whose box comes within 8 sigma of some source (ascending).  Beyond
// 8 sigma the density is below exp(-32) = 1.3e-14 of its peak and the mass
// outside that ball below 1e-13 of the total, so the omitted element loads are
// below the rounding of the kept ones.  Also true when the list would cover
// most of the mesh.
bool source_elements(const dpg_ctx *c, std::vector<int32_t> &list) {
  list.clear();
  for (const LoadDesc &d : c->ld_h)
    if (d.amp[0] != 0.0 || d.amp[1] != 0.0 || d.u0_off >= 0) return true;
  const int N = c->N;
  const double h = c->side / N;
  std::vector<char> mark((size_t)N * N * N, 0);
  for (size_t k = 0; 6 * k + 5 < c->src_h.size(); ++k) {
    const double *S = c->src_h.data() + 6 * k;   // (x, y, z, sigma > 0, re a, im a)
    const double R = 8.0 * S[3];
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::max(0, (int)std::floor((S[d] - R - c->org[d]) / h));
      hi[d] = std::min(N - 1, (int)std::floor((S[d] + R - c->org[d]) / h));
    }
    for (int kz = lo[2]; kz <= hi[2]; ++kz)
      for (int jy = lo[1]; jy <= hi[1]; ++jy)
        for (int ix = lo[0]; ix <= hi[0]; ++ix) {
          const int cell[3] = {ix, jy, kz};
          double d2 = 0.0;   // squared distance from the centre to the element box
          for (int d = 0; d < 3; ++d) {
            const double a = c->org[d] + h * cell[d], b = a + h;
            const double t = S[d] < a ? a - S[d] : S[d] > b ? S[d] - b : 0.0;
            d2 += t * t;
          }
          if (d2 <= R * R) mark[ix + (size_t)N * (jy + (size_t)N * kz)] = 1;
        }
  }
  for (size_t e = 0; e < mark.size(); ++e)
    if (mark[e]) list.push_back((int32_t)e);
  return 4 * list.size() > 3 * mark.size();
}

// Throws DPG_ENOTPD for the first item whose Cholesky met a non-positive
// pivot (info[i] = j + 1 for pivot j of item i).
void check_infos(const int *info, int64_t count, hipStream_t s, const char *what) {
  if (count <= 0) return;
  std::vector<int> h(count);
  HIP_OK(hipMemcpyAsync(h.data(), info, count * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  for (int64_t i = 0; i < count; ++i)
    if (h[i] != 0)
      throw DpgError(DPG_ENOTPD, std::string(what) + " " + std::to_string(i) +
                                     ": Cholesky pivot " + std::to_string(h[i] - 1) +
                                     " is not positive");
}

// Make stream b wait for everything queued on stream a so far.
void stream_wait(hipStream_t a, hipStream_t b, hipEvent_t ev) {
  HIP_OK(hipEventRecord(ev, a));
  HIP_OK(hipStreamWaitEvent(b, ev, 0));
}

// ---- element stage -----------------------------------------------------------------

// Grow-only device buffer: reallocated only when more room is needed, so
// that plans for meshes of different sizes share the largest allocation.
template <typename T> void grow(DevBuf<T> &b, int64_t n, Budget *bd) {
  if (b.n < n) b.alloc(n, bd);
}

// Element-stage plan for nel elements with nr load columns.
void plan_elements(dpg_ctx *c, int nel, int nr) {
  ElemPlan &P = c->ep;
  const int nt = c->n_test, nf = c->n_field, mp = c->m + nr;
  if (P.mp == mp && P.nel == nel) return;
  const int64_t per = 16LL * ((int64_t)nt * nt + (int64_t)nt * mp + (int64_t)mp * mp);
  // a multiple of NS about equal chunks, so that every stream gets the same
  // work; element stage at 16^3 / p = 3 over two streams 38.4 ms, three 37.8,
  // four 37.2
  const int NS = 4;
  const int64_t cmax = std::max<int64_t>(1, std::min<int64_t>(2500000000LL / per, 65535));
  const int64_t groups = (nel + NS * cmax - 1) / (NS * cmax);
  const int C = (int)std::max<int64_t>(1, (nel + NS * groups - 1) / (NS * groups));
  P.ns = NS;
  Budget *bd = &c->bud;
  for (int k = 0; k < NS; ++k) {
    grow(P.G[k], (int64_t)C * nt * nt, bd);
    grow(P.BL[k], (int64_t)C * nt * mp, bd);
    grow(P.K[k], (int64_t)C * mp * mp, bd);
    grow(P.wk[k], dense_work_size(C, nt), bd);
  }
  std::vector<PotrfItem> pG(C), pK(C);
  std::vector<TrsmItem> tG(C), tK(C);
  std::vector<GemmItem> gK(C), gS(C);
  for (int i = 0; i < C; ++i) {
    const int64_t oG = (int64_t)i * nt * nt, oB = (int64_t)i * nt * mp, oK = (int64_t)i * mp * mp;
    pG[i] = {oG, nt, nt};
    tG[i] = {oG, oB, nt, mp, nt, nt};
    gK[i] = {oB, oB, oK, mp, mp, nt, nt, nt, mp};
    pK[i] = {oK, nf, mp};
    tK[i] = {oK, oK + (int64_t)nf * mp, nf, mp - nf, mp, mp};
    gS[i] = {oK + (int64_t)nf * mp, oK + (int64_t)nf * mp, oK + nf + (int64_t)nf * mp,
             mp - nf, mp - nf, nf, mp, mp, mp};
  }
  P.pG.upload(pG, bd, c->stream);
  P.pK.upload(pK, bd, c->stream);
  P.tG.upload(tG, bd, c->stream);
  P.tK.upload(tK, bd, c->stream);
  P.gK.upload(gK, bd, c->stream);
  P.gS.upload(gS, bd, c->stream);
  grow(P.info, 2LL * nel, bd);
  HIP_OK(hipStreamSynchronize(c->stream));
  P.C = C;
  P.mp = mp;
  P.nel = nel;
}

// Error-indicator pass of the element stage: trace solutions x (nr <= the
// context's loads columns of n_trace entries, device) and the output
// eta2 [nr][nel] (device).
struct IndicatorArgs {
  const double2 *x;
  int nr;
  double *eta2;
};

// Per element (Sec. 1.2): Gram matrix G and [B | l]; G = L L^H;
// W = L^-1 [B | l]; K = W^H W; static condensation of the field block of K.
// Chunks of elements are dealt round-robin to four streams.  Level L (the
// finest mesh) with the context's loads; a coarser level l < L (the "store"
// coarse operators) with no loads, writing only its element matrices.
// With ind (finest level only), the pass computes the DPG residual error
// indicator instead of condensing: after K_ff = L_f L_f^H and
// Y = L_f^-1 [K_ft | b], the unknowns [x_f; x_t] of every element
// (x_f = L_f^-H (Y_b - Y_t x_t)), the residual W_l - W_B [x_f; x_t] =
// L^-1 (l - B [x_f; x_t]), and eta^2 = its squared norm = r^H G^-1 r.
// With elist (device, nlist entries; finest level, loads only), the pass
// covers only the listed elements and writes their condensed loads (the
// caller zeroes the others).
void element_stage(dpg_ctx *c, int l, bool write_matrices, const IndicatorArgs *ind = nullptr,
                   const int32_t *elist = nullptr, int nlist = 0) {
  const bool fine = l == c->L;
  LevelData &f = c->lv[l];
  const int nr = fine ? c->nrhs : 0;
  plan_elements(c, f.nel, nr);
  ElemPlan &P = c->ep;
  const int nt = c->n_test, nf = c->n_field, ntr = c->n_tr, m = c->m;
  const int mp = m + nr, C = P.C, nel = f.nel;
  if (elist && (!fine || ind || write_matrices))
    throw DpgError(DPG_EINVAL, "element lists are for load updates only");
  const int total = elist ? nlist : nel;
  if (ind) {
    if (!fine || ind->nr < 1 || ind->nr > nr) throw DpgError(DPG_EINVAL, "bad indicator columns");
    for (int k = 0; k < P.ns; ++k) grow(P.X[k], (int64_t)C * m * ind->nr, &c->bud);
    if (P.gR_nr != ind->nr || P.gR_C != C) {
      std::vector<GemmItem> gR(C);
      for (int i = 0; i < C; ++i)
        gR[i] = {(int64_t)i * nt * mp, (int64_t)i * m * ind->nr, (int64_t)i * nt * mp + (int64_t)m * nt,
                 nt, ind->nr, m, nt, m, nt};
      P.gR.upload(gR, &c->bud, c->stream);
      HIP_OK(hipStreamSynchronize(c->stream));
      P.gR_nr = ind->nr;
      P.gR_C = C;
    }
  }
  const double *kap = fine ? c->kappa.p : f.kappa.p, *Zel = fine ? c->Zel.p : f.Zel.p;
  ElemGeom g{f.N, c->side / f.N, c->omega, 1.0, {c->org[0], c->org[1], c->org[2]}, elist};
  // one stream while kernels are profiled, so that each launch's events time it alone
  const int NS = c->prof.on ? 1 : P.ns;
  const hipStream_t xs[4] = {c->stream, c->aux, c->paux[0], c->paux[1]};
  const DenseProf dG{&c->prof, nullptr, nt, nullptr, mp}, dK{&c->prof, nullptr, nf, nullptr, mp - nf};
  const hipEvent_t xj[4] = {nullptr, c->ev_join, c->ev_pjoin[0], c->ev_pjoin[1]};
  for (int k = 1; k < NS; ++k) stream_wait(c->stream, xs[k], c->ev_fork);
  for (int e0 = 0, k = 0; e0 < total; e0 += C, ++k) {
    const int cnt = std::min(C, total - e0), u = k % NS;
    const hipStream_t s = xs[u];
    double2 *G = P.G[u].p, *BL = P.BL[u].p, *K = P.K[u].p, *wk = P.wk[u].p;
    {
      ProfScope ps(&c->prof, DPG_K_GRAM, 0, s);
      launch_gram(c->tables.p, c->testd.p, nt, g, kap, e0, cnt, G, s);
    }
    {
      ProfScope ps(&c->prof, DPG_K_BMAT, 0, s);
      launch_bmat(c->tables.p, c->testd.p, c->triald.p, nt, m, g, kap, Zel, e0, cnt,
                  BL, (int64_t)nt * mp, s);
    }
    if (nr > 0) {
      ProfScope ps(&c->prof, DPG_K_LOAD, 0, s);
      launch_load(c->tables.p, nt, m, g, Zel, c->ld.p, c->src.p, c->u0q.p, nr, e0, cnt, BL,
                  (int64_t)nt * mp, s);
    }
    {
      ProfScope ps(&c->prof, DPG_K_POTRF, cnt * f_potrf(nt), s);
      potrf_batched(G, P.pG.p, cnt, P.info.p + e0, nt, wk, s, &dG);
    }
    {
      ProfScope ps(&c->prof, DPG_K_TRSM, cnt * f_trsm(nt, mp), s);
      trsm_batched(G, BL, P.tG.p, cnt, nt, mp, false, wk, true, s, &dG);
    }
    {
      ProfScope ps(&c->prof, DPG_K_GEMM, cnt * f_herk(mp, nt), s);
      gemm_batched(OP_C, OP_N, mk(1, 0), BL, BL, mk(0, 0), K, P.gK.p, cnt, mp, mp, s, GEMM_HERM);
    }
    {
      ProfScope ps(&c->prof, DPG_K_POTRF, cnt * f_potrf(nf), s);
      potrf_batched(K, P.pK.p, cnt, P.info.p + nel + e0, nf, wk, s, &dK);
    }
    {
      ProfScope ps(&c->prof, DPG_K_TRSM, cnt * f_trsm(nf, mp - nf), s);
      trsm_batched(K, K, P.tK.p, cnt, nf, mp - nf, false, wk, true, s, &dK);
    }
    if (ind) {
      const int q = ind->nr;
      const int64_t nT = f.num.n;
      {
        ProfScope ps(&c->prof, DPG_K_OTHER, 0, s);
        launch_indicator_x(K, (int64_t)mp * mp, mp, nf, ntr, q, f.edofs.p + (int64_t)e0 * ntr, cnt,
                           ind->x, nT, P.X[u].p, s);
      }
      {
        ProfScope ps(&c->prof, DPG_K_GEMM, cnt * f_gemm(nt, q, m), s);
        gemm_batched(OP_N, OP_N, mk(-1, 0), BL, P.X[u].p, mk(1, 0), BL, P.gR.p, cnt, nt, q, s);
      }
      ProfScope ps(&c->prof, DPG_K_OTHER, 0, s);
      launch_colnorm2(BL, (int64_t)nt * mp, nt, nt, m, q, e0, cnt, nel, ind->eta2, s);
      continue;
    }
    {
      ProfScope ps(&c->prof, DPG_K_GEMM, cnt * f_herk(mp - nf, nf), s);
      gemm_batched(OP_C, OP_N, mk(-1, 0), K, K, mk(1, 0), K, P.gS.p, cnt, mp - nf, mp - nf, s,
                   GEMM_HERM);
    }
    if (write_matrices)
      launch_copy_sub(K, (int64_t)mp * mp, mp, nf, nf, ntr, ntr, f.E.p + (int64_t)e0 * ntr * ntr,
                      (int64_t)ntr * ntr, ntr, cnt, s);
    const int32_t *dl = elist ? elist + e0 : nullptr;   // destination elements
    const int64_t eo = elist ? 0 : e0;
    for (int r = 0; r < nr; ++r)
      launch_copy_sub(K, (int64_t)mp * mp, mp, nf, m + r, ntr, 1,
                      c->s_elem.p + ((int64_t)r * nel + eo) * ntr, ntr, ntr, cnt, s, dl);
    if (fine && c->keep_recovery) {
      if (write_matrices) {   // L = chol(K_ff) and Y_t = L^-1 K_ft (load independent)
        launch_copy_sub(K, (int64_t)mp * mp, mp, 0, 0, nf, nf, c->rec_L.p + eo * nf * nf,
                        (int64_t)nf * nf, nf, cnt, s);
        launch_copy_sub(K, (int64_t)mp * mp, mp, 0, nf, nf, ntr, c->rec_Y.p + eo * nf * ntr,
                        (int64_t)nf * ntr, nf, cnt, s);
      }
      if (nr > 0)             // Y_b = L^-1 b_f
        launch_copy_sub(K, (int64_t)mp * mp, mp, 0, m, nf, nr, c->rec_Yb.p + eo * nf * nr,
                        (int64_t)nf * nr, nf, cnt, s, dl);
    }
  }
  for (int k = 1; k < NS; ++k) stream_wait(xs[k], c->stream, xj[k]);
  if (!fine || ind) {
    check_infos(P.info.p, nel, c->stream, fine ? "element Gram matrix" : "coarse-mesh element Gram matrix");
    check_infos(P.info.p + nel, nel, c->stream, fine ? "element field block" : "coarse-mesh element field block");
    return;
  }
  // assembled loads
  for (int r = 0; r < nr; ++r)
    launch_assemble_vec(f.num.n, c->asm_ptr.p, c->asm_ent.p, c->s_elem.p + (int64_t)r * nel * ntr,
                        0, c->s_asm.p + (int64_t)r * f.num.n, c->stream);
  check_infos(P.info.p, total, c->stream, elist ? "listed element (Gram matrix)" : "element Gram matrix");
  check_infos(P.info.p + nel, total, c->stream, elist ? "listed element (field block)" : "element field block");
}

// ---- load updates by element-class maps ---------------------------------------------

// More classes than this (a wave speed varying from element to element) keep
// the load updates on the element chain.
constexpr int kMaxLoadClasses = 512;

// Classes of the finest elements by (wave speed, faces on Gamma) and one
// representative element of each; false when there are too many.
bool classify_elements(const dpg_ctx *c, std::vector<int32_t> &cls, std::vector<int32_t> &rep) {
  const int N = c->N;
  std::map<std::pair<double, int>, int32_t> id;
  cls.assign((size_t)N * N * N, 0);
  rep.clear();
  for (int k = 0; k < N; ++k)
    for (int j = 0; j < N; ++j)
      for (int i = 0; i < N; ++i) {
        const int e = i + N * (j + N * k);
        const int mask = (i == 0) | (i == N - 1) << 1 | (j == 0) << 2 | (j == N - 1) << 3 |
                         (k == 0) << 4 | (k == N - 1) << 5;
        const auto key = std::make_pair(c->c_h[e], mask);
        auto it = id.find(key);
        if (it == id.end()) {
          if ((int)rep.size() >= kMaxLoadClasses) return false;
          it = id.emplace(key, (int32_t)rep.size()).first;
          rep.push_back(e);
        }
        cls[e] = it->second;
      }
  return true;
}

// The class maps: the element chain on one element per class with the n_test
// identity columns as loads, W = L^-1 [B | I], K = W^H W, the field block of
// K factored and condensed; T_c and F_c are then blocks of the condensed K.
void build_load_maps(dpg_ctx *c) {
  LoadMaps &M = c->lm;
  std::vector<int32_t> rep;
  if (!classify_elements(c, M.cls_h, rep)) {
    M.state = -1;
    M.cls_h.clear();
    return;
  }
  const hipStream_t s = c->stream;
  Budget *bd = &c->bud;
  const int nt = c->n_test, nf = c->n_field, ntr = c->n_tr, m = c->m, mp = m + nt;
  const int nc = (int)rep.size();
  DevBuf<double2> G, BL, K, wk;
  DevBuf<int> info;
  DevBuf<int32_t> rl;
  DevBuf<int64_t> idoff;
  DevBuf<int32_t> idn;
  DevBuf<PotrfItem> pG, pK;
  DevBuf<TrsmItem> tG, tK;
  DevBuf<GemmItem> gK, gS;
  G.alloc((int64_t)nc * nt * nt, bd);
  BL.alloc((int64_t)nc * nt * mp, bd);
  K.alloc((int64_t)nc * mp * mp, bd);
  wk.alloc(dense_work_size(nc, nt), bd);
  info.alloc(2LL * nc, bd);
  std::vector<PotrfItem> hpG(nc), hpK(nc);
  std::vector<TrsmItem> htG(nc), htK(nc);
  std::vector<GemmItem> hgK(nc), hgS(nc);
  std::vector<int64_t> hoff(nc);
  std::vector<int32_t> hn(nc, nt);
  for (int i = 0; i < nc; ++i) {
    const int64_t oG = (int64_t)i * nt * nt, oB = (int64_t)i * nt * mp, oK = (int64_t)i * mp * mp;
    hpG[i] = {oG, nt, nt};
    htG[i] = {oG, oB, nt, mp, nt, nt};
    hgK[i] = {oB, oB, oK, mp, mp, nt, nt, nt, mp};
    hpK[i] = {oK, nf, mp};
    htK[i] = {oK, oK + (int64_t)nf * mp, nf, mp - nf, mp, mp};
    hgS[i] = {oK + (int64_t)nf * mp, oK + (int64_t)nf * mp, oK + nf + (int64_t)nf * mp,
              mp - nf, mp - nf, nf, mp, mp, mp};
    hoff[i] = oB + (int64_t)m * nt;   // the identity load columns of item i
  }
  rl.upload(rep, bd, s);
  pG.upload(hpG, bd, s);
  pK.upload(hpK, bd, s);
  tG.upload(htG, bd, s);
  tK.upload(htK, bd, s);
  gK.upload(hgK, bd, s);
  gS.upload(hgS, bd, s);
  idoff.upload(hoff, bd, s);
  idn.upload(hn, bd, s);
  LevelData &f = c->lv[c->L];
  ElemGeom g{f.N, c->side / f.N, c->omega, 1.0, {c->org[0], c->org[1], c->org[2]}, rl.p};
  launch_gram(c->tables.p, c->testd.p, nt, g, c->kappa.p, 0, nc, G.p, s);
  launch_bmat(c->tables.p, c->testd.p, c->triald.p, nt, m, g, c->kappa.p, c->Zel.p, 0, nc, BL.p,
              (int64_t)nt * mp, s);
  launch_identity(idoff.p, idn.p, nc, nt, BL.p, s);
  potrf_batched(G.p, pG.p, nc, info.p, nt, wk.p, s);
  trsm_batched(G.p, BL.p, tG.p, nc, nt, mp, false, wk.p, true, s);
  gemm_batched(OP_C, OP_N, mk(1, 0), BL.p, BL.p, mk(0, 0), K.p, gK.p, nc, mp, mp, s, GEMM_HERM);
  potrf_batched(K.p, pK.p, nc, info.p + nc, nf, wk.p, s);
  trsm_batched(K.p, K.p, tK.p, nc, nf, mp - nf, false, wk.p, true, s);
  gemm_batched(OP_C, OP_N, mk(-1, 0), K.p, K.p, mk(1, 0), K.p, gS.p, nc, mp - nf, mp - nf, s,
               GEMM_HERM);
  M.T.alloc((int64_t)nc * ntr * nt, bd);
  launch_copy_sub(K.p, (int64_t)mp * mp, mp, nf, m, ntr, nt, M.T.p, (int64_t)ntr * nt, ntr, nc, s);
  if (c->keep_recovery) {
    M.F.alloc((int64_t)nc * nf * nt, bd);
    launch_copy_sub(K.p, (int64_t)mp * mp, mp, 0, m, nf, nt, M.F.p, (int64_t)nf * nt, nf, nc, s);
  }
  check_infos(info.p, 2LL * nc, s, "element class (load maps)");
  M.nclass = nc;
  M.state = 1;
}

// Condensed loads (and field-recovery data) of the listed finest elements
// (every element when list is empty and all is set) by the class maps:
// l_e from the load kernel, then s_e = T_c l_e and Yb_e = F_c l_e, in chunks
// of about 1 GB of load vectors.  s_elem (and rec_Yb) must be zero outside
// the list.
void load_by_maps(dpg_ctx *c, const std::vector<int32_t> &list, const int32_t *list_dev,
                  bool all) {
  LoadMaps &M = c->lm;
  LevelData &f = c->lv[c->L];
  const hipStream_t s = c->stream;
  Budget *bd = &c->bud;
  const int nt = c->n_test, nf = c->n_field, ntr = c->n_tr, nr = c->nrhs, nel = f.nel;
  const int total = all ? nel : (int)list.size();
  if (total > 0) {
    const int64_t per = (int64_t)nt * nr;
    const int C = (int)std::max<int64_t>(1, std::min<int64_t>(total, 62500000LL / per));
    grow(M.lbuf, (int64_t)C * per, bd);
    const bool rec = c->keep_recovery && M.F.p;
    std::vector<GemmItem> it((size_t)total * (rec ? 2 : 1));
    for (int k = 0; k < total; ++k) {
      const int e = all ? k : list[k];
      const int64_t cl = M.cls_h[e], lo = (int64_t)(k % C) * per;
      it[k] = {cl * ntr * nt, lo, (int64_t)e * ntr, ntr, nr, nt, ntr, nt, nel * ntr};
      if (rec) it[(size_t)total + k] = {cl * nf * nt, lo, (int64_t)e * nf * nr, nf, nr, nt, nf, nt, nf};
    }
    M.items.upload(it, bd, s);
    ElemGeom g{f.N, c->side / f.N, c->omega, 1.0, {c->org[0], c->org[1], c->org[2]},
               all ? nullptr : list_dev};
    for (int e0 = 0; e0 < total; e0 += C) {
      const int cnt = std::min(C, total - e0);
      {
        ProfScope ps(&c->prof, DPG_K_LOAD, 0, s);
        launch_load(c->tables.p, nt, 0, g, c->Zel.p, c->ld.p, c->src.p, c->u0q.p, nr, e0, cnt,
                    M.lbuf.p, per, s);
      }
      ProfScope ps(&c->prof, DPG_K_GEMM, 8.0 * cnt * (double)(ntr + (rec ? nf : 0)) * nt * nr, s);
      gemm_batched(OP_N, OP_N, mk(1, 0), M.T.p, M.lbuf.p, mk(0, 0), c->s_elem.p, M.items.p + e0,
                   cnt, ntr, nr, s);
      if (rec)
        gemm_batched(OP_N, OP_N, mk(1, 0), M.F.p, M.lbuf.p, mk(0, 0), c->rec_Yb.p,
                     M.items.p + total + e0, cnt, nf, nr, s);
    }
    HIP_OK(hipStreamSynchronize(s));   // the host item list and M.items may be reused next
  }
  for (int r = 0; r < nr; ++r)
    launch_assemble_vec(f.num.n, c->asm_ptr.p, c->asm_ent.p, c->s_elem.p + (int64_t)r * nel * ntr,
                        0, c->s_asm.p + (int64_t)r * f.num.n, s);
}

// ---- hierarchy -------------------------------------------------------------------------

// The full (nBf x nBf) macro blocks of a level: its element matrices on an
// order level, the condensed blocks otherwise.
const double2 *mfull(const LevelData &f) { return f.order ? f.E.p : f.Mfull.p; }

// Chunk size of the macro blocks of a level and the shared workspace sizes.
int macro_chunk(dpg_ctx *c, const LevelData &f) {
  const int ntr = f.ntr_c, nBf = f.nBf, nI = f.nI, nT = nBf + nI;
  const int64_t per = 16LL * ((int64_t)nT * nT + (int64_t)nI * nI + (int64_t)nBf * ntr);
  const int64_t cmax = std::max<int64_t>(1, std::min<int64_t>(2500000000LL / per, 65535));
  if (f.nblk <= cmax) return f.nblk;
  const int64_t pairs = (f.nblk + 2 * cmax - 1) / (2 * cmax);   // an even number of chunks
  return (int)((f.nblk + 2 * pairs - 1) / (2 * pairs));
}

void plan_macro(dpg_ctx *c, int l) {
  LevelData &f = c->lv[l];
  MacroPlan &P = f.mp;
  if (P.ready) return;
  const hipStream_t s = c->stream;
  Budget *bd = &c->bud;
  // ntr: element size of the coarser level (the Galerkin products' output)
  const int ntr = f.ntr_c, nBf = f.nBf, nI = f.nI, nT = nBf + nI, nblk = f.nblk;
  const bool ord = f.order;   // order level: the blocks are the element matrices
  const int CB = macro_chunk(c, f);
  std::vector<double2> ploc_h(f.P.local.size());
  for (size_t i = 0; i < ploc_h.size(); ++i) ploc_h[i] = mk(f.P.local[i], 0.0);
  P.Ploc.upload(ploc_h, bd, s);
  std::vector<PotrfItem> pII(CB);
  std::vector<TrsmItem> tIB(CB), tLi(CB);
  std::vector<GemmItem> gS(CB), gTi(CB), gWH(CB), gX(CB), gA(CB);
  std::vector<int64_t> idoff(CB);
  std::vector<int32_t> idn(CB, nI);
  for (int i = 0; i < CB; ++i) {
    const int64_t oT = (int64_t)i * nT * nT, oL = (int64_t)i * nI * nI;
    const int64_t oII = oT + nBf + (int64_t)nBf * nT, oIB = oT + nBf;
    pII[i] = {oII, nI, nT};
    tIB[i] = {oII, oIB, nI, nBf, nT, nT};
    gS[i] = {oIB, oIB, oT, nBf, nBf, nI, nT, nT, nT};
    tLi[i] = {oII, oL, nI, nI, nT, nI};
    gTi[i] = {oL, oL, oL, nI, nI, nI, nI, nI, nI};
    gWH[i] = {oIB, oL, (int64_t)i * nBf * nI, nBf, nI, nI, nT, nI, nBf};
    gX[i] = {oT, 0, (int64_t)i * nBf * ntr, nBf, ntr, nBf, nT, nBf, nBf};
    gA[i] = {0, (int64_t)i * nBf * ntr, (int64_t)i * ntr * ntr, ntr, ntr, nBf, nBf, nBf, ntr};
    idoff[i] = oL;
  }
  P.pII.upload(pII, bd, s);
  P.tIB.upload(tIB, bd, s);
  P.tLi.upload(tLi, bd, s);
  P.gS.upload(gS, bd, s);
  P.gTi.upload(gTi, bd, s);
  P.gWH.upload(gWH, bd, s);
  P.gX.upload(gX, bd, s);
  P.gA.upload(gA, bd, s);
  P.idoff.upload(idoff, bd, s);
  P.idn.upload(idn, bd, s);
  if (!ord) {
    std::vector<int32_t> cinv((size_t)8 * nT, -1);
    for (int ch = 0; ch < 8; ++ch)
      for (int k = 0; k < f.ntr; ++k) {
        const int32_t slot = f.mc.child_map[(size_t)ch * f.ntr + k];
        if (slot < 0 || slot >= nT || cinv[(size_t)ch * nT + slot] >= 0)
          throw DpgError(-1, "child map is not one-to-one");
        cinv[(size_t)ch * nT + slot] = k;
      }
    P.cmap.upload(cinv, bd, s);
  }
  std::vector<int64_t> soff(nblk), moff(nblk);
  std::vector<int32_t> sld(nblk, nBf);
  for (int b = 0; b < nblk; ++b) {
    soff[b] = (int64_t)b * nBf * nBf;
    moff[b] = f.mc.blkB_ptr[b];
  }
  P.soff.upload(soff, bd, s);
  P.moff.upload(moff, bd, s);
  P.sld.upload(sld, bd, s);
  P.map.upload(f.mc.blkB_present, bd, s);
  P.info.ensure(nblk, bd);
  // level outputs and the shared workspaces (the finest level has the most blocks)
  LevelData &cl = c->lv[l - 1];
  cl.E.ensure((int64_t)nblk * ntr * ntr, bd);
  if (!ord) {
    f.Mfull.ensure((int64_t)nblk * nBf * nBf, bd);
    f.Tinv.ensure((int64_t)nblk * nI * nI, bd);
    f.WH.ensure((int64_t)nblk * nBf * nI, bd);
  }
  if (c->opt.precision == DPG_MIXED && l < c->L && !ord) {
    f.Tinv32.ensure(f.Tinv.n, bd);
    f.WH32.ensure(f.WH.n, bd);
  }
  for (int h = 0; h < (nblk > CB ? 2 : 1); ++h) {
    if (!ord && c->mT[h].n < (int64_t)CB * nT * nT) c->mT[h].alloc((int64_t)CB * nT * nT, bd);
    if (c->mLinv[h].n < (int64_t)CB * nI * nI) c->mLinv[h].alloc((int64_t)CB * nI * nI, bd);
    if (c->mX[h].n < (int64_t)CB * nBf * ntr) c->mX[h].alloc((int64_t)CB * nBf * ntr, bd);
    if (c->mwk[h].n < dense_work_size(CB, nI)) c->mwk[h].alloc(dense_work_size(CB, nI), bd);
  }
  HIP_OK(hipStreamSynchronize(s));
  P.CB = CB;
  P.ready = true;
}

// Macro condensation of level l (Sec. 3) and, unless the coarse operators are
// stored (assembled on their own meshes), the Galerkin element matrices of
// level l - 1.  Chunks of coarse elements alternate between the two streams
// (each with its own workspaces); on return the main stream has everything.
void build_macro_level(dpg_ctx *c, int l) {
  LevelData &f = c->lv[l];
  LevelData &cl = c->lv[l - 1];
  MacroPlan &P = f.mp;
  const int ntr = f.ntr_c, nBf = f.nBf, nI = f.nI, nT = nBf + nI, nblk = f.nblk, CB = P.CB;
  const bool two = nblk > CB;
  const bool one_stream = c->prof.on;   // profiled launches are timed alone
  const DenseProf dI{&c->prof, nullptr, nI, nullptr, nBf}, dL{&c->prof, nullptr, nI, nullptr, nI};
  if (two && !one_stream) stream_wait(c->stream, c->aux, c->ev_fork);
  for (int b0 = 0, k = 0; b0 < nblk; b0 += CB, ++k) {
    const int cnt = std::min(CB, nblk - b0), u = two ? (k & 1) : 0;
    const hipStream_t s = u && !one_stream ? c->aux : c->stream;
    double2 *T = c->mT[u].p, *Linv = c->mLinv[u].p, *X = c->mX[u].p, *wk = c->mwk[u].p;
    if (f.order) {
      // order level: the blocks are the element matrices themselves (nothing
      // condensed); only the Galerkin products below
      T = f.E.p + (int64_t)b0 * nT * nT;
    } else {
    {
      ProfScope ps(&c->prof, DPG_K_MACRO_ASM, 0, s);
      launch_macro_assemble(f.E.p, f.ntr, P.cmap.p, f.N, b0, cnt, nT, T, s);
    }
    {
      ProfScope ps(&c->prof, DPG_K_POTRF, cnt * f_potrf(nI), s);
      potrf_batched(T, P.pII.p, cnt, P.info.p + b0, nI, wk, s, &dI);
    }
    {
      ProfScope ps(&c->prof, DPG_K_TRSM, cnt * f_trsm(nI, nBf), s);
      trsm_batched(T, T, P.tIB.p, cnt, nI, nBf, false, wk, true, s, &dI);
    }
    {
      ProfScope ps(&c->prof, DPG_K_GEMM, cnt * f_herk(nBf, nI), s);
      gemm_batched(OP_C, OP_N, mk(-1, 0), T, T, mk(1, 0), T, P.gS.p, cnt, nBf, nBf, s, GEMM_HERM);
    }
    {
      ProfScope ps(&c->prof, DPG_K_OTHER, 0, s);
      launch_identity(P.idoff.p, P.idn.p, cnt, nI, Linv, s);
    }
    {
      ProfScope ps(&c->prof, DPG_K_TRSM, cnt * f_trsm(nI, nI), s);
      trsm_batched(T, Linv, P.tLi.p, cnt, nI, nI, true, wk, true, s, &dL);
    }
    {
      ProfScope ps(&c->prof, DPG_K_GEMM, cnt * f_herk(nI, nI), s);
      gemm_batched(OP_C, OP_N, mk(1, 0), Linv, Linv, mk(0, 0), f.Tinv.p + (int64_t)b0 * nI * nI,
                   P.gTi.p, cnt, nI, nI, s, GEMM_HERM_LOWTRI);
    }
    {
      ProfScope ps(&c->prof, DPG_K_GEMM, cnt * f_gemm(nBf, nI, nI), s);
      gemm_batched(OP_C, OP_N, mk(1, 0), T, Linv, mk(0, 0), f.WH.p + (int64_t)b0 * nBf * nI,
                   P.gWH.p, cnt, nBf, nI, s);
    }
    {
      ProfScope ps(&c->prof, DPG_K_OTHER, 0, s);
      launch_copy_sub(T, (int64_t)nT * nT, nT, 0, 0, nBf, nBf, f.Mfull.p + (int64_t)b0 * nBf * nBf,
                      (int64_t)nBf * nBf, nBf, cnt, s);
    }
    }
    if (!(c->opt.flags & DPG_STORE_COARSE)) {
      ProfScope ps(&c->prof, DPG_K_GEMM, cnt * (f_gemm(nBf, ntr, nBf) + f_gemm(ntr, ntr, nBf)), s);
      gemm_batched(OP_N, OP_N, mk(1, 0), T, P.Ploc.p, mk(0, 0), X, P.gX.p, cnt, nBf, ntr, s);
      gemm_batched(OP_T, OP_N, mk(1, 0), P.Ploc.p, X, mk(0, 0), cl.E.p + (int64_t)b0 * ntr * ntr,
                   P.gA.p, cnt, ntr, ntr, s);
    }
  }
  if (two && !one_stream) stream_wait(c->aux, c->stream, c->ev_join);
  const hipStream_t s = c->stream;
  if (c->opt.precision == DPG_MIXED && l < c->L && !f.order) {
    launch_to32(f.Tinv.n, f.Tinv.p, f.Tinv32.p, s);
    launch_to32(f.WH.n, f.WH.p, f.WH32.p, s);
  }
  // macro blocks -> packed tiles (present slots only)
  f.Mset.pack(mfull(f), P.soff.p, P.sld.p, P.moff.p, P.map.p, s);
}

// Each level's patch work is cut into this many parts of equal factorisation
// work, each on a stream of its own (three extra streams and the main one), so
// that the latency-bound diagonal-block steps of one part overlap the
// matrix-core updates of the others.  Hierarchy time at 16^3 / p = 3: two
// parts 50.8 ms, three 50.4, four 49.5.
constexpr int kPatchParts = 4;

void plan_patches(dpg_ctx *c, int l) {
  LevelData &f = c->lv[l];
  PatchPlan &P = f.pp;
  if (P.ready) return;
  const hipStream_t s = c->stream;
  Budget *bd = &c->bud;
  const int np = (int)f.mc.patch_ptr.size() - 1;
  std::vector<int32_t> nv(np);
  int nv_max = 0;
  int64_t maxent = 0;
  for (int v = 0; v < np; ++v) {
    nv[v] = (int32_t)(f.mc.patch_ptr[v + 1] - f.mc.patch_ptr[v]);
    nv_max = std::max(nv_max, (int)nv[v]);
    maxent = std::max<int64_t>(maxent, (int64_t)nv[v] * nv[v]);
  }
  // parts of equal factorisation work (sum n^3), one per stream, each cut
  // into batches that fit its workspaces (S and X: 3 GB each).  With the
  // inverses recomputed in every smoothing step, one part on the main stream
  // and workspaces of 0.5 GB.
  const bool rec = c->opt.flags & DPG_RECOMPUTE_PATCHES;
  const int64_t ws = std::max<int64_t>((rec ? 500000000LL : 3000000000LL) / 16, maxent);
  const int NP = rec ? 1 : kPatchParts;
  double tot = 0.0;
  for (int v = 0; v < np; ++v) tot += (double)nv[v] * nv[v] * nv[v];
  std::vector<int> vcut(NP + 1, np);
  vcut[0] = 0;
  {
    int v = 0;
    double acc = 0.0;
    for (int k = 1; k < NP; ++k) {
      while (v < np && acc < tot * k / NP) {
        acc += (double)nv[v] * nv[v] * nv[v];
        ++v;
      }
      vcut[k] = v;
    }
  }
  std::vector<int64_t> soff_all(np, 0);
  int maxcnt[4] = {0, 0, 0, 0};
  int64_t maxuse[4] = {0, 0, 0, 0};   // largest batch footprint of each part (entries)
  for (int half = 0; half < NP; ++half) {
    int v0 = vcut[half];
    const int vend = vcut[half + 1];
    while (v0 < vend) {
      int cnt = 0;
      int64_t used = 0;
      while (v0 + cnt < vend && cnt < 65535 &&
             (cnt == 0 || used + (int64_t)nv[v0 + cnt] * nv[v0 + cnt] <= ws)) {
        used += (int64_t)nv[v0 + cnt] * nv[v0 + cnt];
        ++cnt;
      }
      PatchBatch B;
      B.half = half;
      B.v0 = v0;
      B.cnt = cnt;
      std::vector<int64_t> off(cnt);
      std::vector<int32_t> nn(cnt);
      std::vector<PotrfItem> pi(cnt);
      std::vector<TrsmItem> ti(cnt);
      std::vector<GemmItem> gi(cnt);
      int64_t o = 0;
      for (int i = 0; i < cnt; ++i) {
        const int n = nv[v0 + i];
        off[i] = o;
        nn[i] = n;
        B.nmax = std::max(B.nmax, n);
        pi[i] = {o, n, n};
        ti[i] = {o, o, n, n, n, n};
        gi[i] = {o, o, o, n, n, n, n, n, n};
        soff_all[v0 + i] = o;
        o += (int64_t)n * n;
        B.fp += f_potrf(n);
        B.ft += f_trsm(n, n) / 3.0;   // identity right-hand side: L^-1 only
        B.fg += f_herk(n, n) / 3.0;   // X^H X with X triangular
      }
      B.off.upload(off, bd, s);
      B.nn.upload(nn, bd, s);
      B.hn = nn;
      B.pi.upload(pi, bd, s);
      B.ti.upload(ti, bd, s);
      B.gi.upload(gi, bd, s);
      if (rec) {   // t_v = X_v x_v, y_v = X_v^H t_v on the local vectors of the patch set
        // nr columns, local vectors column by column (leading dimension nloc)
        const int64_t nloc = f.Sset.nloc;
        std::vector<GemmItem> gyc((size_t)kMaxCols * cnt), gzc((size_t)kMaxCols * cnt);
        for (int q = 1; q <= kMaxCols; ++q)
          for (int i = 0; i < cnt; ++i) {
            const int n = nn[i];
            const int64_t lo = f.Sset.loc_off_h[v0 + i];
            gyc[(size_t)(q - 1) * cnt + i] = {off[i], lo, lo, n, q, n, n, (int)nloc, (int)nloc};
            gzc[(size_t)(q - 1) * cnt + i] = {off[i], lo, lo, n, q, n, n, (int)nloc, (int)nloc};
          }
        B.gyc.upload(gyc, bd, s);
        B.gzc.upload(gzc, bd, s);
      }
      B.t0 = f.Sset.tile_off_h[v0];
      B.t1 = (v0 + cnt < np) ? f.Sset.tile_off_h[v0 + cnt] : f.Sset.ntiles;
      maxcnt[half] = std::max(maxcnt[half], cnt);
      maxuse[half] = std::max(maxuse[half], used);
      P.batches.push_back(std::move(B));
      v0 += cnt;
    }
  }
  P.soff_all.upload(soff_all, bd, s);
  P.ld_all.upload(nv, bd, s);
  P.info.ensure(np, bd);
  if (rec) grow(c->ptmp, f.Sset.nloc, bd);
  for (int h = 0; h < NP; ++h) {
    if (!maxcnt[h]) continue;
    if (c->pS[h].n < maxuse[h]) c->pS[h].alloc(maxuse[h], bd);
    if (c->pX[h].n < maxuse[h]) c->pX[h].alloc(maxuse[h], bd);
    if (c->pwk[h].n < dense_work_size(maxcnt[h], nv_max))
      c->pwk[h].alloc(dense_work_size(maxcnt[h], nv_max), bd);
  }
  HIP_OK(hipStreamSynchronize(s));
  P.ready = true;
}

// Patch blocks of level l (Sec. 3 smoother): gather, Cholesky, explicit
// inverse, packed tiles; the batches of one half, on stream s.
void build_patches(dpg_ctx *c, int l, int half, hipStream_t s) {
  LevelData &f = c->lv[l];
  PatchPlan &P = f.pp;
  double2 *S = c->pS[half].p, *X = c->pX[half].p, *wk = c->pwk[half].p;
  for (PatchBatch &B : P.batches) {
    if (B.half != half) continue;
    const DenseProf dp{&c->prof, B.hn.data(), 0, B.hn.data(), 0};
    {
      ProfScope ps(&c->prof, DPG_K_PATCH_GATHER, 0, s);
      launch_patch_gather(mfull(f), f.nBf, f.mc.Nc, f.patch_ptr.p, f.patch_slot.p, B.v0, B.cnt,
                          B.nmax, B.off.p, S, s);
    }
    {
      ProfScope ps(&c->prof, DPG_K_POTRF, B.fp, s);
      potrf_batched(S, B.pi.p, B.cnt, P.info.p + B.v0, B.nmax, wk, s, &dp);
    }
    {
      ProfScope ps(&c->prof, DPG_K_OTHER, 0, s);
      launch_identity(B.off.p, B.nn.p, B.cnt, B.nmax, X, s);
    }
    {
      ProfScope ps(&c->prof, DPG_K_TRSM, B.ft, s);
      trsm_batched(S, X, B.ti.p, B.cnt, B.nmax, B.nmax, true, wk, true, s, &dp);
    }
    {
      ProfScope ps(&c->prof, DPG_K_GEMM, B.fg, s);
      gemm_batched(OP_C, OP_N, mk(1, 0), X, X, mk(0, 0), S, B.gi.p, B.cnt, B.nmax, B.nmax, s,
                   GEMM_UPPER_LOWTRI);
    }
    f.Sset.pack(S, P.soff_all.p, P.ld_all.p, nullptr, nullptr, s, B.t0, B.t1 - B.t0);
  }
}

// Patch factors of level l without keeping them: gather and Cholesky of every
// patch block, to report a non-positive pivot at build time (DPG_ENOTPD) when
// the smoother recomputes its inverses in every application.
void check_patches(dpg_ctx *c, int l) {
  LevelData &f = c->lv[l];
  PatchPlan &P = f.pp;
  const hipStream_t s = c->stream;
  for (PatchBatch &B : P.batches) {
    double2 *S = c->pS[B.half].p, *wk = c->pwk[B.half].p;
    launch_patch_gather_tiles(f.Mset.t64.p, f.Mset.ent_off.p, f.mpidx.p, f.nBf, f.mc.Nc,
                              f.patch_ptr.p, f.patch_slot.p, B.v0, B.cnt, B.nmax, B.off.p, S, s);
    potrf_batched(S, B.pi.p, B.cnt, P.info.p + B.v0, B.nmax, wk, s);
  }
}

// The smoother of level l with its patch inverses recomputed from the macro
// blocks (DPG_RECOMPUTE_PATCHES; none is stored), for nr interleaved columns
// (x, y, r: vectors of the level, nr = 1 the single-column ones):
// y <- epilogue(sum_v R_v^T S_v^-1 R_v x) batch by batch -- gather S_v from
// the packed macro-block tiles the matvec streams anyway, S_v = L L^H,
// X = L^-1, then S_v^-1 x_v = X^H (X x_v).  Every patch block is gathered and
// factored once per smoothing step for all nr columns, and X multiplies an
// n x nr panel (the local vectors stored column by column), so the
// refactorisation is amortised over the right-hand sides of a block solve.
// The same operator as the stored inverses, rounded differently; HBM traffic
// and memory traded for matrix-core work.
void smooth_recompute(dpg_ctx *c, int l, const double2 *x, double2 *y, const double2 *r,
                      int mode, double theta, int nr) {
  LevelData &f = c->lv[l];
  PatchPlan &P = f.pp;
  HermSet &H = f.Sset;
  const hipStream_t s = c->stream;
  if (nr < 1 || nr > kMaxCols || (nr > 1 && nr > f.Sb.cap))
    throw DpgError(DPG_EINVAL, "bad column count");
  double2 *xl = nr == 1 ? H.xl64.p : f.Sb.xl64.p, *yl = nr == 1 ? H.yl64.p : f.Sb.yl64.p;
  herm_gather_cols(H, x, xl, nr, s);
  for (PatchBatch &B : P.batches) {
    double2 *S = c->pS[B.half].p, *X = c->pX[B.half].p, *wk = c->pwk[B.half].p;
    const DenseProf dp{&c->prof, B.hn.data(), 0, B.hn.data(), 0};
    {
      PROF(DPG_K_PATCH_GATHER, 0);
      launch_patch_gather_tiles(f.Mset.t64.p, f.Mset.ent_off.p, f.mpidx.p, f.nBf, f.mc.Nc,
                                f.patch_ptr.p, f.patch_slot.p, B.v0, B.cnt, B.nmax, B.off.p, S,
                                s);
    }
    {
      PROF(DPG_K_POTRF, B.fp);
      potrf_batched(S, B.pi.p, B.cnt, P.info.p + B.v0, B.nmax, wk, s, &dp);
    }
    {
      PROF(DPG_K_OTHER, 0);
      launch_identity(B.off.p, B.nn.p, B.cnt, B.nmax, X, s);
    }
    {
      PROF(DPG_K_TRSM, B.ft);
      trsm_batched(S, X, B.ti.p, B.cnt, B.nmax, B.nmax, true, wk, true, s, &dp);
    }
    PROF(DPG_K_GEMM, 0);
    const GemmItem *gy = B.gyc.p + (int64_t)(nr - 1) * B.cnt;
    const GemmItem *gz = B.gzc.p + (int64_t)(nr - 1) * B.cnt;
    gemm_batched(OP_N, OP_N, mk(1, 0), X, xl, mk(0, 0), c->ptmp.p, gy, B.cnt, B.nmax, nr, s);
    gemm_batched(OP_C, OP_N, mk(1, 0), X, c->ptmp.p, mk(0, 0), yl, gz, B.cnt, B.nmax, nr, s);
  }
  herm_scatter_cols(H, yl, y, r, mode, theta, nr, s);
}

void plan_coarsest(dpg_ctx *c) {
  if (c->zpi.p) return;
  LevelData &z = c->lv[0];
  const hipStream_t s = c->stream;
  Budget *bd = &c->bud;
  const int n0 = (int)z.num.n;
  c->T0.ensure((int64_t)n0 * n0, bd);
  c->zF.ensure((int64_t)n0 * n0, bd);
  c->zLi.ensure((int64_t)n0 * n0, bd);
  c->zTi.ensure((int64_t)n0 * n0, bd);
  c->zwk.ensure(dense_work_size(1, n0), bd);
  c->zpi.upload(std::vector<PotrfItem>{{0, n0, n0}}, bd, s);
  c->zti.upload(std::vector<TrsmItem>{{0, 0, n0, n0, n0, n0}}, bd, s);
  c->zgi.upload(std::vector<GemmItem>{{0, 0, 0, n0, n0, n0, n0, n0, n0}}, bd, s);
  c->zoff.upload(std::vector<int64_t>{0}, bd, s);
  c->znn.upload(std::vector<int32_t>{n0}, bd, s);
  c->zld.upload(std::vector<int32_t>{n0}, bd, s);
  c->zinfo.ensure(1, bd);
  HIP_OK(hipStreamSynchronize(s));
}

// Coarsest operator T_0: assembled, Cholesky, explicit inverse, packed tiles.
void build_coarsest(dpg_ctx *c) {
  LevelData &z = c->lv[0];
  const hipStream_t s = c->stream;
  const int n0 = (int)z.num.n;
  launch_assemble_dense(z.E.p, z.ntr, z.edofs.p, z.nel, n0, c->T0.p, s);
  HIP_OK(hipMemcpyAsync(c->zF.p, c->T0.p, (size_t)n0 * n0 * 16, hipMemcpyDeviceToDevice, s));
  const DenseProf dz{&c->prof, nullptr, n0, nullptr, n0};
  potrf_batched(c->zF.p, c->zpi.p, 1, c->zinfo.p, n0, c->zwk.p, s, &dz);
  launch_identity(c->zoff.p, c->znn.p, 1, n0, c->zLi.p, s);
  trsm_batched(c->zF.p, c->zLi.p, c->zti.p, 1, n0, n0, true, c->zwk.p, true, s, &dz);
  gemm_batched(OP_C, OP_N, mk(1, 0), c->zLi.p, c->zLi.p, mk(0, 0), c->zTi.p, c->zgi.p, 1, n0, n0,
               s, GEMM_UPPER_LOWTRI);
  c->T0set.pack(c->zTi.p, c->zoff.p, c->zld.p, nullptr, nullptr, s);
}

// The whole hierarchy: macro levels one after the other on the main stream;
// the patches of level l need only that level's macro blocks.  Three quarters
// of them (by work) run on the three extra streams as soon as the level's
// blocks exist, overlapping the coarser levels; the last quarter on the main
// stream after the coarsest level, so that the latency-bound steps of one part
// overlap the matrix-core updates of the others.
void build_hierarchy(dpg_ctx *c) {
  for (int l = c->L; l >= 1; --l) {
    plan_macro(c, l);
    plan_patches(c, l);
  }
  plan_coarsest(c);
  if (c->opt.flags & DPG_STORE_COARSE)   // coarse operators assembled on their own meshes
    for (int l = c->L - 1; l >= 0; --l) element_stage(c, l, true);
  if ((int)c->ev_level.size() < c->L + 1) {
    for (int l = (int)c->ev_level.size(); l <= c->L; ++l) {
      hipEvent_t e;
      HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      c->ev_level.push_back(e);
    }
  }
  const int NX = kPatchParts - 1;   // parts on the extra streams
  hipStream_t xs[3] = {c->aux, c->paux[0], c->paux[1]};
  hipEvent_t xj[3] = {c->ev_join, c->ev_pjoin[0], c->ev_pjoin[1]};
  if (c->opt.flags & DPG_RECOMPUTE_PATCHES) {   // no stored inverses: check the factors only
    for (int l = c->L; l >= 1; --l) {
      build_macro_level(c, l);
      check_patches(c, l);
    }
    build_coarsest(c);
  } else {
    // while kernels are profiled, every part runs on the main stream (each
    // launch's events then time it alone)
    if (c->prof.on)
      for (int k = 0; k < NX; ++k) xs[k] = c->stream;
    for (int k = 0; k < NX && !c->prof.on; ++k) stream_wait(c->stream, xs[k], c->ev_fork);
    for (int l = c->L; l >= 1; --l) {
      build_macro_level(c, l);
      for (int k = 0; k < NX; ++k) {
        if (!c->prof.on) stream_wait(c->stream, xs[k], c->ev_level[l]);
        build_patches(c, l, k, xs[k]);
      }
    }
    build_coarsest(c);
    for (int l = c->L; l >= 1; --l) build_patches(c, l, NX, c->stream);
    for (int k = 0; k < NX && !c->prof.on; ++k) stream_wait(xs[k], c->stream, xj[k]);
  }
  for (int l = c->L; l >= 1; --l) {
    if (!c->lv[l].order)   // an order level factors no interior block
      check_infos(c->lv[l].mp.info.p, c->lv[l].nblk, c->stream, "interior block of coarse element");
    check_infos(c->lv[l].pp.info.p, (int64_t)c->lv[l].mc.patch_ptr.size() - 1, c->stream,
                "vertex patch");
  }
  check_infos(c->zinfo.p, 1, c->stream, "coarsest operator");
}

// ---- V-cycle -----------------------------------------------------------------------------

template <typename T> struct LB;
template <> struct LB<double> {
  static double2 *r(LevelData &f) { return f.r64.p; }
  static double2 *x(LevelData &f) { return f.x64.p; }
  static double2 *res(LevelData &f) { return f.res64.p; }
  static double2 *rc(LevelData &f) { return f.rc64.p; }
  static double2 *ec(LevelData &f) { return f.ec64.p; }
  static double2 *cc(LevelData &f) { return f.c64.p; }
  static const double2 *WH(LevelData &f) { return f.WH.p; }
  static const double2 *Ti(LevelData &f) { return f.Tinv.p; }
  static const double *Pv(LevelData &f) { return f.Pval.p; }
  static const double *Ptv(LevelData &f) { return f.Ptval.p; }
};
template <> struct LB<float> {
  static float2 *r(LevelData &f) { return f.r32.p; }
  static float2 *x(LevelData &f) { return f.x32.p; }
  static float2 *res(LevelData &f) { return f.res32.p; }
  static float2 *rc(LevelData &f) { return f.rc32.p; }
  static float2 *ec(LevelData &f) { return f.ec32.p; }
  static float2 *cc(LevelData &f) { return f.c32.p; }
  static const float2 *WH(LevelData &f) { return f.WH32.p; }
  static const float2 *Ti(LevelData &f) { return f.Tinv32.p; }
  static const float *Pv(LevelData &f) { return f.Pval32.p; }
  static const float *Ptv(LevelData &f) { return f.Ptval32.p; }
};

// The smoother's patch sum on level l: stored inverses, or recomputed ones.
template <typename T>
void smooth_apply(dpg_ctx *c, int l, const cplx_t<T> *x, cplx_t<T> *y, int mode, T theta,
                  bool gathered = false, HermSet *fwd = nullptr) {
  if constexpr (sizeof(T) == 8) {
    if (c->opt.flags & DPG_RECOMPUTE_PATCHES) {
      if (gathered || fwd) throw DpgError(-1, "recomputed patches take no forwarded vectors");
      smooth_recompute(c, l, x, y, nullptr, mode, theta, 1);
      return;
    }
  }
  herm_apply<T>(c->lv[l].Sset, x, y, nullptr, mode, theta, c->stream, gathered, fwd);
}

// Condensation of the macro-grid interior unknowns of level g (Sec. 3): the
// macro right-hand side from nr interleaved full trace columns (cc: the
// per-block partial products).  On an order level nothing is condensed (the
// macro unknowns are the level's traces, in order): a copy.
template <typename T>
void condense_level(const LevelData &g, const cplx_t<T> *WH, const cplx_t<T> *full, cplx_t<T> *cc,
                    cplx_t<T> *out, int nr, hipStream_t s) {
  if (g.order) {
    HIP_OK(hipMemcpyAsync(out, full, g.nM * nr * sizeof(cplx_t<T>), hipMemcpyDeviceToDevice, s));
  } else if (nr == 1) {
    launch_condense_local<T>(WH, g.nI, g.nBf, g.blkI.p, g.nblk, full, cc, s);
    launch_condense_reduce<T>(g.nM, g.macroB.p, g.cred_ptr.p, g.cred_ent.p, full, cc, out, s);
  } else {
    launch_condense_blk<T>(WH, g.nI, g.nBf, g.blkI.p, g.nblk, g.nM, g.macroB.p, g.cred_ptr.p,
                           g.cred_ent.p, full, cc, out, nr, s);
  }
}

// Expansion: the full trace columns from the macro solution xm and the
// loads full (interior recovery); on an order level a copy of xm.
template <typename T>
void expand_level(const LevelData &g, const cplx_t<T> *WH, const cplx_t<T> *Ti,
                  const cplx_t<T> *full, const cplx_t<T> *xm, cplx_t<T> *out, int nr,
                  hipStream_t s) {
  if (g.order) {
    HIP_OK(hipMemcpyAsync(out, xm, g.nM * nr * sizeof(cplx_t<T>), hipMemcpyDeviceToDevice, s));
  } else if (nr == 1) {
    launch_expand<T>(WH, Ti, g.nI, g.nBf, g.blkI.p, g.blkBm.p, g.nblk, full, xm, g.nM, g.macroB.p,
                     out, s);
  } else {
    launch_expand_blk<T>(WH, Ti, g.nI, g.nBf, g.blkI.p, g.blkBm.p, g.nblk, full, xm, g.nM,
                         g.macroB.p, out, nr, s);
  }
}

template <typename T> void vcycle(dpg_ctx *c, int l) {
  using B = LB<T>;
  LevelData &f = c->lv[l];
  const hipStream_t s = c->stream;
  const T th = (T)c->opt.theta;
  auto r = B::r(f), x = B::x(f), res = B::res(f), rc = B::rc(f), ec = B::ec(f);
  // With stored patch inverses every smoother application forwards the new x
  // to the residual's block set and every residual forwards r - Mx to the
  // smoother's (the scatter writes their local vectors), so neither gathers.
  const bool fw = sizeof(T) == 4 || !(c->opt.flags & DPG_RECOMPUTE_PATCHES);
  HermSet *toM = fw ? &f.Mset : nullptr, *toS = fw ? &f.Sset : nullptr;
  if (c->opt.nu_pre == 0) launch_zero(f.nM, x, s);
  for (int k = 0; k < c->opt.nu_pre; ++k) {
    if (k == 0) {
      smooth_apply<T>(c, l, r, x, RED_SET_SCALED, th, false, toM);
    } else {
      herm_apply<T>(f.Mset, x, res, r, RED_RESID, (T)0, s, fw, toS);
      smooth_apply<T>(c, l, res, x, RED_AXPY, th, fw, toM);
    }
  }
  herm_apply<T>(f.Mset, x, res, r, RED_RESID, (T)0, s, fw && c->opt.nu_pre > 0);
  LevelData &g = c->lv[l - 1];
  {
    PROF(DPG_K_TRANSFER, 0);
    launch_csr<T>(g.num.n, f.Ptptr.p, f.Ptcol.p, B::Ptv(f), res, rc, 0, s);
  }
  if (l - 1 == 0) {
    herm_apply<T>(c->T0set, rc, ec, nullptr, RED_SET, (T)1, s);
  } else {
    {
      PROF(DPG_K_CONDENSE, 0);
      condense_level<T>(g, B::WH(g), rc, B::cc(g), B::r(g), 1, s);
    }
    vcycle<T>(c, l - 1);
    PROF(DPG_K_EXPAND, 0);
    expand_level<T>(g, B::WH(g), B::Ti(g), rc, B::x(g), ec, 1, s);
  }
  {
    PROF(DPG_K_TRANSFER, 0);
    launch_csr<T>(f.nM, f.Pptr.p, f.Pcol.p, B::Pv(f), ec, x, 1, s);
  }
  for (int k = 0; k < c->opt.nu_post; ++k) {
    herm_apply<T>(f.Mset, x, res, r, RED_RESID, (T)0, s, fw && k > 0, toS);
    smooth_apply<T>(c, l, res, x, RED_AXPY, th, fw, k + 1 < c->opt.nu_post ? toM : nullptr);
  }
}

// z = V(r) on the finest macro grid (FP64 vectors in and out).
void precondition(dpg_ctx *c, const double2 *r, double2 *z) {
  LevelData &top = c->lv[c->L];
  const hipStream_t s = c->stream;
  if (c->opt.precision == DPG_MIXED) {
    launch_to32(top.nM, r, top.r32.p, s);
    vcycle<float>(c, c->L);
    launch_to64(top.nM, top.x32.p, z, s);
  } else {
    HIP_OK(hipMemcpyAsync(top.r64.p, r, top.nM * 16, hipMemcpyDeviceToDevice, s));
    vcycle<double>(c, c->L);
    HIP_OK(hipMemcpyAsync(z, top.x64.p, top.nM * 16, hipMemcpyDeviceToDevice, s));
  }
}

void read_sc(dpg_ctx *c, const double *sc) {
  HIP_OK(hipMemcpyAsync(c->host_sc, sc, 8 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
}

// Capture the launches of f on stream s into an executable graph.  A capture
// that fails is ended and discarded, so the stream is never left capturing.
template <class F> hipGraphExec_t capture(hipStream_t s, F &&f) {
  HIP_OK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  hipGraph_t g = nullptr;
  try {
    f();
  } catch (...) {
    if (hipStreamEndCapture(s, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
    throw;
  }
  HIP_OK(hipStreamEndCapture(s, &g));
  hipGraphExec_t e = nullptr;
  const hipError_t st = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIP_OK(st);
  return e;
}

// PCG on the finest macro grid for one trace right-hand side s (device);
// full trace solution into xout (device).  Returns DPG_OK / ENOCONV.
// partial (2 kDotBlocks doubles) and sc (8 doubles) hold the reduction
// partials and the CG scalars; graphs: replay the iteration as HIP graphs
// (instantiated per call) instead of launching every kernel.
int solve_one(dpg_ctx *c, const double2 *sv, double tol, double2 *xout, int32_t *iters,
              double *relres, double *partial, double *sc, bool graphs) {
  LevelData &top = c->lv[c->L];
  const hipStream_t s = c->stream;
  const int64_t nM = top.nM;
  condense_level<double>(top, top.WH.p, sv, top.c64.p, c->b.p, 1, s);
  launch_zero(4, reinterpret_cast<double2 *>(sc), s);   // the 8 scalars
  dot_re(nM, c->b.p, c->b.p, partial, sc + 5, s);
  launch_zero(nM, c->x.p, s);
  HIP_OK(hipMemcpyAsync(c->r.p, c->b.p, nM * 16, hipMemcpyDeviceToDevice, s));
  read_sc(c, sc);
  const double bb = c->host_sc[5];
  int it = 0;
  double rr = 0.0;
  int status = DPG_OK;
  if (!std::isfinite(bb)) throw DpgError(DPG_EINVAL, "right-hand side is not finite");
  if (bb > 0.0) {
    double2 *z = c->z.p, *zo = c->zo.p;
    precondition(c, c->r.p, z);
    dot_re(nM, c->r.p, z, partial, sc + 0, s);
    HIP_OK(hipMemcpyAsync(c->pv.p, z, nM * 16, hipMemcpyDeviceToDevice, s));
    rr = 1.0;
    // One iteration is two fixed launch sequences around the host's
    // convergence check: (A) matvec, alpha, x and r; (B) V-cycle, beta, p.
    // Without per-kernel profiling they are captured once per solve as HIP
    // graphs and replayed (B in two versions: z and z_old swap every
    // iteration), which removes the launch gaps between the ~105 kernels.
    auto part_a = [&]() {
      herm_apply<double>(top.Mset, c->pv.p, c->q.p, nullptr, RED_SET, 1.0, s);
      PROF(DPG_K_CG, 0);
      cg_alpha(nM, c->pv.p, c->q.p, partial, sc, s);
      cg_update_xr(nM, c->x.p, c->r.p, c->pv.p, c->q.p, partial, sc, s);
    };
    auto part_b = [&](double2 *zn, double2 *zp) {
      precondition(c, c->r.p, zn);
      PROF(DPG_K_CG, 0);
      cg_beta(nM, c->r.p, zn, zp, partial, sc, s);
      cg_update_p(nM, c->pv.p, zn, sc, s);
    };
    GraphSet gs;
    graphs = graphs && !c->prof.on;
    if (graphs) {
      gs.a = capture(s, part_a);
      gs.b[0] = capture(s, [&]() { part_b(c->zo.p, c->z.p); });   // odd iterations
      gs.b[1] = capture(s, [&]() { part_b(c->z.p, c->zo.p); });   // even iterations
    }
    while (it < c->opt.maxit) {
      if (graphs) HIP_OK(hipGraphLaunch(gs.a, s));
      else part_a();
      ++it;
      read_sc(c, sc);
      if (c->host_sc[6] != 0.0)
        throw DpgError(DPG_EBREAKDOWN, "CG breakdown at iteration " + std::to_string(it) +
                                           " (p^H M p = " + std::to_string(c->host_sc[1]) + ")");
      rr = std::sqrt(c->host_sc[4] / bb);
      if (!std::isfinite(rr)) throw DpgError(DPG_EBREAKDOWN, "residual is not finite");
      if (rr <= tol) break;
      std::swap(z, zo);
      if (graphs) HIP_OK(hipGraphLaunch(gs.b[it & 1 ? 0 : 1], s));
      else part_b(z, zo);
    }
    if (rr > tol) status = DPG_ENOCONV;
  }
  expand_level<double>(top, top.WH.p, top.Tinv.p, sv, c->x.p, xout, 1, s);
  HIP_OK(hipStreamSynchronize(s));
  if (iters) *iters = it;
  if (relres) *relres = rr;
  return status;
}

// Columns solved one after the other (solve_one), rhs / x_out staged through
// the context's trace vectors when they are host memory.
int solve_columns(dpg_ctx *c, const double *rhs, int nrhs, double tol, double *x_out,
                  int32_t *iters_out, double *relres_out, double *partial, double *sc,
                  bool graphs) {
  const int64_t nT = c->lv[c->L].num.n;
  const bool dev = c->opt.flags & DPG_DEVICE_PTRS;
  int status = DPG_OK;
  for (int k = 0; k < nrhs; ++k) {
    const double2 *sv;
    if (rhs) {
      HIP_OK(hipMemcpyAsync(c->sB.p, rhs + 2 * nT * k, nT * 16,
                            dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
      sv = c->sB.p;
    } else {
      sv = c->s_asm.p + nT * k;
    }
    int32_t it = 0;
    double rr = 0;
    const int st = solve_one(c, sv, tol, c->xfull.p, &it, &rr, partial, sc, graphs);
    if (st != DPG_OK) status = st;
    if (iters_out) iters_out[k] = it;
    if (relres_out) relres_out[k] = rr;
    if (x_out) {
      HIP_OK(hipMemcpyAsync(x_out + 2 * nT * k, c->xfull.p, nT * 16,
                            dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
      HIP_OK(hipStreamSynchronize(c->stream));
    }
  }
  return status;
}

// ---- multi-right-hand-side solve -------------------------------------------------------------

template <typename T> struct LBB;
template <> struct LBB<double> {
  static double2 *r(LevelData &f) { return f.br64.p; }
  static double2 *x(LevelData &f) { return f.bx64.p; }
  static double2 *res(LevelData &f) { return f.bres64.p; }
  static double2 *rc(LevelData &f) { return f.brc64.p; }
  static double2 *ec(LevelData &f) { return f.bec64.p; }
  static double2 *cc(LevelData &f) { return f.bc64.p; }
};
template <> struct LBB<float> {
  static float2 *r(LevelData &f) { return f.br32.p; }
  static float2 *x(LevelData &f) { return f.bx32.p; }
  static float2 *res(LevelData &f) { return f.bres32.p; }
  static float2 *rc(LevelData &f) { return f.brc32.p; }
  static float2 *ec(LevelData &f) { return f.bec32.p; }
  static float2 *cc(LevelData &f) { return f.bc32.p; }
};

// Block work vectors for nr columns on every level (same shapes as the
// single-column ones, times nr).
void ensure_block(dpg_ctx *c, int nr) {
  if (nr <= c->bcap) return;
  const bool mixed = c->opt.precision == DPG_MIXED;
  Budget *bd = &c->bud;
  for (int l = 1; l <= c->L; ++l) {
    LevelData &f = c->lv[l];
    const int64_t nc = c->lv[l - 1].num.n, nM = f.nM, ncb = (int64_t)f.nblk * f.nBf;
    if (mixed) {
      f.br32.alloc(nM * nr, bd);
      f.bx32.alloc(nM * nr, bd);
      f.bres32.alloc(nM * nr, bd);
      f.brc32.alloc(nc * nr, bd);
      f.bec32.alloc(nc * nr, bd);
      f.bc32.alloc(ncb * nr, bd);
    } else {
      f.br64.alloc(nM * nr, bd);
      f.bx64.alloc(nM * nr, bd);
      f.bres64.alloc(nM * nr, bd);
      f.brc64.alloc(nc * nr, bd);
      f.bec64.alloc(nc * nr, bd);
    }
    if (!mixed || l == c->L) f.bc64.alloc(ncb * nr, bd);
    f.Mb.ensure(f.Mset, nr, f.Mset.t64.p != nullptr, f.Mset.t32.p != nullptr, bd, c->stream);
    const bool rec = c->opt.flags & DPG_RECOMPUTE_PATCHES;   // local vectors of the
                                                             // recomputed smoother
    f.Sb.ensure(f.Sset, nr, f.Sset.t64.p != nullptr || rec, f.Sset.t32.p != nullptr, bd,
                c->stream);
    if (rec) grow(c->ptmp, f.Sset.nloc * nr, bd);
    f.bcap = nr;
  }
  c->T0b.ensure(c->T0set, nr, c->T0set.t64.p != nullptr, c->T0set.t32.p != nullptr, bd,
                c->stream);
  LevelData &top = c->lv[c->L];
  const int64_t nM = top.nM, nT = top.num.n;
  for (auto *v : {&c->bb, &c->bx, &c->br, &c->bz, &c->bzo, &c->bp, &c->bq}) v->alloc(nM * nr, bd);
  for (auto *v : {&c->bsv, &c->bxf, &c->bcols}) v->alloc(nT * nr, bd);
  c->bpartial.alloc(2LL * kColDotBlocks * kMaxCols, bd);
  c->bsc.alloc(8 * kMaxCols, bd);
  c->bact.alloc(kMaxCols, bd);
  if (!c->host_bsc) {
    HIP_OK(hipHostMalloc((void **)&c->host_bsc, 8 * kMaxCols * sizeof(double), 0));
    HIP_OK(hipHostMalloc((void **)&c->host_bact, kMaxCols * sizeof(int), 0));
  }
  c->bcap = nr;
}

// The smoother's patch sum on level l for nr columns: stored inverses, or
// inverses recomputed in the application (FP64).
template <typename T>
void smooth_apply_blk(dpg_ctx *c, int l, const cplx_t<T> *x, cplx_t<T> *y, const cplx_t<T> *r,
                      int mode, T theta, int nr, bool gathered = false, bool fwd = false) {
  LevelData &f = c->lv[l];
  if constexpr (sizeof(T) == 8) {
    if (c->opt.flags & DPG_RECOMPUTE_PATCHES) {
      if (gathered || fwd) throw DpgError(-1, "recomputed patches take no forwarded vectors");
      smooth_recompute(c, l, x, y, r, mode, theta, nr);
      return;
    }
  }
  herm_apply_blk<T>(f.Sset, f.Sb, x, y, r, mode, theta, nr, c->stream, gathered,
                    fwd ? &f.Mset : nullptr, fwd ? &f.Mb : nullptr);
}

template <typename T> void vcycle_blk(dpg_ctx *c, int l, int nr) {
  using B = LB<T>;
  using BB = LBB<T>;
  LevelData &f = c->lv[l];
  const hipStream_t s = c->stream;
  const T th = (T)c->opt.theta;
  auto r = BB::r(f), x = BB::x(f), res = BB::res(f), rc = BB::rc(f), ec = BB::ec(f);
  // forwarding between the smoother and the residual as in vcycle
  const bool fw = sizeof(T) == 4 || !(c->opt.flags & DPG_RECOMPUTE_PATCHES);
  HermSet *toS = fw ? &f.Sset : nullptr;
  HermBlockBufs *bS = fw ? &f.Sb : nullptr;
  if (c->opt.nu_pre == 0) launch_zero(f.nM * nr, x, s);
  for (int k = 0; k < c->opt.nu_pre; ++k) {
    if (k == 0) {
      smooth_apply_blk<T>(c, l, r, x, nullptr, RED_SET_SCALED, th, nr, false, fw);
    } else {
      herm_apply_blk<T>(f.Mset, f.Mb, x, res, r, RED_RESID, (T)0, nr, s, fw, toS, bS);
      smooth_apply_blk<T>(c, l, res, x, nullptr, RED_AXPY, th, nr, fw, fw);
    }
  }
  herm_apply_blk<T>(f.Mset, f.Mb, x, res, r, RED_RESID, (T)0, nr, s, fw && c->opt.nu_pre > 0);
  LevelData &g = c->lv[l - 1];
  {
    PROF(DPG_K_TRANSFER, 0);
    launch_csr_blk<T>(g.num.n, f.Ptptr.p, f.Ptcol.p, B::Ptv(f), res, rc, 0, nr, s);
  }
  if (l - 1 == 0) {
    herm_apply_blk<T>(c->T0set, c->T0b, rc, ec, nullptr, RED_SET, (T)1, nr, s);
  } else {
    {
      PROF(DPG_K_CONDENSE, 0);
      condense_level<T>(g, B::WH(g), rc, BB::cc(g), BB::r(g), nr, s);
    }
    vcycle_blk<T>(c, l - 1, nr);
    PROF(DPG_K_EXPAND, 0);
    expand_level<T>(g, B::WH(g), B::Ti(g), rc, BB::x(g), ec, nr, s);
  }
  {
    PROF(DPG_K_TRANSFER, 0);
    launch_csr_blk<T>(f.nM, f.Pptr.p, f.Pcol.p, B::Pv(f), ec, x, 1, nr, s);
  }
  for (int k = 0; k < c->opt.nu_post; ++k) {
    herm_apply_blk<T>(f.Mset, f.Mb, x, res, r, RED_RESID, (T)0, nr, s, fw && k > 0, toS, bS);
    smooth_apply_blk<T>(c, l, res, x, nullptr, RED_AXPY, th, nr, fw, fw && k + 1 < c->opt.nu_post);
  }
}

void precondition_blk(dpg_ctx *c, const double2 *r, double2 *z, int nr) {
  LevelData &top = c->lv[c->L];
  const hipStream_t s = c->stream;
  const int64_t n = top.nM * nr;
  if (c->opt.precision == DPG_MIXED) {
    launch_to32(n, r, top.br32.p, s);
    vcycle_blk<float>(c, c->L, nr);
    launch_to64(n, top.bx32.p, z, s);
  } else {
    HIP_OK(hipMemcpyAsync(top.br64.p, r, n * 16, hipMemcpyDeviceToDevice, s));
    vcycle_blk<double>(c, c->L, nr);
    HIP_OK(hipMemcpyAsync(z, top.bx64.p, n * 16, hipMemcpyDeviceToDevice, s));
  }
}

// ---- block PCG with columns that join and leave (continuous batching) -----------------
//
// The block vectors (trace right-hand sides bsv, and x, r, p, z, z_old on the
// finest macro grid) hold the session's width w columns interleaved.  Each
// column runs its own CG recurrence (its own alpha and beta; a finished
// column is frozen: alpha = beta = 0).  One iteration is (B) the V-cycle on
// all columns, beta and the search directions, then (A) the block matvec,
// alpha and the x / r updates; a column that joins starts with x = p = z =
// z_old = 0, r = b and rz = 1, so that its first (B) sets p = z and
// rz = r^H z -- the first step of PCG -- while the other columns go on.

void batch_close(dpg_ctx *c) {
  BatchSession &S = c->bs;
  S.graphs.reset();
  S.gw = 0;
  S.open = false;
  S.max = S.w = 0;
  S.done.clear();   // finished slots not taken (dpg_solve's block path takes none)
}

void batch_open(dpg_ctx *c, int max_slots) {
  if (max_slots < 1 || max_slots > kMaxCols)
    throw DpgError(DPG_EINVAL, "a batch holds 1 to 32 columns");
  batch_close(c);
  ensure_block(c, max_slots);
  BatchSession &S = c->bs;
  LevelData &top = c->lv[c->L];
  const hipStream_t s = c->stream;
  for (auto *v : {&c->bx, &c->br, &c->bp, &c->bz, &c->bzo}) launch_zero(top.nM * max_slots, v->p, s);
  launch_zero(top.num.n * max_slots, c->bsv.p, s);
  launch_zero(4 * kMaxCols, reinterpret_cast<double2 *>(c->bsc.p), s);
  for (int k = 0; k < kMaxCols; ++k) {
    S.state[k] = 0;
    S.iters[k] = 0;
    S.bb[k] = S.rr[k] = 0.0;
    S.tol[k] = 0.0;
    c->host_bact[k] = 0;
  }
  S.act_dirty = true;
  S.max = max_slots;
  S.w = 1;
  S.cur = 0;
  S.open = true;
}

// Width w_new (columns beyond it must be free): the block vectors are laid
// out again through the matvec output, which holds nothing between steps.
void batch_width(dpg_ctx *c, int w_new) {
  BatchSession &S = c->bs;
  if (w_new == S.w) return;
  LevelData &top = c->lv[c->L];
  const hipStream_t s = c->stream;
  const int64_t nM = top.nM, nT = top.num.n;
  for (auto *v : {&c->bx, &c->br, &c->bp, &c->bz, &c->bzo}) {
    HIP_OK(hipMemcpyAsync(c->bq.p, v->p, nM * S.w * 16, hipMemcpyDeviceToDevice, s));
    launch_rewidth(nM, S.w, w_new, c->bq.p, v->p, s);
  }
  HIP_OK(hipMemcpyAsync(c->bxf.p, c->bsv.p, nT * S.w * 16, hipMemcpyDeviceToDevice, s));
  launch_rewidth(nT, S.w, w_new, c->bxf.p, c->bsv.p, s);
  S.w = w_new;
}

// A right-hand side sv (trace vector, device) joins in the lowest free slot.
int batch_add(dpg_ctx *c, const double2 *sv, double tol) {
  BatchSession &S = c->bs;
  int k = 0;
  while (k < S.max && S.state[k] != 0) ++k;
  if (k == S.max) throw DpgError(DPG_EINVAL, "every slot of the batch is in use");
  if (k >= S.w) {
    int w = 1;
    while (w <= k) w *= 2;
    batch_width(c, std::min(w, S.max));
  }
  LevelData &top = c->lv[c->L];
  const hipStream_t s = c->stream;
  const int64_t nM = top.nM, nT = top.num.n;
  launch_set_col(nT, S.w, k, sv, c->bsv.p, s);
  condense_level<double>(top, top.WH.p, sv, top.c64.p, c->b.p, 1, s);
  launch_zero(4, reinterpret_cast<double2 *>(c->sc.p), s);
  dot_re(nM, c->b.p, c->b.p, c->partial.p, c->sc.p + 5, s);
  launch_set_col(nM, S.w, k, c->b.p, c->br.p, s);
  for (auto *v : {&c->bx, &c->bp, &c->bz, &c->bzo}) launch_set_col(nM, S.w, k, nullptr, v->p, s);
  cgb_reset_col(c->bsc.p, k, s);
  read_sc(c, c->sc.p);
  const double bb = c->host_sc[5];
  if (!std::isfinite(bb)) throw DpgError(DPG_EINVAL, "right-hand side is not finite");
  S.bb[k] = bb;
  S.tol[k] = tol;
  S.iters[k] = 0;
  if (bb > 0.0) {
    S.state[k] = 1;
    S.rr[k] = 1.0;
    c->host_bact[k] = 1;
    S.act_dirty = true;
  } else {            // zero right-hand side: x = 0 after no iteration
    S.state[k] = 2;
    S.rr[k] = 0.0;
    S.done.push_back(k);
  }
  return k;
}

// Iterations of the running columns until one of them finishes or max_iters
// have run; appends the slots that finished to S.done.
void batch_step(dpg_ctx *c, int max_iters) {
  BatchSession &S = c->bs;
  LevelData &top = c->lv[c->L];
  const hipStream_t s = c->stream;
  const int64_t nM = top.nM;
  double *Sc = c->host_bsc;
  int *act = c->host_bact;
  const size_t done0 = S.done.size();
  for (int it = 0; it < max_iters && S.done.size() == done0; ++it) {
    int running = 0;
    for (int k = 0; k < S.w; ++k) running += S.state[k] == 1;
    if (!running) break;
    if (S.act_dirty) {
      HIP_OK(hipMemcpyAsync(c->bact.p, act, kMaxCols * sizeof(int), hipMemcpyHostToDevice, s));
      S.act_dirty = false;
    }
    const int w = S.w;
    auto part_a = [&]() {
      herm_apply_blk<double>(top.Mset, top.Mb, c->bp.p, c->bq.p, nullptr, RED_SET, 1.0, w, s);
      PROF(DPG_K_CG, 0);
      cgb_alpha(nM, w, c->bp.p, c->bq.p, c->bpartial.p, c->bsc.p, c->bact.p, s);
      cgb_update_xr(nM, w, c->bx.p, c->br.p, c->bp.p, c->bq.p, c->bpartial.p, c->bsc.p, s);
    };
    auto part_b = [&](double2 *zn, double2 *zp) {
      precondition_blk(c, c->br.p, zn, w);
      PROF(DPG_K_CG, 0);
      cgb_beta(nM, w, c->br.p, zn, zp, c->bpartial.p, c->bsc.p, c->bact.p, s);
      cgb_update_p(nM, w, c->bp.p, zn, c->bsc.p, s);
    };
    double2 *zb[2] = {c->bz.p, c->bzo.p};
    // HIP graphs of the three launch sequences, captured once per width
    // (B in two versions: z and z_old swap every iteration)
    const bool graphs = !c->prof.on;
    if (graphs && S.gw != w) {
      S.graphs.reset(new GraphSet());
      S.graphs->a = capture(s, part_a);
      S.graphs->b[0] = capture(s, [&]() { part_b(zb[0], zb[1]); });
      S.graphs->b[1] = capture(s, [&]() { part_b(zb[1], zb[0]); });
      S.gw = w;
    }
    S.cur ^= 1;
    if (graphs) {
      HIP_OK(hipGraphLaunch(S.graphs->b[S.cur], s));
      HIP_OK(hipGraphLaunch(S.graphs->a, s));
    } else {
      part_b(zb[S.cur], zb[S.cur ^ 1]);
      part_a();
    }
    HIP_OK(hipMemcpyAsync(Sc, c->bsc.p, 8 * kMaxCols * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (int k = 0; k < w; ++k) {
      if (S.state[k] != 1) continue;
      ++S.iters[k];
      const double rr = std::sqrt(Sc[4 * kMaxCols + k] / S.bb[k]);
      if (Sc[6 * kMaxCols + k] != 0.0 || !std::isfinite(rr)) {
        S.state[k] = 4;                      // breakdown (p^H M p <= 0 or not finite)
      } else {
        S.rr[k] = rr;
        if (rr <= S.tol[k]) S.state[k] = 2;
        else if (S.iters[k] >= c->opt.maxit) S.state[k] = 3;
      }
      if (S.state[k] != 1) {
        act[k] = 0;
        S.act_dirty = true;
        S.done.push_back(k);
      }
    }
  }
}

// Solution of a finished slot: its macro-grid column expanded to the full
// trace vector (recovery of the condensed unknowns) into xout (device); the
// slot becomes free and the width shrinks while its upper half is free.
int batch_take(dpg_ctx *c, int k, double2 *xout, int32_t *iters, double *relres) {
  BatchSession &S = c->bs;
  if (k < 0 || k >= S.max || S.state[k] < 2)
    throw DpgError(DPG_ESTATE, "slot " + std::to_string(k) + " holds no finished solve");
  LevelData &top = c->lv[c->L];
  const hipStream_t s = c->stream;
  const int64_t nM = top.nM, nT = top.num.n;
  launch_get_col(nM, S.w, k, c->bx.p, c->x.p, s);
  launch_get_col(nT, S.w, k, c->bsv.p, c->sB.p, s);
  expand_level<double>(top, top.WH.p, top.Tinv.p, c->sB.p, c->x.p, xout, 1, s);
  if (iters) *iters = S.iters[k];
  if (relres) *relres = S.rr[k];
  const int st = S.state[k] == 2 ? DPG_OK : S.state[k] == 3 ? DPG_ENOCONV : DPG_EBREAKDOWN;
  S.state[k] = 0;
  for (size_t i = 0; i < S.done.size(); ++i)
    if (S.done[i] == k) {
      S.done.erase(S.done.begin() + i);
      break;
    }
  int w = S.w;
  while (w > 1) {
    bool upper_free = true;
    for (int j = w / 2; j < w; ++j) upper_free = upper_free && S.state[j] == 0;
    if (!upper_free) break;
    w /= 2;
  }
  batch_width(c, w);
  return st;
}

// All nr columns of a freshly opened batch at once ([nr][n_trace], device): the block
// condensation and one reduction for every column, one host sync.
void batch_add_all(dpg_ctx *c, const double2 *sv_cols, int nr, double tol) {
  BatchSession &S = c->bs;
  LevelData &top = c->lv[c->L];
  const hipStream_t s = c->stream;
  const int64_t nM = top.nM, nT = top.num.n;
  S.w = nr;   // the vectors of a freshly opened batch are zero in every layout
  launch_interleave(nT, nr, sv_cols, c->bsv.p, s);
  condense_level<double>(top, top.WH.p, c->bsv.p, top.bc64.p, c->br.p, nr, s);
  for (int k = 0; k < nr; ++k) cgb_reset_col(c->bsc.p, k, s);
  cgb_dot(nM, nr, c->br.p, c->br.p, c->bpartial.p, c->bsc.p, 5, s);
  HIP_OK(hipMemcpyAsync(c->host_bsc, c->bsc.p, 8 * kMaxCols * sizeof(double),
                        hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  for (int k = 0; k < nr; ++k) {
    const double bb = c->host_bsc[5 * kMaxCols + k];
    if (!std::isfinite(bb)) throw DpgError(DPG_EINVAL, "right-hand side is not finite");
    S.bb[k] = bb;
    S.tol[k] = tol;
    S.iters[k] = 0;
    if (bb > 0.0) {
      S.state[k] = 1;
      S.rr[k] = 1.0;
      c->host_bact[k] = 1;
    } else {
      S.state[k] = 2;
      S.rr[k] = 0.0;
      S.done.push_back(k);
    }
  }
  S.act_dirty = true;
}

// dpg_solve's block path: nr <= kMaxCols loads sv_cols ([nr][n_trace],
// device) through one batch, full trace solutions to xcols likewise (block
// expansion of all columns).
int solve_block(dpg_ctx *c, const double2 *sv_cols, int nr, double tol, double2 *xcols,
                int32_t *iters, double *relres) {
  batch_open(c, nr);
  batch_add_all(c, sv_cols, nr, tol);
  BatchSession &S = c->bs;
  LevelData &top = c->lv[c->L];
  const int64_t nT = top.num.n;
  int status = DPG_OK;
  for (;;) {
    int running = 0;
    for (int k = 0; k < S.w; ++k) running += S.state[k] == 1;
    if (!running) break;
    batch_step(c, c->opt.maxit);
    for (int k = 0; k < S.w; ++k)
      if (S.state[k] == 4)
        throw DpgError(DPG_EBREAKDOWN, "CG breakdown in column " + std::to_string(k) +
                                           " at iteration " + std::to_string(S.iters[k]));
  }
  expand_level<double>(top, top.WH.p, top.Tinv.p, c->bsv.p, c->bx.p, c->bxf.p, nr, c->stream);
  launch_deinterleave(nT, nr, c->bxf.p, xcols, c->stream);
  for (int k = 0; k < nr; ++k) {
    iters[k] = S.iters[k];
    relres[k] = S.rr[k];
    if (S.state[k] == 3) status = DPG_ENOCONV;
  }
  HIP_OK(hipStreamSynchronize(c->stream));
  batch_close(c);
  return status;
}

template <typename V> int64_t put(const std::vector<V> &v, void *out, int64_t cap) {
  if (out && cap > 0) std::memcpy(out, v.data(), sizeof(V) * std::min<int64_t>(cap, (int64_t)v.size()));
  return (int64_t)v.size();
}
template <typename V> std::vector<int64_t> widen(const std::vector<V> &v) {
  return std::vector<int64_t>(v.begin(), v.end());
}
}  // namespace

// ---- API ------------------------------------------------------------------------------------

extern "C" {

void dpg_default_options(dpg_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = DPG_FP64;
  o->nu_pre = 1;
  o->nu_post = 1;
  o->nlevels = 0;
  o->maxit = 500;
  o->flags = 0;
  o->theta = 0.2;
  o->hbm_budget = 0;
  o->stream = nullptr;
}

int dpg_setup(const dpg_mesh *mesh, int p, int dp, double omega, const dpg_material *mat,
              const dpg_load *loads, int nrhs, const dpg_options *opt, dpg_ctx **out) {
  if (!out) return DPG_EINVAL;
  *out = nullptr;
  if (!mesh || mesh->n < 1 || p < 1 || dp < 1 || !(omega > 0) || !(mesh->side > 0) || nrhs < 0 ||
      (nrhs > 0 && !loads))
    return DPG_EINVAL;
  dpg_ctx *c = new dpg_ctx();
  int rc = guarded(c, [&]() {
    auto t0 = clk::now();
    if (opt) c->opt = *opt;
    else dpg_default_options(&c->opt);
    if (!(c->opt.theta > 0.0 && c->opt.theta < 0.25))
      throw DpgError(DPG_EINVAL, "smoother damping must lie in (0, 1/4)");
    if (c->opt.nu_pre < 0 || c->opt.nu_post < 0 || c->opt.maxit < 1)
      throw DpgError(DPG_EINVAL, "bad smoothing counts or maxit");
    if (c->opt.precision != DPG_FP64 && c->opt.precision != DPG_MIXED)
      throw DpgError(DPG_EINVAL, "unknown precision mode");
    if ((c->opt.flags & DPG_RECOMPUTE_PATCHES) && c->opt.precision != DPG_FP64)
      throw DpgError(DPG_EINVAL, "recomputed patch inverses are an FP64 path");
    HIP_OK(hipGetDevice(&c->device));
    (void)scratch_device_ptr(c->device, true);   // once per device, with it current
    c->stream = (hipStream_t)c->opt.stream;
    if (!c->stream) {
      // an own stream (blocking, so ordered with the caller's null-stream
      // work): the solve captures launch sequences as graphs, which the
      // null stream does not allow
      HIP_OK(hipStreamCreate(&c->own_stream));
      c->stream = c->own_stream;
    }
    HIP_OK(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
    HIP_OK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    for (int k = 0; k < 2; ++k) {   // third and fourth setup streams (elements, patches)
      HIP_OK(hipStreamCreateWithFlags(&c->paux[k], hipStreamNonBlocking));
      HIP_OK(hipEventCreateWithFlags(&c->ev_pjoin[k], hipEventDisableTiming));
    }
    c->bud.limit = c->opt.hbm_budget;
    c->N = mesh->n;
    c->p = p;
    c->dp = dp;
    c->omega = omega;
    c->side = mesh->side;
    for (int k = 0; k < 3; ++k) c->org[k] = mesh->origin[k];
    const int64_t nel = (int64_t)c->N * c->N * c->N;
    c->c_h.assign(nel, 1.0);
    if (mat && mat->c)
      for (int64_t e = 0; e < nel; ++e) {
        if (!(mat->c[e] > 0)) throw DpgError(DPG_EINVAL, "wave speed must be positive");
        c->c_h[e] = mat->c[e];
      }
    std::vector<double> kap(nel), Z(nel);
    for (int64_t e = 0; e < nel; ++e) {
      kap[e] = 1.0 / (c->c_h[e] * c->c_h[e]);
      Z[e] = c->c_h[e];
    }
    c->kappa.upload(kap, &c->bud, c->stream);
    c->Zel.upload(Z, &c->bud, c->stream);
    c->el.build(p);
    build_elem_tables(p, dp, c->tables_h);
    c->tables.upload(std::vector<ElemTables>{c->tables_h}, &c->bud, c->stream);
    std::vector<int4> test, trial;
    build_descriptors(p, dp, test, trial);
    c->n_test = (int)test.size();
    c->n_field = 4 * p * p * p;
    c->n_tr = c->el.n_tr;
    c->m = c->n_field + c->n_tr;
    if ((int)trial.size() != c->m) throw DpgError(DPG_EINVAL, "descriptor size mismatch");
    c->testd.upload(test, &c->bud, c->stream);
    c->triald.upload(trial, &c->bud, c->stream);
    set_loads(c, loads, nrhs);
    if (c->opt.p_min < 0 || c->opt.p_min > p)
      throw DpgError(DPG_EINVAL, "p_min must lie in [1, p] (0: no order levels)");
    const std::vector<std::pair<int, int>> plan =
        level_plan(c->N, p, c->opt.p_min, c->opt.nlevels);
    if (plan.size() < 2)
      throw DpgError(DPG_EINVAL, "no coarser level (an even mesh size or p_min < p is needed)");
    if ((c->opt.flags & DPG_STORE_COARSE) && plan.back().second != p)
      throw DpgError(DPG_EINVAL, "stored coarse operators are for mesh levels only");
    c->L = (int)plan.size() - 1;
    c->lv.resize(c->L + 1);
    const bool mixed = c->opt.precision == DPG_MIXED;
    const hipStream_t s = c->stream;
    for (int l = 0; l <= c->L; ++l) {
      LevelData &f = c->lv[l];
      f.N = plan[c->L - l].first;
      f.q = plan[c->L - l].second;
      f.el.build(f.q);
      f.ntr = f.el.n_tr;
      f.nel = f.N * f.N * f.N;
      f.num.build(f.N, f.q);
      f.edofs_h = element_dofs(f.num, f.el);
      f.edofs.upload(f.edofs_h, &c->bud, s);
    }
    for (int l = 1; l <= c->L; ++l) {
      LevelData &f = c->lv[l];
      LevelData &g = c->lv[l - 1];
      f.macro = true;
      f.order = g.N == f.N;
      f.ntr_c = g.ntr;
      if (f.order) {
        f.mc.build_order(f.num, f.el);
        f.P.build_order(f.mc, f.num, g.num, f.el, g.el);
      } else {
        f.mc.build(f.num, f.el);
        f.P.build(f.mc, f.num, g.num, f.el);
      }
      f.nblk = f.mc.Nc * f.mc.Nc * f.mc.Nc;
      f.nBf = f.mc.nBf;
      f.nI = f.mc.nI;
      f.nM = f.mc.nM;
      f.macroB.upload(f.mc.macro_B, &c->bud, s);
      f.blkI.upload(f.mc.blkI, &c->bud, s);
      std::vector<int32_t> bm(f.mc.blkB.size());
      for (size_t k = 0; k < bm.size(); ++k) bm[k] = f.mc.blkB[k] >= 0 ? f.mc.macro_of[f.mc.blkB[k]] : -1;
      f.blkBm.upload(bm, &c->bud, s);
      // condensation reduction lists: (block, slot) holding each macro unknown
      std::vector<int32_t> cnt(f.nM + 1, 0), ent;
      for (size_t k = 0; k < bm.size(); ++k)
        if (bm[k] >= 0) cnt[bm[k] + 1]++;
      for (int64_t mm = 0; mm < f.nM; ++mm) cnt[mm + 1] += cnt[mm];
      ent.assign(cnt[f.nM], 0);
      std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
      for (size_t k = 0; k < bm.size(); ++k)
        if (bm[k] >= 0) ent[fill[bm[k]]++] = (int32_t)k;
      f.cred_ptr.upload(cnt, &c->bud, s);
      f.cred_ent.upload(ent, &c->bud, s);
      f.patch_ptr.upload(f.mc.patch_ptr, &c->bud, s);
      f.patch_slot.upload(f.mc.patch_slot, &c->bud, s);
      f.Pptr.upload(f.P.ptr, &c->bud, s);
      f.Pcol.upload(f.P.col, &c->bud, s);
      f.Pval.upload(f.P.val, &c->bud, s);
      f.Ptptr.upload(f.P.tptr, &c->bud, s);
      f.Ptcol.upload(f.P.tcol, &c->bud, s);
      f.Ptval.upload(f.P.tval, &c->bud, s);
      if (mixed) {
        std::vector<float> pv(f.P.val.begin(), f.P.val.end()), ptv(f.P.tval.begin(), f.P.tval.end());
        f.Pval32.upload(pv, &c->bud, s);
        f.Ptval32.upload(ptv, &c->bud, s);
      }
      // block sets
      std::vector<int32_t> msz(f.nblk), midx;
      for (int b = 0; b < f.nblk; ++b) {
        msz[b] = (int32_t)(f.mc.blkB_ptr[b + 1] - f.mc.blkB_ptr[b]);
        for (int64_t k = f.mc.blkB_ptr[b]; k < f.mc.blkB_ptr[b + 1]; ++k)
          midx.push_back(f.mc.macro_of[f.mc.blkB[(int64_t)b * f.nBf + f.mc.blkB_present[k]]]);
      }
      f.Mset.build(msz, midx, f.nM, !mixed || l == c->L, mixed, &c->bud, s);
      const int np = (int)f.mc.patch_ptr.size() - 1;
      std::vector<int32_t> psz(np);
      for (int v = 0; v < np; ++v) psz[v] = (int32_t)(f.mc.patch_ptr[v + 1] - f.mc.patch_ptr[v]);
      if (c->opt.flags & DPG_RECOMPUTE_PATCHES) {   // no tiles: the inverses are recomputed
        std::vector<int32_t> pidx((size_t)f.nblk * f.nBf, -1);   // slot -> packed position
        for (int b = 0; b < f.nblk; ++b)
          for (int64_t k = f.mc.blkB_ptr[b]; k < f.mc.blkB_ptr[b + 1]; ++k)
            pidx[(size_t)b * f.nBf + f.mc.blkB_present[k]] = (int32_t)(k - f.mc.blkB_ptr[b]);
        f.mpidx.upload(pidx, &c->bud, s);
        f.Sset.build(psz, f.mc.patch_idx, f.nM, false, false, &c->bud, s);
        f.Sset.xl64.alloc(f.Sset.nloc, &c->bud);
        f.Sset.yl64.alloc(f.Sset.nloc, &c->bud);
      } else {
        f.Sset.build(psz, f.mc.patch_idx, f.nM, !mixed, mixed, &c->bud, s);
      }
      f.Mset.prof = &c->prof;
      f.Sset.prof = &c->prof;
      // work vectors
      const int64_t nc = c->lv[l - 1].num.n;
      if (mixed) {
        f.r32.alloc(f.nM, &c->bud);
        f.x32.alloc(f.nM, &c->bud);
        f.res32.alloc(f.nM, &c->bud);
        f.rc32.alloc(nc, &c->bud);
        f.ec32.alloc(nc, &c->bud);
        f.c32.alloc((int64_t)f.nblk * f.nBf, &c->bud);
      } else {
        f.r64.alloc(f.nM, &c->bud);
        f.x64.alloc(f.nM, &c->bud);
        f.res64.alloc(f.nM, &c->bud);
        f.rc64.alloc(nc, &c->bud);
        f.ec64.alloc(nc, &c->bud);
      }
      if (!mixed || l == c->L) f.c64.alloc((int64_t)f.nblk * f.nBf, &c->bud);
    }
    if (c->opt.flags & DPG_STORE_COARSE) {
      // "store" coarse operators (Sec. 3, alternative construction): each
      // coarser mesh gets its own element material, which must be uniform
      // over the fine elements a coarse element covers
      for (int l = 0; l < c->L; ++l) {
        LevelData &f = c->lv[l];
        const int r = c->N / f.N;
        std::vector<double> kl(f.nel), zl(f.nel);
        for (int e = 0; e < f.nel; ++e) {
          const int i = e % f.N, j = (e / f.N) % f.N, k = e / (f.N * f.N);
          const double c0 = c->c_h[(int64_t)i * r + (int64_t)c->N * (j * r + (int64_t)c->N * k * r)];
          for (int a = 0; a < r; ++a)
            for (int b = 0; b < r; ++b)
              for (int d = 0; d < r; ++d) {
                const int64_t fe = (int64_t)(i * r + a) +
                                   (int64_t)c->N * ((j * r + b) + (int64_t)c->N * (k * r + d));
                if (c->c_h[fe] != c0)
                  throw DpgError(DPG_EINVAL,
                                 "stored coarse operators need a wave speed that is constant on "
                                 "every element of every coarser mesh");
              }
          kl[e] = 1.0 / (c0 * c0);
          zl[e] = c0;
        }
        f.kappa.upload(kl, &c->bud, s);
        f.Zel.upload(zl, &c->bud, s);
      }
    }
    {
      const int64_t n0 = c->lv[0].num.n;
      std::vector<int32_t> sz{(int32_t)n0}, id(n0);
      for (int64_t i = 0; i < n0; ++i) id[i] = (int32_t)i;
      c->T0set.build(sz, id, n0, !mixed, mixed, &c->bud, s);
      c->T0set.prof = &c->prof;
    }
    // element load assembly lists of the finest mesh
    LevelData &top = c->lv[c->L];
    {
      const int64_t n = top.num.n;
      std::vector<int32_t> cnt(n + 1, 0), ent;
      for (int32_t t : top.edofs_h)
        if (t >= 0) cnt[t + 1]++;
      for (int64_t t = 0; t < n; ++t) cnt[t + 1] += cnt[t];
      ent.assign(cnt[n], 0);
      std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
      for (size_t k = 0; k < top.edofs_h.size(); ++k)
        if (top.edofs_h[k] >= 0) ent[fill[top.edofs_h[k]]++] = (int32_t)k;
      c->asm_ptr.upload(cnt, &c->bud, s);
      c->asm_ent.upload(ent, &c->bud, s);
    }
    const int64_t nM = top.nM, nT = top.num.n;
    for (auto *v : {&c->b, &c->x, &c->r, &c->z, &c->zo, &c->pv, &c->q}) v->alloc(nM, &c->bud);
    c->xfull.alloc(nT, &c->bud);
    c->sB.alloc(nT, &c->bud);
    c->partial.alloc(2 * kDotBlocks, &c->bud);
    c->sc.alloc(8, &c->bud);
    HIP_OK(hipHostMalloc((void **)&c->host_sc, 8 * sizeof(double), 0));
    const int64_t rec_bytes = 16LL * top.nel * ((int64_t)c->n_field * c->n_field +
                                                (int64_t)c->n_field * (c->n_tr + c->nrhs));
    c->keep_recovery = rec_bytes <= 4000000000LL;
    HIP_OK(hipStreamSynchronize(s));
    c->ms[0] = ms_since(t0);
    c->stage = 1;
    return DPG_OK;
  });
  if (rc != DPG_OK) {
    std::string m = c->err;
    delete c;
    // no context to hold the message: report through stderr-free path (code only)
    (void)m;
    return rc;
  }
  *out = c;
  return DPG_OK;
}

int dpg_assemble(dpg_ctx *c) {
  if (!c) return DPG_EINVAL;
  return guarded(c, [&]() {
    if (c->stage < 1) throw DpgError(DPG_ESTATE, "dpg_setup first");
    if (c->released) throw DpgError(DPG_ESTATE, "setup data released");
    auto t0 = clk::now();
    LevelData &top = c->lv[c->L];
    top.E.ensure((int64_t)top.nel * c->n_tr * c->n_tr, &c->bud);
    c->s_elem.ensure(std::max<int64_t>(1, (int64_t)c->nrhs * top.nel * c->n_tr), &c->bud);
    c->s_asm.ensure(std::max<int64_t>(1, (int64_t)c->nrhs * top.num.n), &c->bud);
    if (c->keep_recovery) {
      c->rec_L.ensure((int64_t)top.nel * c->n_field * c->n_field, &c->bud);
      c->rec_Y.ensure((int64_t)top.nel * c->n_field * c->n_tr, &c->bud);
      c->rec_Yb.ensure(std::max<int64_t>(1, (int64_t)top.nel * c->n_field * c->nrhs), &c->bud);
    }
    element_stage(c, c->L, true);
    c->prof.flush();
    c->ms[1] = ms_since(t0);
    c->stage = 2;
    return DPG_OK;
  });
}

int dpg_build_hierarchy(dpg_ctx *c) {
  if (!c) return DPG_EINVAL;
  return guarded(c, [&]() {
    if (c->stage < 2) throw DpgError(DPG_ESTATE, "dpg_assemble first");
    if (c->released) throw DpgError(DPG_ESTATE, "setup data released");
    auto t0 = clk::now();
    build_hierarchy(c);
    c->prof.flush();
    c->ms[2] = ms_since(t0);
    c->stage = 3;
    return DPG_OK;
  });
}

int dpg_release_setup(dpg_ctx *c) {
  if (!c) return DPG_EINVAL;
  return guarded(c, [&]() {
    if (c->stage < 3) throw DpgError(DPG_ESTATE, "dpg_build_hierarchy first");
    HIP_OK(hipStreamSynchronize(c->stream));
    HIP_OK(hipStreamSynchronize(c->aux));
    for (hipStream_t x : c->paux)
      if (x) HIP_OK(hipStreamSynchronize(x));
    const bool rec = c->opt.flags & DPG_RECOMPUTE_PATCHES;   // the smoother needs the
                                                             // patch work areas
    for (LevelData &f : c->lv) {
      f.E.release();
      f.Mfull.release();
    }
    for (int k = 0; k < 2; ++k) {
      c->mT[k].release();
      c->mLinv[k].release();
      c->mX[k].release();
      c->mwk[k].release();
    }
    for (int k = 0; k < 4 && !rec; ++k) {
      c->pS[k].release();
      c->pX[k].release();
      c->pwk[k].release();
    }
    c->zF.release();
    c->zLi.release();
    c->zTi.release();
    c->zwk.release();
    c->T0.release();
    // load updates go through the class maps from now on, so the element-stage
    // work areas can go too (a later element pass, the error indicator,
    // plans and allocates them again)
    if (c->lm.state == 0) build_load_maps(c);
    if (c->lm.state == 1) {
      ElemPlan &P = c->ep;
      for (int k = 0; k < 4; ++k) {
        P.G[k].release();
        P.BL[k].release();
        P.K[k].release();
        P.wk[k].release();
        P.X[k].release();
      }
      P.mp = -1;
      P.nel = -1;
      P.gR_nr = 0;
    }
    c->released = true;
    return DPG_OK;
  });
}

int dpg_load_rhs(dpg_ctx *c, const dpg_load *loads, int nrhs, double *s_out) {
  if (!c) return DPG_EINVAL;
  return guarded(c, [&]() {
    if (c->stage < 2) throw DpgError(DPG_ESTATE, "dpg_assemble first");
    if (nrhs < 1 || !loads) throw DpgError(DPG_EINVAL, "need at least one load");
    LevelData &top = c->lv[c->L];
    set_loads(c, loads, nrhs);
    c->s_elem.ensure((int64_t)nrhs * top.nel * c->n_tr, &c->bud);
    c->s_asm.ensure((int64_t)nrhs * top.num.n, &c->bud);
    if (c->keep_recovery)
      c->rec_Yb.ensure((int64_t)top.nel * c->n_field * c->nrhs, &c->bud);
    std::vector<int32_t> list;
    const bool everywhere = source_elements(c, list);
    if (c->lm.state == 0) build_load_maps(c);
    if (c->lm.state == 1) {
      // the class maps: the load kernel and one product per element
      const hipStream_t s = c->stream;
      if (!everywhere) {
        launch_zero(c->s_elem.n, c->s_elem.p, s);
        if (c->keep_recovery) launch_zero(c->rec_Yb.n, c->rec_Yb.p, s);
        grow(c->elist, std::max<int64_t>(1, (int64_t)list.size()), &c->bud);
        if (!list.empty())
          HIP_OK(hipMemcpyAsync(c->elist.p, list.data(), list.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, s));
      }
      load_by_maps(c, list, c->elist.p, everywhere);
    } else if (everywhere) {
      element_stage(c, c->L, false);
    } else {
      // point sources only: the elements near a source carry the whole load
      const hipStream_t s = c->stream;
      launch_zero(c->s_elem.n, c->s_elem.p, s);
      if (c->keep_recovery) launch_zero(c->rec_Yb.n, c->rec_Yb.p, s);
      grow(c->elist, std::max<int64_t>(1, (int64_t)list.size()), &c->bud);
      if (!list.empty())
        HIP_OK(hipMemcpyAsync(c->elist.p, list.data(), list.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, s));
      HIP_OK(hipStreamSynchronize(s));
      element_stage(c, c->L, false, nullptr, c->elist.p, (int)list.size());
    }
    c->prof.flush();
    if (s_out) {
      const bool dev = c->opt.flags & DPG_DEVICE_PTRS;
      HIP_OK(hipMemcpyAsync(s_out, c->s_asm.p, (size_t)nrhs * top.num.n * 16,
                            dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
      HIP_OK(hipStreamSynchronize(c->stream));
    }
    return DPG_OK;
  });
}

int dpg_solve(dpg_ctx *c, const double *rhs, int nrhs, double tol, double *x_out,
              int32_t *iters_out, double *relres_out) {
  if (!c) return DPG_EINVAL;
  return guarded(c, [&]() {
    if (c->stage < 3) throw DpgError(DPG_ESTATE, "dpg_build_hierarchy first");
    if (nrhs < 1 || !(tol >= 0.0)) throw DpgError(DPG_EINVAL, "bad nrhs or tol");
    if (!rhs && nrhs > c->nrhs) throw DpgError(DPG_EINVAL, "more columns than assembled loads");
    auto t0 = clk::now();
    LevelData &top = c->lv[c->L];
    const int64_t nT = top.num.n;
    const bool dev = c->opt.flags & DPG_DEVICE_PTRS;
    int status = DPG_OK;
    if (nrhs > 1 && !(c->opt.flags & DPG_COLUMNWISE)) {
      if (c->bs.open) throw DpgError(DPG_ESTATE, "a batch is open (dpg_batch_close first)");
      for (int k0 = 0; k0 < nrhs; k0 += kMaxCols) {
        const int nr = std::min(kMaxCols, nrhs - k0);
        ensure_block(c, nr);
        const double2 *sv;
        if (rhs) {
          HIP_OK(hipMemcpyAsync(c->bcols.p, rhs + 2 * nT * k0, nT * nr * 16,
                                dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
          sv = c->bcols.p;
        } else {
          sv = c->s_asm.p + nT * k0;
        }
        std::vector<int32_t> it(nr);
        std::vector<double> rr(nr);
        const int st = solve_block(c, sv, nr, tol, c->bcols.p, it.data(), rr.data());
        if (st != DPG_OK) status = st;
        for (int k = 0; k < nr; ++k) {
          if (iters_out) iters_out[k0 + k] = it[k];
          if (relres_out) relres_out[k0 + k] = rr[k];
        }
        if (x_out) {
          HIP_OK(hipMemcpyAsync(x_out + 2 * nT * k0, c->bcols.p, nT * nr * 16,
                                dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
          HIP_OK(hipStreamSynchronize(c->stream));
        }
      }
    } else {
      status = solve_columns(c, rhs, nrhs, tol, x_out, iters_out, relres_out, c->partial.p,
                             c->sc.p, true);
    }
    c->prof.flush();
    c->ms[3] = ms_since(t0);
    if (status == DPG_ENOCONV) c->err = "maximum number of iterations reached";
    return status;
  });
}

int dpg_solve_noalloc(dpg_ctx *c, const double *rhs, int nrhs, double tol, double *x_out,
                      int32_t *iters_out, double *relres_out) {
  if (!c) return DPG_EINVAL;
  return guarded(c, [&]() {
    if (c->stage < 3) throw DpgError(DPG_ESTATE, "dpg_build_hierarchy first");
    if (nrhs < 1 || !(tol >= 0.0)) throw DpgError(DPG_EINVAL, "bad nrhs or tol");
    if (!rhs && nrhs > c->nrhs) throw DpgError(DPG_EINVAL, "more columns than assembled loads");
    if (c->prof.on)
      throw DpgError(DPG_ESTATE, "kernel profiling creates events: switch it off for this call");
    // The scratch holds the reductions of one column; columns are solved one
    // after the other, so every size the context accepts fits.
    static_assert(2 * kDotBlocks + 8 <= kScratchDoubles, "solve scratch too small");
    double *sp = scratch_device_ptr(c->device, false);
    if (!sp) throw DpgError(DPG_ESTATE, "solve scratch not set up on this device");
    auto t0 = clk::now();
    const int status =
        solve_columns(c, rhs, nrhs, tol, x_out, iters_out, relres_out, sp, sp + 2 * kDotBlocks,
                      false);
    c->ms[3] = ms_since(t0);
    if (status == DPG_ENOCONV) c->err = "maximum number of iterations reached";
    return status;
  });
}

int dpg_get_fields(dpg_ctx *c, const double *x, int nrhs, double *fields_out) {
  if (!c) return DPG_EINVAL;
  return guarded(c, [&]() -> int {
    if (c->stage < 2) throw DpgError(DPG_ESTATE, "dpg_assemble first");
    if (!c->keep_recovery) throw DpgError(DPG_ENOMEM, "recovery data was not kept (too large)");
    if (!x || !fields_out || nrhs < 1 || nrhs > c->nrhs)
      throw DpgError(DPG_EINVAL, "need x and fields_out, 1 <= nrhs <= assembled loads");
    LevelData &top = c->lv[c->L];
    const int64_t nT = top.num.n, nfe = (int64_t)top.nel * c->n_field;
    const bool dev = c->opt.flags & DPG_DEVICE_PTRS;
    DevBuf<double2> out;
    out.alloc(nfe, &c->bud);
    for (int k = 0; k < nrhs; ++k) {
      HIP_OK(hipMemcpyAsync(c->sB.p, x + 2 * nT * k, nT * 16,
                            dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
      launch_fields(c->rec_L.p, c->rec_Y.p, c->rec_Yb.p, c->n_field, c->n_tr, c->nrhs, k, top.edofs.p,
                    top.nel, c->sB.p, out.p, c->stream);
      HIP_OK(hipMemcpyAsync(fields_out + 2 * nfe * k, out.p, nfe * 16,
                            dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
      HIP_OK(hipStreamSynchronize(c->stream));
    }
    return DPG_OK;
  });
}

int dpg_batch_open(dpg_ctx *c, int max_slots) {
  if (!c) return DPG_EINVAL;
  return guarded(c, [&]() {
    if (c->stage < 3) throw DpgError(DPG_ESTATE, "dpg_build_hierarchy first");
    batch_open(c, max_slots);
    return DPG_OK;
  });
}

int dpg_batch_add(dpg_ctx *c, const double *rhs, int load_col, double tol, int32_t *slot_out) {
  if (!c) return DPG_EINVAL;
  return guarded(c, [&]() {
    if (!c->bs.open) throw DpgError(DPG_ESTATE, "dpg_batch_open first");
    if (!(tol >= 0.0)) throw DpgError(DPG_EINVAL, "bad tol");
    const int64_t nT = c->lv[c->L].num.n;
    const double2 *sv;
    if (rhs) {
      const bool dev = c->opt.flags & DPG_DEVICE_PTRS;
      HIP_OK(hipMemcpyAsync(c->sB.p, rhs, nT * 16,
                            dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
      sv = c->sB.p;
    } else {
      if (load_col < 0 || load_col >= c->nrhs)
        throw DpgError(DPG_EINVAL, "load column out of range");
      sv = c->s_asm.p + nT * load_col;
    }
    const int k = batch_add(c, sv, tol);
    if (slot_out) *slot_out = k;
    return DPG_OK;
  });
}

int dpg_batch_step(dpg_ctx *c, int max_iters, int32_t *done_out, int32_t *ndone_out) {
  if (!c) return DPG_EINVAL;
  return guarded(c, [&]() {
    if (!c->bs.open) throw DpgError(DPG_ESTATE, "dpg_batch_open first");
    if (max_iters < 0) throw DpgError(DPG_EINVAL, "bad max_iters");
    auto t0 = clk::now();
    batch_step(c, max_iters);
    c->prof.flush();
    c->ms[3] = ms_since(t0);
    const BatchSession &S = c->bs;
    if (done_out)
      for (size_t i = 0; i < S.done.size(); ++i) done_out[i] = S.done[i];
    if (ndone_out) *ndone_out = (int32_t)S.done.size();
    return DPG_OK;
  });
}

int dpg_batch_take(dpg_ctx *c, int slot, double *x_out, int32_t *iters_out, double *relres_out) {
  if (!c) return DPG_EINVAL;
  return guarded(c, [&]() {
    if (!c->bs.open) throw DpgError(DPG_ESTATE, "dpg_batch_open first");
    const int64_t nT = c->lv[c->L].num.n;
    const int st = batch_take(c, slot, c->xfull.p, iters_out, relres_out);
    if (x_out) {
      const bool dev = c->opt.flags & DPG_DEVICE_PTRS;
      HIP_OK(hipMemcpyAsync(x_out, c->xfull.p, nT * 16,
                            dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    }
    HIP_OK(hipStreamSynchronize(c->stream));
    if (st == DPG_ENOCONV) c->err = "maximum number of iterations reached";
    if (st == DPG_EBREAKDOWN) c->err = "CG breakdown in slot " + std::to_string(slot);
    return st;
  });
}

int dpg_batch_close(dpg_ctx *c) {
  if (!c) return DPG_EINVAL;
  return guarded(c, [&]() {
    HIP_OK(hipStreamSynchronize(c->stream));
    batch_close(c);
    return DPG_OK;
  });
}

int dpg_error_indicator(dpg_ctx *c, const double *x, int nrhs, double *eta2_out) {
  if (!c) return DPG_EINVAL;
  return guarded(c, [&]() -> int {
    if (c->stage < 2) throw DpgError(DPG_ESTATE, "dpg_assemble first");
    if (!x || !eta2_out || nrhs < 1 || nrhs > c->nrhs)
      throw DpgError(DPG_EINVAL, "need x and eta2_out, 1 <= nrhs <= assembled loads");
    LevelData &top = c->lv[c->L];
    const int64_t nT = top.num.n, nel = top.nel;
    const bool dev = c->opt.flags & DPG_DEVICE_PTRS;
    DevBuf<double2> xs;
    DevBuf<double> eta;
    const double2 *xd = reinterpret_cast<const double2 *>(x);
    double *ed = eta2_out;
    if (!dev) {
      xs.alloc(nT * nrhs, &c->bud);
      HIP_OK(hipMemcpyAsync(xs.p, x, (size_t)nT * nrhs * 16, hipMemcpyHostToDevice, c->stream));
      eta.alloc(nel * nrhs, &c->bud);
      xd = xs.p;
      ed = eta.p;
    }
    IndicatorArgs ia{xd, nrhs, ed};
    element_stage(c, c->L, false, &ia);
    if (!dev)
      HIP_OK(hipMemcpyAsync(eta2_out, eta.p, (size_t)nel * nrhs * 8, hipMemcpyDeviceToHost,
                            c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    c->prof.flush();
    return DPG_OK;
  });
}

int64_t dpg_boundary_points(const dpg_ctx *cc, double *xyz, int64_t cap) {
  dpg_ctx *c = const_cast<dpg_ctx *>(cc);
  if (!c) return DPG_EINVAL;
  if (c->stage < 1) return DPG_ESTATE;
  int64_t rc = 0;
  const int st = guarded(c, [&]() -> int {
    const int N = c->N, nq = c->tables_h.nql;
    const double h = c->side / N;
    rc = boundary_points(c);
    if (!xyz || cap <= 0) return DPG_OK;
    int64_t k = 0;
    for (int d = 0; d < 3; ++d)
      for (int s = 0; s < 2; ++s) {
        const int f1 = d == 0 ? 1 : 0, f2 = d == 2 ? 1 : 2;
        for (int c2 = 0; c2 < N; ++c2)
          for (int c1 = 0; c1 < N; ++c1)
            for (int p2 = 0; p2 < nq; ++p2)
              for (int p1 = 0; p1 < nq; ++p1, ++k) {
                if (k >= cap) return DPG_OK;
                double X[3];
                X[d] = c->org[d] + (s ? c->side : 0.0);
                X[f1] = c->org[f1] + h * c1 + (c->tables_h.xq[p1] + 1.0) * 0.5 * h;
                X[f2] = c->org[f2] + h * c2 + (c->tables_h.xq[p2] + 1.0) * 0.5 * h;
                for (int a = 0; a < 3; ++a) xyz[3 * k + a] = X[a];
              }
      }
    return DPG_OK;
  });
  return st == DPG_OK ? rc : st;
}

int dpg_info(const dpg_ctx *c, dpg_info_t *info) {
  if (!c || !info) return DPG_EINVAL;
  std::memset(info, 0, sizeof(*info));
  if (c->stage < 1) return DPG_ESTATE;
  const auto &top = c->lv[c->L];
  info->n_trace = top.num.n;
  info->n_macro = top.nM;
  info->nlevels = c->L + 1;
  for (int k = 0; k <= c->L && k < 16; ++k) {
    const auto &f = c->lv[c->L - k];
    info->level_n[k] = f.N;
    info->level_p[k] = f.q;
    info->level_ntrace[k] = f.num.n;
    info->level_nmacro[k] = f.nM;
  }
  info->resident_bytes = c->bud.used;
  info->n_test = c->n_test;
  info->n_field = c->n_field;
  info->n_tr = c->n_tr;
  for (int k = 0; k < 4; ++k) info->setup_ms[k] = c->ms[k];
  return DPG_OK;
}

const char *dpg_last_error(const dpg_ctx *c) { return c ? c->err.c_str() : "no context"; }

int dpg_profile(dpg_ctx *c, int enable) {
  if (!c) return DPG_EINVAL;
  return guarded(c, [&]() {
    c->prof.reset();
    c->prof.on = enable != 0;
    return DPG_OK;
  });
}

int dpg_kernel_stats(const dpg_ctx *cc, int cls, dpg_kstat *out) {
  dpg_ctx *c = const_cast<dpg_ctx *>(cc);
  if (!c || !out || cls < 0 || cls >= DPG_K_NCLASS) return DPG_EINVAL;
  return guarded(c, [&]() {
    c->prof.flush();
    out->launches = c->prof.stat[cls].n;
    out->total_ms = c->prof.stat[cls].ms;
    out->work = c->prof.stat[cls].work;
    return DPG_OK;
  });
}


int64_t dpg_export(const dpg_ctx *cc, int what, int level, void *out, int64_t cap) {
  dpg_ctx *c = const_cast<dpg_ctx *>(cc);
  if (!c) return DPG_EINVAL;
  if (c->stage < 1) return DPG_ESTATE;
  if (level < 0 || level > c->L) return DPG_EINVAL;
  int64_t rc = DPG_EINVAL;
  int st = guarded(c, [&]() -> int {
    LevelData &f = c->lv[c->L - level];
    const hipStream_t s = c->stream;
    auto need_macro = [&]() {
      if (!f.macro) throw DpgError(DPG_EINVAL, "the coarsest mesh has no macro grid");
    };
    switch (what) {
      case DPG_X_ELEM_DOFS: rc = put(widen(f.edofs_h), out, cap); break;
      case DPG_X_MACRO_B: need_macro(); rc = put(f.mc.macro_B, out, cap); break;
      case DPG_X_BLOCK_B:
      case DPG_X_BLOCK_I: {
        need_macro();
        std::vector<int64_t> v(f.nblk + 1, 0), body;
        for (int b = 0; b < f.nblk; ++b) {
          if (what == DPG_X_BLOCK_B) {
            for (int64_t k = f.mc.blkB_ptr[b]; k < f.mc.blkB_ptr[b + 1]; ++k)
              body.push_back(f.mc.macro_of[f.mc.blkB[(int64_t)b * f.nBf + f.mc.blkB_present[k]]]);
          } else {
            for (int i = 0; i < f.nI; ++i) body.push_back(f.mc.blkI[(int64_t)b * f.nI + i]);
          }
          v[b + 1] = (int64_t)body.size();
        }
        v.insert(v.end(), body.begin(), body.end());
        rc = put(v, out, cap);
        break;
      }
      case DPG_X_PATCHES: {
        need_macro();
        std::vector<int64_t> v(f.mc.patch_ptr);
        v.insert(v.end(), f.mc.patch_idx.begin(), f.mc.patch_idx.end());
        rc = put(v, out, cap);
        break;
      }
      case DPG_X_PROLONG: {
        need_macro();
        std::vector<int64_t> v(f.P.ptr);
        v.insert(v.end(), f.P.col.begin(), f.P.col.end());
        rc = put(v, out, cap);
        break;
      }
      case DPG_X_PROLONG_VAL: need_macro(); rc = put(f.P.val, out, cap); break;
      case DPG_X_ELEM_S:
      case DPG_X_COARSE_E: {
        if (c->released) throw DpgError(DPG_ESTATE, "setup data released");
        if (!f.E.p) throw DpgError(DPG_ESTATE, "element matrices not computed yet");
        rc = put(f.E.download(s), out, cap);
        break;
      }
      case DPG_X_ELEM_RHS: {
        if (c->stage < 2) throw DpgError(DPG_ESTATE, "dpg_assemble first");
        rc = put(c->s_elem.download(s), out, cap);
        break;
      }
      case DPG_X_ASM_RHS: {
        if (c->stage < 2) throw DpgError(DPG_ESTATE, "dpg_assemble first");
        rc = put(c->s_asm.download(s), out, cap);
        break;
      }
      case DPG_X_MACRO_M: {
        need_macro();
        if (c->released) throw DpgError(DPG_ESTATE, "setup data released");
        if (!mfull(f)) throw DpgError(DPG_ESTATE, "dpg_build_hierarchy first");
        std::vector<double2> full = f.order ? f.E.download(s) : f.Mfull.download(s), v;
        for (int b = 0; b < f.nblk; ++b) {
          const int64_t k0 = f.mc.blkB_ptr[b], n = f.mc.blkB_ptr[b + 1] - k0;
          const double2 *Mb = full.data() + (int64_t)b * f.nBf * f.nBf;
          for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i)
              v.push_back(Mb[f.mc.blkB_present[k0 + i] + (int64_t)f.mc.blkB_present[k0 + j] * f.nBf]);
        }
        rc = put(v, out, cap);
        break;
      }
      case DPG_X_PATCH_INV: {
        need_macro();
        if (c->stage < 3) throw DpgError(DPG_ESTATE, "dpg_build_hierarchy first");
        HermSet &H = f.Sset;
        if (!H.t64.p && !H.t32.p)
          throw DpgError(DPG_ESTATE, "patch inverses are not stored (DPG_RECOMPUTE_PATCHES)");
        std::vector<double2> t;
        if (H.t64.p) t = H.t64.download(s);
        else {
          std::vector<float2> t32 = H.t32.download(s);
          t.resize(t32.size());
          for (size_t k = 0; k < t32.size(); ++k) t[k] = mk(t32[k].x, t32[k].y);
        }
        std::vector<double2> v;
        for (int b = 0; b < H.nblk; ++b) {
          const int n = H.n_h[b], nt = (n + 31) / 32;
          std::vector<double2> A((size_t)n * n);
          for (int J = 0; J < nt; ++J)
            for (int I = 0; I <= J; ++I) {
              const double2 *tp = t.data() + H.ent_off_h[b] + tile_entry(I, J);
              for (int e = 0; e < kTileFull; ++e) {
                const int k = e >> 6, lane = e & 63, ra = lane >> 3, cb = lane & 7;
                if (I == J && ra > cb) continue;   // not stored: mirrored from (cb, ra)
                const double2 v = tp[I == J ? k * kDiagSlots + diag_slot(ra, cb) : e];
                const int row = 32 * I + 4 * ra + (k >> 2), col = 32 * J + 4 * cb + (k & 3);
                if (row < n && col < n) {
                  A[row + (size_t)col * n] = v;
                  if (I < J || ra < cb) A[col + (size_t)row * n] = mk(v.x, -v.y);
                }
              }
            }
          v.insert(v.end(), A.begin(), A.end());
        }
        rc = put(v, out, cap);
        break;
      }
      case DPG_X_COARSEST: {
        if (c->stage < 3) throw DpgError(DPG_ESTATE, "dpg_build_hierarchy first");
        if (c->released) throw DpgError(DPG_ESTATE, "setup data released");
        rc = put(c->T0.download(s), out, cap);
        break;
      }
      default: throw DpgError(DPG_EINVAL, "unknown export");
    }
    return DPG_OK;
  });
  return st == DPG_OK ? rc : st;
}

void dpg_destroy(dpg_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  batch_close(c);
  if (c->host_sc) (void)hipHostFree(c->host_sc);
  if (c->aux) {
    (void)hipStreamSynchronize(c->aux);
    (void)hipStreamDestroy(c->aux);
  }
  for (hipStream_t x : c->paux)
    if (x) {
      (void)hipStreamSynchronize(x);
      (void)hipStreamDestroy(x);
    }
  for (hipEvent_t e : {c->ev_fork, c->ev_join, c->ev_pjoin[0], c->ev_pjoin[1]})
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ev_level) (void)hipEventDestroy(e);
  if (c->own_stream) {
    (void)hipStreamSynchronize(c->own_stream);
    (void)hipStreamDestroy(c->own_stream);
    c->own_stream = nullptr;
  }
  if (c->host_bsc) (void)hipHostFree(c->host_bsc);
  if (c->host_bact) (void)hipHostFree(c->host_bact);
  delete c;
}

}  // extern "C"
