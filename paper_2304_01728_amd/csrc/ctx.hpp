// Internal context of libdpgmg.
#pragma once
#include <chrono>
#include <memory>
#include <string>
#include <vector>

#include "../../include/dpgmg.h"
#include "block.hpp"
#include "common.hpp"
#include "dense.hpp"
#include "element.hpp"
#include "hblocks.hpp"
#include "kernels.hpp"
#include "topology.hpp"

namespace dpg {

// Prepared once per mesh (and per number of loads): item tables on the device
// and fixed workspaces, so that the setup phases only queue kernels.

// Element stage: chunks of C elements are dealt to ns streams, each with its
// own G, [B l], K and diagonal-block-inverse buffers.
struct ElemPlan {
  int C = 0, mp = -1, nel = -1, ns = 2;
  DevBuf<double2> G[4], BL[4], K[4], wk[4];   // one set per stream
  DevBuf<PotrfItem> pG, pK;
  DevBuf<TrsmItem> tG, tK;
  DevBuf<GemmItem> gK, gS;
  DevBuf<int> info;    // [2 nel]: Gram factor, then field block, per element
  // error-indicator pass: per-stream element unknowns [C][nr][m] and the
  // residual products' items (for gR_nr columns, chunks of gR_C)
  DevBuf<double2> X[4];
  DevBuf<GemmItem> gR;
  int gR_nr = 0, gR_C = 0;
};

// Load updates by maps per element class.  Elements with equal wave speed and
// the same faces on Gamma have equal G and B (translated boxes), so one linear
// map T_c takes an element's load vector l (over the test functions) to its
// condensed trace load s = K_tl - K_tf K_ff^-1 K_fl, and F_c to its
// field-recovery data L_f^-1 K_fl; both are formed once by the element chain
// with identity load columns on one element of each class.
struct LoadMaps {
  int state = 0;                     // 0 not built, 1 built, -1 not used (too many classes)
  int nclass = 0;
  std::vector<int32_t> cls_h;        // class of every finest element
  DevBuf<double2> T, F;              // [nclass] n_tr x n_test, n_field x n_test (column-major)
  DevBuf<double2> lbuf;              // load vectors of a chunk of elements [C][nr][n_test]
  DevBuf<GemmItem> items;            // per update: s_e = T_c l_e, then Yb_e = F_c l_e
};

// Macro condensation and Galerkin step of one level (workspaces shared by
// all levels: the levels run one after the other on one stream).
struct MacroPlan {
  bool ready = false;
  int CB = 0;
  DevBuf<double2> Ploc;
  DevBuf<PotrfItem> pII;
  DevBuf<TrsmItem> tIB, tLi;
  DevBuf<GemmItem> gS, gTi, gWH, gX, gA;
  DevBuf<int64_t> idoff, soff, moff;
  DevBuf<int32_t> idn, cmap, sld, map;
  DevBuf<int> info;    // [nblk]
};

// Patch factors and inverses of one level, in batches that fit the patch
// workspaces.
struct PatchBatch {
  int half = 0;                      // part: 0 .. 2 on the extra streams, 3 on the main
                                     // stream (each part with its own workspaces)
  int v0 = 0, cnt = 0, nmax = 0;
  int64_t t0 = 0, t1 = 0;
  double fp = 0, ft = 0, fg = 0;
  DevBuf<int64_t> off;
  DevBuf<int32_t> nn;
  std::vector<int32_t> hn;           // the orders nn on the host (kernel statistics)
  DevBuf<PotrfItem> pi;
  DevBuf<TrsmItem> ti;
  DevBuf<GemmItem> gi;
  DevBuf<GemmItem> gyc, gzc;         // recomputed inverses, t = X x_v and y_v = X^H t for
                                     // nr = 1 .. kMaxCols columns stored column by
                                     // column: items (nr - 1) cnt + i
};
struct PatchPlan {
  bool ready = false;
  std::vector<PatchBatch> batches;
  DevBuf<int64_t> soff_all;
  DevBuf<int32_t> ld_all;
  DevBuf<int> info;    // [npatch]
};

// One mesh of the hierarchy.  Level 0 is the coarsest mesh, level L the finest.
struct LevelData {
  int N = 0, nel = 0;
  int q = 0, ntr = 0, ntr_c = 0;     // order, element trace size, that of the coarser level
  bool order = false;                // the coarser level has the same mesh (order q - 1)
  ElementLayout el;
  Numbering num;
  std::vector<int32_t> edofs_h;
  DevBuf<int32_t> edofs;
  DevBuf<double2> E;                 // element matrices [nel][n_tr^2]
  DevBuf<double> kappa, Zel;         // per element c^-2 and Z on a coarser mesh whose
                                     // operator is assembled directly ("store")
  // macro grid (levels >= 1)
  bool macro = false;
  MacroLevel mc;
  Prolongation P;
  int nblk = 0, nBf = 0, nI = 0;
  int64_t nM = 0;
  DevBuf<double2> Mfull;             // [nblk][nBf^2] condensed blocks, full local layout
  DevBuf<double2> Tinv, WH;          // [nblk][nI^2], [nblk][nBf nI]
  DevBuf<float2> Tinv32, WH32;
  DevBuf<int32_t> blkI, blkBm;       // [nblk][nI] canonical, [nblk][nBf] macro index / -1
  DevBuf<int64_t> macroB;            // [nM] canonical index of each macro unknown
  DevBuf<int32_t> cred_ptr, cred_ent;
  DevBuf<int64_t> patch_ptr;
  DevBuf<int32_t> patch_slot;
  DevBuf<int32_t> mpidx;             // [nblk][nBf] packed position of each macro-block slot
                                     // (recomputed patch inverses)
  HermSet Mset, Sset;
  DevBuf<int64_t> Pptr, Ptptr;
  DevBuf<int32_t> Pcol, Ptcol;
  DevBuf<double> Pval, Ptval;
  DevBuf<float> Pval32, Ptval32;
  // V-cycle work vectors: r, x, res on this macro grid; rc, ec on the coarser
  // mesh's traces; c = per-block condensation contributions of this level.
  DevBuf<double2> r64, x64, res64, rc64, ec64, c64;
  DevBuf<float2> r32, x32, res32, rc32, ec32, c32;
  // the same for block (multi-right-hand-side) solves, bcap columns
  int bcap = 0;
  DevBuf<double2> br64, bx64, bres64, brc64, bec64, bc64;
  DevBuf<float2> br32, bx32, bres32, brc32, bec32, bc32;
  HermBlockBufs Mb, Sb;
  MacroPlan mp;
  PatchPlan pp;
};

// Instantiated HIP graphs of the PCG iteration: (A) matvec, alpha, x and r;
// (B) V-cycle, beta, search direction, in two versions (z and z_old swap
// every iteration).  Destroyed with the object.
struct GraphSet {
  hipGraphExec_t a = nullptr, b[2] = {nullptr, nullptr};
  GraphSet() = default;
  GraphSet(const GraphSet &) = delete;
  GraphSet &operator=(const GraphSet &) = delete;
  ~GraphSet() {
    for (hipGraphExec_t g : {a, b[0], b[1]})
      if (g) (void)hipGraphExecDestroy(g);
  }
};

// A block PCG whose columns join and leave while it runs (continuous
// batching; dpg_batch_* and the block path of dpg_solve).  Slot k is column
// k of the interleaved block vectors of the context (width w).
struct BatchSession {
  bool open = false;
  int max = 0, w = 0;                // capacity, current width (a power of two or max)
  int cur = 0;                       // which of bz / bzo holds z
  int state[kMaxCols] = {};          // 0 free, 1 running, 2 converged, 3 maxit, 4 breakdown
  int iters[kMaxCols] = {};
  double tol[kMaxCols] = {}, bb[kMaxCols] = {}, rr[kMaxCols] = {};
  bool act_dirty = true;
  std::vector<int> done;             // finished slots not taken yet, in finishing order
  std::unique_ptr<GraphSet> graphs;  // captured for width gw
  int gw = 0;
};

}  // namespace dpg

struct dpg_ctx {
  std::string err;
  int stage = 0;                     // 1 set up, 2 assembled, 3 hierarchy built
  bool released = false;             // setup-only data freed (dpg_release_setup)
  int N = 0, p = 0, dp = 1, nrhs = 0;
  double omega = 0, side = 1, org[3] = {0, 0, 0};
  dpg_options opt{};
  int device = 0;                    // the device current at dpg_setup
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;  // created when the options give no stream
  hipStream_t aux = nullptr;         // second stream of the setup phases
  hipStream_t paux[2] = {nullptr, nullptr};   // third and fourth setup streams
  hipEvent_t ev_pjoin[2] = {nullptr, nullptr};
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::vector<hipEvent_t> ev_level;  // per level: macro blocks ready for the patches
  dpg::Budget bud;
  dpg::ElementLayout el;
  int n_test = 0, n_field = 0, n_tr = 0, m = 0;
  std::vector<double> c_h;
  dpg::DevBuf<double> kappa, Zel;
  dpg::ElemTables tables_h{};
  dpg::DevBuf<dpg::ElemTables> tables;
  dpg::DevBuf<int4> testd, triald;
  std::vector<dpg::LoadDesc> ld_h;
  std::vector<double> src_h;
  dpg::DevBuf<dpg::LoadDesc> ld;
  dpg::DevBuf<double> src;
  dpg::DevBuf<double2> u0q;          // impedance data at the boundary load points, all loads
  std::vector<dpg::LevelData> lv;
  int L = 0;
  bool keep_recovery = false;
  dpg::DevBuf<double2> s_elem;       // [nrhs][nel][n_tr] condensed element loads
  dpg::DevBuf<double2> s_asm;        // [nrhs][n_trace] assembled loads
  dpg::DevBuf<int32_t> asm_ptr, asm_ent;
  dpg::DevBuf<double2> rec_L, rec_Y, rec_Yb;  // [nel][nf^2], [nel][nf n_tr], [nel][nrhs nf]
  dpg::DevBuf<int32_t> elist;        // elements of a point-source load update
  dpg::LoadMaps lm;                  // load updates without the element chain
  // coarsest mesh
  dpg::DevBuf<double2> T0;
  dpg::HermSet T0set;
  // setup-phase plans and workspaces
  dpg::ElemPlan ep;
  dpg::DevBuf<double2> mT[2], mLinv[2], mX[2], mwk[2];   // macro levels, one set per stream
  dpg::DevBuf<double2> pS[4], pX[4], pwk[4];       // patches, one set per part
  dpg::DevBuf<double2> ptmp;                       // recomputed inverses: X x_v, local layout
  dpg::DevBuf<double2> zF, zLi, zTi, zwk;          // coarsest
  dpg::DevBuf<dpg::PotrfItem> zpi;
  dpg::DevBuf<dpg::TrsmItem> zti;
  dpg::DevBuf<dpg::GemmItem> zgi;
  dpg::DevBuf<int64_t> zoff;
  dpg::DevBuf<int32_t> znn, zld;
  dpg::DevBuf<int> zinfo;
  // outer CG (FP64, finest macro grid)
  dpg::DevBuf<double2> b, x, r, z, zo, pv, q, xfull, sB;
  dpg::DevBuf<double> partial, sc;
  double *host_sc = nullptr;         // pinned
  // block PCG (interleaved [n][nr] vectors), allocated at the first block solve
  int bcap = 0;
  dpg::HermBlockBufs T0b;
  dpg::DevBuf<double2> bb, bx, br, bz, bzo, bp, bq, bsv, bxf, bcols;
  dpg::DevBuf<double> bpartial, bsc;
  dpg::DevBuf<int> bact;
  double *host_bsc = nullptr;        // pinned, 8 x kMaxCols
  int *host_bact = nullptr;          // pinned, kMaxCols
  dpg::BatchSession bs;
  double ms[4] = {0, 0, 0, 0};
  dpg::Prof prof;
};
