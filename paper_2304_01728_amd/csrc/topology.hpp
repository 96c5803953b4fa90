// Host-side mesh topology of the DPG multigrid hierarchy: canonical trace
// numbering, element maps, macro-grid sets, vertex patches and the
// natural-inclusion prolongation (Sec. 3 "Prolongation" and "V-cycle and
// smoother" of arXiv 2304.01728), plus the 1-D shape-function tables the
// element kernels read.  Integer bookkeeping and small constant tables only;
// all floating-point work of the solver runs in the HIP kernels.
#pragma once
#include <cstdint>
#include <vector>

namespace dpg {

// 1-D rules and functions on [-1, 1].
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);
double legendre(int n, double x);                 // P_n(x)
double legendre_d(int n, double x);               // P_n'(x)
double h1_fun(int r, int a, double x);            // hierarchical H1 function a of order r
double h1_fun_d(int r, int a, double x);

// Two-scale coefficients, 1-D.  R1: [2r+1][r+1] (fine H1 lattice of the two
// halves x coarse H1 function); R0: [2r][r] (fine Legendre (half, degree) x
// coarse degree).  Exact zeros are cleaned to 0.
std::vector<double> twoscale_h1(int r);
std::vector<double> twoscale_leg(int r);

inline int64_t n_trace(int64_t N, int64_t p) {
  return (N * p + 1) * (N * p + 1) * (N * p + 1) - N * N * N * (p - 1) * (p - 1) * (p - 1) +
         3 * N * N * (N - 1) * p * p;
}

// Canonical numbering of the trace unknowns of an N^3 mesh of order p.
struct Numbering {
  int N = 0, p = 0, M = 0;          // M = N p
  int64_t n_h1 = 0, n_fam = 0, n = 0;
  std::vector<int32_t> h1_index;    // [(M+1)^3] lattice (Z,Y,X) -> index or -1
  std::vector<int64_t> h1_lat;      // [n_h1] packed lattice id (Z*(M+1)+Y)*(M+1)+X
  void build(int N_, int p_);
  int64_t h1(int X, int Y, int Z) const {
    return h1_index[((int64_t)Z * (M + 1) + Y) * (M + 1) + X];
  }
  int64_t flux(int d, int s, int T1, int T2) const {
    return n_h1 + d * n_fam + ((int64_t)(s - 1) * M + T2) * M + T1;
  }
  // inverse: kind 0 = H1 with (X,Y,Z); kind 1..3 = flux family with (s,T1,T2)
  void describe(int64_t idx, int &kind, int c[3]) const;
};

// Element-local trace layout: H1 boundary lattice of [0,p]^3 (a fastest),
// then faces x-, x+, y-, y+, z-, z+ with p^2 fluxes each (first in-plane
// degree fastest).
struct ElementLayout {
  int p = 0, n_h1 = 0, n_tr = 0;
  std::vector<int> lat;             // 3 ints per boundary lattice point
  void build(int p_);
};

// Element-to-trace map of an N^3 mesh: [N^3][n_tr], -1 where a flux is on Gamma.
std::vector<int32_t> element_dofs(const Numbering &num, const ElementLayout &el);

// Macro grid of a fine mesh with N even and its coarse mesh N/2.
struct MacroLevel {
  int N = 0, Nc = 0, p = 0;
  int nBf = 0, nI = 0;              // full local B layout size, interior count
  int64_t nM = 0;
  std::vector<int32_t> macro_of;    // [n_trace] -> macro index or -1
  std::vector<int64_t> macro_B;     // [nM] canonical index of each macro unknown
  // per coarse element: canonical index of each local B slot (-1 absent),
  // and of each interior unknown (ascending canonical order)
  std::vector<int32_t> blkB;        // [Nc^3][nBf]
  std::vector<int32_t> blkI;        // [Nc^3][nI]
  std::vector<int32_t> blkB_present;  // CSR of present local slots per block
  std::vector<int64_t> blkB_ptr;
  // child local dof -> position in [B slots | I] of the parent block
  std::vector<int32_t> child_map;   // [8][n_tr]
  // vertex patches: CSR of macro indices; for each member the local B slot in
  // each of the 8 cells around the vertex (-1 where the cell does not hold it
  // or does not exist), cells ordered (dx, dy, dz) with dx fastest, cell =
  // vertex - 1 + d.
  std::vector<int64_t> patch_ptr;
  std::vector<int32_t> patch_idx;
  std::vector<int32_t> patch_slot;  // [members][8]
  std::vector<int> bslot_tab;       // [(2p+1)^3] block lattice -> B slot or -1
  void build(const Numbering &fine, const ElementLayout &el);
  // The level of a hierarchy that lowers the order on one mesh (its coarser
  // level has the same mesh and order p - 1): nothing is condensed (the macro
  // grid is every trace unknown), the blocks are the elements (slots = the
  // element-local layout, present ones listed by ascending canonical index),
  // nI = 0, and the patches are the vertex patches of the mesh itself (cells =
  // elements, Nc = N).  child_map and bslot_tab stay empty.
  void build_order(const Numbering &num, const ElementLayout &el);
  // local B slot of canonical unknown t in coarse cell (ci,cj,ck), or -1
  int slot_in_block(const Numbering &fine, int64_t t, int ci, int cj, int ck) const;
};

// Prolongation of a macro level: coarse trace vector -> fine macro vector.
struct Prolongation {
  std::vector<int64_t> ptr;         // CSR over macro rows
  std::vector<int32_t> col;
  std::vector<double> val;
  std::vector<int64_t> tptr;        // CSR of the transpose over coarse rows
  std::vector<int32_t> tcol;
  std::vector<double> tval;
  std::vector<double> local;        // dense [n_tr (coarse element)][nBf] column-major nBf x n_tr
  void build(const MacroLevel &mc, const Numbering &fine, const Numbering &coarse,
             const ElementLayout &el);
  // Order level (MacroLevel::build_order): the inclusion of the order p - 1
  // traces of the same mesh, an injection with hierarchical bases (lattice
  // X' = (p-1) cell + a' -> p cell + a'; flux degrees kept).  local is the
  // element-local injection [n_tr(p-1)][n_tr(p)].
  void build_order(const MacroLevel &mc, const Numbering &fine, const Numbering &coarse,
                   const ElementLayout &el_fine, const ElementLayout &el_coarse);
};

}  // namespace dpg
