// Element DPG matrices on the GPU (Sec. 2 of arXiv 2304.01728): Gram matrix
// of the adjoint graph test norm (eq. Gnorm, alpha = 1), the ultraweak form B
// on [fields | traces], and loads (Gaussian point sources, plane-wave
// impedance data).  Test functions: orthonormal Legendre products spanning
// q in Q^{p+dp} and v in RT_{p+dp}; fields: Legendre products in Q^{p-1};
// traces: hierarchical H1 (pressure) and Legendre (flux), element-local
// layout as in the topology code.
#pragma once
#include "common.hpp"

namespace dpg {

constexpr int kMX = 10;   // max 1-D test functions (p + dp + 1)
constexpr int kMQ = 14;   // max load quadrature points per direction

struct ElemTables {
  int P1;                 // 1-D test functions: degrees 0..P1-1
  int p;                  // order
  int nql;                // load quadrature points per direction
  // 1-D integrals on [-1,1] of orthonormal Legendre test functions Lt_a:
  double KK[kMX * kMX];   // int Lt_a' Lt_b'
  double DM[kMX * kMX];   // int Lt_a' Lt_b      (derivative on the first)
  double fM[kMX * kMX];   // int Lt_a P_n        (field / flux Legendre, n < p)
  double fD[kMX * kMX];   // int Lt_a' P_n
  double hM[kMX * kMX];   // int Lt_a psi_c      (H1 function c <= p)
  double tEnd[kMX * 2];   // Lt_a(-1), Lt_a(+1)
  double hEnd[kMX * 2];   // psi_c(-1), psi_c(+1)
  double xq[kMQ], wq[kMQ];
  double Lq[kMX * kMQ];   // Lt_a(xq[q])
};

// Per-rhs load description on the device.
struct LoadDesc {
  double dir[3];
  double amp[2];
  int src0, nsrc;         // sources src[6*src0 ...]
  int64_t u0_off;         // impedance data at the boundary load points: u0q[u0_off ...]
                          // (canonical boundary point order), -1 = none
};

// Boundary load points of an N^3 mesh: faces of Gamma in the order axis d,
// side s (low, high), cell coordinates (c1, c2) along the two other axes in
// ascending order, c1 fastest; nql x nql Gauss points per face, the first
// in-plane axis fastest.  Face index ((2 d + s) N + c2) N + c1.
__host__ __device__ inline int64_t boundary_face(int d, int s, int c1, int c2, int N) {
  return ((int64_t)(2 * d + s) * N + c2) * N + c1;
}

struct ElemGeom {
  int N;
  double h, omega, alpha;
  double org[3];
  const int32_t *elist;   // device list of the elements to process (index e0 + i of a
                          // launch), or null for the elements e0 + i themselves
};

void build_elem_tables(int p, int dp, ElemTables &t);
// test descriptors (type 0 = q, 1..3 = v component; degrees a,b,c) and trial
// descriptors (0 = p, 1..3 = u_d fields with degrees; 4 = H1 trace lattice
// point; 5..10 = flux on face 0..5 with in-plane degrees (m, n, 0)).
void build_descriptors(int p, int dp, std::vector<int4> &test, std::vector<int4> &trial);

// G[e][nt x nt] for elements e0 .. e0+count-1 (column-major per element);
// only the lower triangle (diagonal included) is written.
void launch_gram(const ElemTables *tb, const int4 *test, int nt, ElemGeom g, const double *kappa,
                 int e0, int count, double2 *G, hipStream_t s);
// B part of [B | l]: nt x m columns of BL[e] (leading dimension nt).
void launch_bmat(const ElemTables *tb, const int4 *test, const int4 *trial, int nt, int m,
                 ElemGeom g, const double *kappa, const double *Zel, int e0, int count,
                 double2 *BL, int64_t strideBL, hipStream_t s);
// load columns m .. m+nrhs-1 of BL[e].
// u0q: impedance data at the boundary load points (complex, indexed by the
// loads' u0_off), may be null when no load uses it.
void launch_load(const ElemTables *tb, int nt, int m, ElemGeom g, const double *Zel,
                 const LoadDesc *ld, const double *src, const double2 *u0q, int nrhs, int e0,
                 int count, double2 *BL, int64_t strideBL, hipStream_t s);

}  // namespace dpg
