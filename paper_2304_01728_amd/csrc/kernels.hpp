// Hierarchy-setup and solve-phase kernels other than the dense batched
// algebra and the Hermitian block sets.
#pragma once
#include "common.hpp"

namespace dpg {

// ---- hierarchy setup (FP64) ----------------------------------------------------

// T[b] (nT x nT, nT = nBf + nI) = sum over the 8 children of coarse element
// b0 + b of their element matrices E (n_tr x n_tr).  child_inv [8][nT] gives
// each position of [B slots | I] its local index in each child, or -1.
void launch_macro_assemble(const double2 *E, int n_tr, const int32_t *child_inv, int N, int b0,
                           int count, int nT, double2 *T, hipStream_t s);

// dst[d(b)][i + j ldd] = src[b][r0 + i + (c0 + j) lds] for i < rows, j < cols,
// b < count, with d(b) = dlist[b] (or b when dlist is null); zeros when src
// is null.
void launch_copy_sub(const double2 *src, int64_t src_stride, int lds, int r0, int c0, int rows,
                     int cols, double2 *dst, int64_t dst_stride, int ldd, int count,
                     hipStream_t s, const int32_t *dlist = nullptr);

// Lower triangle of the patch block S_v (n_v x n_v) gathered from the macro
// blocks of the <= 8 coarse cells around vertex v: S[i,j] = sum_c M_c[slot_c(i),
// slot_c(j)], j <= i.
void launch_patch_gather(const double2 *Mfull, int nBf, int Nc, const int64_t *patch_ptr,
                         const int32_t *patch_slot, int v0, int count, int nmax,
                         const int64_t *dst_off, double2 *S, hipStream_t s);

// The same lower triangle with the macro blocks read from their packed FP64
// Hermitian tiles (a HermSet: block b at tiles + ent_off[b]); pidx[b nBf + s]
// = packed position of local slot s of block b (-1 absent).
void launch_patch_gather_tiles(const double2 *tiles, const int64_t *ent_off, const int32_t *pidx,
                               int nBf, int Nc, const int64_t *patch_ptr,
                               const int32_t *patch_slot, int v0, int count, int nmax,
                               const int64_t *dst_off, double2 *S, hipStream_t s);

// X[b] = identity of size n[b] (column-major, leading dimension n[b]).
void launch_identity(const int64_t *off, const int32_t *n, int count, int nmax, double2 *X,
                     hipStream_t s);

// Dense T0 (n0 x n0) = sum over elements of E scattered by edofs (-1 skipped).
void launch_assemble_dense(const double2 *E, int n_tr, const int32_t *edofs, int nel, int n0,
                           double2 *T0, hipStream_t s);

// ---- solve phase ---------------------------------------------------------------

// y[i] = sum_k val[k] x[col[k]] over CSR rows (mode 0: set, 1: add).
template <typename T>
void launch_csr(int64_t nrows, const int64_t *ptr, const int32_t *col, const T *val,
                const cplx_t<T> *x, cplx_t<T> *y, int add, hipStream_t s);

// Macro condensation of a trace vector rc through the blocks of one level.
// Per block: WH = (T_II^-1 T_IB)^H (nBf x nI), Tinv = T_II^-1 (nI x nI).
// c_b = WH_b rc[I_b] (nBf slots).
template <typename T>
void launch_condense_local(const cplx_t<T> *WH, int nI, int nBf, const int32_t *blkI, int nblk,
                           const cplx_t<T> *rc, cplx_t<T> *c, hipStream_t s);
// rB[m] = rc[macro_B[m]] - sum over (block, slot) holding m of c_b[slot].
template <typename T>
void launch_condense_reduce(int64_t nM, const int64_t *macro_B, const int32_t *red_ptr,
                            const int32_t *red_ent, const cplx_t<T> *rc, const cplx_t<T> *c,
                            cplx_t<T> *rB, hipStream_t s);
// ec[macro_B[m]] = eB[m]; ec[I_b] = Tinv_b rc[I_b] - WH_b^H eB_b.
template <typename T>
void launch_expand(const cplx_t<T> *WH, const cplx_t<T> *Tinv, int nI, int nBf,
                   const int32_t *blkI, const int32_t *blkBm, int nblk, const cplx_t<T> *rc,
                   const cplx_t<T> *eB, int64_t nM, const int64_t *macro_B, cplx_t<T> *ec,
                   hipStream_t s);

// Element loads assembled into a trace vector: s[t] = sum over (elem, local)
// of se[elem][local] (CSR over t, entries elem * n_tr + local).
void launch_assemble_vec(int64_t n, const int32_t *ptr, const int32_t *ent, const double2 *se,
                         int64_t se_stride, double2 *out, hipStream_t s);

// Field recovery (Sec. 1.2, static condensation undone): per element,
// x_f = K_ff^-1 (b_f - K_ft x_t) = L^-H (Y_b - Y_t x_t) with L = chol(K_ff),
// Y_t = L^-1 K_ft ([nel][nf][ntr]) and Y_b = L^-1 b_f ([nel][nrhs][nf]) kept
// from the element stage; load column col.  out[e][nf].
void launch_fields(const double2 *recL, const double2 *recY, const double2 *recYb, int nf,
                   int ntr, int nrhs, int col, const int32_t *edofs, int nel, const double2 *x,
                   double2 *out, hipStream_t s);

// DPG residual error indicator (Sec. 1.2): per element and load column r,
// X(:, r) = [x_f; x_t] with x_t gathered from x + r nvec through edofs and
// x_f = L^-H (Y_b - Y_t x_t), where K (stride ks, leading dimension ld) holds
// L = chol(K_ff) in its first nf columns and Y = L^-1 [K_ft | b] after them.
// X: [count][nr][m], m = nf + ntr.
void launch_indicator_x(const double2 *K, int64_t ks, int ld, int nf, int ntr, int nr,
                        const int32_t *edofs, int count, const double2 *x, int64_t nvec,
                        double2 *X, hipStream_t s);
// out[r nel_out + e0 + e] = sum_i |W[e](i, c0 + r)|^2, i < n, for e < count,
// r < ncols (W per element at stride ws, leading dimension ld).
void launch_colnorm2(const double2 *W, int64_t ws, int ld, int n, int c0, int ncols, int e0,
                     int count, int64_t nel_out, double *out, hipStream_t s);

// a[0..n) = 0 (a kernel, not a memset: safe inside captured graphs).
template <typename C> void launch_zero(int64_t n, C *a, hipStream_t s);

// Conversions between the FP64 and FP32 copies of a vector.
void launch_to32(int64_t n, const double2 *a, float2 *b, hipStream_t s);
void launch_to64(int64_t n, const float2 *a, double2 *b, hipStream_t s);

// ---- CG vector algebra (FP64) ---------------------------------------------------
// Device scalars: sc[0] = rz, sc[1] = pq, sc[2] = alpha, sc[3] = beta,
// sc[4] = ||r||^2, sc[5] = ||b||^2, sc[6] = breakdown flag, sc[7] = r^H z_old.
constexpr int kDotBlocks = 512;
void dot_re(int64_t n, const double2 *a, const double2 *b, double *partial, double *dst,
            hipStream_t s);                                  // dst = Re(a^H b)
void cg_alpha(int64_t n, const double2 *p, const double2 *q, double *partial, double *sc,
              hipStream_t s);                                // pq, alpha = rz / pq
void cg_update_xr(int64_t n, double2 *x, double2 *r, const double2 *p, const double2 *q,
                  double *partial, double *sc, hipStream_t s);  // x += a p, r -= a q, ||r||^2
void cg_beta(int64_t n, const double2 *r, const double2 *z, const double2 *zold, double *partial,
             double *sc, hipStream_t s);                     // beta (flexible), rz <- r^H z
void cg_update_p(int64_t n, double2 *p, const double2 *z, const double *sc, hipStream_t s);

}  // namespace dpg
