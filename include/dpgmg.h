/*
 * libdpgmg -- DPG multigrid solver for ultraweak time-harmonic acoustics on
 * uniform hexahedral meshes, for one AMD Instinct MI355X (gfx950).
 *
 * Method: Badger, Henneking, Petrides, Demkowicz, "Scalable DPG multigrid
 * solver for Helmholtz problems: a study on convergence" (arXiv 2304.01728).
 *
 *   Problem (Sec. 2, eq. helmholtz; rho = 1, wave speed c per element):
 *       i w c^-2 p + div u = f,  i w u + grad p = 0  in the cube,
 *       Z^-1 p - u.n = u0  on its boundary Gamma, Z = c.
 *   Discretisation (Sec. 2): broken ultraweak form, adjoint graph test norm
 *   (eq. Gnorm) with alpha = 1, test order raised by dp; element DPG
 *   matrices B^H G^-1 B condensed onto the trace unknowns (Sec. 1.2).
 *   Solver (Sec. 3): CG on the macro grid preconditioned by a V-cycle with
 *   vertex-patch additive Schwarz smoothing, natural-inclusion prolongation
 *   and coarse operators by Galerkin restriction P^T A P; a direct Cholesky
 *   solve on the coarsest mesh; zero initial guess; stop at relative l2
 *   residual <= tol (Sec. 4 parameters).
 *
 * Conventions
 *   Complex numbers are interleaved (re, im) doubles.  Integers are int32
 *   unless stated.  Arrays are column-major when two-dimensional.
 *   Canonical trace numbering of an N^3 mesh of order p (the order of x in
 *   dpg_solve): H1 pressure-trace lattice points (X,Y,Z) in [0,Np]^3 with a
 *   coordinate divisible by p, X fastest; then flux families x, y, z, each
 *   over interior planes s = 1..N-1 and in-plane (T1,T2) in [0,Np)^2, T1
 *   fastest (x-family in-plane axes (y,z), y-family (x,z), z-family (x,y)).
 *   Shape functions: hierarchical H1 (vertex hats and normalised integrated
 *   Legendre bubbles) for the pressure trace, Legendre polynomials for fluxes
 *   and fields.  Flux unknowns are u.e_d; none lives on Gamma.
 *
 * Ownership: the caller owns every array passed in or out; the library copies
 * inputs during the call.  The context owns all device memory it allocates
 * until dpg_destroy.  By default pointers are host pointers; with
 * DPG_DEVICE_PTRS in dpg_options.flags, the rhs / x / fields arguments of
 * dpg_solve and dpg_get_fields are device pointers (e.g. torch tensors).
 *
 * Errors: every call returns DPG_OK (0) or a negative code; dpg_last_error
 * gives the message of the last failure on that context.  The call order
 * setup -> assemble -> build_hierarchy -> solve is enforced (DPG_ESTATE).
 * One context per host thread; distinct contexts may run concurrently.
 */
#ifndef DPGMG_H
#define DPGMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DPG_OK = 0,
  DPG_EINVAL = -1,     /* bad argument                                       */
  DPG_ENOMEM = -2,     /* device allocation failed or over hbm_budget        */
  DPG_ENOTPD = -3,     /* a Cholesky factorisation met a non-positive pivot  */
  DPG_ENOCONV = -4,    /* maxit reached; x holds the last iterate            */
  DPG_EBREAKDOWN = -5, /* CG breakdown (p^H M p <= 0 or not finite)          */
  DPG_ESTATE = -6,     /* call out of order                                  */
  DPG_EDEVICE = -7     /* HIP runtime error                                  */
};

enum { DPG_FP64 = 0, DPG_MIXED = 1 };       /* dpg_options.precision          */
enum { DPG_DEVICE_PTRS = 1,                 /* dpg_options.flags              */
       DPG_COLUMNWISE = 2,                   /* solve nrhs > 1 column by column */
       DPG_STORE_COARSE = 4,                 /* coarse operators assembled on
                                                their own meshes ("store", the
                                                alternative of Sec. 3 and the
                                                comparison of Sec. 4.2) instead
                                                of Galerkin P^T M P; needs a
                                                wave speed constant on every
                                                coarse element                 */
       DPG_RECOMPUTE_PATCHES = 8 };          /* no stored patch inverses: every
                                                smoothing step refactors the
                                                patch blocks from the macro
                                                blocks (Sec. 5 and Sec. 6: a
                                                GPU code that recomputes the
                                                patches, amortised over several
                                                loads); FP64; a block solve or
                                                batch refactors each patch once
                                                per step for all its columns   */

/* Uniform mesh of the cube [origin, origin + side]^3 into n^3 equal boxes;
 * element e = i + n (j + n k). */
typedef struct {
  int32_t n;
  double origin[3];
  double side;
} dpg_mesh;

/* Per-element wave speed c (length n^3); NULL means c = 1 everywhere. */
typedef struct {
  const double *c;
} dpg_material;

/* One right-hand side (Sec. 2 load l = <u0, q>_Gamma + (f, q), eq. helmholtz
 * data); the parts below are summed:
 *  - impedance data of a plane wave p = A exp(-i w d.x), u = d p, i.e.
 *    u0 = (Z^-1 - d.n) A exp(-i w d.x) on Gamma (A = amp; A = 0: none);
 *  - nsrc Gaussian point sources in the first equation,
 *    f = sum a_s (2 pi s^2)^(-3/2) exp(-|x - x_s|^2 / (2 s^2)), given as
 *    src[6*k .. 6*k+5] = (x, y, z, sigma, re a, im a);
 *  - general impedance data u0 given by its values at the boundary load
 *    points (complex, interleaved; the points and their order are those of
 *    dpg_boundary_points), or NULL. */
typedef struct {
  double dir[3];
  double amp[2];
  int32_t nsrc;
  const double *src;
  const double *u0_qp;
} dpg_load;

typedef struct {
  int32_t precision;  /* DPG_FP64: everything FP64.  DPG_MIXED: V-cycle
                         (matvecs, smoother, transfers) in complex FP32;
                         setup, coarsest factor and outer CG in FP64.        */
  int32_t nu_pre;     /* smoothing sweeps before / after the coarse solve    */
  int32_t nu_post;
  int32_t nlevels;    /* 0: halve while n is even and n > 2 (n = 2: once)    */
  int32_t maxit;      /* outer CG iteration cap                              */
  int32_t flags;      /* DPG_DEVICE_PTRS | DPG_COLUMNWISE | DPG_STORE_COARSE
                         | DPG_RECOMPUTE_PATCHES                              */
  double theta;       /* smoother damping; must be < 1/4                     */
  int64_t hbm_budget; /* bytes the context may allocate; 0 = no limit        */
  void *stream;       /* hipStream_t to launch on; NULL: a stream the context
                         creates (blocking, i.e. ordered with the null stream) */
  int32_t p_min;      /* order levels (Sec. 4.2, uniform p-refinements read as
                         multigrid levels): with 1 <= p_min < p the hierarchy
                         first lowers the order on the finest mesh one step at
                         a time (prolongation: the inclusion of the lower-order
                         traces; nothing condensed; the mesh's own vertex
                         patches), then halves the mesh at order p_min.
                         0: no order levels.                                  */
} dpg_options;

typedef struct dpg_ctx dpg_ctx;

/* Fills opt with the defaults: FP64, V(1,1), theta = 1/5, maxit = 500, no
 * order levels. */
void dpg_default_options(dpg_options *opt);

/* Builds the mesh topology (canonical numbering, element maps, macro sets,
 * vertex patches, prolongation maps) for an n^3 mesh of order p >= 1 with
 * test enrichment dp >= 1 and angular frequency omega > 0, and uploads it.
 * The problem is the one of Sec. 2 (eq. helmholtz: time-harmonic acoustics
 * in first-order form with an impedance condition on Gamma, the ultraweak
 * DPG formulation with the test order raised by dp); the levels, macro grids
 * and patches are those of the solver of Sec. 3.  loads[0..nrhs-1] are the
 * right-hand sides assembled by dpg_assemble.  mat may be NULL.  On success
 * *out owns the context. */
int dpg_setup(const dpg_mesh *mesh, int p, int dp, double omega, const dpg_material *mat,
              const dpg_load *loads, int nrhs, const dpg_options *opt, dpg_ctx **out);

/* The boundary load points where dpg_load.u0_qp gives the impedance data
 * u0 (Sec. 2, eq. helmholtz): the Gauss rule of the load integrals, p + dp + 5
 * points per direction, on every face of Gamma.  Faces in the order axis
 * d = 0, 1, 2 (x, y, z), side low then high (outward normal -e_d, +e_d),
 * cells (c1, c2) along the two other axes in ascending axis order, c1
 * fastest; on each face the points with the first in-plane coordinate
 * fastest.  Writes min(cap, count) points as (x, y, z) triples to xyz (may
 * be NULL) and returns count = 6 n^2 (p + dp + 5)^2, or a negative error. */
int64_t dpg_boundary_points(const dpg_ctx *ctx, double *xyz, int64_t cap);

/* Element DPG work on the GPU, all in FP64 (Sec. 2 and Sec. 1.2): Gram
 * matrix G of the adjoint graph norm, B and loads l; Cholesky G = L L^H;
 * W = L^-1 [B l]; K = W^H W; static condensation of the fields,
 * S = K_tt - K_tf K_ff^-1 K_ft and s likewise.  Errors: DPG_ENOTPD names
 * the element. */
int dpg_assemble(dpg_ctx *ctx);

/* Multigrid hierarchy on the GPU (Sec. 3), FP64: per level, macro
 * condensation of the 8 children of every coarse element, Galerkin coarse
 * element matrices P^T M P (with DPG_STORE_COARSE: the element DPG matrices
 * of the coarser mesh itself, by the element stage of dpg_assemble at that
 * mesh size), vertex-patch blocks factored and inverted (the inverse kept in
 * FP64, plus an FP32 copy in mixed mode); dense Cholesky of the coarsest
 * operator.  Errors: DPG_ENOTPD names the coarse element, patch or level. */
int dpg_build_hierarchy(dpg_ctx *ctx);

/* Replaces the assembled loads by new right-hand sides for the same operator
 * (the loads l_K of Sec. 2 condensed onto the traces as in Sec. 1.2:
 * s = b_t - K_tf K_ff^-1 b_f with b = W^H (L^-1 l)).  Elements with equal
 * wave speed and the same faces on Gamma have equal G and B, so s is one
 * linear map of the element's load vector l per such class (and so are the
 * field-recovery data): the first call (or dpg_release_setup) forms these
 * maps by the element chain with identity loads on one element of each class
 * (up to 512 classes), and every update is then the load integrals of the
 * elements and one matrix product per element.  Over every element when some
 * load has plane-wave or u0_qp data; when all loads are Gaussian point
 * sources only over the elements whose box comes within 8 sigma of a source
 * (the others get zero loads).  With more classes (a wave speed that varies
 * from element to element) every update runs the element chain of
 * dpg_assemble again on those elements.  Output: the condensed trace loads,
 * n_trace x nrhs, if s_out is not NULL. */
int dpg_load_rhs(dpg_ctx *ctx, const dpg_load *loads, int nrhs, double *s_out);

/* Frees what only dpg_assemble and dpg_build_hierarchy use: the element and
 * coarse element matrices, the full condensed macro blocks, the dense
 * coarsest operator and the setup work areas (the element-stage ones too
 * once the load maps of dpg_load_rhs exist; they are formed here if not
 * yet).  Solves, dpg_load_rhs, dpg_get_fields and dpg_error_indicator keep
 * working; dpg_assemble, dpg_build_hierarchy and the exports of the freed
 * matrices return DPG_ESTATE afterwards.  For callers that keep many
 * hierarchies resident (a solve server).  Requires a built hierarchy
 * (DPG_ESTATE otherwise). */
int dpg_release_setup(dpg_ctx *ctx);

/* Solves T x = rhs for nrhs right-hand sides (rhs: n_trace x nrhs trace
 * vectors; NULL: the assembled loads).  PCG on the macro grid with one
 * V(nu_pre, nu_post) cycle per iteration, x0 = 0, stop at
 * ||r|| / ||b|| <= tol (macro-grid residual), then recovery of the
 * condensed unknowns.  Outputs: x (n_trace x nrhs, canonical order),
 * iteration counts and final relative residuals (nrhs each; any may be
 * NULL).  Returns DPG_ENOCONV if some column hit maxit (its x is the last
 * iterate).  With nrhs > 1 the columns are solved together, up to 32 at a
 * time (multi-right-hand-side forms: every stored block streamed once per
 * application for all columns, one V-cycle per iteration for all columns,
 * per-column CG scalars; a converged column stops updating while the others
 * continue); DPG_COLUMNWISE in the options' flags solves them one by one
 * instead.  Both give each column the same iterates up to rounding. */
int dpg_solve(dpg_ctx *ctx, const double *rhs, int nrhs, double tol, double *x_out,
              int32_t *iters_out, double *relres_out);

/* Continuous batching (a block solve whose columns join and leave while it
 * runs): the multi-right-hand-side forms of dpg_solve over a batch of up to
 * max_slots <= 32 columns, each with its own CG recurrence and tolerance.
 * dpg_batch_add puts a right-hand side (rhs: n_trace trace vector, host or
 * device per DPG_DEVICE_PTRS; NULL: column load_col of the loads of
 * dpg_assemble / dpg_load_rhs, copied at the call) into the lowest free slot,
 * also while other columns are part-way through; its first iteration is the
 * first step of PCG from x0 = 0.  dpg_batch_step runs up to max_iters
 * iterations of the running columns (one V-cycle and one block matvec each,
 * every stored block streamed once for all columns, launched as HIP graphs
 * captured per batch width), stopping after the first iteration in which a
 * column finishes; done_out (max_slots entries) receives every finished slot
 * not taken yet, ndone_out their number.  dpg_batch_take writes the full
 * trace solution of a finished slot to x_out (n_trace) with its iteration
 * count and relative residual, frees the slot, and returns DPG_OK,
 * DPG_ENOCONV (maxit reached) or DPG_EBREAKDOWN for that column.  The
 * columns are independent: a column gets the same iterates (up to rounding)
 * whether it runs alone or beside others, joined early or late.  Requires a
 * built hierarchy; dpg_solve with nrhs > 1 uses the same machinery and
 * returns DPG_ESTATE while a batch is open.  dpg_batch_open closes a batch
 * already open; dpg_destroy closes it. */
int dpg_batch_open(dpg_ctx *ctx, int max_slots);
int dpg_batch_add(dpg_ctx *ctx, const double *rhs, int load_col, double tol, int32_t *slot_out);
int dpg_batch_step(dpg_ctx *ctx, int max_iters, int32_t *done_out, int32_t *ndone_out);
int dpg_batch_take(dpg_ctx *ctx, int slot, double *x_out, int32_t *iters_out,
                   double *relres_out);
int dpg_batch_close(dpg_ctx *ctx);

/* For callers that cannot allocate device memory: code run under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and errors as dpg_solve with DPG_COLUMNWISE (columns
 * solved one after the other, each with the same iterates as dpg_solve gives
 * it), but the call allocates nothing: no hipMalloc or hipFree, no HIP graph
 * instantiation (every kernel is launched directly on the context's stream),
 * no library routine that allocates.  The CG reduction partials and scalars
 * live in a static device array of the library (8,256 bytes per GPU, held
 * until the process ends) instead of the context's buffers; the vectors are
 * the ones dpg_setup allocated.  Every size the context accepts fits, since
 * the array holds one column's reductions.  All calls on one GPU share that
 * array: calls that overlap on one GPU (contexts on different streams, or
 * different host threads) race and must be serialised by the caller.
 * DPG_ESTATE while kernel profiling is on (dpg_profile creates events). */
int dpg_solve_noalloc(dpg_ctx *ctx, const double *rhs, int nrhs, double tol, double *x_out,
                      int32_t *iters_out, double *relres_out);

/* Field coefficients of the element-interior unknowns for trace solutions x
 * (n_trace x nrhs): the back-substitution of the static condensation
 * (Sec. 1.2: the field unknowns are eliminated element by element and
 * recovered from the traces), x_f = K_ff^-1 (b_f - K_ft x_t) per element, output
 * [nrhs][n^3][4 p^3] in the order (p, u_x, u_y, u_z), each a Legendre
 * tensor product with x-degree fastest.  Requires the assembled loads. */
int dpg_get_fields(dpg_ctx *ctx, const double *x, int nrhs, double *fields_out);

/* DPG residual error indicator (Sec. 1.2, the method's built-in error
 * estimate; Sec. 3, first paragraph: it drives the refinements that produce
 * the mesh hierarchy): for trace solutions x (n_trace x nrhs, as from
 * dpg_solve for the context's first nrhs loads), per element K
 *     eta_K^2 = r^H G_K^-1 r,   r = l_K - B_K [x_f; x_t],
 * the residual of the element equations in the dual test norm, with the
 * fields x_f recovered from the traces.  Output [nrhs][n^3] doubles.
 * Re-runs the FP64 element stage (Gram and B, both Cholesky factors) on the
 * GPU and allocates a staging copy when the pointers are host memory.
 * sum_K eta_K^2 is the quantity the DPG solution minimises. */
int dpg_error_indicator(dpg_ctx *ctx, const double *x, int nrhs, double *eta2_out);

typedef struct {
  int64_t n_trace;          /* trace unknowns of the finest mesh          */
  int64_t n_macro;          /* macro-grid unknowns of the finest mesh     */
  int32_t nlevels;          /* meshes in the hierarchy (finest included)  */
  int32_t level_n[16];      /* mesh size per level, finest first          */
  int64_t level_ntrace[16];
  int64_t level_nmacro[16]; /* 0 for the coarsest                         */
  int64_t resident_bytes;   /* device memory held by the context          */
  int32_t n_test, n_field, n_tr;
  double setup_ms[4];       /* topology, assemble, hierarchy, last solve  */
  int32_t level_p[16];      /* order per level, finest first              */
} dpg_info_t;

int dpg_info(const dpg_ctx *ctx, dpg_info_t *info);

/* Export of internal arrays, for testing against an independent reference.
 * Writes at most cap elements to out and returns the number of elements the
 * full array has (or a negative error).  `level` indexes meshes finest = 0.
 * Integer arrays are int64; matrices are complex (2 doubles per entry). */
enum {
  DPG_X_ELEM_DOFS = 1,   /* int64 [nel][n_tr], -1 = absent (Gamma flux)          */
  DPG_X_MACRO_B = 2,     /* int64 canonical index of each macro unknown         */
  DPG_X_BLOCK_B = 3,     /* int64 CSR: [nblk+1 offsets][macro indices, ascending]*/
  DPG_X_BLOCK_I = 4,     /* int64 CSR: [nblk+1 offsets][canonical indices]      */
  DPG_X_PATCHES = 5,     /* int64 CSR: [npatch+1 offsets][macro indices]        */
  DPG_X_PROLONG = 6,     /* int64 CSR of P: [nM+1 offsets][coarse trace cols]   */
  DPG_X_ELEM_S = 7,      /* complex [nel][n_tr][n_tr] condensed element matrix  */
  DPG_X_ELEM_RHS = 8,    /* complex [nrhs][nel][n_tr] condensed element loads   */
  DPG_X_MACRO_M = 9,     /* complex per block n_B x n_B (ascending macro order) */
  DPG_X_COARSE_E = 10,   /* complex [nel][n_tr][n_tr] Galerkin element matrices */
  DPG_X_PATCH_INV = 11,  /* complex per patch n x n inverse of the patch block  */
  DPG_X_COARSEST = 12,   /* complex n0 x n0 coarsest operator T_0               */
  DPG_X_PROLONG_VAL = 13,/* double values of P, in the order of DPG_X_PROLONG   */
  DPG_X_ASM_RHS = 14     /* complex [nrhs][n_trace] assembled condensed loads   */
};
int64_t dpg_export(const dpg_ctx *ctx, int what, int level, void *out, int64_t cap);

/* Kernel timing.  dpg_profile(ctx, 1) resets the counters and brackets every
 * later kernel launch of the context with HIP events on its stream;
 * dpg_profile(ctx, 0) stops.  While profiling is on, the setup runs on the
 * context's stream alone (no overlap of its four setup streams), so that each
 * launch's events time that launch.  dpg_kernel_stats returns, for one kernel
 * class, the launches timed so far, their summed duration and their summed
 * algorithmic work: bytes for the single-column block-apply kernels (packed
 * Hermitian blocks, each read once), flops for the dense kernels (LAPACK
 * counts) and for the multi-column block applies (8 n^2 nr real flops per
 * block of order n applied to nr columns).  Classes follow the kernel
 * symbols; DPG_K_POTRF and DPG_K_TRSM time whole Cholesky and forward-solve
 * routines (several kernels each), and DPG_K_POTRF_DIAG ... DPG_K_TRSM_UPDATE
 * their kernels one by one, each launch with its share of the routine's
 * LAPACK count split by the steps of the blocked algorithm (diagonal block,
 * panel, updates; solves with the diagonal-block inverses, updates). */
enum {
  DPG_K_GRAM = 0, DPG_K_BMAT = 1, DPG_K_LOAD = 2, DPG_K_POTRF = 3, DPG_K_TRSM = 4,
  DPG_K_GEMM = 5, DPG_K_MACRO_ASM = 6, DPG_K_PATCH_GATHER = 7, DPG_K_APPLY64 = 8,
  DPG_K_APPLY32 = 9, DPG_K_REDUCE = 10, DPG_K_CONDENSE = 11, DPG_K_EXPAND = 12,
  DPG_K_TRANSFER = 13, DPG_K_CG = 14, DPG_K_OTHER = 15, DPG_K_APPLYB64 = 16,
  DPG_K_APPLYB32 = 17, DPG_K_POTRF_DIAG = 18, DPG_K_POTRF_PANEL = 19,
  DPG_K_POTRF_UPDATE = 20, DPG_K_TRSM_INV = 21, DPG_K_TRSM_SOLVE = 22,
  DPG_K_TRSM_UPDATE = 23, DPG_K_NCLASS = 24
};
typedef struct {
  int64_t launches;
  double total_ms;
  double work;
} dpg_kstat;
int dpg_profile(dpg_ctx *ctx, int enable);
int dpg_kernel_stats(const dpg_ctx *ctx, int cls, dpg_kstat *out);

const char *dpg_last_error(const dpg_ctx *ctx);

void dpg_destroy(dpg_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* DPGMG_H */
