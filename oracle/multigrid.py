"""DPG-MG: macro grids, Galerkin coarse operators, V-cycle, PCG (oracle).

Sec. 3 of the paper, restated:
  * The hierarchy comes from uniform refinement; here N_L -> N_L/2 -> ...,
    halving while N is even and N > 2 (a mesh with N = 2 is halved once).
  * Two-stage prolongation ("Prolongation"): on mesh l, the trace unknowns
    not on the skeleton of mesh l-1 are statically condensed (macro grid),
    then the natural inclusion P_l maps the trace unknowns of mesh l-1 onto
    the macro-grid unknowns.
  * Coarse operators by restriction ("Alternative construction"):
    T_{l-1} = P_l^T M_l P_l, formed coarse element by coarse element; or,
    for the comparison the paper makes (Sec. 3 and 4.2), assembled directly
    on the coarse mesh from its own element DPG matrices ("store").
  * Smoother ("V-cycle and smoother"): additive Schwarz over the macro-grid
    unknowns supported in each coarse-grid vertex patch, damped by theta.
    CG and smoothing both act on the macro grid.
  * Coarsest mesh: a direct Cholesky solve inside the V-cycle.
  * Outer iteration: CG preconditioned by one V(nu_pre, nu_post) cycle, zero
    initial guess, stopped at relative l2 residual <= tol (Sec. 4 parameters).

Order levels (Sec. 4.2, uniform p-refinements): optionally the order is
lowered on the finest mesh before the mesh is coarsened; between two orders
on one mesh the prolongation is the inclusion of the lower-order traces
(hierarchical bases: an injection), nothing is condensed, and the patches
are the vertex patches of the mesh itself.

Readings where the paper is silent: damping theta = 1/5.  Colouring the
coarse vertices by index parity gives 8 classes of pairwise M-orthogonal
patches, so lambda_max(S M) <= 8, and the bound is attained by unknowns on a
boundary face of a boundary coarse cell (they lie in all 8 patches around
it); theta must stay below 1/4 for the V-cycle to be positive definite.
Flexible Polak-Ribiere beta, equal to Fletcher-Reeves in exact arithmetic;
Re() of the Hermitian inner products.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import dpg, topology


def level_plan(N, p, p_min=None, nlevels=0):
    """(mesh size, order) of every level, finest first: with p_min < p the
    order is lowered on the finest mesh one step at a time down to p_min (the
    uniform p-refinements of Sec. 4.2 read from coarse to fine), then the mesh
    is halved as in level_sizes."""
    p_min = p if p_min is None else p_min
    plan = [(N, q) for q in range(p, p_min, -1)] + [(n, p_min) for n in level_sizes(N)]
    return plan[:nlevels] if nlevels > 0 else plan


def level_sizes(N):
    """Mesh sizes from finest to coarsest."""
    sizes = [N]
    while N % 2 == 0 and (N > 2 or len(sizes) == 1):
        N //= 2
        sizes.append(N)
    return sizes


class Level:
    def __init__(self, N, p, E):
        self.N, self.p = N, p
        self.num = topology.Numbering(N, p)
        self.edofs = topology.element_dofs(self.num)
        self.E = E                      # element matrices [nel, n_tr, n_tr]
        self.n = self.num.n


def condense_block(lv, mc, kc):
    """Coarse element kc: M_K = T_BB - T_BI T_II^-1 T_IB from its 8 children.

    Returns (M_K, Cholesky factor of T_II, T_IB)."""
    Bd, Id = mc.blocks_B[kc], mc.blocks_I[kc]
    dofs = np.concatenate([Bd, Id])
    pos = {int(d): i for i, d in enumerate(dofs)}
    T = np.zeros((dofs.size, dofs.size), dtype=np.complex128)
    for e in mc.children[kc]:
        d = lv.edofs[e]
        ok = np.nonzero(d >= 0)[0]
        loc = np.array([pos[int(d[i])] for i in ok])
        T[np.ix_(loc, loc)] += lv.E[e][np.ix_(ok, ok)]
    nb = Bd.size
    TBB, TBI, TIB, TII = T[:nb, :nb], T[:nb, nb:], T[nb:, :nb], T[nb:, nb:]
    c = sla.cho_factor(TII, lower=True)
    M = TBB - TBI @ sla.cho_solve(c, TIB)
    return 0.5 * (M + M.conj().T), c, TIB


def assemble_macro(mc, blocks, Mblocks):
    """Sparse macro operator sum_K E_K^T M_K E_K over the given blocks."""
    rows, cols, vals = [], [], []
    for kc, M in zip(blocks, Mblocks):
        m = mc.macro_of[mc.blocks_B[kc]]
        rows.append(np.repeat(m, m.size))
        cols.append(np.tile(m, m.size))
        vals.append(M.ravel())
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(mc.nM, mc.nM)).tocsr()


def order_blocks(lv):
    """An order level (mesh unchanged below it): the macro grid is the whole
    trace space, its blocks are the element matrices (unknowns in ascending
    canonical order), nothing is condensed."""
    mc = topology.OrderLevel(lv.num)
    lv.macro = mc
    lv.Mblocks = []
    for e in range(len(mc.children)):
        d = lv.edofs[e]
        loc = np.nonzero(d >= 0)[0]
        loc = loc[np.argsort(d[loc])]
        lv.Mblocks.append(lv.E[e][np.ix_(loc, loc)])
    lv.TII, lv.TIB = None, None
    lv.M = assemble_macro(mc, range(len(mc.children)), lv.Mblocks)


def macro_condense(lv):
    """Macro condensation of every coarse element of the level."""
    mc = topology.MacroLevel(lv.num)
    lv.macro = mc
    lv.Mblocks, lv.TII, lv.TIB = [], [], []
    for kc in range(len(mc.children)):
        M, c, TIB = condense_block(lv, mc, kc)
        lv.Mblocks.append(M)
        lv.TII.append(c)
        lv.TIB.append(TIB)
    lv.M = assemble_macro(mc, range(len(mc.children)), lv.Mblocks)


def galerkin_block(mc, P, Mk, kc, coarse_edofs):
    """A_Kc = P_Kc^T M_Kc P_Kc of coarse element kc."""
    rows = mc.macro_of[mc.blocks_B[kc]]
    cd = coarse_edofs[kc]
    Pk = np.zeros((rows.size, cd.size))
    ok = cd >= 0
    Pk[:, ok] = P[rows][:, cd[ok]].toarray()
    Ak = Pk.T @ Mk @ Pk
    return 0.5 * (Ak + Ak.conj().T)


def galerkin(lv, coarse_num, coarse_edofs):
    """Coarse element matrices of every coarse element."""
    mc = lv.macro
    return np.array([galerkin_block(mc, lv.P, lv.Mblocks[kc], kc, coarse_edofs)
                     for kc in range(len(mc.children))])


def patch_inverse(M, idx):
    """Inverse of the principal submatrix of M on the patch unknowns idx."""
    S = M[idx][:, idx].toarray()
    c = sla.cho_factor(S, lower=True)
    Si = sla.cho_solve(c, np.eye(idx.size, dtype=np.complex128))
    return 0.5 * (Si + Si.conj().T)


def build_patches(lv):
    Md = lv.M.tocsr()
    lv.Sinv = [patch_inverse(Md, idx) for idx in lv.macro.patches]


class Hierarchy:
    """All levels, finest last: levels[0] is the coarsest mesh."""

    def __init__(self, N, p, S_fine, theta=0.2, nu_pre=1, nu_post=1, nlevels=0, coarse=None,
                 p_min=None):
        """coarse: None for coarse operators by restriction (Galerkin P^T M P);
        else a function n -> element matrices of the n^3 mesh assembled
        directly ("store", the approach the paper compares against).
        p_min: lowest order of the order levels above the mesh levels
        (level_plan); None = no order levels."""
        plan = level_plan(N, p, p_min, nlevels)
        if coarse is not None and plan[0][1] != plan[-1][1]:
            raise ValueError("stored coarse operators are for mesh levels only")
        self.theta, self.nu_pre, self.nu_post = theta, nu_pre, nu_post
        self.p = p
        self.plan = plan
        L = len(plan) - 1
        self.L = L
        levels = [None] * (L + 1)
        E = S_fine
        for l in range(L, 0, -1):
            (Nl, ql), (Nc, qc) = plan[L - l], plan[L - l + 1]
            lv = Level(Nl, ql, E)
            coarse_num = topology.Numbering(Nc, qc)
            lv.order_level = Nc == Nl
            if lv.order_level:
                order_blocks(lv)
                lv.P = topology.order_injection(lv.num, coarse_num)
            else:
                macro_condense(lv)
                lv.P = topology.prolongation(lv.macro, coarse_num)
            build_patches(lv)
            if coarse is None:
                E = galerkin(lv, coarse_num, topology.element_dofs(coarse_num))
            else:
                E = coarse(Nc)
            levels[l] = lv
        lv0 = Level(*plan[L], E)
        lv0.T = dpg.assemble(lv0.edofs, E, lv0.n).toarray()
        lv0.chol = sla.cho_factor(lv0.T, lower=True)
        levels[0] = lv0
        self.levels = levels

    # -- pieces of the V-cycle ------------------------------------------------
    def smooth(self, lv, r, x):
        """x + theta * sum_v R_v^T S_v^-1 R_v (r - M x)."""
        res = r - lv.M @ x
        dx = np.zeros_like(x)
        for idx, Si in zip(lv.macro.patches, lv.Sinv):
            dx[idx] += Si @ res[idx]
        return x + self.theta * dx

    def condense_rhs(self, lv, rc):
        """Macro right-hand side r_B - sum_K T_BI T_II^-1 r_I of a trace vector."""
        if getattr(lv, 'order_level', False):
            return rc.copy()
        mc = lv.macro
        rB = rc[mc.B].copy()
        for kc in range(len(mc.children)):
            w = sla.cho_solve(lv.TII[kc], rc[mc.blocks_I[kc]])
            rB[mc.macro_of[mc.blocks_B[kc]]] -= lv.TIB[kc].conj().T @ w
        return rB

    def expand(self, lv, rc, eB):
        """Trace vector with B part eB and I part T_II^-1 (r_I - T_IB e_B)."""
        if getattr(lv, 'order_level', False):
            return eB.copy()
        mc = lv.macro
        e = np.zeros(lv.n, dtype=np.complex128)
        e[mc.B] = eB
        for kc in range(len(mc.children)):
            rhs = rc[mc.blocks_I[kc]] - lv.TIB[kc] @ eB[mc.macro_of[mc.blocks_B[kc]]]
            e[mc.blocks_I[kc]] = sla.cho_solve(lv.TII[kc], rhs)
        return e

    def vcycle(self, l, r):
        lv = self.levels[l]
        x = np.zeros_like(r)
        for _ in range(self.nu_pre):
            x = self.smooth(lv, r, x)
        rc = lv.P.T @ (r - lv.M @ x)
        if l - 1 == 0:
            ec = sla.cho_solve(self.levels[0].chol, rc)
        else:
            lc = self.levels[l - 1]
            eB = self.vcycle(l - 1, self.condense_rhs(lc, rc))
            ec = self.expand(lc, rc, eB)
        x = x + lv.P @ ec
        for _ in range(self.nu_post):
            x = self.smooth(lv, r, x)
        return x

    # -- outer iteration --------------------------------------------------------
    def pcg(self, b, tol, maxit=1000):
        """Preconditioned CG on the finest macro operator; returns x, iters, relres."""
        lv = self.levels[self.L]
        x = np.zeros_like(b)
        r = b.copy()
        bnorm = np.linalg.norm(b)
        if bnorm == 0.0:
            return x, 0, 0.0
        z = self.vcycle(self.L, r)
        p = z.copy()
        rz = np.real(np.vdot(r, z))
        it = 0
        relres = 1.0
        while it < maxit:
            q = lv.M @ p
            alpha = rz / np.real(np.vdot(p, q))
            x = x + alpha * p
            r = r - alpha * q
            it += 1
            relres = np.linalg.norm(r) / bnorm
            if relres <= tol:
                break
            zn = self.vcycle(self.L, r)
            beta = np.real(np.vdot(r, zn - z)) / rz
            rz = np.real(np.vdot(r, zn))
            p = zn + beta * p
            z = zn
        return x, it, relres

    def solve(self, s, tol, maxit=1000):
        """Full trace solution of T_L x = s via PCG on the macro grid."""
        lv = self.levels[self.L]
        bM = self.condense_rhs(lv, s)
        xB, it, rr = self.pcg(bM, tol, maxit)
        return self.expand(lv, s, xB), it, rr
