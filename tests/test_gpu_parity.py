"""Parity of the HIP library (through the C ABI) against the oracle.

Integer arrays (numbering, maps, macro sets, patch lists, prolongation
pattern) must be bit-exact; floating-point results of the FP64 path must
match to the tolerances stated per test (relative to the largest entry):
  element matrices                     cond(G) x unit round-off (>= 1e-12)
  hierarchy matrices                   1e-12 (patch inverses 1e-11)
  solution                             1e-10 (both sides at tol 1e-12)
  PCG iteration counts                 +-1 at the workload tolerance
The mixed-precision path (FP32 V-cycle, FP64 outer CG) must stay within 1e-8
of the FP64 oracle at tol 1e-10.
"""
import json
import os

import numpy as np
import pytest

from oracle import dpg, multigrid, topology
from paper_2304_01728_amd import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _D():
    from paper_2304_01728_amd import dpgmg as D
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return D


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def elem_tol(p, omega, h):
    """Tolerance for element matrices: both sides form B^H G^-1 B through a
    Cholesky factor of G, in different test bases; their FP64 results can
    differ by about cond(G) times the unit round-off (cond of the oracle's
    less well-conditioned basis, computed here), never below 1e-12."""
    from oracle import element
    G, _ = element.element_matrices(p, omega, h)
    ev = np.linalg.eigvalsh(G)
    return max(1e-12, ev[-1] / ev[0] * 2.0 ** -53)


class Case:
    """A library context and the oracle for the same plane-wave problem."""

    def __init__(self, N, p, omega, seed, nu=(1, 1), precision="fp64", oracle=True, nlevels=0):
        D = _D()
        self.D = D
        self.N, self.p, self.omega = N, p, omega
        self.d = workloads.plane_wave_direction(seed)
        self.nu = nu
        opt = D.dpg_default_options(nu_pre=nu[0], nu_post=nu[1], nlevels=nlevels,
                                    precision=D.DPG_MIXED if precision == "mixed" else D.DPG_FP64)
        print(f"[case] N={N} p={p} omega={omega:.4f} nu={nu} {precision}", flush=True)
        self.ctx = D.dpg_setup(N, p, omega, [dict(dir=self.d, amp=1.0)], options=opt)
        D.dpg_assemble(self.ctx)
        D.dpg_build_hierarchy(self.ctx)
        if oracle:
            self.pr = dpg.Problem(N, p, omega, [dict(u0=dpg.plane_wave_u0(omega, self.d))])
            self.S, self.s, self.rec = self.pr.condensed()
            self.rhs = dpg.assemble_vector(self.pr.edofs, self.s, self.pr.num.n)[:, 0]
            self.H = multigrid.Hierarchy(N, p, self.S, nu_pre=nu[0], nu_post=nu[1],
                                         nlevels=nlevels)


@pytest.fixture(scope="module")
def two_level():
    return Case(4, 2, 2 * np.pi, 0)


@pytest.fixture(scope="module")
def three_level():
    return Case(8, 2, 4 * np.pi, 5, nu=(2, 2))


@pytest.fixture(scope="module")
def odd_coarsest():
    return Case(6, 1, 3.0, 7, nu=(1, 2))


@pytest.fixture(scope="module")
def order_three():
    return Case(4, 3, 8 * np.pi, 1, nu=(2, 2))


ALL = ["two_level", "three_level", "odd_coarsest", "order_three"]


def _levels(case):
    """(export level index, oracle Level) pairs of the levels with a macro grid."""
    H = case.H
    return [(H.L - l, H.levels[l]) for l in range(H.L, 0, -1)]


@pytest.mark.parametrize("name", ALL)
def test_topology_bit_exact(name, request):
    c = request.getfixturevalue(name)
    D = c.D
    H = c.H
    for k in range(H.L + 1):
        lv = H.levels[H.L - k]
        ed = D.dpg_export(c.ctx, D.X_ELEM_DOFS, k).reshape(lv.edofs.shape)
        assert np.array_equal(ed, lv.edofs)
    for k, lv in _levels(c):
        mc = lv.macro
        assert np.array_equal(D.dpg_export(c.ctx, D.X_MACRO_B, k), mc.B)
        nb = len(mc.blocks_B)
        bb = D.dpg_export(c.ctx, D.X_BLOCK_B, k)
        ptr, body = bb[:nb + 1], bb[nb + 1:]
        for kc in range(nb):
            assert np.array_equal(body[ptr[kc]:ptr[kc + 1]], mc.macro_of[mc.blocks_B[kc]])
        bi = D.dpg_export(c.ctx, D.X_BLOCK_I, k)
        ptr, body = bi[:nb + 1], bi[nb + 1:]
        for kc in range(nb):
            assert np.array_equal(body[ptr[kc]:ptr[kc + 1]], mc.blocks_I[kc])
        pt = D.dpg_export(c.ctx, D.X_PATCHES, k)
        npch = len(mc.patches)
        ptr, body = pt[:npch + 1], pt[npch + 1:]
        for v in range(npch):
            assert np.array_equal(body[ptr[v]:ptr[v + 1]], mc.patches[v])
        P = lv.P.tocsr()
        P.sort_indices()
        pp = D.dpg_export(c.ctx, D.X_PROLONG, k)
        ptr, cols = pp[:mc.nM + 1], pp[mc.nM + 1:]
        assert np.array_equal(ptr, P.indptr) and np.array_equal(cols, P.indices)
        vals = D.dpg_export(c.ctx, D.X_PROLONG_VAL, k)
        assert np.abs(vals - P.data).max() <= 1e-14


@pytest.mark.parametrize("name", ALL)
def test_element_matrices_and_loads(name, request):
    c = request.getfixturevalue(name)
    D = c.D
    n_tr = c.pr.n_tr
    tol = elem_tol(c.p, c.omega, 1.0 / c.N)
    S = D.dpg_export(c.ctx, D.X_ELEM_S).reshape(c.pr.nel, n_tr, n_tr).transpose(0, 2, 1)
    assert rel(S, c.S) <= tol
    s = D.dpg_export(c.ctx, D.X_ELEM_RHS).reshape(c.pr.nel, n_tr)
    assert rel(s, c.s[:, :, 0]) <= tol
    sa = D.dpg_export(c.ctx, D.X_ASM_RHS)
    assert rel(sa, c.rhs) <= tol


@pytest.mark.parametrize("name", ALL)
def test_hierarchy_matrices(name, request):
    c = request.getfixturevalue(name)
    D = c.D
    n_tr = c.pr.n_tr
    for k, lv in _levels(c):
        M = D.dpg_export(c.ctx, D.X_MACRO_M, k)
        o = 0
        for Mo in lv.Mblocks:
            n = Mo.shape[0]
            assert rel(M[o:o + n * n].reshape(n, n).T, Mo) <= 1e-12
            o += n * n
        Si = D.dpg_export(c.ctx, D.X_PATCH_INV, k)
        o = 0
        for So in lv.Sinv:
            n = So.shape[0]
            assert rel(Si[o:o + n * n].reshape(n, n).T, So) <= 1e-11
            o += n * n
        Ec = D.dpg_export(c.ctx, D.X_COARSE_E, k + 1).reshape(-1, n_tr, n_tr).transpose(0, 2, 1)
        assert rel(Ec, c.H.levels[c.H.L - k - 1].E) <= 1e-12
    n0 = c.H.levels[0].n
    T0 = D.dpg_export(c.ctx, D.X_COARSEST).reshape(n0, n0).T
    assert rel(T0, c.H.levels[0].T) <= 1e-12


@pytest.mark.parametrize("name", ALL)
def test_solution_and_iterations(name, request):
    c = request.getfixturevalue(name)
    D = c.D
    x, it, rr, code = D.dpg_solve(c.ctx, tol=1e-12)
    xo, ito, rro = c.H.solve(c.rhs, 1e-12)
    assert code == D.DPG_OK and rr[0] <= 1e-12
    assert np.linalg.norm(x[0] - xo) <= 1e-10 * np.linalg.norm(xo)
    assert abs(int(it[0]) - ito) <= 1
    for tol in (1e-6, 1e-8, 1e-10):
        _, it, _, _ = D.dpg_solve(c.ctx, tol=tol)
        _, ito, _ = c.H.solve(c.rhs, tol)
        assert abs(int(it[0]) - ito) <= 1, (tol, it[0], ito)


def test_solution_matches_direct_solve(two_level):
    c = two_level
    D = c.D
    T = dpg.assemble(c.pr.edofs, c.S, c.pr.num.n)
    xd = dpg.direct_solve(T, c.rhs[:, None])[:, 0]
    x, it, rr, code = D.dpg_solve(c.ctx, tol=1e-13)
    assert np.linalg.norm(x[0] - xd) <= 1e-10 * np.linalg.norm(xd)


def test_fields(two_level):
    c = two_level
    D = c.D
    x, _, _, _ = D.dpg_solve(c.ctx, tol=1e-12)
    f = D.dpg_get_fields(c.ctx, x[0])
    fo = dpg.recover_fields(c.rec, c.pr.edofs, x[0][:, None])[:, :, 0]
    assert rel(f[0], fo) <= 1e-10


def test_explicit_rhs_zero_rhs_and_iteration_cap(two_level):
    c = two_level
    D = c.D
    x1, it1, _, _ = D.dpg_solve(c.ctx, tol=1e-10)
    # the same right-hand side passed explicitly: bitwise the same (deterministic kernels)
    own = D.dpg_export(c.ctx, D.X_ASM_RHS)
    x2, it2, _, _ = D.dpg_solve(c.ctx, rhs=own[None, :], tol=1e-10)
    assert it1[0] == it2[0] and np.array_equal(x2, x1)
    # the oracle's right-hand side: same iterations, solution to round-off
    x3, it3, _, _ = D.dpg_solve(c.ctx, rhs=c.rhs[None, :], tol=1e-10)
    assert abs(int(it3[0]) - int(it1[0])) <= 1 and rel(x3, x1) <= 1e-11
    x0, it0, rr0, code0 = D.dpg_solve(c.ctx, rhs=np.zeros((1, c.pr.num.n)), tol=1e-10)
    assert it0[0] == 0 and np.all(x0 == 0) and code0 == D.DPG_OK
    opt = D.dpg_default_options(maxit=2)
    ctx = D.dpg_setup(4, 2, 2 * np.pi, [dict(dir=c.d, amp=1.0)], options=opt)
    D.dpg_assemble(ctx)
    D.dpg_build_hierarchy(ctx)
    x, it, rr, code = D.dpg_solve(ctx, tol=1e-14)
    assert code == D.DPG_ENOCONV and it[0] == 2 and rr[0] > 1e-14


def test_call_order_enforced():
    D = _D()
    ctx = D.dpg_setup(4, 2, 2 * np.pi, [dict(dir=(1, 0, 0), amp=1.0)])
    with pytest.raises(D.DPGError) as e:
        D.dpg_solve(ctx, tol=1e-8)
    assert e.value.code == D.DPG_ESTATE
    with pytest.raises(D.DPGError) as e:
        D.dpg_build_hierarchy(ctx)
    assert e.value.code == D.DPG_ESTATE


def test_mixed_precision_error_vs_fp64_oracle(two_level):
    c = two_level
    m = Case(4, 2, 2 * np.pi, 0, precision="mixed", oracle=False)
    D = c.D
    xm, itm, rrm, code = D.dpg_solve(m.ctx, tol=1e-10)
    xo, ito, _ = c.H.solve(c.rhs, 1e-12)
    assert code == D.DPG_OK
    assert np.linalg.norm(xm[0] - xo) <= 1e-8 * np.linalg.norm(xo)
    assert abs(int(itm[0]) - c.H.solve(c.rhs, 1e-10)[1]) <= 2


def test_multiple_rhs_point_sources():
    """Several Gaussian point sources, homogeneous impedance data, solved as a
    block: every column matches the oracle, and its own single-column solve."""
    D = _D()
    N, p, omega = 4, 2, 3 * np.pi
    cen = workloads.source_centres(3, 3)
    loads = [dict(dir=(0, 0, 1), amp=0.0, sources=[[*c0, 0.08, 1.0, 0.5]]) for c0 in cen]
    ctx = D.dpg_setup(N, p, omega, loads)
    D.dpg_assemble(ctx)
    D.dpg_build_hierarchy(ctx)
    x, it, rr, code = D.dpg_solve(ctx, nrhs=3, tol=1e-12)
    pr = dpg.Problem(N, p, omega, [dict(f=dpg.gaussian_sources([c0], 0.08, [1.0 + 0.5j]))
                                   for c0 in cen])
    S, s, rec = pr.condensed()
    rhs = dpg.assemble_vector(pr.edofs, s, pr.num.n)
    H = multigrid.Hierarchy(N, p, S)
    for k in range(3):
        xo, ito, _ = H.solve(rhs[:, k], 1e-12)
        assert np.linalg.norm(x[k] - xo) <= 1e-10 * np.linalg.norm(xo)
        assert abs(int(it[k]) - ito) <= 1
        # the single-column path sums the products in another order
        xs, _, _, _ = D.dpg_solve(ctx, rhs=rhs[:, k][None, :], tol=1e-12)
        assert rel(xs[0], x[k]) <= 1e-10
    f = D.dpg_get_fields(ctx, x)
    fo = dpg.recover_fields(rec, pr.edofs, x.T)
    assert rel(f, fo.transpose(2, 0, 1)) <= 1e-10


def test_load_rhs_replaces_loads(two_level):
    c = two_level
    D = c.D
    d2 = workloads.plane_wave_direction(11)
    s_new = D.dpg_load_rhs(c.ctx, [dict(dir=d2, amp=0.5 - 0.25j)])
    pr = dpg.Problem(4, 2, 2 * np.pi, [dict(u0=dpg.plane_wave_u0(2 * np.pi, d2, amp=0.5 - 0.25j))])
    _, s, _ = pr.condensed()
    ref = dpg.assemble_vector(pr.edofs, s, pr.num.n)[:, 0]
    assert rel(s_new[0], ref) <= 1e-12
    x, _, _, _ = D.dpg_solve(c.ctx, tol=1e-12)
    xo, _, _ = c.H.solve(ref, 1e-12)
    assert np.linalg.norm(x[0] - xo) <= 1e-10 * np.linalg.norm(xo)
    D.dpg_load_rhs(c.ctx, [dict(dir=c.d, amp=1.0)])       # restore for later tests


def test_full_size_workload_against_stored_oracle_values():
    """16^3, p = 3, omega = 8 pi, V(2,2), FP64.  Iteration counts, sampled
    entries and the whole solution vector against values the oracle wrote
    (tests/golden/make_golden.py); topology bit-exact against the oracle
    computed here; sampled element matrices against the oracle."""
    D = _D()
    path = os.path.join(HERE, "golden", "plane_wave_16.json")
    g = json.load(open(path))
    w = workloads.plane_wave_16()
    opt = D.dpg_default_options(nu_pre=w.nu_pre, nu_post=w.nu_post, theta=w.theta)
    print("[case] full size 16^3 p=3", flush=True)
    ctx = D.dpg_setup(w.N, w.p, w.omega, [dict(dir=w.direction, amp=1.0)], options=opt)
    D.dpg_assemble(ctx)
    D.dpg_build_hierarchy(ctx)
    x8, it8, _, _ = D.dpg_solve(ctx, tol=1e-8)
    assert abs(int(it8[0]) - g["iters_tol_1e-8"]) <= 1
    x12, it12, _, _ = D.dpg_solve(ctx, tol=1e-12)
    assert abs(int(it12[0]) - g["iters_tol_1e-12"]) <= 1
    pos = np.array(g["sample_pos"])
    ref = np.array(g["x12_sample_re"]) + 1j * np.array(g["x12_sample_im"])
    assert np.abs(x12[0][pos] - ref).max() <= 1e-10 * g["x_inf_norm"]
    # the whole solution vector
    xo = np.load(os.path.join(HERE, "golden", "plane_wave_16_x12.npy"))
    assert xo.shape == x12[0].shape
    assert np.linalg.norm(x12[0] - xo) <= 1e-10 * np.linalg.norm(xo)
    sref = np.array(g["s_sample_re"]) + 1j * np.array(g["s_sample_im"])
    sa = D.dpg_export(ctx, D.X_ASM_RHS)
    assert np.abs(sa[pos] - sref).max() <= elem_tol(w.p, w.omega, 1.0 / w.N) * np.abs(sa).max()
    # topology of the finest level
    num = topology.Numbering(w.N, w.p)
    ed = topology.element_dofs(num)
    assert np.array_equal(D.dpg_export(ctx, D.X_ELEM_DOFS, 0).reshape(ed.shape), ed)
    mc = topology.MacroLevel(num)
    assert np.array_equal(D.dpg_export(ctx, D.X_MACRO_B, 0), mc.B)
    pt = D.dpg_export(ctx, D.X_PATCHES, 0)
    npch = len(mc.patches)
    assert np.array_equal(pt[npch + 1:], np.concatenate(mc.patches))
    # element matrices of a corner, an edge, a face and an interior element
    pr = dpg.Problem(w.N, w.p, w.omega, [dict(u0=dpg.plane_wave_u0(w.omega, w.direction))])
    N = w.N
    sample = [0, 5, 5 + N * 7, 5 + N * (7 + N * 9), N ** 3 - 1]
    S, s, _ = pr.condensed(elements=sample)
    Sg = D.dpg_export(ctx, D.X_ELEM_S).reshape(pr.nel, pr.n_tr, pr.n_tr)
    tol = elem_tol(w.p, w.omega, 1.0 / w.N)
    for e in sample:
        assert rel(Sg[e].T, S[e]) <= tol


# ---- DPG residual error indicator (Sec. 1.2) -------------------------------------------------

def test_error_indicator_matches_oracle(two_level):
    """eta_K^2 of every element for the GPU solution, against the oracle's
    residual of the same solution.  The residual l - Bx cancels, so the bound
    is relative to the largest eta_K^2."""
    c = two_level
    D = c.D
    x, _, _, _ = D.dpg_solve(c.ctx, tol=1e-12)
    eta2 = D.dpg_error_indicator(c.ctx, x)
    ref = dpg.error_indicator(c.pr, x[0][:, None], c.rec)[:, 0]
    assert np.abs(eta2[0] - ref).max() <= 1e-9 * ref.max()


def test_error_indicator_several_loads_and_falls_with_h():
    D = _D()
    N, p, omega = 4, 2, 3 * np.pi
    cen = workloads.source_centres(3, 2)
    loads = [dict(dir=(0, 0, 1), amp=0.0, sources=[[*c0, 0.08, 1.0, 0.5]]) for c0 in cen]
    ctx = D.dpg_setup(N, p, omega, loads)
    D.dpg_assemble(ctx)
    D.dpg_build_hierarchy(ctx)
    x, _, _, _ = D.dpg_solve(ctx, nrhs=2, tol=1e-12)
    eta2 = D.dpg_error_indicator(ctx, x)
    pr = dpg.Problem(N, p, omega, [dict(f=dpg.gaussian_sources([c0], 0.08, [1.0 + 0.5j]))
                                   for c0 in cen])
    _, _, rec = pr.condensed()
    ref = dpg.error_indicator(pr, x.T, rec)
    for k in range(2):
        assert np.abs(eta2[k] - ref[:, k]).max() <= 1e-9 * ref[:, k].max()
    ctx.close()
    # plane waves: the total falls with h
    d = workloads.plane_wave_direction(4)
    tot = []
    for N in (4, 8):
        ctx = D.dpg_setup(N, 2, 2 * np.pi, [dict(dir=d, amp=1.0)])
        D.dpg_assemble(ctx)
        D.dpg_build_hierarchy(ctx)
        x, _, _, _ = D.dpg_solve(ctx, tol=1e-10)
        tot.append(D.dpg_error_indicator(ctx, x).sum())
        ctx.close()
    assert tot[1] < 0.25 * tot[0]


# ---- impedance data given at the boundary load points (Sec. 2, eq. helmholtz) ---------------

def _boundary_normals(count, N, nq):
    face = np.arange(count) // (nq * nq)
    d = face // (2 * N * N)
    s = (face // (N * N)) % 2
    n = np.zeros((count, 3))
    n[np.arange(count), d] = np.where(s == 1, 1.0, -1.0)
    return n


def test_impedance_data_at_boundary_points():
    D = _D()
    N, p, omega = 4, 2, 2 * np.pi
    dvec = workloads.plane_wave_direction(0)
    ctx0 = D.dpg_setup(N, p, omega, [dict(dir=dvec, amp=1.0)])
    X = D.dpg_boundary_points(ctx0)
    nq = p + 1 + 5
    assert X.shape == (6 * N * N * nq * nq, 3)
    nrm = _boundary_normals(X.shape[0], N, nq)
    assert np.all(np.abs(np.sum(X * np.abs(nrm), axis=1) - (nrm.sum(axis=1) > 0)) == 0)
    pw = (1.0 - nrm @ dvec) * np.exp(-1j * omega * (X @ dvec))
    # the plane wave given point by point equals the built-in plane-wave load
    ctx1 = D.dpg_setup(N, p, omega, [dict(amp=0.0, u0_qp=pw)])
    for ctx in (ctx0, ctx1):
        D.dpg_assemble(ctx)
    s0, s1 = D.dpg_export(ctx0, D.X_ASM_RHS), D.dpg_export(ctx1, D.X_ASM_RHS)
    assert rel(s1, s0) <= 1e-13
    # general data (plus half a plane wave, summed) against the oracle
    g = lambda X, n: (X[:, 0] + 2j * X[:, 1] - X[:, 2] ** 2) * (1.0 + n @ np.array([0.3, 0.5, 0.7]))
    ctx2 = D.dpg_setup(N, p, omega, [dict(dir=dvec, amp=0.5, u0_qp=g(X, nrm))])
    D.dpg_assemble(ctx2)
    D.dpg_build_hierarchy(ctx2)
    u0pw = dpg.plane_wave_u0(omega, dvec, amp=0.5)
    pr = dpg.Problem(N, p, omega, [dict(u0=lambda Y, n: g(Y, n[None, :].repeat(len(Y), 0))
                                        + u0pw(Y, n))])
    S, s, _ = pr.condensed()
    rhs = dpg.assemble_vector(pr.edofs, s, pr.num.n)[:, 0]
    assert rel(D.dpg_export(ctx2, D.X_ASM_RHS), rhs) <= elem_tol(p, omega, 1.0 / N)
    x, _, _, _ = D.dpg_solve(ctx2, tol=1e-12)
    xo, _, _ = multigrid.Hierarchy(N, p, S).solve(rhs, 1e-12)
    assert np.linalg.norm(x[0] - xo) <= 1e-10 * np.linalg.norm(xo)
    for ctx in (ctx0, ctx1, ctx2):
        ctx.close()
