"""Stored coarse operators (DPG_STORE_COARSE; the alternative of Sec. 3 that
Sec. 4.2 compares with restriction) against the oracle's store hierarchy.

Tolerances as for the restricted hierarchy: coarse element matrices within
cond(G) x unit round-off of the oracle's (both are element DPG matrices, at the
coarse h), the coarsest operator within the same bound, solutions within 1e-10
at tol 1e-12, iteration counts +-1.
"""
import numpy as np
import pytest

from oracle import dpg, multigrid
from paper_2304_01728_amd import workloads

from test_gpu_parity import elem_tol, rel

pytestmark = pytest.mark.gpu


def _D():
    from paper_2304_01728_amd import dpgmg as D
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return D


def _store(p, omega):
    return lambda n: dpg.Problem(n, p, omega, []).condensed_operator()


@pytest.mark.parametrize("N,p,omega,seed,nu", [(4, 2, 2 * np.pi, 0, (1, 1)),
                                               (8, 2, 4 * np.pi, 5, (2, 2))])
def test_store_hierarchy_matches_oracle(N, p, omega, seed, nu):
    D = _D()
    d = workloads.plane_wave_direction(seed)
    opt = D.dpg_default_options(nu_pre=nu[0], nu_post=nu[1], flags=D.DPG_STORE_COARSE)
    print(f"[store] N={N} p={p} omega={omega:.4f}", flush=True)
    ctx = D.dpg_setup(N, p, omega, [dict(dir=d, amp=1.0)], options=opt)
    D.dpg_assemble(ctx)
    D.dpg_build_hierarchy(ctx)
    pr = dpg.Problem(N, p, omega, [dict(u0=dpg.plane_wave_u0(omega, d))])
    S, s, _ = pr.condensed()
    rhs = dpg.assemble_vector(pr.edofs, s, pr.num.n)[:, 0]
    H = multigrid.Hierarchy(N, p, S, nu_pre=nu[0], nu_post=nu[1], coarse=_store(p, omega))
    n_tr = pr.n_tr
    for k in range(1, H.L + 1):
        lv = H.levels[H.L - k]
        Ec = D.dpg_export(ctx, D.X_COARSE_E, k).reshape(-1, n_tr, n_tr).transpose(0, 2, 1)
        assert rel(Ec, lv.E) <= elem_tol(p, omega, 1.0 / lv.N)
    n0 = H.levels[0].n
    T0 = D.dpg_export(ctx, D.X_COARSEST).reshape(n0, n0).T
    assert rel(T0, H.levels[0].T) <= elem_tol(p, omega, 1.0 / H.levels[0].N)
    x, it, rr, code = D.dpg_solve(ctx, tol=1e-12)
    xo, ito, _ = H.solve(rhs, 1e-12)
    assert code == D.DPG_OK
    assert np.linalg.norm(x[0] - xo) <= 1e-10 * np.linalg.norm(xo)
    assert abs(int(it[0]) - ito) <= 1
    for tol in (1e-8, 1e-10):
        _, it, _, _ = D.dpg_solve(ctx, tol=tol)
        _, ito, _ = H.solve(rhs, tol)
        assert abs(int(it[0]) - ito) <= 1, (tol, it[0], ito)
    ctx.close()


def test_restrict_needs_fewer_iterations_than_store_at_high_frequency():
    """Sec. 4.2: with stored coarse operators the iteration count grows with
    omega much faster than with restriction.  8^3, p = 2, V(2,2), tol 1e-8."""
    D = _D()
    d = np.array([2.0, -1.0, 2.0]) / 3.0
    its = {}
    for omega in (2 * np.pi, 8 * np.pi):
        for name, flags in (("restrict", 0), ("store", D.DPG_STORE_COARSE)):
            opt = D.dpg_default_options(nu_pre=2, nu_post=2, flags=flags)
            ctx = D.dpg_setup(8, 2, omega, [dict(dir=d, amp=1.0)], options=opt)
            D.dpg_assemble(ctx)
            D.dpg_build_hierarchy(ctx)
            _, it, _, code = D.dpg_solve(ctx, tol=1e-8)
            assert code == D.DPG_OK
            its[name, omega] = int(it[0])
            ctx.close()
    lo, hi = 2 * np.pi, 8 * np.pi
    assert its["restrict", lo] <= its["store", lo]
    assert its["restrict", hi] < its["store", hi]
    assert its["store", hi] - its["restrict", hi] > its["store", lo] - its["restrict", lo], its


def test_store_rejects_wave_speed_varying_inside_a_coarse_element():
    D = _D()
    c = np.ones(64)
    c[1] = 2.0                          # element (1, 0, 0): shares a coarse cell with (0, 0, 0)
    opt = D.dpg_default_options(flags=D.DPG_STORE_COARSE)
    with pytest.raises(D.DPGError) as e:
        D.dpg_setup(4, 2, 2 * np.pi, [dict(dir=(1, 0, 0), amp=1.0)], c=c, options=opt)
    assert e.value.code == D.DPG_EINVAL
    # layers aligned with every coarse mesh are accepted
    c = np.repeat([1.0, 2.0], 32)       # z < 1/2 and z > 1/2
    ctx = D.dpg_setup(4, 2, 2 * np.pi, [dict(dir=(1, 0, 0), amp=1.0)], c=c, options=opt)
    ctx.close()


def test_store_mixed_precision_block_solve_matches_oracle():
    """Stored coarse operators with the FP32 V-cycle and three right-hand
    sides in one block solve: each column within 1e-8 of the oracle's store
    hierarchy solution (tol 1e-10), iterations within 2."""
    D = _D()
    N, p, omega, nu = 8, 2, 4 * np.pi, (2, 2)
    d = workloads.plane_wave_direction(5)
    opt = D.dpg_default_options(nu_pre=nu[0], nu_post=nu[1], flags=D.DPG_STORE_COARSE,
                                precision=D.DPG_MIXED)
    print(f"[store mixed block] N={N} p={p}", flush=True)
    ctx = D.dpg_setup(N, p, omega, [dict(dir=d, amp=1.0)], options=opt)
    try:
        D.dpg_assemble(ctx)
        D.dpg_build_hierarchy(ctx)
        pr = dpg.Problem(N, p, omega, [dict(u0=dpg.plane_wave_u0(omega, d))])
        S, s, _ = pr.condensed()
        rhs = dpg.assemble_vector(pr.edofs, s, pr.num.n)[:, 0]
        H = multigrid.Hierarchy(N, p, S, nu_pre=nu[0], nu_post=nu[1], coarse=_store(p, omega))
        rng = np.random.default_rng(3)
        n = rhs.shape[0]
        B = np.stack([rhs, rng.standard_normal(n) + 1j * rng.standard_normal(n), (1 + 1j) * rhs])
        x, it, rr, code = D.dpg_solve(ctx, rhs=B, nrhs=3, tol=1e-10)
        assert code == D.DPG_OK
        for k in range(3):
            xo, _, _ = H.solve(B[k], 1e-12)
            _, ito, _ = H.solve(B[k], 1e-10)
            assert np.linalg.norm(x[k] - xo) <= 1e-8 * np.linalg.norm(xo), k
            assert abs(int(it[k]) - ito) <= 2, (k, it[k], ito)
    finally:
        ctx.close()
