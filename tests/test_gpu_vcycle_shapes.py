"""Single-column solves with V-cycles of other shapes than V(2,2): no
pre-smoothing, no post-smoothing, uneven counts (Sec. 3, "V-cycle and
smoother").  Each shape takes a different chain of residual and smoother
applications on every level, and so a different chain of applications whose
local vectors are filled by the scatter of the application before them.

Bar: FP64 within 1e-10 of the oracle's solution (tol 1e-12) with iteration
counts +-1; mixed precision (tol 1e-10) within 1e-8 of the FP64 oracle, its
iteration count within 2 of the oracle's at that tolerance.  The block path
(three explicit right-hand sides in one solve, the same chains on block
buffers) is held to the same bar column by column.
"""
import numpy as np
import pytest

from oracle import dpg, multigrid
from paper_2304_01728_amd import workloads

pytestmark = pytest.mark.gpu

N, P, OMEGA, SEED = 8, 2, 4 * np.pi, 2


def _D():
    from paper_2304_01728_amd import dpgmg as D
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return D


@pytest.fixture(scope="module")
def problem():
    d = workloads.plane_wave_direction(SEED)
    pr = dpg.Problem(N, P, OMEGA, [dict(u0=dpg.plane_wave_u0(OMEGA, d))])
    S, s, _ = pr.condensed()
    rhs = dpg.assemble_vector(pr.edofs, s, pr.num.n)[:, 0]
    return d, S, rhs, {}


def _hierarchy(problem, nu):
    """The oracle's hierarchy for V(nu) and its solutions so far (cached)."""
    _, S, _, cache = problem
    if nu not in cache:
        cache[nu] = (multigrid.Hierarchy(N, P, S, nu_pre=nu[0], nu_post=nu[1]), {})
    return cache[nu]


def _oracle(problem, nu, tol):
    """The oracle's solution and iteration count for V(nu) at tol (cached)."""
    rhs = problem[2]
    H, sols = _hierarchy(problem, nu)
    if tol not in sols:
        sols[tol] = H.solve(rhs, tol)
    return sols[tol]


@pytest.mark.parametrize("nu,precision", [((1, 3), "fp64"), ((0, 1), "fp64"), ((3, 0), "fp64"),
                                          ((0, 1), "mixed"), ((1, 3), "mixed")])
def test_vcycle_shape_matches_oracle(problem, nu, precision):
    D = _D()
    d = problem[0]
    opt = D.dpg_default_options(nu_pre=nu[0], nu_post=nu[1],
                                precision=D.DPG_MIXED if precision == "mixed" else D.DPG_FP64)
    print(f"[vcycle] N={N} p={P} nu={nu} {precision}", flush=True)
    ctx = D.dpg_setup(N, P, OMEGA, [dict(dir=d, amp=1.0)], options=opt)
    try:
        D.dpg_assemble(ctx)
        D.dpg_build_hierarchy(ctx)
        xo, _, _ = _oracle(problem, nu, 1e-12)
        if precision == "fp64":
            x, it, rr, code = D.dpg_solve(ctx, tol=1e-12)
            ito = _oracle(problem, nu, 1e-12)[1]
            assert code == D.DPG_OK and rr[0] <= 1e-12
            assert np.linalg.norm(x[0] - xo) <= 1e-10 * np.linalg.norm(xo)
            assert abs(int(it[0]) - ito) <= 1, (it[0], ito)
        else:
            x, it, rr, code = D.dpg_solve(ctx, tol=1e-10)
            ito = _oracle(problem, nu, 1e-10)[1]
            assert code == D.DPG_OK
            assert np.linalg.norm(x[0] - xo) <= 1e-8 * np.linalg.norm(xo)
            assert abs(int(it[0]) - ito) <= 2, (it[0], ito)
    finally:
        ctx.close()


@pytest.mark.parametrize("nu,precision", [((1, 3), "fp64"), ((0, 1), "mixed"), ((3, 0), "fp64"),
                                          ((1, 3), "mixed")])
def test_block_vcycle_shape_matches_oracle(problem, nu, precision):
    D = _D()
    d, _, rhs, _ = problem
    opt = D.dpg_default_options(nu_pre=nu[0], nu_post=nu[1],
                                precision=D.DPG_MIXED if precision == "mixed" else D.DPG_FP64)
    print(f"[vcycle block] N={N} p={P} nu={nu} {precision}", flush=True)
    ctx = D.dpg_setup(N, P, OMEGA, [dict(dir=d, amp=1.0)], options=opt)
    try:
        D.dpg_assemble(ctx)
        D.dpg_build_hierarchy(ctx)
        rng = np.random.default_rng(17)
        n = rhs.shape[0]
        B = np.stack([rhs, (rng.standard_normal(n) + 1j * rng.standard_normal(n)),
                      (0.5 - 2j) * rhs + (rng.standard_normal(n) + 1j * rng.standard_normal(n))])
        H = _hierarchy(problem, nu)[0]
        tol, bar = (1e-12, 1e-10) if precision == "fp64" else (1e-10, 1e-8)
        x, it, rr, code = D.dpg_solve(ctx, rhs=B, nrhs=3, tol=tol)
        assert code == D.DPG_OK
        for k in range(3):
            xo, _, _ = H.solve(B[k], 1e-12)
            _, ito, _ = H.solve(B[k], tol)
            assert np.linalg.norm(x[k] - xo) <= bar * np.linalg.norm(xo), k
            assert abs(int(it[k]) - ito) <= (1 if precision == "fp64" else 2), (k, it[k], ito)
    finally:
        ctx.close()
