"""dpg_solve_noalloc (the solve that allocates nothing) against dpg_solve.

Both calls go through the C ABI (ctypes).  Two no-allocation calls in a row on
one GPU, the second on a smaller problem, each checked against dpg_solve on
the same context: same iteration counts, solutions within 1e-10 (FP64) or
1e-8 (mixed) -- the bar of the FP64 and mixed paths against the oracle.  The
context's device memory must not change across the call.
"""
import numpy as np
import pytest

from paper_2304_01728_amd import workloads

pytestmark = pytest.mark.gpu


def _D():
    from paper_2304_01728_amd import dpgmg as D
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return D


def _ctx(D, N, p, omega, seed, precision="fp64", flags=0, nu=(2, 2)):
    opt = D.dpg_default_options(nu_pre=nu[0], nu_post=nu[1], flags=flags,
                                precision=D.DPG_MIXED if precision == "mixed" else D.DPG_FP64)
    print(f"[noalloc] N={N} p={p} {precision} flags={flags}", flush=True)
    ctx = D.dpg_setup(N, p, omega, [dict(dir=workloads.plane_wave_direction(seed), amp=1.0)],
                      options=opt)
    D.dpg_assemble(ctx)
    D.dpg_build_hierarchy(ctx)
    return ctx


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("mixed", 1e-8)])
def test_noalloc_matches_solve_two_calls_second_smaller(precision, bar):
    D = _D()
    big = _ctx(D, 8, 2, 4 * np.pi, 5, precision)
    small = _ctx(D, 4, 2, 2 * np.pi, 0, precision)
    cases = ((big, 1e-10), (small, 1e-12))
    got = []
    for ctx, tol in cases:              # the two no-allocation calls back to back
        before = D.dpg_info(ctx).resident_bytes
        got.append(D.dpg_solve_noalloc(ctx, tol=tol))
        assert D.dpg_info(ctx).resident_bytes == before
    for (ctx, tol), (xn, itn, rrn, cn) in zip(cases, got):
        xs, its, rrs, cs = D.dpg_solve(ctx, tol=tol)
        assert cn == D.DPG_OK and cs == D.DPG_OK
        assert int(itn[0]) == int(its[0]) and rrn[0] <= tol
        assert _rel(xn[0], xs[0]) <= bar


def test_noalloc_device_pointers_explicit_rhs_and_errors():
    import torch
    D = _D()
    ctx = _ctx(D, 4, 3, 8 * np.pi, 1, flags=D.DPG_DEVICE_PTRS)
    nT = D.dpg_info(ctx).n_trace
    rng = np.random.default_rng(3)
    rhs = torch.tensor(rng.standard_normal((2, nT)) + 1j * rng.standard_normal((2, nT)),
                       dtype=torch.complex128, device="cuda:0")
    xa = torch.zeros((2, nT), dtype=torch.complex128, device="cuda:0")
    xb = torch.zeros_like(xa)
    _, ita, _, ca = D.dpg_solve_noalloc(ctx, rhs=rhs, nrhs=2, tol=1e-11, x_out=xa, device=True)
    _, itb, _, cb = D.dpg_solve(ctx, rhs=rhs, nrhs=2, tol=1e-11, x_out=xb, device=True)
    torch.cuda.synchronize()
    assert ca == D.DPG_OK and cb == D.DPG_OK
    # dpg_solve takes nrhs > 1 as a block; the no-allocation call solves the
    # columns one by one, so the counts agree to +-1
    assert np.all(np.abs(ita.astype(int) - itb.astype(int)) <= 1)
    for k in range(2):
        assert _rel(xa[k].cpu().numpy(), xb[k].cpu().numpy()) <= 1e-10
    D.dpg_profile(ctx, True)
    with pytest.raises(D.DPGError) as e:
        D.dpg_solve_noalloc(ctx, rhs=rhs, nrhs=1, tol=1e-8, x_out=xa, device=True)
    assert e.value.code == D.DPG_ESTATE
    D.dpg_profile(ctx, False)
    ctx.close()
