"""Kernel statistics of the setup: with profiling on, the setup runs on one
stream and every dense kernel is timed under its own symbol with its share
of the routine's LAPACK flop count.  The results must not change: the same
kernels on the same data, only the streams differ, so the hierarchy and the
solution agree bitwise with an unprofiled setup, and the per-kernel flop
shares add up to the routine counts."""
import numpy as np
import pytest

from paper_2304_01728_amd import workloads

pytestmark = pytest.mark.gpu


def test_profiled_setup_is_bitwise_equal_and_splits_the_flops():
    from paper_2304_01728_amd import dpgmg as D
    import torch
    assert torch.cuda.is_available()
    N, p, omega = 8, 3, 4 * np.pi
    d = workloads.plane_wave_direction(3)
    opt = D.dpg_default_options(nu_pre=2, nu_post=2)
    out = []
    for prof in (False, True):
        print(f"[profile] N={N} p={p} profiled setup={prof}", flush=True)
        ctx = D.dpg_setup(N, p, omega, [dict(dir=d, amp=1.0)], options=opt)
        if prof:
            D.dpg_profile(ctx, True)
        D.dpg_assemble(ctx)
        D.dpg_build_hierarchy(ctx)
        stats = D.dpg_kernel_stats(ctx) if prof else None
        if prof:
            D.dpg_profile(ctx, False)
        x, it, rr, code = D.dpg_solve(ctx, tol=1e-10)
        assert code == D.DPG_OK
        pinv = D.dpg_export(ctx, D.X_PATCH_INV, 0)
        out.append((x, int(it[0]), pinv, stats))
        ctx.close()
    (x0, it0, p0, _), (x1, it1, p1, st) = out
    assert it0 == it1 and np.array_equal(x0, x1) and np.array_equal(p0, p1)
    for name in ("potrf_diag", "potrf_panel", "potrf_update", "trsm_solve", "trsm_update", "gemm"):
        assert st[name][0] > 0 and st[name][1] > 0 and st[name][2] > 0, name
    # the blocked algorithm's steps add up to the LAPACK counts up to terms of
    # lower order (orders 108 to 1160 here)
    potrf = sum(st[k][2] for k in ("potrf_diag", "potrf_panel", "potrf_update"))
    trsm = sum(st[k][2] for k in ("trsm_solve", "trsm_update"))
    assert abs(potrf / st["potrf"][2] - 1) < 0.05, (potrf, st["potrf"][2])
    assert abs(trsm / st["trsm"][2] - 1) < 0.05, (trsm, st["trsm"][2])
