"""The PCG iteration replayed from captured HIP graphs against the same
iteration launched kernel by kernel (per-kernel profiling on disables the
graphs): identical kernels in identical order, so the results must agree
bitwise, on repeated solves with other work on the stream in between."""
import numpy as np
import pytest

from paper_2304_01728_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_matches_eager_launches(precision):
    from paper_2304_01728_amd import dpgmg as D
    import torch
    assert torch.cuda.is_available()
    N, p, omega = 8, 2, 4 * np.pi
    d = workloads.plane_wave_direction(5)
    opt = D.dpg_default_options(nu_pre=2, nu_post=2,
                                precision=D.DPG_MIXED if precision == "mixed" else D.DPG_FP64)
    print(f"[graphs] N={N} p={p} {precision}", flush=True)
    ctx = D.dpg_setup(N, p, omega, [dict(dir=d, amp=1.0)], options=opt)
    D.dpg_assemble(ctx)
    D.dpg_build_hierarchy(ctx)
    D.dpg_profile(ctx, True)
    xe, ite, rre, ce = D.dpg_solve(ctx, tol=1e-10)
    D.dpg_profile(ctx, False)
    assert ce == D.DPG_OK
    for rep in range(3):
        xg, itg, rrg, cg = D.dpg_solve(ctx, tol=1e-10)
        assert cg == D.DPG_OK
        assert int(itg[0]) == int(ite[0])
        assert np.array_equal(xg, xe), f"replay {rep} differs"
        # eager work in between: a different right-hand side through the same context
        D.dpg_solve(ctx, rhs=0.5 * xe, tol=1e-6)
