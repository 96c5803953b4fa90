"""Parity at the full sizes of the benchmark workloads, in the configuration
bench.py times (the oracle cannot solve these meshes, so it is checked on
what it can compute one element at a time, and the solve by a property that
holds at any size):

- 32^3, p = 4, omega = 16 pi, V(2,2), mixed precision (2,785,665 trace
  unknowns, five levels): finest-level topology bit-exact against the
  oracle (element dofs, macro unknowns, vertex patches); condensed element
  matrices and loads of a corner, edge, face and interior element within
  cond(G) u of the oracle's; the solution's true residual in the FP64 trace
  system assembled here from the element matrices (host NumPy, not the
  library's apply): at most 10 x the solver tolerance relative to the load
  (the solver stops on the macro-grid residual relative to the condensed
  load, whose norm differs from the full load's by a factor of order one);
- 24^3, p = 3, omega = 12 pi, 32 Gaussian point sources of width 0.02, one
  block solve in mixed precision: element loads of the elements holding a
  source against the oracle's, and every column's true residual likewise.
"""
import numpy as np
import pytest

from oracle import dpg, topology
from paper_2304_01728_amd import workloads

from test_gpu_parity import elem_tol, rel

pytestmark = pytest.mark.gpu


def _D():
    from paper_2304_01728_amd import dpgmg as D
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return D


def _ctx(D, w, loads):
    opt = D.dpg_default_options(nu_pre=w.nu_pre, nu_post=w.nu_post, theta=w.theta,
                                precision=D.DPG_MIXED if w.precision == "mixed" else D.DPG_FP64)
    print(f"[full size] {w.name}", flush=True)
    ctx = D.dpg_setup(w.N, w.p, w.omega, loads, dp=w.dp, options=opt)
    D.dpg_assemble(ctx)
    D.dpg_build_hierarchy(ctx)
    return ctx


def _residuals(S, edofs, rhs, x):
    """||s - T x|| / ||s|| per column, T = sum_e R_e^T S_e R_e from the
    exported element matrices (S[e] column-major: S[e][i, j] = (S_e)_ji)."""
    n = rhs.shape[1]
    ok = edofs >= 0
    idx = np.where(ok, edofs, 0)
    out = []
    for k in range(rhs.shape[0]):
        xe = np.where(ok, x[k][idx], 0)
        ye = np.matmul(xe[:, None, :], S)[:, 0, :]
        ye = np.where(ok, ye, 0)
        y = (np.bincount(idx.ravel(), ye.real.ravel(), minlength=n)
             + 1j * np.bincount(idx.ravel(), ye.imag.ravel(), minlength=n))
        out.append(np.linalg.norm(rhs[k] - y) / np.linalg.norm(rhs[k]))
    return np.array(out)


def test_mixed_32_p4_full_size():
    D = _D()
    w = workloads.plane_wave_32_mixed()
    ctx = _ctx(D, w, [dict(dir=w.direction, amp=1.0)])
    info = D.dpg_info(ctx)
    N = w.N
    pr = dpg.Problem(N, w.p, w.omega, [dict(u0=dpg.plane_wave_u0(w.omega, w.direction))])
    assert info.n_trace == pr.num.n and info.n_tr == pr.n_tr
    # finest-level topology
    ed = topology.element_dofs(pr.num)
    edg = D.dpg_export(ctx, D.X_ELEM_DOFS, 0).reshape(ed.shape)
    assert np.array_equal(edg, ed)
    mc = topology.MacroLevel(pr.num)
    assert np.array_equal(D.dpg_export(ctx, D.X_MACRO_B, 0), mc.B)
    pt = D.dpg_export(ctx, D.X_PATCHES, 0)
    npch = len(mc.patches)
    assert np.array_equal(pt[:npch + 1], np.cumsum([0] + [len(q) for q in mc.patches]))
    assert np.array_equal(pt[npch + 1:], np.concatenate(mc.patches))
    del mc, pt
    # element matrices and loads of a corner, an edge, a face and an interior element
    sample = [0, 5, 5 + N * 7, 5 + N * (7 + N * 9), N ** 3 - 1]
    So, so, _ = pr.condensed(elements=sample)
    Sg = D.dpg_export(ctx, D.X_ELEM_S).reshape(pr.nel, pr.n_tr, pr.n_tr)
    sg = D.dpg_export(ctx, D.X_ELEM_RHS).reshape(pr.nel, pr.n_tr)
    tol = elem_tol(w.p, w.omega, 1.0 / N)
    for e in sample:
        assert rel(Sg[e].T, So[e]) <= tol, e
        assert rel(sg[e], so[e][:, 0]) <= tol, e
    del So, so, sg
    # true residual of the FP64 trace system at the workload's tolerance and at 1e-10
    rhs = D.dpg_export(ctx, D.X_ASM_RHS).reshape(1, -1)
    for tol_s in (w.tol, 1e-10):
        x, it, rr, code = D.dpg_solve(ctx, tol=tol_s)
        assert code == D.DPG_OK and rr[0] <= tol_s
        res = _residuals(Sg, edg, rhs, x)
        print(f"[full size] tol {tol_s:g}: {int(it[0])} iterations, true residual {res[0]:.3e}",
              flush=True)
        assert res[0] <= 10 * tol_s
    ctx.close()


def test_point_sources_24_block_full_size():
    D = _D()
    w = workloads.point_sources_24()
    loads = [dict(dir=(0.0, 0.0, 1.0), amp=0.0, sources=[[*c, w.sigma, 1.0, 0.0]])
             for c in w.sources]
    ctx = _ctx(D, w, loads)
    N = w.N
    # the elements holding the first four sources, and a corner element
    hold = [int(c[0] * N) + N * (int(c[1] * N) + N * int(c[2] * N)) for c in w.sources[:4]]
    sample = sorted(set(hold + [0]))
    pr = dpg.Problem(N, w.p, w.omega,
                     [dict(f=dpg.gaussian_sources([c], w.sigma, [1.0])) for c in w.sources])
    So, so, _ = pr.condensed(elements=sample)
    Sg = D.dpg_export(ctx, D.X_ELEM_S).reshape(pr.nel, pr.n_tr, pr.n_tr)
    sg = D.dpg_export(ctx, D.X_ELEM_RHS).reshape(w.nrhs, pr.nel, pr.n_tr)
    tol = elem_tol(w.p, w.omega, 1.0 / N)
    for e in sample:
        assert rel(Sg[e].T, So[e]) <= tol, e
        assert rel(sg[:, e, :], so[e].T) <= tol, e
    for k, e in enumerate(hold):   # each source's own element carries its load
        assert np.abs(sg[k, e]).max() > 0.0
    del So, so, sg
    x, it, rr, code = D.dpg_solve(ctx, nrhs=w.nrhs, tol=w.tol)
    assert code == D.DPG_OK and np.all(rr <= w.tol)
    rhs = D.dpg_export(ctx, D.X_ASM_RHS).reshape(w.nrhs, -1)
    edg = D.dpg_export(ctx, D.X_ELEM_DOFS, 0).reshape(pr.nel, pr.n_tr)
    res = _residuals(Sg, edg, rhs, x)
    print(f"[full size] 32 columns: iterations {int(it.min())}-{int(it.max())}, true residuals "
          f"{res.min():.3e}-{res.max():.3e}", flush=True)
    assert np.all(res <= 10 * w.tol)
    ctx.close()
