"""The highest orders the library takes (p + dp <= 7: element tables of eight
1-D functions, load quadrature of twelve points): p = 5 on a 4^3 mesh with two
levels and p = 6 on a 2^3 mesh, against the oracle -- element matrices within
cond(G) u, hierarchy matrices within 1e-12 (patch inverses 1e-11), the
solution within 1e-10 at tol 1e-12 and iteration counts +-1."""
import numpy as np
import pytest

from test_gpu_parity import Case, _levels, elem_tol, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,p,seed", [(4, 5, 7), (2, 6, 8)])
def test_highest_orders_match_oracle(N, p, seed):
    omega = 2 * np.pi * N / 4          # four elements per wavelength
    c = Case(N, p, omega, seed, nu=(2, 2))
    D = c.D
    n_tr = c.pr.n_tr
    tol = elem_tol(p, omega, 1.0 / N)
    S = D.dpg_export(c.ctx, D.X_ELEM_S).reshape(c.pr.nel, n_tr, n_tr).transpose(0, 2, 1)
    assert rel(S, c.S) <= tol
    s = D.dpg_export(c.ctx, D.X_ELEM_RHS).reshape(c.pr.nel, n_tr)
    assert rel(s, c.s[:, :, 0]) <= tol
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
    x, it, rr, code = D.dpg_solve(c.ctx, tol=1e-12)
    xo, ito, _ = c.H.solve(c.rhs, 1e-12)
    assert code == D.DPG_OK
    assert np.linalg.norm(x[0] - xo) <= 1e-10 * np.linalg.norm(xo)
    assert abs(int(it[0]) - ito) <= 1
    c.ctx.close()


def test_order_beyond_the_tables_is_rejected():
    from paper_2304_01728_amd import dpgmg as D
    import torch
    assert torch.cuda.is_available()
    with pytest.raises(D.DPGError) as e:
        D.dpg_setup(2, 7, 2 * np.pi, [dict(dir=(1.0, 0.0, 0.0), amp=1.0)])
    assert e.value.code == D.DPG_EINVAL
