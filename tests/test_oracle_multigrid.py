"""Pins of the oracle's DPG-MG solver (Sec. 3) against direct solves and
spectral properties."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import dpg, multigrid, topology


def _problem(N, p, omega, seed):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    pr = dpg.Problem(N, p, omega, [dict(u0=dpg.plane_wave_u0(omega, d))])
    S, s, _ = pr.condensed()
    T = dpg.assemble(pr.edofs, S, pr.num.n)
    rhs = dpg.assemble_vector(pr.edofs, s, pr.num.n)[:, 0]
    return pr, S, T, rhs


@pytest.fixture(scope="module")
def two_level():
    pr, S, T, rhs = _problem(4, 2, 2 * np.pi, 0)
    return pr, S, T, rhs, multigrid.Hierarchy(4, 2, S)


@pytest.fixture(scope="module")
def three_level():
    pr, S, T, rhs = _problem(8, 1, 2 * np.pi, 1)
    return pr, S, T, rhs, multigrid.Hierarchy(8, 1, S, nu_pre=2, nu_post=2)


def test_level_sizes():
    assert multigrid.level_sizes(4) == [4, 2]
    assert multigrid.level_sizes(16) == [16, 8, 4, 2]
    assert multigrid.level_sizes(32) == [32, 16, 8, 4, 2]
    assert multigrid.level_sizes(24) == [24, 12, 6, 3]
    assert multigrid.level_sizes(2) == [2, 1]
    assert multigrid.level_sizes(3) == [3]


@pytest.mark.parametrize("fx", ["two_level", "three_level"])
def test_macro_condensation_is_exact(fx, request):
    pr, S, T, rhs, H = request.getfixturevalue(fx)
    lv = H.levels[H.L]
    xd = spla.spsolve(T.tocsc(), rhs)
    xB = spla.spsolve(lv.M.tocsc(), H.condense_rhs(lv, rhs))
    assert np.linalg.norm(H.expand(lv, rhs, xB) - xd) <= 1e-11 * np.linalg.norm(xd)


@pytest.mark.parametrize("fx", ["two_level", "three_level"])
def test_galerkin_elementwise_equals_bruteforce_triple_product(fx, request):
    _, _, _, _, H = request.getfixturevalue(fx)
    for l in range(1, H.L + 1):
        lv, lc = H.levels[l], H.levels[l - 1]
        P = lv.P.toarray()
        brute = P.T @ lv.M.toarray() @ P
        elementwise = dpg.assemble(lc.edofs, lc.E, lc.n).toarray()
        assert np.abs(brute - elementwise).max() <= 1e-13 * np.abs(brute).max()


def _vcycle_matrix(H):
    n = H.levels[H.L].macro.nM
    V = np.zeros((n, n), dtype=complex)
    for i in range(n):
        e = np.zeros(n, dtype=complex)
        e[i] = 1.0
        V[:, i] = H.vcycle(H.L, e)
    return V


def test_vcycle_hermitian_positive_definite(two_level):
    _, _, _, _, H = two_level
    V = _vcycle_matrix(H)
    assert np.abs(V - V.conj().T).max() <= 1e-12 * np.abs(V).max()
    M = H.levels[H.L].M.toarray()
    ev = np.linalg.eigvals(V @ M).real
    assert ev.min() > 0.3 and ev.max() < 1.0 + 1e-10


def test_eight_colour_bound_attained_so_quarter_damping_is_singular(two_level):
    """lambda_max(S M) = 8 exactly: Gamma-face unknowns of a boundary coarse cell
    lie in all 8 patches around it.  With theta = 1/4 the smoother flips them
    (I - theta S M = -I there), and the V-cycle becomes singular."""
    pr, S, _, _, H = two_level
    lv = H.levels[H.L]
    n = lv.macro.nM
    SM = np.zeros((n, n), dtype=complex)
    for idx, Si in zip(lv.macro.patches, lv.Sinv):
        SM[np.ix_(idx, idx)] += Si
    lam = np.linalg.eigvals(SM @ lv.M.toarray()).real
    assert abs(lam.max() - 8.0) < 1e-9
    Hq = multigrid.Hierarchy(4, 2, S, theta=0.25)
    ev = np.linalg.eigvals(_vcycle_matrix(Hq) @ lv.M.toarray()).real
    assert ev.min() < 1e-10


@pytest.mark.parametrize("fx", ["two_level", "three_level"])
def test_pcg_matches_direct_solve(fx, request):
    pr, S, T, rhs, H = request.getfixturevalue(fx)
    xd = spla.spsolve(T.tocsc(), rhs)
    x, it, rr = H.solve(rhs, 1e-12)
    assert rr <= 1e-12
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    assert 0 < it < 40


def test_pcg_zero_rhs_and_iteration_cap(two_level):
    _, _, _, rhs, H = two_level
    x, it, rr = H.solve(np.zeros_like(rhs), 1e-8)
    assert it == 0 and np.all(x == 0)
    x, it, rr = H.solve(rhs, 0.0, maxit=3)
    assert it == 3 and rr > 0
