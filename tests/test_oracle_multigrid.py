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


# ---- "store" coarse operators (Sec. 3, alternative construction; Sec. 4.2) ----------------------

def _store(p, omega):
    return lambda n: dpg.Problem(n, p, omega, []).condensed_operator()


def test_store_coarse_operator_is_the_coarse_mesh_dpg_operator(two_level):
    """With store, the coarse operator is the DPG trace operator of the coarse
    mesh itself (the 2^3 problem's own condensed matrix): Hermitian positive
    definite, and different from the Galerkin operator P^T M P."""
    pr, S, _, rhs, H = two_level
    Hs = multigrid.Hierarchy(4, 2, S, coarse=_store(2, 2 * np.pi))
    Ts, Tr = Hs.levels[0].T, H.levels[0].T
    assert np.abs(Ts - Ts.conj().T).max() <= 1e-13 * np.abs(Ts).max()
    assert np.linalg.eigvalsh(Ts).min() > 0
    assert np.abs(Ts - Tr).max() > 1e-3 * np.abs(Tr).max()
    # the coarse mesh's own solve: the 2^3 problem of the same data
    pc = dpg.Problem(2, 2, 2 * np.pi, pr.loads)
    Sc, sc, _ = pc.condensed()
    assert np.abs(dpg.assemble(pc.edofs, Sc, pc.num.n).toarray() - Ts).max() <= \
        1e-13 * np.abs(Ts).max()


def test_store_vcycle_hermitian_positive_definite_and_pcg_exact(two_level):
    pr, S, T, rhs, H = two_level
    Hs = multigrid.Hierarchy(4, 2, S, coarse=_store(2, 2 * np.pi))
    V = _vcycle_matrix(Hs)
    assert np.abs(V - V.conj().T).max() <= 1e-12 * np.abs(V).max()
    assert np.linalg.eigvals(V @ Hs.levels[Hs.L].M.toarray()).real.min() > 0
    xd = spla.spsolve(T.tocsc(), rhs)
    x, it, rr = Hs.solve(rhs, 1e-12)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)


@pytest.mark.slow
def test_restrict_beats_store_and_the_gap_grows_with_frequency():
    """The paper's comparison (Sec. 4.2, uniform h-refinements): coarse
    operators by restriction need fewer PCG iterations than stored (directly
    assembled) ones, increasingly so as omega grows.  8^3, p = 2, V(2,2)."""
    d = np.array([2.0, -1.0, 2.0]) / 3.0
    gaps = []
    for omega in (2 * np.pi, 8 * np.pi):
        pr = dpg.Problem(8, 2, omega, [dict(u0=dpg.plane_wave_u0(omega, d))])
        S, s, _ = pr.condensed()
        rhs = dpg.assemble_vector(pr.edofs, s, pr.num.n)[:, 0]
        Hr = multigrid.Hierarchy(8, 2, S, nu_pre=2, nu_post=2)
        Hs = multigrid.Hierarchy(8, 2, S, nu_pre=2, nu_post=2, coarse=_store(2, omega))
        xr, itr, _ = Hr.solve(rhs, 1e-10)
        xs, its, _ = Hs.solve(rhs, 1e-10)
        assert np.linalg.norm(xr - xs) <= 1e-8 * np.linalg.norm(xr)
        assert itr < its
        gaps.append(its - itr)
    assert gaps[1] > gaps[0]
