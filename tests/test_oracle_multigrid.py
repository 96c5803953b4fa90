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


# ---- order levels (Sec. 4.2, uniform p-refinements read as multigrid levels) -------------------

from oracle import basis1d, element  # noqa: E402


def _trace_values(num, x, e, d, s, pts):
    """The H1 trace and the flux trace given by the coefficient vector x on
    face (axis d, side s) of element e, at reference points pts [n, 2] of the
    face (first in-plane axis first), evaluated from the shape functions."""
    N, q = num.N, num.p
    ed = topology.element_dofs(num)[e]
    lat = element.h1_boundary_lattice(q)
    ip = [a for a in range(3) if a != d]
    xi = np.zeros((len(pts), 3))
    xi[:, d] = 1.0 if s else -1.0
    xi[:, ip[0]], xi[:, ip[1]] = pts[:, 0], pts[:, 1]
    H = [basis1d.h1(q, xi[:, a]) for a in range(3)]
    ph = np.zeros(len(pts), dtype=complex)
    for k, (a, b, c) in enumerate(lat):
        ph += x[ed[k]] * H[0][a] * H[1][b] * H[2][c]
    un = np.zeros(len(pts), dtype=complex)
    c0 = len(lat) + (2 * d + s) * q * q
    if ed[c0] >= 0:
        Lm = basis1d.legendre(q, pts[:, 0])
        Ln = basis1d.legendre(q, pts[:, 1])
        for n in range(q):
            for m in range(q):
                un += x[ed[c0 + n * q + m]] * Lm[m] * Ln[n]
    return ph, un


@pytest.mark.parametrize("N,q", [(2, 2), (2, 3), (3, 4)])
def test_order_injection_reproduces_lower_order_traces(N, q):
    """P x is the order-q coefficient vector of the same trace functions as the
    order-(q-1) vector x: pressure and flux traces agree at random points of
    every face of every element."""
    fine, coarse = topology.Numbering(N, q), topology.Numbering(N, q - 1)
    P = topology.order_injection(fine, coarse)
    assert P.shape == (fine.n, coarse.n) and np.all(P.sum(axis=0) == 1)
    rng = np.random.default_rng(N + 10 * q)
    xc = rng.standard_normal(coarse.n) + 1j * rng.standard_normal(coarse.n)
    xf = P @ xc
    pts = rng.uniform(-1, 1, size=(7, 2))
    for e in range(N ** 3):
        for d in range(3):
            for s in range(2):
                pc, uc = _trace_values(coarse, xc, e, d, s, pts)
                pf, uf = _trace_values(fine, xf, e, d, s, pts)
                assert np.abs(pf - pc).max() <= 1e-12 * np.abs(pc).max()
                assert np.abs(uf - uc).max() <= 1e-12 * max(np.abs(uc).max(), 1.0)


def test_order_level_patches_by_definition():
    """Unknown t is in the patch of vertex v iff every element holding t
    contains v (the support rule, with the elements as the cells)."""
    N, q = 3, 2
    num = topology.Numbering(N, q)
    ol = topology.OrderLevel(num)
    ed = topology.element_dofs(num)
    holders = [set() for _ in range(num.n)]
    for e in range(N ** 3):
        for t in ed[e][ed[e] >= 0]:
            holders[t].add(e)
    for vz in range(N + 1):
        for vy in range(N + 1):
            for vx in range(N + 1):
                around = {(vx - 1 + a) + N * ((vy - 1 + b) + N * (vz - 1 + c))
                          for c in range(2) for b in range(2) for a in range(2)
                          if 0 <= vx - 1 + a < N and 0 <= vy - 1 + b < N and 0 <= vz - 1 + c < N}
                want = [t for t in range(num.n) if holders[t] <= around]
                got = ol.patches[(vz * (N + 1) + vy) * (N + 1) + vx]
                assert list(got) == want


@pytest.fixture(scope="module")
def order_levels():
    N, p = 2, 3
    pr = dpg.Problem(N, p, 2 * np.pi, [dict(u0=dpg.plane_wave_u0(2 * np.pi, [0.6, 0.0, 0.8]))])
    S, s, _ = pr.condensed()
    T = dpg.assemble(pr.edofs, S, pr.num.n)
    rhs = dpg.assemble_vector(pr.edofs, s, pr.num.n)[:, 0]
    return pr, S, T, rhs, multigrid.Hierarchy(N, p, S, nu_pre=2, nu_post=2, p_min=2)


def test_order_levels_galerkin_vcycle_and_pcg(order_levels):
    pr, S, T, rhs, H = order_levels
    assert H.plan == [(2, 3), (2, 2), (1, 2)]
    lv, lc = H.levels[H.L], H.levels[H.L - 1]
    assert lv.order_level and not lc.order_level
    P = lv.P.toarray()
    brute = P.T @ lv.M.toarray() @ P
    assert np.abs(brute - dpg.assemble(lc.edofs, lc.E, lc.n).toarray()).max() <= \
        1e-13 * np.abs(brute).max()
    assert np.abs(lv.M.toarray() - T.toarray()).max() <= 1e-14 * np.abs(T).max()
    V = _vcycle_matrix(H)
    assert np.abs(V - V.conj().T).max() <= 1e-12 * np.abs(V).max()
    ev = np.linalg.eigvals(V @ lv.M.toarray()).real
    assert ev.min() > 0 and ev.max() < 1.0 + 1e-10
    xd = spla.spsolve(T.tocsc(), rhs)
    x, it, rr = H.solve(rhs, 1e-12)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
