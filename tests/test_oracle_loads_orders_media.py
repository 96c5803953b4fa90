"""More pins of the oracle: the point-source load, order 4, piecewise media,
and plane-wave h-convergence at orders 2 and 3.

* Gaussian point source (Sec. 5 source model; read as f in the first
  equation, a Gaussian of standard deviation sigma with unit mass times its
  amplitude): its mass, first and second moments by a spectrally accurate
  trapezoid rule on a fine grid, with no Gauss rule and none of the oracle's
  load code.  The load code itself is pinned separately: polynomial data
  integrated against the test functions equal exact integrals done by
  polynomial arithmetic, and the total mass of a source reaches the constant
  test functions.
* Order 4 (the 32^3 workload's order): the Kronecker route of the element
  matrices and exact polynomial reproduction.
* Piecewise constant wave speed and impedance (the layered media of the
  serving stream, Sec. 2 eq. helmholtz with c per element, Z = c): a global
  polynomial solution with element-wise data f = i w c_K^-2 p + div u and
  u0 = Z_K^-1 p - u.n is reproduced exactly.
* Plane waves at p = 2, 3 on N = 2, 4, 8: L2 field errors fall like h^p.
"""
import numpy as np
import pytest
from numpy.polynomial import Legendre

from oracle import dpg, element

from test_oracle_dpg import _monomial_field, _plane_wave_error, _solve, _element_points
from test_oracle_element import _kron_route, _block


# ---- the Gaussian source ---------------------------------------------------------------------

def _trapezoid_grid(c, sigma, half=9.0, per_sigma=4):
    """Tensor trapezoid rule on [c - half sigma, c + half sigma]^3."""
    n = int(2 * half * per_sigma) + 1
    ax = [np.linspace(c[d] - half * sigma, c[d] + half * sigma, n) for d in range(3)]
    hstep = ax[0][1] - ax[0][0]
    w1 = np.full(n, hstep)
    w1[0] = w1[-1] = 0.5 * hstep
    g = np.meshgrid(*ax, indexing='ij')
    X = np.stack([g[d].reshape(-1) for d in range(3)], axis=1)
    W = np.einsum('i,j,k->ijk', w1, w1, w1).reshape(-1)
    return X, W


@pytest.mark.parametrize("sigma,amp", [(0.02, 1.0 + 0.0j), (0.05, 0.7 - 1.3j)])
def test_gaussian_source_mass_and_moments(sigma, amp):
    c = np.array([0.31, 0.52, 0.68])
    f = dpg.gaussian_sources([c], sigma, [amp])
    X, W = _trapezoid_grid(c, sigma)
    fx = f(X)
    mass = W @ fx
    assert abs(mass - amp) <= 1e-10 * abs(amp)                      # unit mass x amplitude
    first = (W * fx) @ X
    assert np.abs(first - amp * c).max() <= 1e-10 * abs(amp)         # centred at x_s
    Y = X - c
    cov = (Y * (W * fx)[:, None]).T @ Y
    assert np.abs(cov - amp * sigma ** 2 * np.eye(3)).max() <= 1e-9 * abs(amp) * sigma ** 2


def test_gaussian_sources_superpose():
    cs = np.array([[0.3, 0.3, 0.3], [0.6, 0.5, 0.4]])
    amps = [1.0, -0.5 + 2.0j]
    f = dpg.gaussian_sources(cs, 0.04, amps)
    X = np.random.default_rng(1).uniform(0, 1, size=(500, 3))
    one = [dpg.gaussian_sources([c0], 0.04, [a])(X) for c0, a in zip(cs, amps)]
    assert np.abs(f(X) - one[0] - one[1]).max() <= 1e-14 * np.abs(f(X)).max()


def _leg_coef_poly(coef, p):
    """The monomial field sum c[a,b,c] x^a y^b z^c, as 1-D factors on the reference
    interval of an element [x0, x0 + h]: returns a function of (x0, h) that yields
    the list of separable terms (c, poly_x, poly_y, poly_z) in xi."""
    def terms(x0, h):
        out = []
        for a in range(p):
            for b in range(p):
                for cc in range(p):
                    ps = []
                    for d, e in enumerate((a, b, cc)):
                        # x = x0 + (xi + 1) h / 2
                        lin = Legendre([x0[d] + h / 2.0, h / 2.0])
                        ps.append(lin ** e if e else Legendre([1.0]))
                    out.append((coef[a, b, cc], ps))
        return out
    return terms


def test_element_load_of_polynomial_data_is_exact():
    """(f, q_i) for a polynomial f through the oracle's load quadrature equals
    the exact integral by polynomial arithmetic (pins the physical-point map,
    the weights and the test-function rows of the load code)."""
    p, h = 2, 0.25
    x0 = np.array([0.25, 0.5, 0.0])
    rng = np.random.default_rng(7)
    coef = rng.standard_normal((p, p, p)) + 1j * rng.standard_normal((p, p, p))
    f = lambda X: _monomial_field(coef, p, X)
    l = element.element_load(p, h, x0, f=f)
    P = p + 1
    Lt = [Legendre.basis(k) for k in range(P + 1)]
    ref = np.zeros((P + 1) ** 3, dtype=complex)
    for cf, ps in _leg_coef_poly(coef, p)(x0, h):
        I = []
        for d in range(3):
            row = []
            for q in Lt:
                F = (q * ps[d]).integ()
                row.append((F(1.0) - F(-1.0)) * h / 2.0)
            I.append(np.array(row))
        ref += cf * np.kron(I[2], np.kron(I[1], I[0]))
    nq = (P + 1) ** 3
    assert np.abs(l[:nq] - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.all(l[nq:] == 0)                              # f pairs with q only


def test_gaussian_source_load_total_mass():
    """The constant test function of every element (Legendre degree 0 in q)
    collects (f, 1) over the element; summed over the mesh that is the source's
    mass times its amplitude when the source is well inside the cube."""
    N, p = 4, 3
    amp = 0.8 + 0.6j
    pr = dpg.Problem(N, p, 5.0, [dict(f=dpg.gaussian_sources([[0.45, 0.55, 0.5]], 0.07, [amp]))])
    tot = sum(pr.element_load(e)[0, 0] for e in range(pr.nel))
    assert abs(tot - amp) <= 1e-6 * abs(amp)


# ---- order 4 ---------------------------------------------------------------------------------

@pytest.mark.slow
def test_order_four_element_matrices_match_kronecker_route():
    p, omega, h, kappa = 4, 16 * np.pi, 1 / 32, 0.7
    G, B = element.element_matrices(p, omega, h, kappa=kappa)
    Gk, Bk = _kron_route(p, omega, h, kappa)
    assert np.abs(G - Gk).max() <= 1e-13 * np.abs(Gk).max()
    nf = 4 * p ** 3
    assert np.abs(B[:, :nf] - Bk).max() <= 1e-13 * np.abs(Bk).max()


def _reproduce(N, p, omega, kap, Zel, seed):
    """Global polynomial (p, u) of degree p-1 per coordinate with per-element
    wave speed data: returns the largest field and trace errors and the scale."""
    rng = np.random.default_rng(seed)
    cp = rng.standard_normal((p, p, p)) + 1j * rng.standard_normal((p, p, p))
    cu = rng.standard_normal((3, p, p, p)) + 1j * rng.standard_normal((3, p, p, p))
    h = 1.0 / N

    def elem_of(X):
        ijk = np.clip(np.floor(X / h).astype(int), 0, N - 1)
        return ijk[:, 0] + N * (ijk[:, 1] + N * ijk[:, 2])

    P = lambda X: _monomial_field(cp, p, X)
    U = lambda X: np.stack([_monomial_field(cu[d], p, X) for d in range(3)], axis=1)
    f = lambda X: (1j * omega * kap[elem_of(X)] * P(X)
                   + sum(_monomial_field(cu[d], p, X, d) for d in range(3)))
    g = lambda X: 1j * omega * U(X) + np.stack([_monomial_field(cp, p, X, d) for d in range(3)], 1)
    u0 = lambda X, n: P(X) / Zel[elem_of(X - 0.25 * h * n)] - U(X) @ n
    pr = dpg.Problem(N, p, omega, [dict(f=f, g=g, u0=u0)], kappa=kap, Zel=Zel)
    x, fields, T = _solve(pr)
    err = scale = 0.0
    for e in range(pr.nel):
        X, w, F = _element_points(pr, e, p + 1)
        ex = [P(X)] + [U(X)[:, d] for d in range(3)]
        for c in range(4):
            got = F.T @ fields[e, c * p ** 3:(c + 1) * p ** 3, 0]
            err = max(err, np.abs(got - ex[c]).max())
            scale = max(scale, np.abs(ex[c]).max())
    num = pr.num
    M = num.M
    pts = np.array([(X_, Y_, Z_) for Z_ in range(M + 1) for Y_ in range(M + 1)
                    for X_ in range(M + 1) if all(v % p == 0 for v in (X_, Y_, Z_))])
    terr = np.abs(x[num.h1_index[pts[:, 2], pts[:, 1], pts[:, 0]], 0] - P(pts / M)).max()
    return err, terr, scale


@pytest.mark.slow
def test_order_four_polynomial_reproduction():
    err, terr, scale = _reproduce(2, 4, 6.0, np.full(8, 1.3), np.full(8, 0.8), 41)
    assert err <= 1e-9 * scale and terr <= 1e-9 * scale


@pytest.mark.parametrize("N,p", [(2, 2), (3, 2), (2, 3)])
def test_polynomial_reproduction_piecewise_wave_speed(N, p):
    """Layered (z) and fully random per-element wave speeds, Z = c."""
    nel = N ** 3
    rng = np.random.default_rng(100 + N * 10 + p)
    k = np.arange(nel) // (N * N)                       # z-layer index
    layers = rng.uniform(1.0, 4.0, size=N)
    for c in (layers[k], rng.uniform(1.0, 4.0, size=nel)):
        err, terr, scale = _reproduce(N, p, 4.0, c ** -2.0, c, N * 7 + p)
        assert err <= 1e-10 * scale and terr <= 1e-10 * scale, (err, terr, scale)


# ---- plane-wave h-rates ----------------------------------------------------------------------

@pytest.mark.slow
@pytest.mark.parametrize("p", [2, 3])
def test_plane_wave_h_rates_orders_two_and_three(p):
    omega = 2 * np.pi
    d = np.array([2.0, -1.0, 2.0]) / 3.0
    errs = [_plane_wave_error(N, p, omega, d) for N in (2, 4, 8)]
    e = [a for a, _ in errs]
    assert e[0] > e[1] > e[2]
    rate = np.log2(e[1] / e[2])
    assert rate > p - 0.35, (e, rate)
    for a, b in errs:
        assert a < 3.0 * b
