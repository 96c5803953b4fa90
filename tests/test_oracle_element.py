"""Pins of the oracle's element matrices (Sec. 2: forms, test norm eq. Gnorm).

The oracle integrates with Gauss quadrature at tensor points.  These tests
rebuild the same matrices along a second route: Kronecker products of 1-D
integrals computed by exact polynomial arithmetic (no quadrature), plus Green's
formula for the trace pairing.
"""
import numpy as np
import pytest
import scipy.linalg as sla
from numpy.polynomial import Legendre

from oracle import basis1d, dpg, element


def _poly_h1(r, a):
    """Hierarchical H1 function a of order r as a numpy polynomial."""
    if a == 0:
        return Legendre([0.5, -0.5])
    if a == r:
        return Legendre([0.5, 0.5])
    k = a + 1
    return Legendre.basis(k - 1).integ(lbnd=-1) * np.sqrt((2 * k - 1) / 2.0)


def _I1(rows, cols, drow, dcol, h):
    """1-D integrals (h/2) (2/h)^(drow+dcol) int f_a^(drow) g_b^(dcol) over [-1,1]."""
    out = np.zeros((len(rows), len(cols)))
    for i, f in enumerate(rows):
        for j, g in enumerate(cols):
            prod = (f.deriv(drow) if drow else f) * (g.deriv(dcol) if dcol else g)
            F = prod.integ()
            out[i, j] = F(1.0) - F(-1.0)
    return out * (h / 2.0) * (2.0 / h) ** (drow + dcol)


def _block(rows3, cols3, drow3, dcol3, h):
    """3-D tensor block: x fastest, so kron(z, kron(y, x))."""
    I = [_I1(rows3[a], cols3[a], drow3[a], dcol3[a], h) for a in range(3)]
    return np.kron(I[2], np.kron(I[1], I[0]))


def _kron_route(p, omega, h, kappa, alpha=1.0, dp=1):
    P = p + dp
    leg = lambda n: [Legendre.basis(k) for k in range(n)]
    Lt, Lr, Lf = leg(P + 1), leg(P), leg(p)
    q3 = (Lt, Lt, Lt)
    v3 = []
    for d in range(3):
        f = [Lr, Lr, Lr]
        f[d] = Lt
        v3.append(tuple(f))
    f3 = (Lf, Lf, Lf)
    z = (0, 0, 0)
    e = [tuple(1 if a == d else 0 for a in range(3)) for d in range(3)]
    iw = 1j * omega
    # Gram blocks
    Gqq = (omega ** 2 * kappa ** 2 + alpha) * _block(q3, q3, z, z, h)
    for d in range(3):
        Gqq = Gqq + _block(q3, q3, e[d], e[d], h)
    Gqv = [(-iw * kappa) * _block(q3, v3[d], z, e[d], h) + iw * _block(q3, v3[d], e[d], z, h)
           for d in range(3)]
    Gvv = [[_block(v3[r], v3[c], e[r], e[c], h)
            + ((omega ** 2 + alpha) * _block(v3[r], v3[c], z, z, h) if r == c else 0)
            for c in range(3)] for r in range(3)]
    G = np.block([[Gqq] + Gqv] + [[Gqv[r].conj().T] + Gvv[r] for r in range(3)])
    # B volume blocks (columns p, u_x, u_y, u_z)
    Bq = [iw * kappa * _block(q3, f3, z, z, h)] + [-_block(q3, f3, e[d], z, h) for d in range(3)]
    Bv = [[-_block(v3[r], f3, e[r], z, h)]
          + [iw * _block(v3[r], f3, z, z, h) if d == r else np.zeros((len(Lt) * len(Lr) ** 2, p ** 3))
             for d in range(3)] for r in range(3)]
    Bvol = np.block([Bq] + Bv)
    return G, Bvol


@pytest.mark.parametrize("p,omega,h,kappa", [(1, 3.0, 0.5, 1.0), (2, 2 * np.pi, 0.25, 1.0),
                                             (3, 8 * np.pi, 1 / 16, 0.3)])
def test_gram_and_volume_terms_match_kronecker_route(p, omega, h, kappa):
    G, B = element.element_matrices(p, omega, h, kappa=kappa)
    Gk, Bk = _kron_route(p, omega, h, kappa)
    assert np.abs(G - Gk).max() <= 1e-13 * np.abs(Gk).max()
    nf = 4 * p ** 3
    assert np.abs(B[:, :nf] - Bk).max() <= 1e-13 * np.abs(Bk).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_gram_hermitian_positive_definite(p):
    G, _ = element.element_matrices(p, 8 * np.pi, 1 / 16, gamma=(True, False) * 3)
    assert np.abs(G - G.conj().T).max() <= 1e-15 * np.abs(G).max()
    sla.cholesky(G, lower=True)                  # raises if not positive definite
    n_test, n_field, n_tr = element.sizes(p)
    assert G.shape == (n_test, n_test)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_pressure_trace_pairing_by_greens_formula(p):
    """<phat, v.n>_dK = (grad w, v) + (w, div v) for the H1 extension w of phat."""
    h, omega = 0.5, 2.0
    _, B = element.element_matrices(p, omega, h)
    n_test, n_field, n_tr = element.sizes(p)
    P = p + 1
    Lt, Lr = [Legendre.basis(k) for k in range(P + 1)], [Legendre.basis(k) for k in range(P)]
    H = [_poly_h1(p, a) for a in range(p + 1)]
    lat = element.h1_boundary_lattice(p)
    lat_idx = [(c * (p + 1) + b) * (p + 1) + a for (a, b, c) in lat]
    z = (0, 0, 0)
    nq = (P + 1) ** 3
    blocks = []
    for d in range(3):
        v = [Lr, Lr, Lr]
        v[d] = Lt
        e = tuple(1 if a == d else 0 for a in range(3))
        blk = _block(tuple(v), (H, H, H), z, e, h) + _block(tuple(v), (H, H, H), e, z, h)
        blocks.append(blk[:, lat_idx])
    ref = np.vstack([np.zeros((nq, len(lat)))] + blocks)
    got = B[:, n_field:n_field + len(lat)]
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_optimal_test_product_independent_of_test_basis():
    """K = B^H G^-1 B does not change under an invertible change of test basis."""
    p = 2
    G, B = element.element_matrices(p, 5.0, 0.5, gamma=(True,) * 6)
    rng = np.random.default_rng(3)
    n = G.shape[0]
    C = np.eye(n) + 0.1 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    K1, _ = dpg.optimal_test_product(G, B, np.zeros((n, 1)))
    K2, _ = dpg.optimal_test_product(C.conj().T @ G @ C, C.conj().T @ B, np.zeros((n, 1)))
    assert np.abs(K1 - K2).max() <= 1e-9 * np.abs(K1).max()
    # K is Hermitian and the Gamma-face flux columns vanish
    assert np.abs(K1 - K1.conj().T).max() <= 1e-14 * np.abs(K1).max()
    n_field = 4 * p ** 3
    n_h1 = (p + 1) ** 3 - (p - 1) ** 3
    assert np.all(K1[:, n_field + n_h1:] == 0)


def test_sizes_closed_form():
    assert element.sizes(2) == (172, 32, 50)
    assert element.sizes(3) == (365, 108, 110)
    assert element.sizes(4) == (666, 256, 194)
