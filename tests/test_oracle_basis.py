"""Pins of the oracle's 1-D building blocks against closed forms."""
import numpy as np
import pytest
from numpy.polynomial import Legendre, Polynomial

from oracle import basis1d


@pytest.mark.parametrize("n", [1, 2, 3, 5, 9])
def test_gauss_exact_to_degree_2n_minus_1(n):
    x, w = basis1d.gauss(n)
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(w @ x ** k - exact) < 1e-14
    k = 2 * n                                   # first degree that is not exact
    assert abs(w @ x ** k - 2.0 / (k + 1)) > 1e-6


@pytest.mark.parametrize("r", [1, 2, 3, 4, 5])
def test_h1_family_shape_and_orthonormal_derivatives(r):
    ends = basis1d.h1(r, np.array([-1.0, 1.0]))
    assert np.allclose(ends[0], [1.0, 0.0]) and np.allclose(ends[r], [0.0, 1.0])
    assert np.allclose(ends[1:r], 0.0, atol=1e-15)           # bubbles vanish at the ends
    x, w = basis1d.gauss(r + 1)
    D = basis1d.h1_deriv(r, x)[1:r]
    assert np.allclose(D @ (w[:, None] * D.T), np.eye(r - 1), atol=1e-14)
    # derivative of phi_k is sqrt((2k-1)/2) P_{k-1}
    for a in range(1, r):
        k = a + 1
        ref = np.sqrt((2 * k - 1) / 2.0) * basis1d.legendre(k, x)[k - 1]
        assert np.allclose(basis1d.h1_deriv(r, x)[a], ref, atol=1e-13)


def test_legendre_against_textbook_polynomials():
    x = np.linspace(-1, 1, 7)
    P = basis1d.legendre(4, x)
    assert np.allclose(P[2], (3 * x ** 2 - 1) / 2)
    assert np.allclose(P[3], (5 * x ** 3 - 3 * x) / 2)
    dP = basis1d.legendre_deriv(4, x)
    assert np.allclose(dP[3], (15 * x ** 2 - 3) / 2)


def test_twoscale_closed_forms():
    # Legendre: on the left half xi = (eta-1)/2, so P1 = eta/2 - 1/2 = P1/2 - P0/2;
    # on the right half P1 = P1/2 + P0/2.  P0 is P0 on both halves.
    r = 3
    R0 = basis1d.twoscale_leg(r)
    assert np.allclose(R0[:, 0], [1, 0, 0, 1, 0, 0])
    assert np.allclose(R0[:, 1], [-0.5, 0.5, 0, 0.5, 0.5, 0])
    # P2(xi) on the left half: (3 (eta-1)^2/4 - 1)/2 = (3 eta^2 - 6 eta - 1)/8
    # = P2/4 - 3 P1/4 (using 3 eta^2 = 2 P2 + 1).
    assert np.allclose(R0[:3, 2], [0.0, -0.75, 0.25])
    # H1: the coarse left vertex function is linear: 1 at -1, 1/2 at the midpoint.
    R1 = basis1d.twoscale_h1(2)
    assert np.allclose(R1[:, 0], [1, 0, 0.5, 0, 0])
    # coarse bubble phi_2 = 3 (xi^2 - 1)/(2 sqrt 6): value -3/(2 sqrt 6) at the
    # midpoint and 1/4 of the fine bubble on each half (leading term halves twice).
    assert np.allclose(R1[:, 1], [0, 0.25, -3 / (2 * np.sqrt(6)), 0.25, 0])


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_twoscale_reproduces_coarse_functions_pointwise(r):
    """Brute force: sum of fine functions times R equals the coarse function."""
    rng = np.random.default_rng(r)
    R1 = basis1d.twoscale_h1(r)
    R0 = basis1d.twoscale_leg(r)
    for side in (0, 1):
        eta = rng.uniform(-1, 1, 11)
        xi = (eta - 1) / 2 if side == 0 else (eta + 1) / 2
        fine = basis1d.h1(r, eta)                      # local fine functions on that half
        rows = np.arange(r + 1) + side * r
        assert np.allclose(R1[rows].T @ fine, basis1d.h1(r, xi), atol=1e-13)
        fl = basis1d.legendre(r, eta)
        assert np.allclose(R0[side * r:(side + 1) * r].T @ fl, basis1d.legendre(r, xi), atol=1e-13)


def test_h1_functions_match_independent_polynomial_construction():
    """phi_k from the integrated Legendre polynomial, built by numpy polynomials."""
    r = 5
    x = np.linspace(-1, 1, 13)
    for a in range(1, r):
        k = a + 1
        prim = Legendre.basis(k - 1).integ(lbnd=-1)        # int_{-1}^{xi} P_{k-1}
        ref = np.sqrt((2 * k - 1) / 2.0) * prim(x)
        assert np.allclose(basis1d.h1(r, x)[a], ref, atol=1e-13)
    assert np.allclose(basis1d.h1(r, x)[0], Polynomial([0.5, -0.5])(x))
