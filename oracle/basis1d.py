"""1-D building blocks of the tensor-product shape functions (oracle).

Reference interval xi in [-1, 1].

* Legendre polynomials P_n: the L2 (discontinuous) family used for fields,
  normal traces and the broken test space.
* Hierarchical H1 family of order r (index a = 0..r): a = 0 is (1-xi)/2,
  a = r is (1+xi)/2, and 1 <= a <= r-1 is the normalised integrated Legendre
  polynomial phi_{a+1} = (P_{a+1} - P_{a-1}) / sqrt(2(2a+1)), whose
  derivatives are L2-orthonormal on [-1, 1].  These span the exact-sequence
  H1 space of order r used for the pressure trace (Sec. 2, the trace spaces).
* Two-scale matrices: a coarse-cell function written in the basis of the two
  half cells.  They express coarse basis functions as combinations of fine
  ones, i.e. the natural inclusion of Sec. 3 ("Prolongation") in 1-D.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def gauss(n):
    """Gauss-Legendre rule with n points on [-1, 1] (exact to degree 2n-1)."""
    return npleg.leggauss(n)


def legendre(n, x):
    """Values of P_0..P_{n-1} at x: array [n, len(x)]."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty((n, x.size))
    for k in range(n):
        c = np.zeros(k + 1)
        c[k] = 1.0
        out[k] = npleg.legval(x, c)
    return out


def legendre_deriv(n, x):
    """Derivatives of P_0..P_{n-1} at x: array [n, len(x)]."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty((n, x.size))
    for k in range(n):
        c = np.zeros(k + 1)
        c[k] = 1.0
        out[k] = npleg.legval(x, npleg.legder(c)) if k > 0 else 0.0
    return out


def _h1_coeffs(r):
    """Legendre-series coefficients of the r+1 hierarchical H1 functions."""
    coefs = []
    for a in range(r + 1):
        c = np.zeros(r + 1)
        if a == 0:
            c[0], c[1] = 0.5, -0.5          # (1 - xi)/2
        elif a == r:
            c[0], c[1] = 0.5, 0.5           # (1 + xi)/2
        else:
            k = a + 1                       # phi_k, degree k
            s = 1.0 / np.sqrt(2.0 * (2 * k - 1))
            c[k] += s
            c[k - 2] -= s
        coefs.append(c)
    return coefs


def h1(r, x):
    """Values of the order-r hierarchical H1 functions at x: [r+1, len(x)]."""
    x = np.asarray(x, dtype=np.float64)
    return np.array([npleg.legval(x, c) for c in _h1_coeffs(r)])


def h1_deriv(r, x):
    """Derivatives of the order-r hierarchical H1 functions: [r+1, len(x)]."""
    x = np.asarray(x, dtype=np.float64)
    return np.array([npleg.legval(x, npleg.legder(c)) for c in _h1_coeffs(r)])


def _fit_on_half(values_fn, fine_fn, nfun, side):
    """Coefficients c[fine, coarse] with coarse(xi) = sum fine(eta) c on a half.

    side = 0 is the left half xi = (eta - 1)/2, side = 1 the right half
    xi = (eta + 1)/2.  Both families are polynomial spaces of the same
    dimension, so collocation at nfun distinct points is exact.
    """
    eta, _ = gauss(nfun)
    xi = (eta - 1.0) / 2.0 if side == 0 else (eta + 1.0) / 2.0
    V = fine_fn(eta)            # [nfun, npts]
    F = values_fn(xi)           # [ncoarse, npts]
    # solve V^T c = F^T  -> c [nfun_fine, ncoarse]
    return np.linalg.solve(V.T, F.T)


def twoscale_h1(r):
    """Local H1 two-scale matrix R1 of shape [2r+1, r+1].

    Row X indexes the fine lattice of one coarse cell split in two:
    X = 0 left vertex, 1..r-1 left-cell bubbles, X = r the midpoint vertex,
    r+1..2r-1 right-cell bubbles, X = 2r right vertex.  Column a is the coarse
    H1 function a.  Entry = coefficient of fine function X in coarse function a.
    """
    cl = _fit_on_half(lambda t: h1(r, t), lambda t: h1(r, t), r + 1, 0)
    cr = _fit_on_half(lambda t: h1(r, t), lambda t: h1(r, t), r + 1, 1)
    R = np.zeros((2 * r + 1, r + 1))
    R[0:r + 1] = cl            # left cell local 0..r -> lattice 0..r
    R[r:2 * r + 1] = cr        # right cell local 0..r -> lattice r..2r
    # the midpoint row appears in both halves; both give the coarse value there
    assert np.allclose(cl[r], cr[0], atol=1e-13)
    return _clean(R)


def twoscale_leg(r):
    """Local Legendre two-scale matrix R0 of shape [2r, r].

    Row T = r*half + n (half 0 = left, 1 = right; n = fine degree), column m =
    coarse degree.  Entry = coefficient of fine P_n (on that half) in coarse P_m.
    """
    cl = _fit_on_half(lambda t: legendre(r, t), lambda t: legendre(r, t), r, 0)
    cr = _fit_on_half(lambda t: legendre(r, t), lambda t: legendre(r, t), r, 1)
    return _clean(np.vstack([cl, cr]))


def _clean(R):
    """Set round-off residue of exactly-zero coefficients to zero.

    Coefficients vanish exactly by parity or support; collocation leaves
    residues near 1e-16 there, which would blur the sparsity pattern.
    """
    R = R.copy()
    R[np.abs(R) < 1e-13] = 0.0
    return R
