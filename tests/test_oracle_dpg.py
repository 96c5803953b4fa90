"""Pins of the oracle's discretisation (Sec. 2) against exact solutions.

* Polynomial reproduction: a global solution whose fields lie in Q^{p-1} is in
  the trial space, and the DPG solution (a minimum-residual solution, unique)
  must reproduce it to round-off -- fields and traces, including the
  impedance reading on Gamma and the flux orientation signs.
* Plane waves: field errors fall like h^p and stay within a fixed factor of
  the L2-projection error (quasi-optimality of a minimum-residual method).
* Static condensation: the trace part of the uncondensed global solve.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import basis1d, dpg, element, topology


def _monomial_field(coef, p, X, der=None):
    """sum c[a,b,c] x^a y^b z^c (or its derivative along axis `der`)."""
    out = np.zeros(X.shape[0], dtype=complex)
    for a in range(p):
        for b in range(p):
            for c in range(p):
                e = [a, b, c]
                if der is not None:
                    if e[der] == 0:
                        continue
                    fac = e[der]
                    e[der] -= 1
                else:
                    fac = 1
                out += fac * coef[a, b, c] * X[:, 0] ** e[0] * X[:, 1] ** e[1] * X[:, 2] ** e[2]
    return out


def _element_points(pr, e, n):
    xg, wg = basis1d.gauss(n)
    x0 = pr.element_origin(e)
    g = np.meshgrid(*(x0[d] + (xg + 1) * pr.h / 2 for d in range(3)), indexing='ij')
    X = np.stack([g[d].transpose(2, 1, 0).reshape(-1) for d in range(3)], axis=1)
    w = np.einsum('i,j,k->kji', wg, wg, wg).reshape(-1) * (pr.h / 2) ** 3
    Lf = basis1d.legendre(pr.p, xg)
    F = np.einsum('ai,bj,ck->cbakji', Lf, Lf, Lf).reshape(pr.p ** 3, -1)
    return X, w, F


def _solve(pr):
    S, s, rec = pr.condensed()
    T = dpg.assemble(pr.edofs, S, pr.num.n)
    rhs = dpg.assemble_vector(pr.edofs, s, pr.num.n)
    x = dpg.direct_solve(T, rhs)
    return x, dpg.recover_fields(rec, pr.edofs, x), T


@pytest.mark.parametrize("N,p,omega,kappa,Z", [(2, 1, 3.0, 1.0, 1.0), (2, 2, 2 * np.pi, 1.0, 1.0),
                                               (2, 3, 5.0, 0.5, 1.7), (3, 2, 4.0, 2.0, 0.6)])
def test_polynomial_reproduction(N, p, omega, kappa, Z):
    rng = np.random.default_rng(N * 10 + p)
    cp = rng.standard_normal((p, p, p)) + 1j * rng.standard_normal((p, p, p))
    cu = rng.standard_normal((3, p, p, p)) + 1j * rng.standard_normal((3, p, p, p))
    P = lambda X: _monomial_field(cp, p, X)
    U = lambda X: np.stack([_monomial_field(cu[d], p, X) for d in range(3)], axis=1)
    f = lambda X: 1j * omega * kappa * P(X) + sum(_monomial_field(cu[d], p, X, d) for d in range(3))
    g = lambda X: 1j * omega * U(X) + np.stack([_monomial_field(cp, p, X, d) for d in range(3)], 1)
    u0 = lambda X, n: P(X) / Z - U(X) @ n
    nel = N ** 3
    pr = dpg.Problem(N, p, omega, [dict(f=f, g=g, u0=u0)], kappa=np.full(nel, kappa),
                     Zel=np.full(nel, Z))
    x, fields, T = _solve(pr)
    err = 0.0
    scale = 0.0
    for e in range(nel):
        X, w, F = _element_points(pr, e, p + 1)
        ex = [P(X)] + [U(X)[:, d] for d in range(3)]
        for c in range(4):
            got = F.T @ fields[e, c * p ** 3:(c + 1) * p ** 3, 0]
            err = max(err, np.abs(got - ex[c]).max())
            scale = max(scale, np.abs(ex[c]).max())
    assert err <= 1e-10 * scale
    # pressure trace: evaluate the H1 trace at skeleton lattice points and compare
    num = pr.num
    M = num.M
    pts = np.array([(X, Y, Z_) for Z_ in range(M + 1) for Y in range(M + 1) for X in range(M + 1)
                    if min(X % p, Y % p, Z_ % p) == 0 and all(v % p == 0 for v in (X, Y, Z_))])
    # at vertex lattice points only the vertex function is nonzero: coefficient = value
    vals = x[num.h1_index[pts[:, 2], pts[:, 1], pts[:, 0]], 0]
    assert np.abs(vals - P(pts / M)).max() <= 1e-10 * scale
    assert np.abs(T - T.getH()).max() <= 1e-14 * abs(T).max()


def _plane_wave_error(N, p, omega, d):
    pr = dpg.Problem(N, p, omega, [dict(u0=dpg.plane_wave_u0(omega, d))])
    _, fields, _ = _solve(pr)
    err2 = proj2 = norm2 = 0.0
    for e in range(pr.nel):
        X, w, F = _element_points(pr, e, p + 6)
        pex = np.exp(-1j * omega * (X @ d))
        ph = F.T @ fields[e, :p ** 3, 0]
        # L2 projection onto Q^{p-1}: Legendre coefficients by quadrature
        mass = (F * w) @ F.T
        cproj = np.linalg.solve(mass, (F * w) @ pex)
        err2 += w @ np.abs(ph - pex) ** 2
        proj2 += w @ np.abs(F.T @ cproj - pex) ** 2
        norm2 += w @ np.abs(pex) ** 2
    return np.sqrt(err2 / norm2), np.sqrt(proj2 / norm2)


@pytest.mark.parametrize("p", [1, 2])
def test_plane_wave_convergence_rate_and_quasi_optimality(p):
    omega = np.pi
    d = np.array([1.0, 2.0, 2.0]) / 3.0
    errs = [_plane_wave_error(N, p, omega, d) for N in (1, 2, 4)]
    e = [a for a, _ in errs]
    rate = np.log2(e[-2] / e[-1])
    assert rate > p - 0.35, (e, rate)
    for a, b in errs:
        assert a < 3.0 * b                       # within a fixed factor of the best fit


def test_static_condensation_matches_uncondensed_solve():
    N, p, omega = 2, 2, 2 * np.pi
    d = np.array([0.0, 0.6, 0.8])
    pr = dpg.Problem(N, p, omega, [dict(u0=dpg.plane_wave_u0(omega, d))])
    nf = pr.n_field
    nT = pr.num.n
    rows, cols, vals = [], [], []
    rhs = np.zeros(pr.nel * nf + nT, dtype=complex)
    for e in range(pr.nel):
        K, b = pr.element_system(e)
        gidx = np.concatenate([nT + e * nf + np.arange(nf), pr.edofs[e]])
        ok = gidx >= 0
        Kk = K[np.ix_(ok, ok)]
        gi = gidx[ok]
        rows.append(np.repeat(gi, gi.size))
        cols.append(np.tile(gi, gi.size))
        vals.append(Kk.ravel())
        np.add.at(rhs, gi, b[ok, 0])
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(rhs.size,) * 2).tocsc()
    full = spla.spsolve(A, rhs)
    x, fields, _ = _solve(pr)
    assert np.abs(full[:nT] - x[:, 0]).max() <= 1e-10 * np.abs(x).max()
    assert np.abs(full[nT:].reshape(pr.nel, nf) - fields[:, :, 0]).max() <= 1e-10 * np.abs(fields).max()


def test_condensed_element_matrices_hermitian_positive_semidefinite():
    pr = dpg.Problem(2, 2, 2 * np.pi, [dict(u0=dpg.plane_wave_u0(2 * np.pi, [1, 0, 0]))])
    S, s, _ = pr.condensed()
    for e in range(pr.nel):
        assert np.abs(S[e] - S[e].conj().T).max() <= 1e-15 * np.abs(S[e]).max()
        ok = pr.edofs[e] >= 0
        ev = np.linalg.eigvalsh(S[e][np.ix_(ok, ok)])
        assert ev.min() > 0
        assert np.all(S[e][~ok] == 0) and np.all(S[e][:, ~ok] == 0)


# ---- the DPG residual error indicator (Sec. 1.2; Sec. 3, first paragraph) ----------------------

def test_error_indicator_vanishes_for_reproduced_polynomials():
    """A solution in the trial space satisfies every element equation exactly,
    so its residual -- and the indicator of every element -- is zero."""
    N, p, omega, kappa, Z = 2, 2, 3.0, 0.7, 1.3
    rng = np.random.default_rng(5)
    cp = rng.standard_normal((p, p, p)) + 1j * rng.standard_normal((p, p, p))
    cu = rng.standard_normal((3, p, p, p)) + 1j * rng.standard_normal((3, p, p, p))
    P = lambda X: _monomial_field(cp, p, X)
    U = lambda X: np.stack([_monomial_field(cu[d], p, X) for d in range(3)], axis=1)
    f = lambda X: 1j * omega * kappa * P(X) + sum(_monomial_field(cu[d], p, X, d) for d in range(3))
    g = lambda X: 1j * omega * U(X) + np.stack([_monomial_field(cp, p, X, d) for d in range(3)], 1)
    u0 = lambda X, n: P(X) / Z - U(X) @ n
    pr = dpg.Problem(N, p, omega, [dict(f=f, g=g, u0=u0)], kappa=np.full(8, kappa),
                     Zel=np.full(8, Z))
    S, s, rec = pr.condensed()
    T = dpg.assemble(pr.edofs, S, pr.num.n)
    x = dpg.direct_solve(T, dpg.assemble_vector(pr.edofs, s, pr.num.n))
    eta2 = dpg.error_indicator(pr, x, rec)
    # scale: the load in the same dual norm
    lnorm = sum(np.real(np.vdot(l, sla.cho_solve(pr._operator(e)[2], l)))
                for e, l in ((e, pr.element_load(e)[:, 0]) for e in range(8)))
    assert eta2.max() <= 1e-20 * lnorm


def test_error_indicator_is_the_minimised_residual():
    """The DPG solution minimises the residual sum_K eta_K^2 over the trial
    space, so moving the traces by d (fields re-recovered) raises it by exactly
    d^H T d, T the condensed operator: the cross term vanishes at the optimum."""
    N, p, omega = 2, 2, 2 * np.pi
    d = np.array([0.48, 0.6, 0.64])
    pr = dpg.Problem(N, p, omega, [dict(u0=dpg.plane_wave_u0(omega, d))])
    S, s, rec = pr.condensed()
    T = dpg.assemble(pr.edofs, S, pr.num.n)
    x = dpg.direct_solve(T, dpg.assemble_vector(pr.edofs, s, pr.num.n))
    J0 = dpg.error_indicator(pr, x, rec).sum()
    rng = np.random.default_rng(2)
    dx = 1e-3 * (rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape))
    J1 = dpg.error_indicator(pr, x + dx, rec).sum()
    quad = np.real(np.vdot(dx[:, 0], T @ dx[:, 0]))
    assert J0 > 0
    assert abs((J1 - J0) - quad) <= 1e-8 * quad


def test_error_indicator_falls_with_h_on_plane_waves():
    omega, p = np.pi, 2
    d = np.array([1.0, 2.0, 2.0]) / 3.0
    tot = []
    for N in (1, 2, 4):
        pr = dpg.Problem(N, p, omega, [dict(u0=dpg.plane_wave_u0(omega, d))])
        S, s, rec = pr.condensed()
        T = dpg.assemble(pr.edofs, S, pr.num.n)
        x = dpg.direct_solve(T, dpg.assemble_vector(pr.edofs, s, pr.num.n))
        tot.append(dpg.error_indicator(pr, x, rec).sum())
    assert tot[0] > tot[1] > tot[2]
    assert np.log2(np.sqrt(tot[1] / tot[2])) > p - 0.5
