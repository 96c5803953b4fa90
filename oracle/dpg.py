"""Optimal test product, static condensation, assembly, solve (oracle).

Practical DPG (Sec. 2, first paragraph): the optimal test functions are
obtained by inverting the Riesz map of the enriched broken test space element
by element, so each element contributes the Hermitian positive definite
matrix K = B^H G^-1 B and the load b = B^H G^-1 l, where G is the Gram matrix
of the test norm (eq. Gnorm).  Field unknowns are interior to an element and
are statically condensed onto the traces (Sec. 1.2):
    S = K_tt - K_tf K_ff^-1 K_ft,    s = b_t - K_tf K_ff^-1 b_f.
The condensed trace system T x = s assembles S by gather/scatter over the
element-to-trace maps (orientation signs live inside B).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import element, topology


def optimal_test_product(G, B, l):
    """K = B^H G^-1 B and b = B^H G^-1 l, through the Cholesky factor of G."""
    c = sla.cho_factor(G, lower=True)
    GiB = sla.cho_solve(c, B)
    Gil = sla.cho_solve(c, l)
    K = B.conj().T @ GiB
    b = B.conj().T @ Gil
    return 0.5 * (K + K.conj().T), b


def condense(K, b, n_field):
    """Schur complement onto the traces; also returns the recovery data."""
    f = slice(0, n_field)
    t = slice(n_field, K.shape[0])
    nt = K.shape[0] - n_field
    c = sla.cho_factor(K[f, f], lower=True)
    X = sla.cho_solve(c, np.column_stack([K[f, t], b[f]]))
    S = K[t, t] - K[t, f] @ X[:, :nt]
    s = b[t] - K[t, f] @ X[:, nt:]
    return 0.5 * (S + S.conj().T), s, (c, K[f, t], b[f])


def plane_wave_u0(omega, direction, amp=1.0, Z=1.0):
    """Impedance data of p = A exp(-i w d.x), u = d p:  u0 = (Z^-1 - d.n) p."""
    d = np.asarray(direction, dtype=np.float64)

    def u0(X, n):
        return (1.0 / Z - d @ n) * amp * np.exp(-1j * omega * (X @ d))
    return u0


def gaussian_sources(centers, sigma, amps):
    """f = sum_s a_s (2 pi sigma^2)^(-3/2) exp(-|x - x_s|^2 / (2 sigma^2))."""
    centers = np.atleast_2d(np.asarray(centers, dtype=np.float64))
    amps = np.atleast_1d(np.asarray(amps, dtype=np.complex128))
    sigma = np.atleast_1d(np.asarray(sigma, dtype=np.float64)) * np.ones(len(centers))

    def f(X):
        out = np.zeros(X.shape[0], dtype=np.complex128)
        for c, s, a in zip(centers, sigma, amps):
            r2 = np.sum((X - c) ** 2, axis=1)
            out += a * (2 * np.pi * s * s) ** -1.5 * np.exp(-r2 / (2 * s * s))
        return out
    return f


class Problem:
    """Uniform N^3 mesh of a cube [origin, origin + side]^3, order p.

    kappa: per-element c^-2 (None = 1); Zel: per-element impedance (None = 1).
    loads: list of dicts with optional keys f, g, u0 (one per right-hand side).
    """

    def __init__(self, N, p, omega, loads, dp=1, side=1.0, origin=(0.0, 0.0, 0.0),
                 kappa=None, Zel=None, alpha=1.0):
        self.N, self.p, self.dp, self.omega = N, p, dp, omega
        self.h = side / N
        self.origin = np.asarray(origin, dtype=np.float64)
        self.num = topology.Numbering(N, p)
        self.edofs = topology.element_dofs(self.num)
        self.nel = N ** 3
        self.kappa = np.ones(self.nel) if kappa is None else np.asarray(kappa, float)
        self.Zel = np.ones(self.nel) if Zel is None else np.asarray(Zel, float)
        self.loads = loads
        self.alpha = alpha
        self.n_test, self.n_field, self.n_tr = element.sizes(p, dp)

    def element_gamma(self, e):
        N = self.N
        i, j, k = e % N, (e // N) % N, e // (N * N)
        g = []
        for c in (i, j, k):
            g += [c == 0, c == N - 1]
        return tuple(g)

    def element_origin(self, e):
        N = self.N
        i, j, k = e % N, (e // N) % N, e // (N * N)
        return self.origin + self.h * np.array([i, j, k], dtype=np.float64)

    def _operator(self, e):
        """Element matrices that do not depend on the load: G, B and what the
        condensation reuses.  They depend only on (kappa, Z, Gamma faces), so
        they are computed once per distinct triple (memoised pure function)."""
        key = (float(self.kappa[e]), float(self.Zel[e]), self.element_gamma(e))
        cache = self.__dict__.setdefault('_opcache', {})
        if key not in cache:
            G, B = element.element_matrices(self.p, self.omega, self.h, self.dp,
                                            kappa=key[0], Z=key[1], gamma=key[2],
                                            alpha=self.alpha)
            cache[key] = (G, B, sla.cho_factor(G, lower=True))
        return cache[key]

    def element_load(self, e):
        """Element load vectors l [n_test, nrhs]."""
        gam = self.element_gamma(e)
        x0 = self.element_origin(e)
        return np.column_stack([element.element_load(self.p, self.h, x0, self.dp, gam,
                                                     f=ld.get('f'), g=ld.get('g'),
                                                     u0=ld.get('u0'))
                                for ld in self.loads])

    def element_system(self, e):
        """Element K [m, m] and b [m, nrhs], m = n_field + n_tr."""
        G, B, _ = self._operator(e)
        return optimal_test_product(G, B, self.element_load(e))

    def condensed_operator(self):
        """Per-element condensed matrices S [nel, n_tr, n_tr] without loads: the
        operator of this mesh assembled directly (used for the "store" coarse
        operators of the multigrid hierarchy)."""
        S = np.zeros((self.nel, self.n_tr, self.n_tr), dtype=np.complex128)
        scache = {}
        for e in range(self.nel):
            G, B, cG = self._operator(e)
            key = id(cG)
            if key not in scache:
                K, _ = optimal_test_product(G, B, np.zeros((G.shape[0], 1)))
                scache[key] = condense(K, np.zeros((K.shape[0], 1)), self.n_field)[0]
            S[e] = scache[key]
        return S

    def condensed(self, elements=None):
        """Per-element S [nel, n_tr, n_tr], s [nel, n_tr, nrhs], recovery data.

        K and S are memoised per element class like G and B; the loads are
        computed for every element.  `elements` restricts the work to a subset
        (the other rows stay zero).
        """
        S = np.zeros((self.nel, self.n_tr, self.n_tr), dtype=np.complex128)
        s = np.zeros((self.nel, self.n_tr, len(self.loads)), dtype=np.complex128)
        rec = [None] * self.nel
        scache = {}
        for e in (range(self.nel) if elements is None else elements):
            G, B, cG = self._operator(e)
            key = id(cG)
            l = self.element_load(e)
            if key not in scache:
                K, _ = optimal_test_product(G, B, l)
                scache[key] = condense(K, np.zeros((K.shape[0], l.shape[1])), self.n_field)
            Se, _, (cK, Kft, _) = scache[key]
            b = B.conj().T @ sla.cho_solve(cG, l)
            f = slice(0, self.n_field)
            S[e] = Se
            s[e] = b[self.n_field:] - Kft.conj().T @ sla.cho_solve(cK, b[f])
            rec[e] = (cK, Kft, b[f])
        return S, s, rec


def assemble(edofs, E, n):
    """Sparse sum_K E_K^T M_K E_K over element maps (absent entries skipped)."""
    rows, cols, vals = [], [], []
    for e in range(edofs.shape[0]):
        d = edofs[e]
        ok = d >= 0
        dd = d[ok]
        M = E[e][np.ix_(ok, ok)]
        rows.append(np.repeat(dd, dd.size))
        cols.append(np.tile(dd, dd.size))
        vals.append(M.ravel())
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsr()


def assemble_vector(edofs, s, n):
    out = np.zeros((n, s.shape[2]), dtype=np.complex128)
    for e in range(edofs.shape[0]):
        d = edofs[e]
        ok = d >= 0
        np.add.at(out, d[ok], s[e][ok])
    return out


def direct_solve(T, rhs):
    return spla.spsolve(T.tocsc(), rhs).reshape(rhs.shape)


def recover_fields(rec, edofs, x):
    """Field coefficients x_f = K_ff^-1 (b_f - K_ft x_t) per element [nel, n_field, nrhs]."""
    out = []
    for e in range(edofs.shape[0]):
        c, Kft, bf = rec[e]
        d = edofs[e]
        xt = np.zeros((d.size,) + x.shape[1:], dtype=np.complex128)
        xt[d >= 0] = x[d[d >= 0]]
        out.append(sla.cho_solve(c, bf - Kft @ xt))
    return np.array(out)


def error_indicator(pr, x, rec):
    """DPG residual error indicator of every element (Sec. 1.2, the built-in
    error estimate; Sec. 3, first paragraph): the residual of the element
    equations in the dual test norm, eta_K^2 = r^H G^-1 r with
    r = l_K - B_K [x_f; x_t], for the trace solution x [n_trace, nrhs] and the
    fields recovered from it.  Returns eta^2 [nel, nrhs]."""
    fields = recover_fields(rec, pr.edofs, x)
    out = np.zeros((pr.nel, x.shape[1]))
    for e in range(pr.nel):
        G, B, cG = pr._operator(e)
        d = pr.edofs[e]
        xt = np.zeros((d.size, x.shape[1]), dtype=np.complex128)
        xt[d >= 0] = x[d[d >= 0]]
        r = pr.element_load(e) - B @ np.vstack([fields[e], xt])
        out[e] = np.real(np.sum(r.conj() * sla.cho_solve(cG, r), axis=0))
    return out

