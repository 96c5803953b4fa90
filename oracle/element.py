"""Element matrices of the broken ultraweak acoustics formulation (oracle).

Problem (Sec. 2, eq. helmholtz, with wave speed c per element, rho = 1):
    i w c^-2 p + div u = f,   i w u + grad p = g   in Omega,
    Z^-1 p - u.n = u0                               on Gamma,   Z = c.

Forms (Sec. 2, "Broken ultraweak formulation"), all sesquilinear, (a, b) =
int a conj(b):
    b((u,p),(q,v))  = (i w c^-2 p, q) - (u, grad q) + (i w u, v) - (p, div v)
    bhat            = <uhat_n, q> + <phat, v.n>   on every element boundary
    l(q, v)         = (f, q) + (g, v) + <u0, q>_Gamma
Test norm (Sec. 2, eq. Gnorm), alpha = 1:
    ||(q,v)||^2 = ||i w c^-2 q + div v||^2 + ||grad q + i w v||^2
                  + alpha (||q||^2 + ||v||^2).
Reading of the impedance condition (the paper constrains both the traces and
the test functions on Gamma): no flux unknown lives on Gamma; there the flux
pairing <uhat_n, q> is replaced by <Z^-1 phat, q>, and the test space is left
unconstrained.  The exact solution then satisfies b + bhat = l for every test
function (integration by parts gives <Z^-1 p - u.n, q> = <u0, q> on Gamma).

Discrete spaces for "order p" (exact sequence) with test enrichment dp
(Sec. 2: the test order is raised by one):
    fields p, u_x, u_y, u_z  in Q^{p-1}          (Legendre tensor products)
    phat  trace of H1 Q^p    (hierarchical H1 tensor products, boundary lattice)
    uhat  Q^{p-1} per face   (Legendre in the two in-plane directions)
    q in Q^{p+dp},  v in RT_{p+dp}  (v_x in Q^{p+dp, p+dp-1, p+dp-1}, ...)
The test basis is any basis of the broken test space (Legendre products
here); the optimal-test product does not depend on that choice.

Element-local trace layout (n_tr entries):
    [H1 boundary lattice (a,b,c) in [0,p]^3 with a coordinate in {0,p},
     a fastest] + [faces x-, x+, y-, y+, z-, z+, each p^2 Legendre pairs
     (m, n) with m fastest; x-faces (m,n) = (y,z) degrees, y-faces (x,z),
     z-faces (x,y)].
On a Gamma face the flux unknowns are absent: their columns of B are zero.
Flux orientation: the unknown is u.e_d for the global axis d; on the element's
high face the outward normal is +e_d (sign +1), on its low face -e_d (-1).

Quadrature: p+dp+1 Gauss points per direction for the matrices (exact, the
data are constant per element); p+dp+5 points for loads.
"""
import numpy as np

from . import basis1d


def sizes(p, dp=1):
    P = p + dp
    n_test = (P + 1) ** 3 + 3 * (P + 1) * P * P
    n_field = 4 * p ** 3
    n_tr = (p + 1) ** 3 - (p - 1) ** 3 + 6 * p * p
    return n_test, n_field, n_tr


def h1_boundary_lattice(p):
    """Local H1 lattice points (a, b, c) on the element boundary, a fastest."""
    pts = []
    for c in range(p + 1):
        for b in range(p + 1):
            for a in range(p + 1):
                if a in (0, p) or b in (0, p) or c in (0, p):
                    pts.append((a, b, c))
    return pts


def _t3(fx, fy, fz):
    """Tensor products: rows (c,b,a) with a fastest, points (k,j,i), i fastest."""
    na, nx = fx.shape
    nb, ny = fy.shape
    nc, nz = fz.shape
    return np.einsum('ai,bj,ck->cbakji', fx, fy, fz).reshape(na * nb * nc, nx * ny * nz)


def _test_functions(p, dp, h, pts):
    """Test functions (q, v) at tensor points pts (1-D nodes on [-1,1] per axis).

    Returns dict with 'q', 'dq' (3 arrays), 'v' (3 arrays, component d rows only
    nonzero in block d), 'div', each of shape [n_test, npts] over the full test
    list [q | v_x | v_y | v_z].
    """
    P = p + dp
    x, y, z = pts
    L = [basis1d.legendre(P + 1, t) for t in (x, y, z)]
    dL = [basis1d.legendre_deriv(P + 1, t) * (2.0 / h) for t in (x, y, z)]
    nq = (P + 1) ** 3
    nv = (P + 1) * P * P
    npts = x.size * y.size * z.size
    n_test = nq + 3 * nv
    out = {'q': np.zeros((n_test, npts)), 'dq': [np.zeros((n_test, npts)) for _ in range(3)],
           'v': [np.zeros((n_test, npts)) for _ in range(3)], 'div': np.zeros((n_test, npts))}
    out['q'][:nq] = _t3(L[0], L[1], L[2])
    out['dq'][0][:nq] = _t3(dL[0], L[1], L[2])
    out['dq'][1][:nq] = _t3(L[0], dL[1], L[2])
    out['dq'][2][:nq] = _t3(L[0], L[1], dL[2])
    for d in range(3):
        f = [L[e][:P] for e in range(3)]
        f[d] = L[d]
        g = [L[e][:P] for e in range(3)]
        g[d] = dL[d]
        rows = slice(nq + d * nv, nq + (d + 1) * nv)
        out['v'][d][rows] = _t3(*f)
        out['div'][rows] = _t3(*g)
    return out


def _volume_rule(n, h):
    xg, wg = basis1d.gauss(n)
    w = np.einsum('i,j,k->kji', wg, wg, wg).reshape(-1) * (h / 2.0) ** 3
    return xg, w


def _face_points(d, s, xg):
    """1-D node arrays per axis for face (axis d, side s) of the reference cube."""
    pts = [xg, xg, xg]
    pts[d] = np.array([-1.0 if s == 0 else 1.0])
    return pts


def _face_weights(d, wg, h):
    # points are (k,j,i) flattened with the fixed axis of size 1
    w = [wg, wg, wg]
    w[d] = np.array([1.0])
    return np.einsum('i,j,k->kji', w[0], w[1], w[2]).reshape(-1) * (h / 2.0) ** 2


def _phys(pts, x0, h):
    """Physical coordinates [npts, 3] of reference tensor points, (k,j,i) order."""
    X = [x0[d] + (pts[d] + 1.0) * h / 2.0 for d in range(3)]
    g = np.meshgrid(X[0], X[1], X[2], indexing='ij')          # [i, j, k]
    return np.stack([g[d].transpose(2, 1, 0).reshape(-1) for d in range(3)], axis=1)


def element_matrices(p, omega, h, dp=1, kappa=1.0, Z=1.0, gamma=(False,) * 6, alpha=1.0):
    """Gram matrix G [n_test, n_test] and B [n_test, n_field + n_tr].

    kappa = c^-2 of the element, Z = impedance used on its Gamma faces,
    gamma[2*d + s] tells whether face (axis d, side s) lies on Gamma.
    """
    n_test, n_field, n_tr = sizes(p, dp)
    nq1 = p + dp + 1
    xg, w = _volume_rule(nq1, h)
    T = _test_functions(p, dp, h, (xg, xg, xg))
    iw = 1j * omega
    A1 = iw * kappa * T['q'] + T['div']
    A2 = [T['dq'][d] + iw * T['v'][d] for d in range(3)]
    G = np.conj(A1) @ (w[:, None] * A1.T)
    for d in range(3):
        G += np.conj(A2[d]) @ (w[:, None] * A2[d].T)
    G += alpha * (T['q'] @ (w[:, None] * T['q'].T))
    for d in range(3):
        G += alpha * (T['v'][d] @ (w[:, None] * T['v'][d].T))

    B = np.zeros((n_test, n_field + n_tr), dtype=np.complex128)
    Lf = basis1d.legendre(p, xg)
    F = _t3(Lf, Lf, Lf)                                   # [p^3, npts]
    nfp = p ** 3
    # b = (i w kappa p, q) - (p, div v) - (u, grad q) + (i w u, v)
    B[:, 0:nfp] = (iw * kappa * T['q'] - T['div']) @ (w[:, None] * F.T)
    for d in range(3):
        cols = slice(nfp * (d + 1), nfp * (d + 2))
        B[:, cols] = (-T['dq'][d] + iw * T['v'][d]) @ (w[:, None] * F.T)

    # trace terms
    lat = h1_boundary_lattice(p)
    n_h1 = len(lat)
    lat_rows = [(c * (p + 1) + b) * (p + 1) + a for (a, b, c) in lat]
    xgf, wgf = basis1d.gauss(nq1)
    for d in range(3):
        for s in range(2):
            pts = _face_points(d, s, xgf)
            wf = _face_weights(d, wgf, h)
            Tf = _test_functions(p, dp, h, pts)
            Hf = _t3(*(basis1d.h1(p, t) for t in pts))[lat_rows]    # [n_h1, npts]
            sign = 1.0 if s == 1 else -1.0                            # n_K . e_d
            # <phat, v.n> on every face
            B[:, n_field:n_field + n_h1] += (sign * Tf['v'][d]) @ (wf[:, None] * Hf.T)
            fidx = 2 * d + s
            if gamma[fidx]:
                # <Z^-1 phat, q> replaces the flux pairing on Gamma
                B[:, n_field:n_field + n_h1] += (Tf['q'] / Z) @ (wf[:, None] * Hf.T)
            else:
                inplane = [e for e in range(3) if e != d]
                Lm = basis1d.legendre(p, pts[inplane[0]])
                Ln = basis1d.legendre(p, pts[inplane[1]])
                # rows (n, m) with m fastest, points ordered like the face rule
                U = np.einsum('mj,nk->nmkj', Lm, Ln).reshape(p * p, -1)
                c0 = n_field + n_h1 + fidx * p * p
                B[:, c0:c0 + p * p] += (sign * Tf['q']) @ (wf[:, None] * U.T)
    return G, B


def element_load(p, h, x0, dp=1, gamma=(False,) * 6, f=None, g=None, u0=None, nq_extra=4):
    """Load vector l [n_test] = (f, q) + (g, v) + <u0, q>_Gamma.

    f(X) -> [npts] complex, g(X) -> [npts, 3] complex, u0(X, n) -> [npts]
    complex, with X the physical points [npts, 3] and n the outward normal.
    """
    n_test, _, _ = sizes(p, dp)
    nql = p + dp + 1 + nq_extra
    xg, w = _volume_rule(nql, h)
    l = np.zeros(n_test, dtype=np.complex128)
    if f is not None or g is not None:
        T = _test_functions(p, dp, h, (xg, xg, xg))
        X = _phys((xg, xg, xg), x0, h)
        if f is not None:
            l += T['q'] @ (w * f(X))
        if g is not None:
            gv = g(X)
            for d in range(3):
                l += T['v'][d] @ (w * gv[:, d])
    if u0 is not None:
        for d in range(3):
            for s in range(2):
                if not gamma[2 * d + s]:
                    continue
                pts = _face_points(d, s, xg)
                wf = _face_weights(d, basis1d.gauss(nql)[1], h)
                Tf = _test_functions(p, dp, h, pts)
                X = _phys(pts, x0, h)
                n = np.zeros(3)
                n[d] = 1.0 if s == 1 else -1.0
                l += Tf['q'] @ (wf * u0(X, n))
    return l
