"""Canonical numbering, macro grids, vertex patches, prolongation (oracle).

Mesh: the unit cube (or a cube of side `side`) split into N^3 equal boxes;
element e = i + N (j + N k).  Order p.

Trace unknowns of the mesh, in canonical order:
  * H1 (pressure trace): lattice points (X, Y, Z) in [0, Np]^3 with at least
    one coordinate divisible by p, ordered with X fastest, then Y, then Z.
  * Flux (normal velocity trace) families x, y, z: interior planes
    s = 1..N-1 of global normal e_d, in-plane index (T1, T2) in [0, Np)^2 with
    T = p*cell + Legendre degree; T1 fastest, then T2, then s.  In-plane axes:
    x-family (y, z), y-family (x, z), z-family (x, y).
  * Global vector = [H1 | flux x | flux y | flux z].

Macro grid of a mesh with N even (Sec. 3, "Prolongation"): trace unknowns on
the skeleton of the twice-coarser mesh (some H1 coordinate divisible by 2p;
flux planes with even s) form the set B, numbered by ascending canonical
index; the others are interior to exactly one coarse element (set I) and are
condensed.

Vertex patches (Sec. 3, "V-cycle and smoother"): for each vertex of the
coarse mesh (X fastest), the B unknowns whose support lies inside the union
of the coarse elements sharing that vertex.

Prolongation (Sec. 3, natural inclusion): coarse trace functions written in
the fine basis, restricted to B rows: tensor products of the 1-D two-scale
matrices.
"""
import numpy as np
import scipy.sparse as sp

from . import basis1d


def n_trace(N, p):
    return (N * p + 1) ** 3 - N ** 3 * (p - 1) ** 3 + 3 * N * N * (N - 1) * p * p


class Numbering:
    """Canonical indices of the trace unknowns of an N^3 mesh of order p."""

    def __init__(self, N, p):
        self.N, self.p = N, p
        M = N * p
        self.M = M
        g = np.arange(M + 1)
        Zc, Yc, Xc = np.meshgrid(g, g, g, indexing='ij')          # [Z, Y, X]
        mask = (Xc % p == 0) | (Yc % p == 0) | (Zc % p == 0)
        self.h1_index = np.full(mask.shape, -1, dtype=np.int64)  # [Z, Y, X]
        self.h1_index[mask] = np.arange(int(mask.sum()))
        self.n_h1 = int(mask.sum())
        self.n_fam = (N - 1) * M * M
        self.n = self.n_h1 + 3 * self.n_fam
        assert self.n == n_trace(N, p)

    def h1(self, X, Y, Z):
        return self.h1_index[Z, Y, X]

    def flux(self, d, s, T1, T2):
        """Index of flux unknown of family d on plane s (1..N-1)."""
        return self.n_h1 + d * self.n_fam + ((s - 1) * self.M + T2) * self.M + T1

    def describe(self):
        """Per-unknown records: kind (0 = H1, 1..3 = flux family + 1) and coords.

        For H1: (X, Y, Z).  For flux: (s, T1, T2).
        """
        kind = np.zeros(self.n, dtype=np.int64)
        coord = np.zeros((self.n, 3), dtype=np.int64)
        Z, Y, X = np.nonzero(self.h1_index >= 0)
        idx = self.h1_index[Z, Y, X]
        coord[idx] = np.stack([X, Y, Z], axis=1)
        for d in range(3):
            for s in range(1, self.N):
                for T2 in range(self.M):
                    T1 = np.arange(self.M)
                    i = self.flux(d, s, T1, T2)
                    kind[i] = d + 1
                    coord[i, 0] = s
                    coord[i, 1] = T1
                    coord[i, 2] = T2
        return kind, coord


def element_dofs(num):
    """Global trace index per element-local trace unknown, -1 where absent.

    Array [N^3, n_tr]; element-local layout as in ``element``.
    """
    N, p = num.N, num.p
    lat = []
    for c in range(p + 1):
        for b in range(p + 1):
            for a in range(p + 1):
                if a in (0, p) or b in (0, p) or c in (0, p):
                    lat.append((a, b, c))
    n_tr = len(lat) + 6 * p * p
    out = np.full((N ** 3, n_tr), -1, dtype=np.int64)
    for k in range(N):
        for j in range(N):
            for i in range(N):
                e = i + N * (j + N * k)
                cell = (i, j, k)
                row = [num.h1(i * p + a, j * p + b, k * p + c) for (a, b, c) in lat]
                for d in range(3):
                    ip = [q for q in range(3) if q != d]
                    for s in range(2):
                        plane = cell[d] + s
                        for n in range(p):
                            for m in range(p):
                                if 0 < plane < N:
                                    T1 = cell[ip[0]] * p + m
                                    T2 = cell[ip[1]] * p + n
                                    row.append(num.flux(d, plane, T1, T2))
                                else:
                                    row.append(-1)
                out[e] = row
    return out


class MacroLevel:
    """Macro-grid sets, blocks and vertex patches of a fine mesh with N even."""

    def __init__(self, num):
        N, p = num.N, num.p
        assert N % 2 == 0
        Nc = N // 2
        self.num, self.N, self.Nc, self.p = num, N, Nc, p
        kind, coord = num.describe()
        self.kind, self.coord = kind, coord
        isB = np.zeros(num.n, dtype=bool)
        h1 = kind == 0
        isB[h1] = np.any(coord[h1] % (2 * p) == 0, axis=1)
        fl = kind > 0
        isB[fl] = coord[fl, 0] % 2 == 0
        self.isB = isB
        self.B = np.nonzero(isB)[0]                     # canonical indices, ascending
        self.macro_of = np.full(num.n, -1, dtype=np.int64)
        self.macro_of[self.B] = np.arange(self.B.size)
        self.nM = self.B.size
        # Support of every B unknown, as an interval [lo, hi] of coarse cells per
        # axis.  H1 factor at fine lattice X: a coarse vertex (X % 2p == 0)
        # touches the cells on both sides, any other point only its own cell.
        # Flux unknown: the two cells beside its plane, one cell in-plane.
        lo = np.zeros((self.nM, 3), dtype=np.int64)
        hi = np.zeros((self.nM, 3), dtype=np.int64)
        kB, cB = kind[self.B], coord[self.B]
        hb = kB == 0
        for a in range(3):
            X = cB[hb, a]
            atv = X % (2 * p) == 0
            lo[hb, a] = np.where(atv, np.maximum(X // (2 * p) - 1, 0), X // (2 * p))
            hi[hb, a] = np.where(atv, np.minimum(X // (2 * p), Nc - 1), X // (2 * p))
        for d in range(3):
            m = kB == d + 1
            ip = [q for q in range(3) if q != d]
            lo[m, d] = cB[m, 0] // 2 - 1
            hi[m, d] = cB[m, 0] // 2
            for a, col in ((ip[0], 1), (ip[1], 2)):
                lo[m, a] = cB[m, col] // (2 * p)
                hi[m, a] = cB[m, col] // (2 * p)
        self.support_lo, self.support_hi = lo, hi
        # coarse-element blocks from the children's element maps
        edofs = element_dofs(num)
        self.edofs = edofs
        self.children, self.blocks_B, self.blocks_I = [], [], []
        for kc in range(Nc):
            for jc in range(Nc):
                for ic in range(Nc):
                    kids = [(2 * ic + a) + N * ((2 * jc + b) + N * (2 * kc + c))
                            for c in range(2) for b in range(2) for a in range(2)]
                    dofs = np.unique(edofs[kids].ravel())
                    dofs = dofs[dofs >= 0]
                    self.children.append(kids)
                    self.blocks_B.append(dofs[isB[dofs]])
                    self.blocks_I.append(dofs[~isB[dofs]])
        # Vertex patches of the coarse mesh.  The patch of vertex v covers the
        # cells v-1 and v on each axis (those that exist); an unknown belongs to
        # it iff its support interval is inside, i.e. hi <= v <= lo + 1 on every
        # axis.  Members are listed by ascending macro index.
        members = [[] for _ in range((Nc + 1) ** 3)]
        for dz in range(2):
            for dy in range(2):
                for dx in range(2):
                    v = hi + np.array([dx, dy, dz])
                    ok = np.all(v <= lo + 1, axis=1) & np.all(v <= Nc, axis=1)
                    vid = (v[:, 2] * (Nc + 1) + v[:, 1]) * (Nc + 1) + v[:, 0]
                    for mi in np.nonzero(ok)[0]:
                        members[vid[mi]].append(mi)
        self.patches = [np.array(sorted(m), dtype=np.int64) for m in members]


def _global_twoscale_h1(Nc, p):
    R = basis1d.twoscale_h1(p)
    G = np.zeros((2 * Nc * p + 1, Nc * p + 1))
    for c in range(Nc):
        # neighbouring cells overlap only in the shared-vertex entry (value 1)
        G[2 * c * p:2 * c * p + 2 * p + 1, c * p:c * p + p + 1] = R
    return G


def _global_twoscale_leg(Nc, p):
    R = basis1d.twoscale_leg(p)
    G = np.zeros((2 * Nc * p, Nc * p))
    for c in range(Nc):
        G[2 * c * p:2 * c * p + 2 * p, c * p:c * p + p] = R
    return G


def prolongation(level, coarse_num):
    """Sparse P [nM, n_trace(coarse mesh)]: natural inclusion onto B rows."""
    p, Nc = level.p, level.Nc
    num = level.num
    R1 = sp.csr_matrix(_global_twoscale_h1(Nc, p))
    R0 = sp.csr_matrix(_global_twoscale_leg(Nc, p))
    # H1 part: full-lattice Kronecker product, X fastest in both index spaces
    K1 = sp.kron(sp.kron(R1, R1), R1).tocsr()          # rows (Z,Y,X), cols (Zc,Yc,Xc)
    Mf, Mc = num.M, coarse_num.M
    fine_rows = np.zeros(level.nM, dtype=np.int64)
    rows_h1, lat_rows = [], []
    for mi, t in enumerate(level.B):
        if level.kind[t] == 0:
            X, Y, Z = level.coord[t]
            rows_h1.append(mi)
            lat_rows.append((Z * (Mf + 1) + Y) * (Mf + 1) + X)
    Zc, Yc, Xc = np.nonzero(coarse_num.h1_index >= 0)
    lat_cols = (Zc * (Mc + 1) + Yc) * (Mc + 1) + Xc
    col_ids = coarse_num.h1_index[Zc, Yc, Xc]
    Ph1 = K1[np.array(lat_rows)][:, lat_cols].tocoo()
    rows = [np.array(rows_h1)[Ph1.row]]
    cols = [col_ids[Ph1.col]]
    vals = [Ph1.data]
    # flux part: in-plane Kronecker product of the Legendre two-scale matrices
    K0 = sp.kron(R0, R0).tocsr()                        # rows (T2,T1), cols (T2c,T1c)
    for mi, t in enumerate(level.B):
        k = level.kind[t]
        if k == 0:
            continue
        d = k - 1
        s, T1, T2 = level.coord[t]
        r = K0.getrow(T2 * Mf + T1)
        for c, v in zip(r.indices, r.data):
            T2c, T1c = divmod(c, Mc)
            rows.append(np.array([mi]))
            cols.append(np.array([coarse_num.flux(d, s // 2, T1c, T2c)]))
            vals.append(np.array([v]))
    P = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(level.nM, coarse_num.n)).tocsr()
    P.eliminate_zeros()
    return P


class OrderLevel:
    """The level of a hierarchy that coarsens the order on one mesh (the
    uniform p-refinements of Sec. 4.2 read as multigrid levels): mesh N,
    order q, next coarser level (N, q - 1).

    Every trace unknown of the mesh stays on the coarse skeleton (the meshes
    coincide), so nothing is condensed: the macro grid is the whole trace
    space, the blocks are the elements (their unknowns in ascending canonical
    order) and the vertex patches are those of the mesh itself -- an unknown
    belongs to the patch of vertex v iff every element its support touches
    contains v.  Attribute names follow MacroLevel."""

    def __init__(self, num):
        N, q = num.N, num.p
        self.num, self.N, self.Nc, self.p = num, N, N, q
        kind, coord = num.describe()
        self.kind, self.coord = kind, coord
        self.B = np.arange(num.n)
        self.macro_of = np.arange(num.n)
        self.nM = num.n
        self.isB = np.ones(num.n, dtype=bool)
        # support intervals (element index per axis), as in MacroLevel with the
        # elements in the place of the coarse cells
        lo = np.zeros((num.n, 3), dtype=np.int64)
        hi = np.zeros((num.n, 3), dtype=np.int64)
        hb = kind == 0
        for a in range(3):
            X = coord[hb, a]
            atv = X % q == 0
            lo[hb, a] = np.where(atv, np.maximum(X // q - 1, 0), X // q)
            hi[hb, a] = np.where(atv, np.minimum(X // q, N - 1), X // q)
        for d in range(3):
            m = kind == d + 1
            ip = [k for k in range(3) if k != d]
            lo[m, d] = coord[m, 0] - 1
            hi[m, d] = coord[m, 0]
            for a, col in ((ip[0], 1), (ip[1], 2)):
                lo[m, a] = coord[m, col] // q
                hi[m, a] = coord[m, col] // q
        edofs = element_dofs(num)
        self.edofs = edofs
        self.children = [[e] for e in range(N ** 3)]
        self.blocks_B = [np.sort(edofs[e][edofs[e] >= 0]) for e in range(N ** 3)]
        self.blocks_I = [np.zeros(0, dtype=np.int64) for _ in range(N ** 3)]
        members = [[] for _ in range((N + 1) ** 3)]
        for dz in range(2):
            for dy in range(2):
                for dx in range(2):
                    v = hi + np.array([dx, dy, dz])
                    ok = np.all(v <= lo + 1, axis=1) & np.all(v <= N, axis=1)
                    vid = (v[:, 2] * (N + 1) + v[:, 1]) * (N + 1) + v[:, 0]
                    for mi in np.nonzero(ok)[0]:
                        members[vid[mi]].append(mi)
        self.patches = [np.array(sorted(m), dtype=np.int64) for m in members]


def order_injection(num, coarse_num):
    """P [n_trace(N, q), n_trace(N, q - 1)]: the natural inclusion of the order
    q - 1 trace space in the order q one on the same mesh.  The hierarchical
    H1 functions (vertex hats and integrated Legendre bubbles) and the
    Legendre flux functions do not depend on the order they belong to, so
    every coarse function is one fine function: lattice coordinate
    X' = (q-1) cell + a' goes to q cell + a' (a' = 0 a vertex, else the same
    bubble), flux in-plane T' = (q-1) cell + m to q cell + m."""
    q = num.p
    assert coarse_num.N == num.N and coarse_num.p == q - 1
    qc = q - 1

    def lat(Xc):
        return q * (Xc // qc) + Xc % qc

    rows, cols = [], []
    Zc, Yc, Xc = np.nonzero(coarse_num.h1_index >= 0)
    rows.append(num.h1_index[lat(Zc), lat(Yc), lat(Xc)])
    cols.append(coarse_num.h1_index[Zc, Yc, Xc])
    for d in range(3):
        for s in range(1, num.N):
            T2c, T1c = np.meshgrid(np.arange(coarse_num.M), np.arange(coarse_num.M),
                                   indexing='ij')
            T1c, T2c = T1c.ravel(), T2c.ravel()
            rows.append(num.flux(d, s, lat(T1c), lat(T2c)))
            cols.append(coarse_num.flux(d, s, T1c, T2c))
    r, c = np.concatenate(rows), np.concatenate(cols)
    assert np.all(r >= 0)
    return sp.coo_matrix((np.ones(r.size), (r, c)), shape=(num.n, coarse_num.n)).tocsr()

