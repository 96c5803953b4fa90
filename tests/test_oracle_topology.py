"""Pins of the oracle's numbering, macro grids, patches and prolongation."""
from collections import Counter

import numpy as np
import pytest

from oracle import basis1d, topology


def _count_trace_bruteforce(N, p):
    M = N * p
    h1 = sum(1 for X in range(M + 1) for Y in range(M + 1) for Z in range(M + 1)
             if X % p == 0 or Y % p == 0 or Z % p == 0)
    return h1 + 3 * (N - 1) * M * M


@pytest.mark.parametrize("N,p", [(1, 1), (2, 2), (3, 3), (4, 2)])
def test_trace_count_formula(N, p):
    assert topology.n_trace(N, p) == _count_trace_bruteforce(N, p)
    assert topology.Numbering(N, p).n == topology.n_trace(N, p)


def test_trace_counts_of_the_workloads():
    assert [topology.n_trace(N, p) for N, p in ((4, 2), (16, 3), (32, 4), (24, 3))] == \
        [1241, 188561, 2785665, 636121]


@pytest.mark.parametrize("N,p", [(2, 2), (3, 1), (3, 3)])
def test_element_maps_cover_and_share_correctly(N, p):
    num = topology.Numbering(N, p)
    ed = topology.element_dofs(num)
    cnt = Counter(ed[ed >= 0].ravel().tolist())
    assert len(cnt) == num.n                                 # every unknown is used
    kind, coord = num.describe()
    for t, c in cnt.items():
        if kind[t] > 0:
            assert c == 2                                    # a flux lives on one interior face
        else:
            X, Y, Z = coord[t]
            # number of elements sharing the H1 function at this lattice point
            mult = 1
            for v in (X, Y, Z):
                mult *= 2 if (v % p == 0 and 0 < v < N * p) else 1
            assert c == mult
    # no element lists an unknown twice
    for row in ed:
        r = row[row >= 0]
        assert r.size == np.unique(r).size


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_macro_block_sizes_closed_form(p):
    N = 4
    lv = topology.MacroLevel(topology.Numbering(N, p))
    nB = (2 * p + 1) ** 3 - (2 * p - 1) ** 3 + 24 * p * p
    nI = (2 * p - 1) ** 3 - 8 * (p - 1) ** 3 + 12 * p * p
    # N = 4: all 8 coarse elements touch 3 Gamma faces, each losing 4 p^2 fluxes
    assert {len(b) for b in lv.blocks_B} == {nB - 12 * p * p}
    assert {len(b) for b in lv.blocks_I} == {nI}
    lv8 = topology.MacroLevel(topology.Numbering(8, p))
    sizes = Counter(len(b) for b in lv8.blocks_B)
    assert sizes == {nB: 8, nB - 4 * p * p: 24, nB - 8 * p * p: 24, nB - 12 * p * p: 8}


def test_macro_and_patch_distribution_at_16_cubed_order_3():
    lv = topology.MacroLevel(topology.Numbering(16, 3))
    assert lv.nM == 102033
    assert Counter(len(b) for b in lv.blocks_B) == {326: 8, 362: 72, 398: 216, 434: 216}
    # interior vertex patch: (4p-1)^3 - (4p-2)^3 pressure unknowns on the three
    # inner planes of the 2x2x2 coarse block, plus 48 p^2 fluxes on them.  A
    # vertex next to Gamma also takes the Gamma-face unknowns of its boundary
    # cells, so the interior size holds for vertices 2..Nc-2 on each axis.
    assert Counter(len(x) for x in lv.patches)[11 ** 3 - 10 ** 3 + 48 * 9] == 5 ** 3
    assert len(lv.patches) == 9 ** 3


@pytest.mark.parametrize("N,p", [(2, 1), (4, 2), (6, 1), (4, 3)])
def test_patches_match_bruteforce_support_definition(N, p):
    """d is in patch(v) iff every coarse cell touched by d's support has vertex v."""
    num = topology.Numbering(N, p)
    lv = topology.MacroLevel(num)
    ed = topology.element_dofs(num)
    Nc = N // 2
    touched = [set() for _ in range(num.n)]
    for e in range(N ** 3):
        i, j, k = e % N, (e // N) % N, e // (N * N)
        for t in ed[e][ed[e] >= 0]:
            touched[t].add((i // 2, j // 2, k // 2))
    for vid, members in enumerate(lv.patches):
        vx, vy, vz = vid % (Nc + 1), (vid // (Nc + 1)) % (Nc + 1), vid // (Nc + 1) ** 2
        cells = {(a, b, c) for a in (vx - 1, vx) for b in (vy - 1, vy) for c in (vz - 1, vz)}
        ref = [m for m, t in enumerate(lv.B) if touched[t] <= cells]
        assert list(members) == ref


def _eval_h1(num, x, pt):
    """Value of the H1 trace field with coefficients x at a physical point pt."""
    N, p = num.N, num.p
    val = 0.0
    cell, loc = [], []
    for a in range(3):
        c = min(int(pt[a] * N), N - 1)
        cell.append(c)
        loc.append(basis1d.h1(p, np.array([2 * (pt[a] * N - c) - 1]))[:, 0])
    for cz in range(p + 1):
        for cy in range(p + 1):
            for cx in range(p + 1):
                idx = num.h1(cell[0] * p + cx, cell[1] * p + cy, cell[2] * p + cz)
                if idx >= 0:
                    val = val + x[idx] * loc[0][cx] * loc[1][cy] * loc[2][cz]
    return val


def _eval_flux(num, x, d, s, pt):
    """Value of the family-d flux field on plane s at a physical point pt of it."""
    N, p = num.N, num.p
    ip = [q for q in range(3) if q != d]
    c1, c2 = (min(int(pt[a] * N), N - 1) for a in ip)
    L1 = basis1d.legendre(p, np.array([2 * (pt[ip[0]] * N - c1) - 1]))[:, 0]
    L2 = basis1d.legendre(p, np.array([2 * (pt[ip[1]] * N - c2) - 1]))[:, 0]
    return sum(x[num.flux(d, s, c1 * p + m, c2 * p + n)] * L1[m] * L2[n]
               for m in range(p) for n in range(p))


@pytest.mark.parametrize("N,p", [(4, 1), (4, 2), (4, 3)])
def test_prolongation_is_exact_inclusion_on_coarse_skeleton(N, p):
    rng = np.random.default_rng(N + p)
    num = topology.Numbering(N, p)
    cnum = topology.Numbering(N // 2, p)
    lv = topology.MacroLevel(num)
    P = topology.prolongation(lv, cnum)
    xc = rng.standard_normal(cnum.n)
    xf = np.zeros(num.n)
    xf[lv.B] = P @ xc
    Nc = N // 2
    for _ in range(40):
        pt = rng.uniform(0, 1, 3)
        a = rng.integers(3)
        pt[a] = rng.integers(0, Nc + 1) / Nc              # a point on a coarse plane
        assert abs(_eval_h1(num, xf, pt) - _eval_h1(cnum, xc, pt)) < 1e-12
        S = rng.integers(1, Nc)                            # interior coarse plane
        pt[a] = S / Nc
        assert abs(_eval_flux(num, xf, a, 2 * S, pt) - _eval_flux(cnum, xc, a, S, pt)) < 1e-12
