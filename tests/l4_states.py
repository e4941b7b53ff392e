"""Brute-force state space of the 4x4 periodic octahedron surface.

Independent of the oracle: works on height functions directly.  A valid surface
is a height function h on the L x L torus with h(0,0) = 0 whose nearest
neighbours differ by exactly 1 (Sec. 2.1: octahedra edges are +-1 slopes).
Slopes follow the bit convention of the slope lattice gas: sx[x,y] = 1 iff
h(x,y) - h(x-1,y) = +1, sy[x,y] = 1 iff h(x,y) - h(x,y-1) = +1.
"""
from __future__ import annotations

import numpy as np


def enumerate_heights(L: int = 4):
    """All height functions with h(0,0) = 0 and |h(r) - h(r')| = 1 for neighbours."""
    sites = [(x, y) for y in range(L) for x in range(L)]
    h = {}
    out = []

    def ok(x, y, v):
        for nx, ny in (((x - 1) % L, y), ((x + 1) % L, y), (x, (y - 1) % L), (x, (y + 1) % L)):
            if (nx, ny) in h and abs(h[(nx, ny)] - v) != 1:
                return False
        return True

    def rec(i):
        if i == len(sites):
            out.append(np.array([[h[(x, y)] for x in range(L)] for y in range(L)], dtype=np.int64))
            return
        x, y = sites[i]
        if i == 0:
            cands = [0]
        elif x > 0:
            cands = [h[(x - 1, y)] - 1, h[(x - 1, y)] + 1]
        else:
            cands = [h[(x, y - 1)] - 1, h[(x, y - 1)] + 1]
        for v in cands:
            if ok(x, y, v):
                h[(x, y)] = v
                rec(i + 1)
                del h[(x, y)]

    rec(0)
    return out


def slopes_from_heights(h: np.ndarray) -> np.ndarray:
    dx = h - np.roll(h, 1, axis=1)
    dy = h - np.roll(h, 1, axis=0)
    assert np.all(np.abs(dx) == 1) and np.all(np.abs(dy) == 1)
    return ((dx == 1).astype(np.uint8) | ((dy == 1).astype(np.uint8) << 1)).copy()


def height_rule(h: np.ndarray, x: int, y: int, dep_ok: bool, rem_ok: bool) -> np.ndarray:
    """The octahedron move on heights: a site lower than all four neighbours
    gains 2 (deposition), one higher than all four loses 2 (removal)."""
    L = h.shape[0]
    nb = [h[y, (x - 1) % L], h[y, (x + 1) % L], h[(y - 1) % L, x], h[(y + 1) % L, x]]
    g = h.copy()
    if all(v > h[y, x] for v in nb) and dep_ok:
        g[y, x] += 2
    elif all(v < h[y, x] for v in nb) and rem_ok:
        g[y, x] -= 2
    return g - g[0, 0]


def w2_of_heights(h: np.ndarray) -> float:
    """Sec. 2.1 roughness: mean of h^2 minus the squared mean."""
    n = h.size
    s1 = int(h.sum())
    s2 = int((h * h).sum())
    return (n * s2 - s1 * s1) / (n * n)


def w2_sub_of_heights(h: np.ndarray) -> float:
    L = h.shape[0]
    par = (np.add.outer(np.arange(L), np.arange(L)) & 1).astype(bool)
    out = 0.0
    for cls in (False, True):
        v = h[par == cls]
        n = v.size
        out += (n * int((v * v).sum()) - int(v.sum()) ** 2) / (n * n)
    return out / 2


class StateSpace:
    """Index of the 990 states of the 4x4 torus and the exact RS master equation."""

    def __init__(self, L: int = 4):
        self.L = L
        self.heights = enumerate_heights(L)
        self.slopes = [slopes_from_heights(h) for h in self.heights]
        self.index = {s.tobytes(): i for i, s in enumerate(self.slopes)}

    def __len__(self):
        return len(self.heights)

    def attempt_matrix(self, p: float, q: float) -> np.ndarray:
        """Transition matrix of one RS attempt at a uniformly chosen site."""
        n, L = len(self), self.L
        T = np.zeros((n, n))
        for i, h in enumerate(self.heights):
            for y in range(L):
                for x in range(L):
                    up = height_rule(h, x, y, True, False)
                    dn = height_rule(h, x, y, False, True)
                    j_up = self.index[slopes_from_heights(up).tobytes()]
                    j_dn = self.index[slopes_from_heights(dn).tobytes()]
                    w = 1.0 / (L * L)
                    if j_up != i:
                        T[i, j_up] += w * p
                        T[i, i] += w * (1 - p)
                    elif j_dn != i:
                        T[i, j_dn] += w * q
                        T[i, i] += w * (1 - q)
                    else:
                        T[i, i] += w
        return T

    def flat_index(self) -> int:
        L = self.L
        h = (np.add.outer(np.arange(L), np.arange(L)) & 1).astype(np.int64)
        return self.index[slopes_from_heights(h).tobytes()]


def site_kernels(space: "StateSpace", p: float, q: float):
    """Sparse one-attempt kernel for each site (x, y) of the 4x4 torus."""
    import scipy.sparse as sp

    n, L = len(space), space.L
    out = {}
    for y in range(L):
        for x in range(L):
            rows, cols, vals = [], [], []
            for i, h in enumerate(space.heights):
                up = space.index[slopes_from_heights(height_rule(h, x, y, True, False)).tobytes()]
                dn = space.index[slopes_from_heights(height_rule(h, x, y, False, True)).tobytes()]
                if up != i:
                    rows += [i, i]; cols += [up, i]; vals += [p, 1 - p]
                elif dn != i:
                    rows += [i, i]; cols += [dn, i]; vals += [q, 1 - q]
                else:
                    rows.append(i); cols.append(i); vals.append(1.0)
            out[(x, y)] = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    return out


def dtr_tiny_evolve(space: "StateSpace", P: np.ndarray, kernels, D: int = 2) -> np.ndarray:
    """Exact one-MCS evolution of the distribution P under DTr with one tile
    covering the 4x4 torus, domains of D x D = 2 x 2 sites and single-hit
    rounds on 2 x 2 cells: the origin is uniform over the 16 sites, the order
    of the four domain sets uniform over the 24 permutations, and each of a
    step's D*D rounds makes one attempt at a uniformly chosen site of the
    active domain (Sec. 3, DTr; Sec. 3.1)."""
    import itertools

    L = space.L
    total = np.zeros_like(P)
    perms = list(itertools.permutations(range(4)))
    for oy in range(L):
        for ox in range(L):
            for perm in perms:
                v = P.copy()
                for k in range(4):
                    a, b = perm[k] & 1, perm[k] >> 1
                    sites = [((ox + a * D + u) % L, (oy + b * D + w) % L)
                             for w in range(D) for u in range(D)]
                    for _ in range(D * D):
                        v = sum(kernels[s_].T @ v for s_ in sites) / len(sites)
                total += v
    return total / (L * L * len(perms))
