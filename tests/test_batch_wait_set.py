"""Pin the batch kernel's dependency neighbourhoods on the CPU by brute force.

A batch launch runs work items (generation g = 4 * MCS + step, tile t) of a
lattice in any order the queue hands them out, with one rule: item (g, t)
starts once tile t and every tile of okpz_batch_wait_set(...) have finished
generation g - 1 (a per-tile count of finished generations; each tile
finishes its generations in order).  Each item stages the window of its
domain in LDS -- the domain plus its +1 column and row (the bits rim
attempts touch), widened to whole 32 x 4-site blocks -- and writes every
word of it back.  The result equals the device-wide step order of Sec. 3.1
iff every earlier item whose window shares a block with (g, t)'s window is
guaranteed finished when (g, t) starts.  This test computes the windows from
first principles for random origins and domain-set orders (the Sec. 3 DTr
schedule: a fresh origin per MCS, the four sets in some order) and checks
that guarantee, closing the wait rule transitively, against the library's
host export of the function the kernel evaluates.
"""
import itertools

import numpy as np
import pytest


def windows(L, Dx, Dy, ox, oy, sa, sb):
    """Each tile's window in one device step as block rectangles on the torus
    of 32 x 4-site blocks: first block column, columns, first band, bands."""
    ntx, nty = L // (2 * Dx), L // (2 * Dy)
    tx = np.tile(np.arange(ntx), nty)
    ty = np.repeat(np.arange(nty), ntx)
    x0 = (ox + 2 * Dx * tx + sa * Dx) % L
    y0 = (oy + 2 * Dy * ty + sb * Dy) % L
    # sites x0 .. x0 + Dx and rows y0 .. y0 + Dy (the domain and its +1 column / row)
    bx0, nbx = x0 // 32, (x0 + Dx) // 32 - x0 // 32 + 1
    by0, nby = y0 // 4, (y0 + Dy) // 4 - y0 // 4 + 1
    return bx0, nbx, by0, nby


def _arcs_meet(a, n, b, m, N):
    """Arcs [a, a+n) and [b, b+m) of a circle of N points share a point
    (broadcast: a, n over rows, b, m over columns)."""
    a, n = a[:, None], n[:, None]
    b, m = b[None, :], m[None, :]
    return ((b - a) % N < n) | ((a - b) % N < m) | (n >= N) | (m >= N)


def shared_blocks(L, w1, w2):
    """(tiles of w1, tiles of w2) matrix: the two windows share a block."""
    return _arcs_meet(w1[0], w1[1], w2[0], w2[1], L // 32) & _arcs_meet(w1[2], w1[3], w2[2], w2[3], L // 4)


def _windows_by_enumeration(L, Dx, Dy, ox, oy, sa, sb):
    ntx, nty = L // (2 * Dx), L // (2 * Dy)
    out = []
    for ty in range(nty):
        for tx in range(ntx):
            x0 = (ox + 2 * Dx * tx + sa * Dx) % L
            y0 = (oy + 2 * Dy * ty + sb * Dy) % L
            out.append({(((y0 + j) % L) // 4, ((x0 + i) % L) // 32) for j in range(Dy + 1) for i in range(Dx + 1)})
    return out


def test_window_rectangles_equal_enumerated_blocks():
    """The rectangle arithmetic above against plain enumeration of the sites."""
    rng = np.random.default_rng(3)
    for L, Dx, Dy in ((64, 8, 8), (128, 16, 32), (256, 64, 8), (128, 32, 32)):
        for _ in range(4):
            ox, oy, s1, s2 = (int(v) for v in (rng.integers(0, L), rng.integers(0, L), rng.integers(0, 4),
                                               rng.integers(0, 4)))
            o2x, o2y = int(rng.integers(0, L)), int(rng.integers(0, L))
            e1 = _windows_by_enumeration(L, Dx, Dy, ox, oy, s1 & 1, s1 >> 1)
            e2 = _windows_by_enumeration(L, Dx, Dy, o2x, o2y, s2 & 1, s2 >> 1)
            got = shared_blocks(L, windows(L, Dx, Dy, ox, oy, s1 & 1, s1 >> 1),
                                windows(L, Dx, Dy, o2x, o2y, s2 & 1, s2 >> 1))
            want = np.array([[bool(a & b) for b in e2] for a in e1])
            assert np.array_equal(got, want)


def wait_tiles(okpz, L, Dx, Dy, t, new_tiling, ox, oy, oxp, oyp):
    ntx, nty = L // (2 * Dx), L // (2 * Dy)
    cx0, ncol, cy0, nrow = okpz.batch_wait_set(L, Dx, Dy, t, new_tiling, ox, oy, oxp, oyp)
    assert 1 <= ncol <= ntx and 1 <= nrow <= nty and cx0 < ntx and cy0 < nty
    s = {t}
    for j in range(nrow):
        for i in range(ncol):
            s.add(((cy0 + j) % nty) * ntx + (cx0 + i) % ntx)
    return sorted(s)


def draw_origins(rng, L, Dx, Dy, n_mcs):
    """Origins of n_mcs MCS: uniform, but half of the moves put the new tile
    corners in the last word (last band) of an old tile, where a new tile's
    window reaches furthest into the old tiling."""
    out = [(int(rng.integers(0, L)), int(rng.integers(0, L)))]
    for _ in range(n_mcs - 1):
        px, py = out[-1]
        if rng.random() < 0.5:
            dx = 2 * Dx - 1 - int(rng.integers(0, min(32, 2 * Dx)))
            dy = 2 * Dy - 1 - int(rng.integers(0, min(4, 2 * Dy)))
            out.append(((px + dx + 2 * Dx * int(rng.integers(0, L // (2 * Dx)))) % L,
                        (py + dy + 2 * Dy * int(rng.integers(0, L // (2 * Dy)))) % L))
        else:
            out.append((int(rng.integers(0, L)), int(rng.integers(0, L))))
    return out


def check_launch(okpz, rng, L, Dx, Dy, n_mcs, last_first=None):
    """One launch of n_mcs MCS; last_first = (s, s') forces the set of the last
    step of MCS 0 and of the first step of MCS 1."""
    ntiles = (L // (2 * Dx)) * (L // (2 * Dy))
    origins = draw_origins(rng, L, Dx, Dy, n_mcs)
    orders = [list(rng.permutation(4)) for _ in range(n_mcs)]
    if last_first is not None:
        for order, want, pos in ((orders[0], last_first[0], 3), (orders[1], last_first[1], 0)):
            i = order.index(want)
            order[i], order[pos] = order[pos], order[i]
    gens = []  # (origin, set) per generation
    for m in range(n_mcs):
        for k in range(4):
            gens.append((origins[m], orders[m][k]))
    win = [windows(L, Dx, Dy, o[0], o[1], s & 1, s >> 1) for o, s in gens]
    # done[g][t, t'] = every generation <= done of tile t' has finished when (g, t) starts
    # (-1: nothing guaranteed); generation 0 of a launch starts after the previous launch
    done = [np.full((ntiles, ntiles), -1, dtype=np.int64)]
    for g in range(1, len(gens)):
        d = np.full((ntiles, ntiles), -1, dtype=np.int64)
        new_tiling = g % 4 == 0
        (ox, oy), (oxp, oyp) = gens[g][0], gens[g - 1][0]
        for t in range(ntiles):
            for u in wait_tiles(okpz, L, Dx, Dy, t, new_tiling, ox, oy, oxp, oyp):
                # u finished g - 1, hence all its earlier generations, and all that
                # its own item of generation g - 1 was guaranteed when it started
                np.maximum(d[t], done[g - 1][u], out=d[t])
                d[t, u] = max(d[t, u], g - 1)
        done.append(d)
        # every earlier item sharing a block with (g, t) must be guaranteed finished
        for gp in range(g):
            share = shared_blocks(L, win[g], win[gp])
            t_idx, u_idx = np.nonzero(share)
            bad = d[t_idx, u_idx] < gp
            assert not bad.any(), (L, Dx, Dy, g, gp, t_idx[bad][:4], u_idx[bad][:4])


# small lattices (every tile waits for every other) and lattices with more
# tiles per row and column than a wait set spans, where a missing tile shows
CASES = [(64, 8, 8), (64, 16, 16), (64, 32, 32), (128, 8, 16), (128, 16, 8), (128, 32, 16),
         (128, 64, 64), (256, 16, 16), (256, 32, 64), (256, 64, 32), (256, 128, 128), (512, 256, 256),
         (512, 32, 32), (256, 8, 32), (256, 8, 8), (512, 16, 16), (1024, 32, 32), (1024, 64, 16),
         (2048, 64, 64)]


@pytest.mark.parametrize("L,Dx,Dy", CASES)
def test_wait_sets_cover_every_conflict(okpz, L, Dx, Dy):
    rng = np.random.default_rng(L * 1000 + Dx * 10 + Dy)
    for last, first in itertools.product(range(4), range(4)):  # every set pair across an MCS boundary
        check_launch(okpz, rng, L, Dx, Dy, n_mcs=2, last_first=(last, first))
    check_launch(okpz, rng, L, Dx, Dy, n_mcs=3)


def test_wait_set_is_tight_enough(okpz):
    """Inside one tiling a D >= 32 tile waits for its 3 x 3 neighbours only
    (so the steps of one lattice overlap across its tiles)."""
    for L, D in ((256, 32), (512, 64), (1024, 256)):
        ntx = L // (2 * D)
        for t in (0, ntx + 1, ntx * ntx - 1):
            assert len(wait_tiles(okpz, L, D, D, t, False, 0, 0, 0, 0)) == min(9, ntx * ntx)


def test_wait_set_rejects_bad_arguments(okpz):
    for args in ((96, 16, 16, 0), (64, 16, 16, 4), (64, 64, 16, 0), (64, 12, 16, 0)):
        with pytest.raises(okpz.OkpzError):
            okpz.batch_wait_set(*args)
    with pytest.raises(okpz.OkpzError):
        okpz.batch_wait_set(64, 16, 16, 0, True, 64, 0, 0, 0)
