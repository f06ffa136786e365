"""Pins of the quadtree relations (Section 3.3.1, Fig. 6-8) and leaf convention."""
import itertools

import numpy as np
import pytest

from oracle import quadtree as qt


def test_box_counts_and_sides():
    root = (0.0, 0.0, 2.0)
    for lev in range(6):
        assert (1 << lev) ** 2 == 4 ** lev  # Fig. 6: 4^l boxes at level l
        assert qt.box_side(root, lev) == 2.0 / 2 ** lev


def test_neighbour_counts():
    lev = 3
    m = 8
    counts = {}
    for ix, iy in itertools.product(range(m), range(m)):
        n = len(qt.neighbours(lev, ix, iy))
        edge = (ix in (0, m - 1)) + (iy in (0, m - 1))
        counts.setdefault(edge, set()).add(n)
    assert counts == {0: {8}, 1: {5}, 2: {3}}  # "at most 8 neighbours"


def test_interaction_list_shapes():
    lev = 4
    offs = set()
    for ix, iy in itertools.product(range(4, 12), range(4, 12)):
        il = qt.interaction_list(lev, ix, iy)
        assert len(il) == 27  # interior boxes: 6x6 children minus 3x3 local list
        for sx, sy in il:
            d = (ix - sx, iy - sy)
            assert max(abs(d[0]), abs(d[1])) in (2, 3)
            offs.add(d)
    assert len(offs) == 40  # [-3,3]^2 minus [-1,1]^2
    assert qt.interaction_list(1, 0, 0) == [] and qt.interaction_list(0, 0, 0) == []
    # level 2: all boxes not adjacent to the target
    for ix, iy in itertools.product(range(4), range(4)):
        il = set(qt.interaction_list(2, ix, iy))
        want = {(a, b) for a in range(4) for b in range(4) if max(abs(a - ix), abs(b - iy)) > 1}
        assert il == want


@pytest.mark.parametrize("levels", [2, 3, 4, 5])
def test_list_cover_invariant(levels):
    """Every (target leaf, source leaf) pair is covered exactly once: by the leaf
    local list, or by one interaction-list pair of their ancestors."""
    m = 1 << levels
    cover = np.zeros((m * m, m * m), np.int32)
    for ix, iy in itertools.product(range(m), range(m)):
        t = iy * m + ix
        for sx, sy in qt.local_list(levels, ix, iy):
            cover[t, sy * m + sx] += 1
    for lev in range(2, levels + 1):
        sh = levels - lev
        for bx, by in itertools.product(range(1 << lev), range(1 << lev)):
            for sx, sy in qt.interaction_list(lev, bx, by):
                tl = [(tx, ty) for tx in range(bx << sh, (bx + 1) << sh) for ty in range(by << sh, (by + 1) << sh)]
                sl = [(ux, uy) for ux in range(sx << sh, (sx + 1) << sh) for uy in range(sy << sh, (sy + 1) << sh)]
                for tx, ty in tl:
                    for ux, uy in sl:
                        cover[ty * m + tx, uy * m + ux] += 1
    assert np.all(cover == 1)


def test_leaf_convention_hand_placed():
    # root [0, 4)^2 given explicitly, level 2: unit boxes
    root = (0.0, 0.0, 4.0)
    x = np.array([0.5, 1.0, 3.999, 4.0, 0.0, 2.0, -0.1])
    y = np.array([0.5, 2.5, 0.2, 4.0, 3.0, 2.0, 5.0])
    ix, iy = qt.leaf_coords(x, y, root, 2)
    assert list(ix) == [0, 1, 3, 3, 0, 2, 0]   # edges go to the upper box, max clamps
    assert list(iy) == [0, 2, 0, 3, 3, 2, 3]
    assert qt.box_centre(root, 2, 1, 2) == complex(1.5, 2.5)


def test_root_square_bounding():
    x = np.array([-1.0, 3.0, 0.0]); y = np.array([0.0, 1.0, 2.0])
    x0, y0, s = qt.root_square(x, y)
    assert s == 4.0 * (1 + 2.0 ** -20)
    assert x0 + s / 2 == 1.0 and y0 + s / 2 == 1.0
    ix, iy = qt.leaf_coords(x, y, (x0, y0, s), 3)
    assert ix.min() >= 0 and ix.max() <= 7 and iy.min() >= 0 and iy.max() <= 7
    # degenerate extent: unit root
    assert qt.root_square(np.array([2.0]), np.array([3.0]))[2] == 1.0
