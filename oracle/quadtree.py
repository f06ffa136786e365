"""Uniform quadtree geometry (Section 3.3, Fig. 6-8).

Test infrastructure (see ``oracle/__init__``).

Level 0 is the root box holding the whole domain; each box splits into four,
so level l has 4^l boxes of side w_l = S / 2^l (Fig. 6).  Boxes are addressed by
integer coordinates (ix, iy), 0 <= ix, iy < 2^l.

Relations (Section 3.3.1):

* parent of (ix, iy) at level l is (ix // 2, iy // 2) at level l - 1;
* neighbours: same-level boxes sharing at least one boundary point (at most 8);
* local list: the box itself plus its neighbours;
* interaction list: children of the parent's neighbours that are not in the
  local list.

Readings of what the paper leaves open:

* root box: the bounding square of the particles, side
  S = max(x-extent, y-extent) (1 + 2^-20), centred on the bounding-box
  midpoint; S = 1 when the extent is zero; a caller may give (x0, y0, S) instead;
* leaf of a particle: ix = clamp(floor(((x - x0) / S) * 2^L), 0, 2^L - 1), the
  same for y (a particle on a box edge goes to the upper/right box);
* expansion centre: the geometric box centre x0 + (ix + 1/2) w_l;
* "children of the parent's neighbours" taken without the parent itself; the
  parent's own children are the box and its siblings, which are all in the
  local list, so the list is the same either way;
* the interaction list is empty at levels 0 and 1.
"""
from __future__ import annotations

import numpy as np


def root_square(x, y, domain=None):
    """Root box as (x0, y0, S): lower-left corner and side length."""
    if domain is not None:
        x0, y0, s = (float(v) for v in domain)
        return x0, y0, s
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64)
    xmin = float(x.min()); xmax = float(x.max())
    ymin = float(y.min()); ymax = float(y.max())
    ext = max(xmax - xmin, ymax - ymin)
    s = ext * (1.0 + 2.0 ** -20) if ext > 0.0 else 1.0
    x0 = 0.5 * (xmin + xmax) - 0.5 * s
    y0 = 0.5 * (ymin + ymax) - 0.5 * s
    return x0, y0, s


def leaf_coords(x, y, root, level):
    """Integer box coordinates (ix, iy) at ``level`` of every particle."""
    x0, y0, s = root
    m = 1 << level
    scale = float(m)
    ix = np.floor((np.asarray(x, np.float64) - x0) / s * scale)
    iy = np.floor((np.asarray(y, np.float64) - y0) / s * scale)
    ix = np.clip(ix, 0, m - 1).astype(np.int64)
    iy = np.clip(iy, 0, m - 1).astype(np.int64)
    return ix, iy


def box_side(root, level):
    return root[2] / float(1 << level)


def box_centre(root, level, ix, iy):
    """Geometric centre of box (ix, iy) at ``level`` as a complex number."""
    x0, y0, _ = root
    w = box_side(root, level)
    return complex(x0 + (ix + 0.5) * w, y0 + (iy + 0.5) * w)


def in_range(level, ix, iy):
    m = 1 << level
    return 0 <= ix < m and 0 <= iy < m


def parent(ix, iy):
    return ix // 2, iy // 2


def children(ix, iy):
    return [(2 * ix + a, 2 * iy + b) for b in (0, 1) for a in (0, 1)]


def neighbours(level, ix, iy):
    """Same-level boxes sharing a boundary point with (ix, iy)."""
    out = []
    for jy in (iy - 1, iy, iy + 1):
        for jx in (ix - 1, ix, ix + 1):
            if (jx, jy) != (ix, iy) and in_range(level, jx, jy):
                out.append((jx, jy))
    return out


def local_list(level, ix, iy):
    """The box itself plus its neighbours."""
    return [(ix, iy)] + neighbours(level, ix, iy)


def interaction_list(level, ix, iy):
    """Children of the parent's neighbours, minus the local list."""
    if level < 2:
        return []
    px, py = parent(ix, iy)
    local = set(local_list(level, ix, iy))
    out = []
    for nx, ny in neighbours(level - 1, px, py):
        for c in children(nx, ny):
            if c not in local:
                out.append(c)
    return out
