"""FMM on an adaptive (non-uniform) quadtree: leaves at the depth that the local
particle density asks for.

Test infrastructure (see ``oracle/__init__``).

The paper builds uniform trees (Section 3.3, Fig. 6: every leaf at level l).
On clustered particles most of the near-field work sits in a few dense leaves
while many leaves are empty or nearly so.  The adaptive tree subdivides a box
only while it holds more than ``s`` particles, down to a deepest level ``Lmax``.
How the paper's method runs on such a tree is not stated; this module's
reading, followed by the GPU path as well:

* tree: the root (level 0) is split; a box of level l < Lmax holding more than
  s particles is split into its four children; a box that is not split and
  whose parent was split is a leaf (boxes holding no particle included, which
  carry no work);
* near field of a particle (eq. 10, first sum): the regularised kernel (eq. 6)
  over the particles of its leaf's local list taken at the leaf's own level
  l -- the 3 x 3 boxes of level l around the leaf (Section 3.3.1), whatever
  the tree does inside them (split boxes, parts of larger leaves);
* far field: the L2P of the leaf's local expansion, which is formed exactly as
  in the uniform method of depth l: M2L over the interaction lists of the leaf
  and of its ancestors at levels 2 .. l (eq. 22), L2L down the ancestors
  (Section 3.3.3).  The multipole expansion of any box is the one of the
  particles it contains (P2M at level Lmax, M2M upward; M2M is exact), so a
  box of an interaction list that lies inside a larger leaf, or that is split
  further, contributes its own particles;
* distance cut-off (optional radius a > 0, Section 4.1's distance): particles
  outside the leaf's local list and closer than a are summed with the
  regularised kernel (the correction Gamma (K_sigma - K')), a being clamped to
  four sides of the target's leaf, as in the uniform method.

Per target this is the uniform method of depth l, the level of its leaf: the
tree chooses l region by region.  (Near is therefore decided on the target's
side: a particle in a small leaf may be far for a neighbour in a large leaf
that is near to it.)  Every pair is covered exactly once, by the local list of
the target's leaf or by one interaction list of the leaf or one of its
ancestors (tested).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import fmm as F
from . import quadtree as qt
from .kernel import regularized_kernel, singular_kernel

MAX_RINGS = 4  # the cut-off radius is clamped to MAX_RINGS sides of the target's leaf


@dataclasses.dataclass
class AdaptiveTree:
    root: tuple
    lmax: int
    s: int
    leaves: list          # (level, ix, iy, count), every leaf of the tree
    level: np.ndarray     # per particle: level of its leaf
    bx: np.ndarray        # per particle: leaf coordinates at that level
    by: np.ndarray


def build_adaptive(x, y, lmax, s, domain=None) -> AdaptiveTree:
    """The tree of the reading above: a box is split while it holds more than
    s particles and lies above level lmax."""
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64)
    root = qt.root_square(x, y, domain)
    coords = [qt.leaf_coords(x, y, root, l) for l in range(lmax + 1)]
    counts = []
    for l in range(lmax + 1):
        ix, iy = coords[l]
        m = 1 << l
        counts.append(np.bincount(iy * m + ix, minlength=m * m).reshape(m, m))
    level = np.full(x.shape[0], -1, np.int64)
    leaves = []
    stack = [(0, 0, 0)]
    while stack:
        l, ix, iy = stack.pop()
        n = int(counts[l][iy, ix])
        if n > s and l < lmax:
            stack.extend((l + 1, cx, cy) for cx, cy in qt.children(ix, iy))
            continue
        leaves.append((l, ix, iy, n))
        if n:
            cx, cy = coords[l]
            level[(cx == ix) & (cy == iy)] = l
    assert np.all(level >= 0)
    bx = np.array([coords[l][0][i] for i, l in enumerate(level)], np.int64)
    by = np.array([coords[l][1][i] for i, l in enumerate(level)], np.int64)
    return AdaptiveTree(root, lmax, s, sorted(leaves), level, bx, by)


def leaf_radius(radius, root, level):
    """The cut-off radius used for targets in a leaf of ``level``."""
    if radius <= 0.0:
        return 0.0
    return min(radius, MAX_RINGS * qt.box_side(root, level))


def fmm_velocity_adaptive(x, y, gamma, sigma, p, lmax, s, domain=None, targets=None,
                          radius=0.0) -> F.FMMResult:
    """The FMM of the reading above at all particles (or at ``targets``)."""
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64)
    gamma = np.asarray(gamma, np.float64)
    z = x + 1j * y
    at = build_adaptive(x, y, lmax, s, domain)
    root = at.root
    tidx = np.arange(len(x)) if targets is None else np.asarray(targets, np.int64)
    # multipoles of every box of levels 2 .. lmax: the uniform upward sweep
    ut = F.build_tree(x, y, lmax, domain=root)
    me = F.upward_sweep(z, gamma, ut, p) if lmax >= 2 else {}
    nu = np.zeros(len(tidx)); nv = np.zeros(len(tidx))
    fu = np.zeros(len(tidx)); fv = np.zeros(len(tidx))
    groups = {}
    for k, i in enumerate(tidx):
        groups.setdefault((int(at.level[i]), int(at.bx[i]), int(at.by[i])), []).append(k)
    trees = {}
    for (l, bx, by), ks in sorted(groups.items()):
        ks = np.asarray(ks, np.int64)
        ti = tidx[ks]
        if l not in trees:
            trees[l] = F.build_tree(x, y, l, domain=root)
        tl = trees[l]
        # far field: the local expansion of the leaf at its level
        if l >= 2:
            le = F.downward_sweep(me, dataclasses.replace(ut, levels=l), p, {(bx, by)})
            w = F.l2p(le[l][(bx, by)], qt.box_centre(root, l, bx, by), z[ti])
            fu[ks] = w.real
            fv[ks] = -w.imag
        # near field: the 3 x 3 boxes of level l around the leaf
        src = [tl.members[b] for b in qt.local_list(l, bx, by) if b in tl.members]
        sj = np.concatenate(src)
        ku, kv = regularized_kernel(x[ti, None] - x[None, sj], y[ti, None] - y[None, sj], sigma)
        self_mask = ti[:, None] == sj[None, :]
        ku[self_mask] = 0.0; kv[self_mask] = 0.0
        nu[ks] = ku @ gamma[sj]
        nv[ks] = kv @ gamma[sj]
        rl = leaf_radius(radius, root, l)
        if rl > 0.0:
            cu, cv = F.cutoff_correction(x, y, gamma, sigma, tl, x[ti], y[ti],
                                         np.full(len(ti), bx), np.full(len(ti), by), rl)
            nu[ks] += cu; nv[ks] += cv
    return F.FMMResult(nu + fu, nv + fv, nu, nv, fu, fv, tidx, ut)


def hybrid_velocity_adaptive(x, y, gamma, sigma, lmax, s, domain=None, targets=None, radius=0.0):
    """The p -> infinity limit of ``fmm_velocity_adaptive``: the regularised
    kernel for sources in the local list of the target's leaf (at the leaf's
    level) or closer than the leaf's cut-off radius, the singular kernel
    (eq. 27) for every other source."""
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64)
    g = np.asarray(gamma, np.float64)
    at = build_adaptive(x, y, lmax, s, domain)
    coords = [qt.leaf_coords(x, y, at.root, l) for l in range(lmax + 1)]
    tidx = np.arange(len(x)) if targets is None else np.asarray(targets, np.int64)
    u = np.zeros(len(tidx)); v = np.zeros(len(tidx))
    for k, i in enumerate(tidx):
        l = int(at.level[i])
        cx, cy = coords[l]
        near = (np.abs(cx - at.bx[i]) <= 1) & (np.abs(cy - at.by[i]) <= 1)
        dx = x[i] - x; dy = y[i] - y
        rl = leaf_radius(radius, at.root, l)
        if rl > 0.0:
            near = near | (dx * dx + dy * dy < rl * rl)
        ru, rv = regularized_kernel(dx, dy, sigma)
        su, sv = singular_kernel(dx, dy)
        ku = np.where(near, ru, su); kv = np.where(near, rv, sv)
        ku[i] = 0.0; kv[i] = 0.0
        u[k] = ku @ g; v[k] = kv @ g
    return u, v


def covering(at: AdaptiveTree, tl, tx, ty, sx, sy):
    """How the pair (target leaf (tl, tx, ty), source box (sx, sy) of level
    lmax) is covered: ("near", l) if the source lies in the local list of the
    target's leaf, ("far", k) for each level k in 2 .. tl at which the source's
    level-k box is in the interaction list of the target's level-k ancestor.
    A correct reading covers every pair exactly once."""
    out = []
    d = at.lmax - tl
    if abs((sx >> d) - tx) <= 1 and abs((sy >> d) - ty) <= 1:
        out.append(("near", tl))
    for k in range(2, tl + 1):
        ax, ay = tx >> (tl - k), ty >> (tl - k)
        bxk, byk = sx >> (at.lmax - k), sy >> (at.lmax - k)
        if (bxk, byk) in qt.interaction_list(k, ax, ay):
            out.append(("far", k))
    return out
