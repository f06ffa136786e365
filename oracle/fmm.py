"""Reference FMM for the velocity of N vortex particles, in the paper's notation.

Test infrastructure (see ``oracle/__init__``).  Plain float64 NumPy, complex
arithmetic, unscaled coefficients, explicit loops over boxes.

The method (Cruz & Barba 2008, Sections 3.1-3.3):

* far-field kernel in complex form: the conjugate velocity of a point vortex
  is [u(y)]* = -(j / 2 pi) Gamma / (y - x) (eq. 14-16, sign read as in eq. 20,
  which is the sign that agrees with eq. 6);
* P2M, eq. 20-21: a_m = sum_i c_i (x_i - x_*)^m, c_i = -j Gamma_i / (2 pi),
  m = 0 .. p-1, and [u(y)]* ~ sum_m a_m (y - x_*)^(-m-1);
* M2M, Section 3.3.2: shifting a child expansion by t = x_parent - x_child,
  a'_n = sum_{k<=n} (-1)^(n-k) C(n, k) t^(n-k) a_k (the binomial re-centring
  whose first lines the paper prints; its last line drops the t power);
* M2L, eq. 22: b_n = sum_k (-1)^n C(n+k, k) t^-(k+n+1) a_k with
  t = target centre - source centre;
* L2L, Section 3.3.3: b'_n = sum_{k>=n} C(k, n) t^(k-n) b_k with
  t = child centre - parent centre;
* L2P: [u(y)]* ~ sum_n b_n (y - c)^n;
* P2P: eq. 10 first sum, the regularised kernel of eq. 6 over the local list;
* sweeps (Section 3.1, Fig. 3): P2M at the leaves (level L), M2M for levels
  L-1 .. 2, then for levels 2 .. L the LE of each box is the L2L-shifted LE of
  its parent (from level 3 on) plus the M2L of every box of its interaction
  list; finally L2P at the leaves plus P2P.

Distance cut-off (optional, ``radius`` > 0): Section 4.1 bounds the error of
using the singular kernel for far pairs by the distance a between them; with a
radius a, far pairs closer than a also use the regularised kernel, added as the
correction Gamma (K_sigma - K') to the expansion result.

Readings: p terms (indices 0 .. p-1) for both ME and LE (eq. 21; the p+1 upper
limits printed for M2L and M2M are taken as the same truncation); M2L starts at
level 2 (Section 3.3.3); with L <= 1 there is no far field and the result is the
direct sum.  The tree conventions are those of ``oracle.quadtree``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import quadtree as qt
from .kernel import TWO_PI, regularized_kernel, singular_kernel


_BINOM = {}


def _binom(n: int) -> np.ndarray:
    """Table C(a, b) for 0 <= a, b < n (zero where b > a)."""
    if n in _BINOM:
        return _BINOM[n]
    t = np.zeros((n, n))
    for a in range(n):
        for b in range(a + 1):
            t[a, b] = float(math.comb(a, b))
    _BINOM[n] = t
    return t


# ----------------------------------------------------------------- expansions

def p2m(z, gamma, centre, p):
    """eq. 20-21: ME coefficients a_m = sum_i c_i (z_i - centre)^m, m < p."""
    c = -1j * np.asarray(gamma, np.float64) / TWO_PI
    d = np.asarray(z, np.complex128) - centre
    a = np.zeros(p, np.complex128)
    pw = np.ones_like(d)
    for m in range(p):
        a[m] = np.sum(c * pw)
        pw = pw * d
    return a


def me_eval(a, centre, y):
    """Evaluate an ME: [u(y)]* = sum_m a_m (y - centre)^(-m-1)."""
    w = 1.0 / (np.asarray(y, np.complex128) - centre)
    out = np.zeros_like(w)
    pw = w.copy()
    for m in range(len(a)):
        out = out + a[m] * pw
        pw = pw * w
    return out


def m2m_matrix(t, p):
    """Section 3.3.2: M2M(t)_{nk} = (-1)^(n-k) C(n, k) t^(n-k) for k <= n, else 0."""
    bn = _binom(p)
    tp = np.ones(p, np.complex128)
    for m in range(1, p):
        tp[m] = tp[m - 1] * t
    n = np.arange(p)[:, None]; k = np.arange(p)[None, :]
    d = np.clip(n - k, 0, p - 1)
    sgn = np.where((n - k) % 2 == 1, -1.0, 1.0)
    return np.where(k <= n, sgn * bn[n, k] * tp[d], 0.0)


def m2m(a_child, child_centre, parent_centre):
    """Section 3.3.2: re-centre a child ME on its parent's centre (t = parent - child)."""
    return m2m_matrix(parent_centre - child_centre, len(a_child)) @ a_child


def m2l_matrix(t, p):
    """eq. 22: M2L(t)_{nk} = (-1)^n C(n+k, k) t^-(k+n+1), n, k < p."""
    bn = _binom(2 * p)
    inv = 1.0 / t
    tp = np.empty(2 * p, np.complex128)  # tp[m] = t^-(m+1)
    tp[0] = inv
    for m in range(1, 2 * p):
        tp[m] = tp[m - 1] * inv
    n = np.arange(p)[:, None]; k = np.arange(p)[None, :]
    sgn = np.where(n % 2 == 1, -1.0, 1.0)
    return sgn * bn[n + k, k] * tp[n + k]


def m2l(a, source_centre, target_centre):
    """eq. 22 applied to an ME: LE coefficients about the target centre."""
    return m2l_matrix(target_centre - source_centre, len(a)) @ a


def l2l_matrix(t, p):
    """Section 3.3.3: L2L(t)_{nk} = C(k, n) t^(k-n) for k >= n, else 0."""
    bn = _binom(p)
    tp = np.ones(p, np.complex128)
    for m in range(1, p):
        tp[m] = tp[m - 1] * t
    n = np.arange(p)[:, None]; k = np.arange(p)[None, :]
    d = np.clip(k - n, 0, p - 1)
    return np.where(k >= n, bn[k, n] * tp[d], 0.0)


def l2l(b_parent, parent_centre, child_centre):
    """Section 3.3.3: re-centre a parent LE on a child's centre (t = child - parent)."""
    return l2l_matrix(child_centre - parent_centre, len(b_parent)) @ b_parent


def l2p(b, centre, y):
    """Evaluate an LE: [u(y)]* = sum_n b_n (y - centre)^n."""
    d = np.asarray(y, np.complex128) - centre
    out = np.zeros_like(d)
    pw = np.ones_like(d)
    for n in range(len(b)):
        out = out + b[n] * pw
        pw = pw * d
    return out


# ----------------------------------------------------------------- tree

@dataclass
class Tree:
    root: tuple
    levels: int
    ix: np.ndarray
    iy: np.ndarray
    members: dict          # (ix, iy) -> int64 indices of the leaf's particles (input order)

    def leaf_key(self):
        return self.iy * (1 << self.levels) + self.ix


def build_tree(x, y, levels, domain=None) -> Tree:
    root = qt.root_square(x, y, domain)
    ix, iy = qt.leaf_coords(x, y, root, levels)
    key = iy * (1 << levels) + ix
    order = np.argsort(key, kind="stable")
    uniq, first = np.unique(key[order], return_index=True)
    parts = np.split(order, first[1:])
    m = 1 << levels
    members = {(int(k % m), int(k // m)): idx.astype(np.int64) for k, idx in zip(uniq, parts)}
    return Tree(root, levels, ix, iy, members)


# ----------------------------------------------------------------- sweeps

@dataclass
class FMMResult:
    u: np.ndarray
    v: np.ndarray
    near_u: np.ndarray
    near_v: np.ndarray
    far_u: np.ndarray
    far_v: np.ndarray
    targets: np.ndarray
    tree: Tree
    me: dict = field(default_factory=dict)   # level -> {(ix, iy): a (complex p)}
    le: dict = field(default_factory=dict)   # level -> {(ix, iy): b (complex p)}


def upward_sweep(z, gamma, tree: Tree, p):
    """P2M at the leaves, then M2M for levels L-1 .. 2 (Fig. 3, upward)."""
    L = tree.levels
    me = {L: {}}
    for box, idx in tree.members.items():
        me[L][box] = p2m(z[idx], gamma[idx], qt.box_centre(tree.root, L, *box), p)
    for lev in range(L - 1, 1, -1):
        me[lev] = {}
        for (cx, cy), a in me[lev + 1].items():
            par = qt.parent(cx, cy)
            shifted = m2m(a, qt.box_centre(tree.root, lev + 1, cx, cy),
                          qt.box_centre(tree.root, lev, *par))
            if par in me[lev]:
                me[lev][par] = me[lev][par] + shifted
            else:
                me[lev][par] = shifted
    return me


def downward_sweep(me, tree: Tree, p, leaves):
    """M2L over interaction lists and L2L for levels 2 .. L (Fig. 3, downward).

    Only the LEs of ``leaves`` and their ancestors are formed.
    """
    L = tree.levels
    need = {L: set(leaves)}
    for lev in range(L, 2, -1):
        need[lev - 1] = {qt.parent(*b) for b in need[lev]}
    le = {}
    for lev in range(2, L + 1):
        le[lev] = {}
        for box in sorted(need[lev]):
            c = qt.box_centre(tree.root, lev, *box)
            if lev > 2:
                par = qt.parent(*box)
                b = l2l(le[lev - 1][par], qt.box_centre(tree.root, lev - 1, *par), c)
            else:
                b = np.zeros(p, np.complex128)
            for src in qt.interaction_list(lev, *box):
                a = me[lev].get(src)
                if a is not None:
                    b = b + m2l(a, qt.box_centre(tree.root, lev, *src), c)
            le[lev][box] = b
    return le


def near_field(x, y, gamma, sigma, tree: Tree, targets):
    """eq. 10, first sum: regularised kernel over the leaf's local list, j != i."""
    L = tree.levels
    nu = np.zeros(len(targets)); nv = np.zeros(len(targets))
    tl = {}
    for pos, i in enumerate(targets):
        tl.setdefault((int(tree.ix[i]), int(tree.iy[i])), []).append(pos)
    for box, poss in tl.items():
        poss = np.asarray(poss, np.int64)
        ti = targets[poss]
        src = [tree.members[b] for b in qt.local_list(L, *box) if b in tree.members]
        sj = np.concatenate(src)
        ku, kv = regularized_kernel(x[ti, None] - x[None, sj], y[ti, None] - y[None, sj], sigma)
        self_mask = ti[:, None] == sj[None, :]
        ku[self_mask] = 0.0; kv[self_mask] = 0.0
        nu[poss] = ku @ gamma[sj]
        nv[poss] = kv @ gamma[sj]
    return nu, nv


def cutoff_correction(x, y, gamma, sigma, tree: Tree, xe, ye, ex, ey, radius):
    """Distance cut-off of the near field (the distance a of Section 4.1): for
    every evaluation point (xe, ye) in leaf (ex, ey) and every particle outside
    that leaf's local list closer than ``radius``, the regularised kernel (eq. 6)
    replaces the singular one (eq. 27) that the expansions carry, i.e. the sum
    adds Gamma_j (K_sigma - K')(z - z_j).

    A particle closer than a to a point of leaf (ex, ey) lies in a leaf at
    Chebyshev distance at most ceil(a / w_L) from it, so the candidates are the
    members of those leaves outside the local list; each pair is then tested
    exactly (r < a)."""
    xe = np.asarray(xe, np.float64); ye = np.asarray(ye, np.float64)
    cu = np.zeros(len(xe)); cv = np.zeros(len(xe))
    if radius <= 0.0 or len(xe) == 0:
        return cu, cv
    L = tree.levels
    m = 1 << L
    reach = int(math.ceil(radius / qt.box_side(tree.root, L)))
    groups = {}
    for k in range(len(xe)):
        groups.setdefault((int(ex[k]), int(ey[k])), []).append(k)
    for (bx, by), ks in groups.items():
        ks = np.asarray(ks, np.int64)
        cand = [tree.members[(sx, sy)]
                for sy in range(max(0, by - reach), min(m, by + reach + 1))
                for sx in range(max(0, bx - reach), min(m, bx + reach + 1))
                if max(abs(sx - bx), abs(sy - by)) > 1 and (sx, sy) in tree.members]
        if not cand:
            continue
        sj = np.concatenate(cand)
        dx = xe[ks, None] - x[None, sj]; dy = ye[ks, None] - y[None, sj]
        close = dx * dx + dy * dy < radius * radius
        ru, rv = regularized_kernel(dx, dy, sigma)
        su, sv = singular_kernel(dx, dy)
        cu[ks] = np.where(close, ru - su, 0.0) @ gamma[sj]
        cv[ks] = np.where(close, rv - sv, 0.0) @ gamma[sj]
    return cu, cv


def fmm_velocity(x, y, gamma, sigma, p, levels, domain=None, targets=None,
                 keep_expansions=False, radius=0.0) -> FMMResult:
    """The paper's FMM evaluation of eq. 9 at all particles (or at ``targets``).

    ``radius`` > 0 adds the distance cut-off of the near field
    (``cutoff_correction``), counted in the near part."""
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64)
    gamma = np.asarray(gamma, np.float64)
    tree = build_tree(x, y, levels, domain)
    tidx = np.arange(len(x)) if targets is None else np.asarray(targets, np.int64)
    me = upward_sweep(x + 1j * y, gamma, tree, p) if levels >= 2 else {}
    return evaluate_targets(x, y, gamma, sigma, p, tree, me, tidx, radius, keep_expansions)


def evaluate_targets(x, y, gamma, sigma, p, tree: Tree, me, tidx, radius=0.0,
                     keep_expansions=False) -> FMMResult:
    """Everything of ``fmm_velocity`` after the upward sweep, for the particles
    ``tidx``: the downward sweep of their leaves and ancestors, L2P, the near
    field and the cut-off correction.  Disjoint target sets can be evaluated
    separately (in parallel) from one tree and one upward sweep ``me``."""
    z = x + 1j * y
    fu = np.zeros(len(tidx)); fv = np.zeros(len(tidx))
    le = {}
    L = tree.levels
    if L >= 2:
        leaves = {(int(tree.ix[i]), int(tree.iy[i])) for i in tidx}
        le = downward_sweep(me, tree, p, leaves)
        for box in leaves:
            sel = np.nonzero((tree.ix[tidx] == box[0]) & (tree.iy[tidx] == box[1]))[0]
            w = l2p(le[L][box], qt.box_centre(tree.root, L, *box), z[tidx[sel]])
            fu[sel] = w.real
            fv[sel] = -w.imag
    nu, nv = near_field(x, y, gamma, sigma, tree, tidx)
    cu, cv = cutoff_correction(x, y, gamma, sigma, tree, x[tidx], y[tidx], tree.ix[tidx],
                               tree.iy[tidx], radius)
    nu = nu + cu; nv = nv + cv
    res = FMMResult(nu + fu, nv + fv, nu, nv, fu, fv, tidx, tree)
    if keep_expansions:
        res.me = me; res.le = le
    return res


def hybrid_velocity(x, y, gamma, sigma, levels, domain=None, targets=None, radius=0.0):
    """The p -> infinity limit of the FMM: eq. 6 inside the leaf's local list (and,
    with ``radius`` > 0, for every pair closer than radius) and the singular
    kernel (eq. 27) everywhere else (Section 4 opening)."""
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64)
    g = np.asarray(gamma, np.float64)
    root = qt.root_square(x, y, domain)
    ix, iy = qt.leaf_coords(x, y, root, levels)
    tidx = np.arange(len(x)) if targets is None else np.asarray(targets, np.int64)
    u = np.zeros(len(tidx)); v = np.zeros(len(tidx))
    cs = max(1, (1 << 21) // max(1, len(x)))
    for s in range(0, len(tidx), cs):
        ti = tidx[s:s + cs]
        dx = x[ti, None] - x[None, :]; dy = y[ti, None] - y[None, :]
        near = (np.abs(ix[ti, None] - ix[None, :]) <= 1) & (np.abs(iy[ti, None] - iy[None, :]) <= 1)
        if radius > 0.0:
            near = near | (dx * dx + dy * dy < radius * radius)
        ru, rv = regularized_kernel(dx, dy, sigma)
        su, sv = singular_kernel(dx, dy)
        ku = np.where(near, ru, su); kv = np.where(near, rv, sv)
        rows = np.arange(len(ti))
        ku[rows, ti] = 0.0; kv[rows, ti] = 0.0
        u[s:s + cs] = ku @ g; v[s:s + cs] = kv @ g
    return u, v


# ----------------------------------------------------------------- evaluation points

def inside_root(xe, ye, root):
    """True where an evaluation point lies in the closed root square."""
    x0, y0, s = root
    xe = np.asarray(xe, np.float64); ye = np.asarray(ye, np.float64)
    return (xe >= x0) & (xe <= x0 + s) & (ye >= y0) & (ye <= y0 + s)


def fmm_velocity_at(x, y, gamma, sigma, p, levels, xe, ye, domain=None, radius=0.0) -> FMMResult:
    """The FMM of eq. 10 evaluated at separate points (eq. 8) instead of at the
    particles (eq. 9).

    The tree is built on the particles.  An evaluation point belongs to the
    leaf given by the same floor-and-clamp rule; its near field is the
    regularised kernel over the particles of that leaf's local list (a particle
    at the point itself contributes zero, the limit of eq. 6), its far field the
    L2P of that leaf's LE.  Points outside the closed root square have no leaf
    whose expansions converge there: their velocity is NaN.  ``radius`` adds
    the distance cut-off (``cutoff_correction``) to the near part.
    """
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64)
    gamma = np.asarray(gamma, np.float64)
    xe = np.asarray(xe, np.float64); ye = np.asarray(ye, np.float64)
    tree = build_tree(x, y, levels, domain)
    L = levels
    ok = inside_root(xe, ye, tree.root)
    ex, ey = qt.leaf_coords(np.where(ok, xe, tree.root[0]), np.where(ok, ye, tree.root[1]),
                            tree.root, L)
    ze = xe + 1j * ye
    ne = len(xe)
    nu = np.zeros(ne); nv = np.zeros(ne); fu = np.zeros(ne); fv = np.zeros(ne)
    boxes = {}
    for k in np.nonzero(ok)[0]:
        boxes.setdefault((int(ex[k]), int(ey[k])), []).append(k)
    me = le = {}
    if L >= 2 and boxes:
        me = upward_sweep(x + 1j * y, gamma, tree, p)
        le = downward_sweep(me, tree, p, set(boxes))
    for box, ks in boxes.items():
        ks = np.asarray(ks, np.int64)
        src = [tree.members[b] for b in qt.local_list(L, *box) if b in tree.members]
        if src:
            sj = np.concatenate(src)
            ku, kv = regularized_kernel(xe[ks, None] - x[None, sj], ye[ks, None] - y[None, sj], sigma)
            nu[ks] = ku @ gamma[sj]
            nv[ks] = kv @ gamma[sj]
        if L >= 2:
            w = l2p(le[L][box], qt.box_centre(tree.root, L, *box), ze[ks])
            fu[ks] = w.real
            fv[ks] = -w.imag
    okk = np.nonzero(ok)[0]
    cu, cv = cutoff_correction(x, y, gamma, sigma, tree, xe[okk], ye[okk], ex[okk], ey[okk], radius)
    nu[okk] += cu; nv[okk] += cv
    bad = ~ok
    for a in (nu, nv, fu, fv):
        a[bad] = np.nan
    return FMMResult(nu + fu, nv + fv, nu, nv, fu, fv, np.arange(ne), tree, me, le)
