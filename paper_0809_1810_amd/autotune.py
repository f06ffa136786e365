"""Autotuner for the launch shapes of the near field (P2P) and of the M2L.

Tunable shape: particles per tile T (64, 32, 16: one, two or four lanes per
target; T is also the source-chunk size of the far-pair test, so smaller tiles
have tighter bounding boxes) and waves per workgroup (1, 2, 4, 8).  For each
workload the tuner times the P2P phase of FP32 evaluations with HIP events
(median of repeated calls) for every shape, keeps the fastest, and writes a
table keyed by log2 of the mean particles per leaf and by the occupancy
spread (``leaf_spread``: log2 of the pair-weighted over the plain mean
particles per leaf, 0 for even leaves; a clustered and an even input with the
same mean take different shapes).  ``apply_for(n, levels, spread=...)`` sets
the library's tuning from the nearest table entry.  With the distance
cut-off only 64-target tiles (one lane per target) cull the ring sources
lane-parallel, so the tuner also times the 64-target shapes with the cut-off
at the radius where one pair's kernel difference is 1e-6 (``cutoff_ms``), and
``apply_for(..., cutoff=True)`` takes the fastest of those (or, for an entry
without them, the fastest 64-target shape of the paper's split).

Symmetric near field (VFMM_TUNE_P2P_SYMMETRIC, 64-target tiles): the tuner
times the 64-target shapes with it too, keyed "64x<waves>s" in ``all_ms`` and
``cutoff_ms``; ``apply_for`` sets it when such a shape is the fastest.

M2L on the matrix cores (FP32, p <= 16): the tile variants of
VFMM_TUNE_M2L_TILE (operands in registers one offset ahead; sources staged in
LDS with 4 or 8 waves) are timed on the M2L + L2L phase of far-only
evaluations, and the fastest is stored per entry (``m2l_tile``, ``m2l_ms``);
``apply_for`` sets it too (0 for an entry without it).

    python -m paper_0809_1810_amd.autotune --out tuning.json
    python -m paper_0809_1810_amd.autotune --m2l-only      (add the M2L timings to the table)
    python -m paper_0809_1810_amd.autotune --sym-only      (add the symmetric near-field timings)
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import vfmm as V

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_PATH = os.path.join(HERE, "tuning.json")
TILES = (64, 32, 16)
WAVES = (1, 2, 4, 8)
M2L_TILES = (0, 1, 2)


CUTOFF_TOL = 1e-6


def time_p2p(x, y, g, sigma, p, levels, tile, waves, reps=5, radius=0.0, sym=0):
    """Median P2P phase time (ms) for one launch shape (radius: near cut-off;
    sym: symmetric near field, 64-target tiles)."""
    V.set_tuning(tile=tile, waves=waves, sym=sym)
    t = V.Tree(x, y, levels, p_max=p)
    t.set_near_radius(radius)
    t.velocity(g, sigma, p, V.FP32)
    t.enable_timing(reps)
    for _ in range(reps):
        t.velocity(g, sigma, p, V.FP32)
    ms = float(np.median([ph["p2p"] for ph in t.read_timing()]))
    t.close()
    V.set_tuning(sym=0)
    return ms


def sym_entry(x, y, g, sigma, p, levels):
    """Timings of the symmetric 64-target shapes, paper split and cut-off."""
    radius = sigma * math.sqrt(2.0 * math.log(1.0 / CUTOFF_TOL))
    split = {f"64x{w}s": round(time_p2p(x, y, g, sigma, p, levels, 64, w, sym=1), 4) for w in WAVES}
    cut = {f"64x{w}s": round(time_p2p(x, y, g, sigma, p, levels, 64, w, radius=radius, sym=1), 4)
           for w in WAVES}
    return split, cut


def time_m2l(x, y, g, sigma, p, levels, mode, reps=10):
    """Median M2L + L2L phase time (ms) of far-only FP32 evaluations for one M2L tile."""
    V.set_tuning(m2l=mode)
    t = V.Tree(x, y, levels, p_max=p)
    t.velocity(g, sigma, p, V.FP32, parts=V.PART_FAR)
    t.enable_timing(reps)
    for _ in range(reps):
        t.velocity(g, sigma, p, V.FP32, parts=V.PART_FAR)
    ms = float(np.median([ph["m2l_l2l"] for ph in t.read_timing()]))
    t.close()
    V.set_tuning(m2l=0)
    return ms


def m2l_entry(x, y, g, sigma, p, levels):
    res = {m: time_m2l(x, y, g, sigma, p, levels, m) for m in M2L_TILES}
    best = min(res, key=res.get)
    return {"m2l_tile": best, "m2l_ms": {str(k): round(v, 4) for k, v in sorted(res.items())}}


def tune_workload(name, P, p, levels, log=print):
    import torch
    x = torch.from_numpy(P.x).cuda(); y = torch.from_numpy(P.y).cuda(); g = torch.from_numpy(P.gamma).cuda()
    res = {}
    for tile in TILES:
        for waves in WAVES:
            res[(tile, waves)] = time_p2p(x, y, g, P.sigma, p, levels, tile, waves)
    best = min(res, key=res.get)
    radius = P.sigma * math.sqrt(2.0 * math.log(1.0 / CUTOFF_TOL))
    cut = {w: time_p2p(x, y, g, P.sigma, p, levels, 64, w, radius=radius) for w in WAVES}
    cbest = min(cut, key=cut.get)
    entry = {"workload": name, "n": P.n, "levels": levels, "p": p,
             "ppl_log2": math.log2(P.n) - 2 * levels,
             "spread": round(leaf_spread(P.x, P.y, levels), 4), "tile": best[0], "waves": best[1],
             "p2p_ms": res[best], "default_ms": res[(64, 4)],
             "all_ms": {f"{k[0]}x{k[1]}": round(v, 4) for k, v in sorted(res.items())},
             "cutoff_radius_sigma": round(radius / P.sigma, 4),
             "cutoff_ms": {f"64x{w}": round(v, 4) for w, v in sorted(cut.items())}}
    entry.update(m2l_entry(x, y, g, P.sigma, p, levels))
    split, cut_s = sym_entry(x, y, g, P.sigma, p, levels)
    entry["all_ms"].update(split)
    entry["cutoff_ms"].update(cut_s)
    log(f"[tune] {name} L={levels}: best tile {best[0]} waves {best[1]} {res[best]:.3f} ms "
        f"(default 64x4 {res[(64, 4)]:.3f} ms); with the cut-off 64x{cbest} {cut[cbest]:.3f} ms")
    return entry


def default_workloads():
    import workloads as W
    return [
        ("clusters_1m", W.config("clusters_1m"), 14, 6),
        ("clusters_1m", W.config("clusters_1m"), 14, 7),
        ("lattice_1024", W.config("lattice_1024"), 14, 6),
        ("lattice_1024", W.config("lattice_1024"), 14, 7),
        ("lattice_1024", W.config("lattice_1024"), 14, 8),
        ("lattice_320", W.config("lattice_320"), 14, 5),
        ("lattice_320", W.config("lattice_320"), 14, 6),
        ("uniform_64k", W.uniform(65536, seed=9, sigma=2.0 / 256 / 0.8), 12, 6),
    ]


def tune_m2l(path=TABLE_PATH, log=print):
    """Adds the M2L tile timings to every entry of an existing table."""
    import torch
    import workloads as W
    table = json.load(open(path))
    work = {(w[0], w[3]): w for w in default_workloads()}
    for e in table["entries"]:
        name, P, p, levels = work[(e["workload"], e["levels"])]
        x = torch.from_numpy(P.x).cuda(); y = torch.from_numpy(P.y).cuda()
        g = torch.from_numpy(P.gamma).cuda()
        e.update(m2l_entry(x, y, g, P.sigma, p, levels))
        log(f"[tune] {name} L={levels}: M2L tile {e['m2l_tile']} {e['m2l_ms']}")
    with open(path, "w") as f:
        json.dump(table, f, indent=1)
    return table


def tune_sym(path=TABLE_PATH, log=print):
    """Adds the symmetric near-field timings to every entry of an existing table."""
    import torch
    table = json.load(open(path))
    work = {(w[0], w[3]): w for w in default_workloads()}
    for e in table["entries"]:
        name, P, p, levels = work[(e["workload"], e["levels"])]
        x = torch.from_numpy(P.x).cuda(); y = torch.from_numpy(P.y).cuda()
        g = torch.from_numpy(P.gamma).cuda()
        split, cut = sym_entry(x, y, g, P.sigma, p, levels)
        e.setdefault("all_ms", {}).update(split)
        e.setdefault("cutoff_ms", {}).update(cut)
        log(f"[tune] {name} L={levels}: symmetric {split}, with the cut-off {cut}")
    with open(path, "w") as f:
        json.dump(table, f, indent=1)
    return table


def tune(out=TABLE_PATH, log=print):
    t0 = time.time()
    entries = [tune_workload(*w, log=log) for w in default_workloads()]
    V.set_tuning(tile=64, waves=4)
    table = {"entries": entries, "seconds": round(time.time() - t0, 1)}
    with open(out, "w") as f:
        json.dump(table, f, indent=1)
    return table


def _parse(key):
    """"64x2" -> (64, 2, 0); "64x2s" (symmetric near field) -> (64, 2, 1)."""
    tile, rest = key.split("x")
    return int(tile), int(rest.rstrip("s")), int(rest.endswith("s"))


def spread_from_counts(counts):
    """Occupancy spread of a leaf population: log2(4^L sum n_b^2 / N^2), i.e.
    the pair-weighted mean particles per leaf over the plain mean, in log2
    units (0 when every leaf holds the same number; a clustered input's near
    field has many more pairs than its mean occupancy suggests)."""
    c = np.asarray(counts, dtype=np.float64)
    n = c.sum()
    if n <= 0:
        return 0.0
    return float(math.log2(c.size * float(np.dot(c, c)) / (n * n)))


def leaf_spread(x, y, levels):
    """``spread_from_counts`` of host positions at level ``levels``, with the
    library's root square (the bounding square of side max extent (1 + 2^-20)
    centred on the bounding box) and floor-and-clamp leaf rule."""
    x = np.asarray(x, dtype=np.float64); y = np.asarray(y, dtype=np.float64)
    if x.size == 0:
        return 0.0
    xl, xh, yl, yh = x.min(), x.max(), y.min(), y.max()
    side = max(xh - xl, yh - yl) * (1.0 + 2.0 ** -20)
    if side == 0.0:
        side = 1.0
    x0 = 0.5 * (xl + xh) - 0.5 * side
    y0 = 0.5 * (yl + yh) - 0.5 * side
    m = 1 << levels
    ix = np.clip(np.floor((x - x0) / side * m), 0, m - 1).astype(np.int64)
    iy = np.clip(np.floor((y - y0) / side * m), 0, m - 1).astype(np.int64)
    return spread_from_counts(np.bincount(iy * m + ix, minlength=m * m))


def _nearest(entries, n, levels, spread):
    ppl = math.log2(max(n, 1)) - 2 * levels
    if spread is None:
        return min(entries, key=lambda e: abs(e["ppl_log2"] - ppl))
    # both in log2 units; entries without a recorded spread count as even
    return min(entries, key=lambda e: abs(e["ppl_log2"] - ppl) + abs(e.get("spread", 0.0) - spread))


def lookup_shape(n, levels, path=TABLE_PATH, cutoff=False, spread=None):
    """(tile, waves, sym) of the table entry nearest in log2 particles per leaf
    (and, given ``spread``, in occupancy spread: the sum of the two distances):
    its fastest timed shape; with ``cutoff`` its fastest 64-target shape (timed
    with the cut-off if it has such timings)."""
    try:
        table = json.load(open(path))
    except (OSError, ValueError):
        return 64, 4, 0
    e = _nearest(table["entries"], n, levels, spread)
    if cutoff:
        t64 = e.get("cutoff_ms") or {k: v for k, v in e.get("all_ms", {}).items()
                                     if k.startswith("64x")}
        if t64:
            return _parse(min(t64, key=t64.get))
        return 64, int(e["waves"]) if int(e["tile"]) == 64 else 4, 0
    if e.get("all_ms"):
        return _parse(min(e["all_ms"], key=e["all_ms"].get))
    return int(e["tile"]), int(e["waves"]), 0


def lookup(n, levels, path=TABLE_PATH, cutoff=False, spread=None):
    """(tile, waves) of ``lookup_shape``."""
    return lookup_shape(n, levels, path, cutoff, spread)[:2]


def lookup_m2l(n, levels, path=TABLE_PATH, spread=None):
    """M2L tile of the nearest table entry (as ``lookup_shape``; 0 without)."""
    try:
        table = json.load(open(path))
    except (OSError, ValueError):
        return 0
    return int(_nearest(table["entries"], n, levels, spread).get("m2l_tile", 0))


def apply_for(n, levels, path=TABLE_PATH, cutoff=False, spread=None):
    """Sets the process-wide tuning from the nearest table entry (``spread``:
    the input's ``leaf_spread`` at ``levels``, None to match on particles per
    leaf alone)."""
    tile, waves, sym = lookup_shape(n, levels, path, cutoff, spread)
    V.set_tuning(tile=tile, waves=waves, m2l=lookup_m2l(n, levels, path, spread), sym=sym)
    return tile, waves


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE_PATH)
    ap.add_argument("--m2l-only", action="store_true",
                    help="time the M2L tiles and add them to the existing table")
    ap.add_argument("--sym-only", action="store_true",
                    help="time the symmetric near field and add it to the existing table")
    a = ap.parse_args(argv)
    if a.m2l_only:
        tune_m2l(a.out, log=lambda m: print(m, flush=True))
    elif a.sym_only:
        tune_sym(a.out, log=lambda m: print(m, flush=True))
    else:
        tune(a.out, log=lambda m: print(m, flush=True))


if __name__ == "__main__":
    sys.exit(main())
