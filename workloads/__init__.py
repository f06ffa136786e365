"""Seeded synthetic inputs for the vortex-particle FMM.

This module only *generates* particle sets (positions, circulations, core size)
and sample indices.  It holds none of the method's arithmetic: no kernel, no
expansion, no tree.  Both the CPU oracle and the GPU path are fed from here, so
the two sides see bit-identical inputs.

All random draws use NumPy's PCG64 (``numpy.random.default_rng(seed)``) in a
fixed draw order, documented per generator.

Workloads follow the set-ups of Cruz & Barba (2008):

* lattice discretisation of a vorticity field with ``Gamma_i = h^2 omega(x_i)``
  (Section 5.1; vortex blobs of eq. 2 with the Gaussian cut-off of eq. 3),
  spacing ``h = 0.8 sigma``;
* the Lamb-Oseen vortex of eq. 32 with nu = 5e-4, t = 4, sigma = 0.02 and the
  lattice sizes of Section 5.1 (N = 3969, 7744, 8836, 11449, 19044);
* the single-source set-up of Section 5.2 (one unit source at the domain
  centre, 8836 lattice evaluation points carrying zero circulation);

plus the larger synthetic distributions used to measure the GPU path
(uniform, cell-centred lattice with a Lamb-Oseen vortex pair, Gaussian
clusters, and a batch of uneven instances).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Particles",
    "uniform",
    "cell_lattice",
    "lamb_oseen_pair",
    "clusters",
    "paper_lamb_oseen",
    "paper_single_source",
    "batch_instances",
    "sample_targets",
    "PAPER_LO_DOMAINS",
]


@dataclass
class Particles:
    """A particle set: SoA float64 positions and circulations plus the core size."""

    x: np.ndarray
    y: np.ndarray
    gamma: np.ndarray
    sigma: float
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def uniform(n: int, seed: int, sigma: float = 0.02, lo: float = -1.0, hi: float = 1.0,
            name: str = "uniform") -> Particles:
    """N particles uniform in [lo, hi]^2 with circulations uniform in [-1, 1].

    Draw order: x (n), y (n), gamma (n).
    """
    rng = np.random.default_rng(seed)
    x = rng.uniform(lo, hi, n)
    y = rng.uniform(lo, hi, n)
    g = rng.uniform(-1.0, 1.0, n)
    return Particles(_f64(x), _f64(y), _f64(g), float(sigma), name,
                     {"seed": seed, "kind": "uniform"})


def cell_lattice(n_side: int, lo: float = -1.0, hi: float = 1.0):
    """Cell-centred n_side x n_side lattice in [lo, hi]^2: x_i = lo + (i + 1/2) h.

    Returns (x, y, h) with x varying fastest.
    """
    h = (hi - lo) / n_side
    c = lo + (np.arange(n_side, dtype=np.float64) + 0.5) * h
    yy, xx = np.meshgrid(c, c, indexing="ij")
    return _f64(xx.ravel()), _f64(yy.ravel()), h


def _gauss_vorticity(r2: np.ndarray, width2: float) -> np.ndarray:
    """omega(r) = exp(-r^2 / width2) / (pi width2): unit total circulation."""
    return np.exp(-r2 / width2) / (math.pi * width2)


def lamb_oseen_pair(n_side: int, offset: float = 0.5, width2: float = 0.04,
                    h_over_sigma: float = 0.8, name: str = "lamb_oseen_pair") -> Particles:
    """Counter-rotating Gaussian vortex pair on a cell-centred lattice in [-1, 1]^2.

    Gamma_i = h^2 [omega(|x_i|) - omega(|x_i - (offset, 0)|)] with
    omega(r) = exp(-r^2/0.04)/(0.04 pi); sigma = h / 0.8.  Deterministic.
    """
    x, y, h = cell_lattice(n_side)
    w1 = _gauss_vorticity(x * x + y * y, width2)
    w2 = _gauss_vorticity((x - offset) ** 2 + y * y, width2)
    g = h * h * (w1 - w2)
    return Particles(x, y, _f64(g), h / h_over_sigma, name,
                     {"kind": "lattice", "n_side": n_side, "h": h})


def clusters(n: int, seed: int, n_clusters: int = 8, sigma: float = 0.005,
             centre_range: float = 0.8, std_range=(0.05, 0.2),
             name: str = "clusters") -> Particles:
    """n_clusters equal isotropic Gaussian clusters.

    Centres uniform in [-centre_range, centre_range]^2, per-cluster standard
    deviation uniform in std_range, circulations N(0, 1) times a random sign per
    cluster.  Draw order: centres (n_clusters x 2), stds (n_clusters), signs
    (n_clusters), then per cluster: positions (m x 2) and circulations (m).
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-centre_range, centre_range, (n_clusters, 2))
    stds = rng.uniform(std_range[0], std_range[1], n_clusters)
    signs = np.where(rng.uniform(0.0, 1.0, n_clusters) < 0.5, -1.0, 1.0)
    base, extra = divmod(n, n_clusters)
    xs, ys, gs = [], [], []
    for c in range(n_clusters):
        m = base + (1 if c < extra else 0)
        pos = rng.normal(0.0, 1.0, (m, 2)) * stds[c] + centres[c]
        g = rng.normal(0.0, 1.0, m) * signs[c]
        xs.append(pos[:, 0]); ys.append(pos[:, 1]); gs.append(g)
    return Particles(_f64(np.concatenate(xs)), _f64(np.concatenate(ys)),
                     _f64(np.concatenate(gs)), float(sigma), name,
                     {"seed": seed, "kind": "clusters", "centres": centres.tolist(),
                      "stds": stds.tolist(), "signs": signs.tolist()})


# Section 5.1: square domains whose lattice sizes reproduce the printed N.
PAPER_LO_DOMAINS = {3969: 1.0, 7744: 1.4, 8836: 1.5, 11449: 1.7, 19044: 2.2}
PAPER_SIGMA = 0.02
PAPER_H = 0.8 * PAPER_SIGMA
PAPER_NU = 5e-4
PAPER_T = 4.0


def _paper_lattice(side: float, h: float = PAPER_H):
    """Lattice -side/2 + k h, k = 0 .. ceil(side/h) - 1, per axis (x fastest)."""
    m = int(math.ceil(side / h - 1e-12))
    c = -0.5 * side + h * np.arange(m, dtype=np.float64)
    yy, xx = np.meshgrid(c, c, indexing="ij")
    return _f64(xx.ravel()), _f64(yy.ravel())


def paper_lamb_oseen(n: int = 8836, gamma0: float = 1.0) -> Particles:
    """Section 5.1 set-up: Lamb-Oseen vortex (eq. 32) on a lattice, h/sigma = 0.8.

    Gamma_i = h^2 omega(r_i, t) with omega = Gamma0/(4 pi nu t) exp(-r^2/(4 nu t)),
    nu = 5e-4, t = 4, sigma = 0.02, h = 0.016.
    """
    side = PAPER_LO_DOMAINS[n]
    x, y = _paper_lattice(side)
    four_nu_t = 4.0 * PAPER_NU * PAPER_T
    w = gamma0 / (math.pi * four_nu_t) * np.exp(-(x * x + y * y) / four_nu_t)
    g = PAPER_H * PAPER_H * w
    return Particles(x, y, _f64(g), PAPER_SIGMA, f"paper_lamb_oseen_{n}",
                     {"kind": "lattice", "side": side, "h": PAPER_H,
                      "nu": PAPER_NU, "t": PAPER_T, "gamma0": gamma0})


def paper_single_source(n_eval: int = 8836, gamma0: float = 1.0) -> Particles:
    """Section 5.2 set-up: one source at the domain centre, lattice evaluation points.

    Particle 0 is the source (Gamma = gamma0 at the origin); the n_eval lattice
    points of the matching Section 5.1 domain carry zero circulation.
    """
    side = PAPER_LO_DOMAINS[n_eval]
    x, y = _paper_lattice(side)
    x = np.concatenate([[0.0], x]); y = np.concatenate([[0.0], y])
    g = np.zeros_like(x); g[0] = gamma0
    return Particles(_f64(x), _f64(y), _f64(g), PAPER_SIGMA, f"paper_single_source_{n_eval}",
                     {"kind": "single_source", "side": side})


def batch_instances(count: int = 256, seed: int = 4, n_range=(2048, 65536),
                    p_range=(5, 20), level_range=(3, 6)):
    """A batch of uneven FMM instances (uniform or cell-centred lattice, 50/50).

    Per instance, in draw order: log-uniform N, kind, p, levels, then positions
    (uniform kind) and circulations uniform in [-1, 1].  Lattice instances use
    n = round(sqrt(N)) points per side, N = n^2.  sigma = h / 0.8 with
    h = 2 / sqrt(N).  Returns a list of (Particles, p, levels).
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        lattice = bool(rng.uniform() < 0.5)
        p = int(rng.integers(p_range[0], p_range[1] + 1))
        lev = int(rng.integers(level_range[0], level_range[1] + 1))
        if lattice:
            side = int(round(math.sqrt(n)))
            x, y, _ = cell_lattice(side)
            n = side * side
        else:
            x = rng.uniform(-1.0, 1.0, n)
            y = rng.uniform(-1.0, 1.0, n)
        g = rng.uniform(-1.0, 1.0, n)
        h = 2.0 / math.sqrt(n)
        parts = Particles(_f64(x), _f64(y), _f64(g), h / 0.8, f"batch_{i}",
                          {"kind": "lattice" if lattice else "uniform", "index": i})
        out.append((parts, p, lev))
    return out


def sample_targets(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct indices in [0, n), drawn without replacement, sorted (int64)."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)


def eval_lattice(n_side: int, square) -> tuple:
    """Evaluation points: the n_side^2 cell centres of the square (x0, y0, S),
    row-major, as (x, y) float64 arrays (the error-map grids of Section 5.2)."""
    x0, y0, s = (float(v) for v in square)
    c = (np.arange(n_side, dtype=np.float64) + 0.5) * (s / n_side)
    gx, gy = np.meshgrid(x0 + c, y0 + c)
    return _f64(gx.ravel()), _f64(gy.ravel())


def eval_points(k: int, seed: int, square) -> tuple:
    """k evaluation points uniform in the square (x0, y0, S), seeded."""
    rng = np.random.default_rng(seed)
    x0, y0, s = (float(v) for v in square)
    return _f64(x0 + s * rng.uniform(size=k)), _f64(y0 + s * rng.uniform(size=k))


def config(name: str) -> Particles:
    """Named workloads used by tests and the benchmark.

    * ``uniform_1k``: N = 1000 uniform in [-1, 1]^2, seed 1, sigma = 0.02.
    * ``lattice_320``: 320^2 cell-centred lattice, Lamb-Oseen pair, sigma = h/0.8.
    * ``clusters_1m``: N = 2^20 in 8 Gaussian clusters, seed 3, sigma = 0.005.
    * ``lattice_2048``: 2048^2 lattice, Lamb-Oseen pair.
    * ``lattice_1024``: 1024^2 lattice, Lamb-Oseen pair.
    """
    if name == "uniform_1k":
        return uniform(1000, seed=1, sigma=0.02, name=name)
    if name == "lattice_320":
        return lamb_oseen_pair(320, name=name)
    if name == "lattice_1024":
        return lamb_oseen_pair(1024, name=name)
    if name == "lattice_2048":
        return lamb_oseen_pair(2048, name=name)
    if name == "clusters_1m":
        return clusters(1 << 20, seed=3, name=name)
    if name.startswith("clusters_"):
        n = int(name.split("_")[1])
        return clusters(n, seed=3, name=name)
    raise KeyError(name)
