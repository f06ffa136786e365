"""Learned (p, levels) selection: data generation, training, selection and audit.

The paper characterises the FMM error against N, the number of levels and the
truncation p by running the method over a grid of parameters and comparing with
a reference (Section 5).  This module automates that design: it runs the
library's FP32 FMM over a grid of (p, L) on seeded synthetic particle sets,
records log10 of the maximum error against the library's FP64 direct sum
(normalised by the maximum velocity, Section 5.1), trains the selector
network with the library's own forward / backward / Adam kernels, and chooses
parameters with ``vfmm_select_and_audit``, which audits every choice with
the direct sum on sampled targets and falls back to the conservative choice
when the audit fails.

Every computation runs in the HIP library; this file only drives it.

    python -m paper_0809_1810_amd.selector generate --instances 400 --out data.npz
    python -m paper_0809_1810_amd.selector generate --instances 160 --seed 2 --nmax-log2 22 \
        --cutoff --out data_cutoff.npz
    python -m paper_0809_1810_amd.selector train --data data.npz,data_cutoff.npz --out weights.npz
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
WEIGHTS_PATH = os.path.join(HERE, "selector_weights.npz")
P_GRID = (4, 6, 8, 10, 12, 14, 16, 18, 20)
LOG10_FLOOR = -9.0


def _torch():
    import torch
    return torch


# ----------------------------------------------------------------- instances

def random_instance(rng, n_range=(2 ** 11, 2 ** 18)):
    """A seeded synthetic particle set of a random kind (positions in ~[-1, 1]^2).

    Kinds: uniform (Gamma ~ U[-1, 1]); cell lattice with a Lamb-Oseen vortex pair;
    Gaussian clusters (1-16 clusters, std 0.02-0.3, Gamma ~ N(0,1) x sign per
    cluster); a single Lamb-Oseen vortex on a lattice.  sigma = ratio * h with
    h = 2 / sqrt(N) and ratio log-uniform in [0.5, 4].
    """
    import workloads as W
    n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
    kind = ["uniform", "lattice_pair", "clusters", "lamb_oseen"][int(rng.integers(0, 4))]
    ratio = math.exp(rng.uniform(math.log(0.5), math.log(4.0)))
    seed = int(rng.integers(0, 2 ** 31))
    if kind == "uniform":
        P = W.uniform(n, seed=seed)
    elif kind == "clusters":
        P = W.clusters(n, seed=seed, n_clusters=int(rng.integers(1, 17)),
                       std_range=(0.02, float(rng.uniform(0.03, 0.3))))
    else:
        side = max(8, int(round(math.sqrt(n))))
        if kind == "lattice_pair":
            P = W.lamb_oseen_pair(side, offset=float(rng.uniform(0.2, 0.8)))
        else:
            x, y, h = W.cell_lattice(side)
            w2 = float(rng.uniform(0.01, 0.1))
            g = h * h * np.exp(-(x * x + y * y) / w2) / (math.pi * w2)
            P = W.Particles(x, y, g, h / 0.8, "lamb_oseen")
        n = P.n
    P.sigma = ratio * 2.0 / math.sqrt(n)
    P.meta["kind"] = kind
    return P


# ----------------------------------------------------------------- data generation

def resolve_radius(r, sigma, tol=1e-6):
    """Near radius of a grid entry: 0 (the paper's split), V.NEAR_RADIUS_AUTO, or
    "tol" for sigma sqrt(2 ln(1/tol)), where one pair's kernel difference
    equals tol."""
    return sigma * math.sqrt(2.0 * math.log(1.0 / tol)) if r == "tol" else float(r)


def evaluate_grid(P, p_grid=P_GRID, max_levels=9, n_targets=2048, seed=0, radii=(0.0,)):
    """Rows (features, log10 e_max, p, L, radius, ms) of FP32 runs of the library
    on P, for every near radius of ``radii`` (see resolve_radius) at the levels
    where NEAR_RINGS_MAX leaf sides reach 6 sigma."""
    torch = _torch()
    x = torch.from_numpy(P.x).cuda(); y = torch.from_numpy(P.y).cuda()
    g = torch.from_numpy(P.gamma).cuda()
    n = P.n
    if n <= 16384:
        tg = None
        ur, vr = V.direct_velocity(x, y, g, P.sigma)
    else:
        rng = np.random.default_rng(seed)
        tg = torch.from_numpy(np.sort(rng.choice(n, n_targets, replace=False)).astype(np.int64)).cuda()
        ur, vr = V.direct_velocity(x, y, g, P.sigma, targets=tg)
    stats = V.particle_stats(x, y, g)
    side = max(stats[9] - stats[8], stats[11] - stats[10]) * (1.0 + 2.0 ** -20)
    rows = []
    lmax = min(max_levels, int(math.log2(4 * n) // 2))
    for L in range(2, lmax + 1):
        tree = V.Tree(x, y, L, p_max=max(p_grid))
        for rr in radii:
            r = resolve_radius(rr, P.sigma)
            if r != 0.0 and V.NEAR_RINGS_MAX * side / 2 ** L < 6.0 * P.sigma:
                continue
            tree.set_near_radius(r)
            for p in p_grid:
                e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                u, v = tree.velocity(g, P.sigma, p, V.FP32)
                e1.record()
                if tg is not None:
                    u = u[tg].contiguous(); v = v[tg].contiguous()
                emax, _, _ = V.error_metrics(u, v, ur, vr)
                f = V.selector_features(stats, n, P.sigma, p, L, r)
                rows.append((f, math.log10(max(emax, 10 ** LOG10_FLOOR)), p, L, r,
                             e0.elapsed_time(e1)))
        tree.close()
    return rows


def generate(n_instances, seed, out, n_range=(2 ** 11, 2 ** 18), log=print, radii=(0.0,)):
    """Training rows of n_instances seeded instances; meta holds (instance, N,
    p, L, ms, radius) per row."""
    rng = np.random.default_rng(seed)
    F, Y, meta = [], [], []
    t0 = time.time()
    for i in range(n_instances):
        P = random_instance(rng, n_range)
        for f, lg, p, L, r, ms in evaluate_grid(P, seed=i, radii=radii):
            F.append(f); Y.append(lg); meta.append((i, P.n, p, L, ms, r))
        if (i + 1) % 5 == 0 or i + 1 == n_instances:
            log(f"[generate] {i + 1}/{n_instances} instances, {len(Y)} rows, {time.time() - t0:.1f} s")
            # written as it goes: a run cut short keeps the instances done so far
            np.savez_compressed(out, features=np.array(F, np.float32),
                                target=np.array(Y, np.float32), meta=np.array(meta, np.float64),
                                seed=seed)
    return len(Y)


# ----------------------------------------------------------------- training

def _he_init(seed):
    """He-style initial parameters (weights N(0, 2/fan_in), zero biases)."""
    rng = np.random.default_rng(seed)
    w1 = rng.normal(0, math.sqrt(2.0 / 10), (10, 64)); w2 = rng.normal(0, math.sqrt(2.0 / 64), (64, 64))
    w3 = rng.normal(0, math.sqrt(1.0 / 64), 64)
    return np.concatenate([w1.ravel(), np.zeros(64), w2.ravel(), np.zeros(64), w3, np.zeros(1)]).astype(np.float32)


def train(data_paths, out, epochs=300, batch=256, lr=3e-3, seed=0, val_frac=0.2, log=print):
    """Trains the selector on the GPU on the rows of one or more data files
    (their instances kept apart); writes params, feature mean/std and metrics."""
    torch = _torch()
    if isinstance(data_paths, str):
        data_paths = data_paths.split(",")
    Fs, Ys, insts = [], [], []
    for k, path in enumerate(data_paths):
        d = np.load(path)
        Fs.append(d["features"].astype(np.float64)); Ys.append(d["target"].astype(np.float64))
        insts.append(d["meta"][:, 0].astype(np.int64) + 1_000_000 * k)
    F = np.concatenate(Fs); Y = np.concatenate(Ys); inst = np.concatenate(insts)
    rng = np.random.default_rng(seed)
    ids = np.unique(inst)
    val_ids = set(rng.choice(ids, max(1, int(len(ids) * val_frac)), replace=False).tolist())
    val = np.array([i in val_ids for i in inst])
    mean = F[~val].mean(0); std = F[~val].std(0)
    std[std == 0] = 1.0
    Z = ((F - mean) / std).astype(np.float32)
    Xt = torch.from_numpy(Z[~val]).cuda(); Tt = torch.from_numpy(Y[~val].astype(np.float32)).cuda()
    Xv = torch.from_numpy(Z[val]).cuda(); Tv = Y[val]
    params = torch.from_numpy(_he_init(seed)).cuda()
    tr = V.MlpTrainer(params, batch)
    nt = Xt.shape[0]
    steps = 0
    t0 = time.time()
    # the parameters with the lowest validation error, checked every 10 epochs
    best = (math.inf, None, 0)
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(nt).astype(np.int64)).cuda()
        lr_ep = lr * 0.5 * (1 + math.cos(math.pi * ep / epochs)) + 1e-5
        for s in range(0, nt - batch + 1, batch):
            idx = perm[s:s + batch]
            tr.step(Xt[idx].contiguous(), Tt[idx].contiguous(), lr_ep)
            steps += 1
        if (ep + 1) % 10 == 0 or ep == epochs - 1:
            pv = V.mlp_forward(tr.params, Xv).cpu().numpy()
            rmse = float(np.sqrt(np.mean((pv - Tv) ** 2)))
            if rmse < best[0]:
                best = (rmse, tr.params.clone(), ep + 1)
            if (ep + 1) % 50 == 0 or ep == epochs - 1:
                log(f"[train] epoch {ep + 1}: val rmse {rmse:.3f} (log10 units), "
                    f"{time.time() - t0:.1f} s")
    tr.params.copy_(best[1])
    log(f"[train] kept the parameters of epoch {best[2]} (val rmse {best[0]:.3f})")
    pv = V.mlp_forward(tr.params, Xv).cpu().numpy()
    pt = V.mlp_forward(tr.params, Xt).cpu().numpy()
    resid = pv - Tv
    metrics = {"train_rmse": float(np.sqrt(np.mean((pt - Y[~val]) ** 2))),
               "val_rmse": float(np.sqrt(np.mean(resid ** 2))),
               "val_q95_underprediction": float(np.quantile(-resid, 0.95)),
               "rows_train": int(nt), "rows_val": int(val.sum()), "steps": steps, "epochs": epochs,
               "kept_epoch": best[2]}
    margin = max(0.3, metrics["val_q95_underprediction"])
    np.savez(out, params=tr.params.cpu().numpy(), mean=mean.astype(np.float32),
             std=std.astype(np.float32), margin=np.float64(margin), metrics=json.dumps(metrics))
    log(f"[train] {json.dumps(metrics)} margin {margin:.3f}")
    return metrics


# ----------------------------------------------------------------- selection

def load_weights(path=WEIGHTS_PATH):
    torch = _torch()
    d = np.load(path)
    return (torch.from_numpy(d["params"].astype(np.float32)).cuda(), d["mean"].astype(np.float32),
            d["std"].astype(np.float32), float(d["margin"]))


def conservative_choice(side, sigma, n):
    """p = 20 and the deepest level whose leaf side is >= 8 sigma."""
    L = 0
    while L + 1 <= V.MAX_LEVELS and side / 2 ** (L + 1) / sigma >= 8.0 and 4 ** (L + 1) <= 4 * n:
        L += 1
    return 20, L


def select_and_audit(x, y, g, sigma, tol, weights=None, n_audit=8192, seed=0, audit=True,
                     slack=0.5, targets=None, reference=None, cutoff=True, time_reps=3):
    """Selected (p, L), audited by the FP64 direct sum on sampled targets
    (``vfmm_select_and_audit``; this function only marshals arguments).

    The network's choice is evaluated in FP32 and accepted if its error on the
    audit targets is <= slack * tol (slack 0.5: the largest error over all
    particles was measured at up to 1.8 times the largest over a sample of
    16384 of them, the truncation error having a thin tail); otherwise p is
    raised by 2 at the same
    level (up to 20) and audited again; if FP32 still misses, the conservative
    choice is evaluated in FP64.  With ``cutoff``, an accepted FP32 choice is
    compared with the same p one or two levels deeper under the distance
    cut-off of the near field (Section 4.1's distance a) at two radii; the
    fastest passing candidate replaces the choice if it is more than 3 % faster.
    The trial trees take the process-wide tuning (set it first, e.g. with
    ``autotune.apply_for``).

    ``targets`` (device int64) and ``reference`` ((u, v) of the direct sum
    there) may be supplied; otherwise n_audit targets are drawn with ``seed``.
    Returns a dict with the choice (p, levels, radius: 0, > 0 or
    NEAR_RADIUS_AUTO, precision), the audited error, the network's prediction
    and the audit trail [p, L, mode, e_max, ms].
    """
    torch = _torch()
    params, mean, std, margin = weights if weights is not None else load_weights()
    n = int(x.shape[0])
    if targets is None:
        rng = np.random.default_rng(seed)
        targets = torch.from_numpy(np.sort(rng.choice(n, min(n, n_audit), replace=False))
                                   .astype(np.int64)).cuda()
    r = V.select_and_audit(x, y, g, sigma, tol, params, mean, std, margin, targets,
                           reference=reference, audit=audit, cutoff=cutoff, slack=slack,
                           time_reps=time_reps)
    out = {"p": r.p, "levels": r.levels, "predicted_log10": r.predicted_log10,
           "fallback": bool(r.used_fallback), "audited": bool(audit),
           "precision": "fp64" if r.precision == V.FP64 else "fp32",
           "radius": r.near_radius,
           "network_choice": [r.network_p, r.network_levels, r.network_radius]}
    if audit:
        trail = []
        for k in range(r.n_steps):
            st = r.steps[k]
            mode = "fp64" if st.precision == V.FP64 else "fp32"
            if st.near_radius != 0.0:
                mode += " +cutoff " + ("auto" if st.near_radius < 0
                                       else f"{st.near_radius / sigma:.2f} sigma")
            trail.append([st.p, st.levels, mode.replace(" +", "+"), st.emax,
                          st.ms if st.ms >= 0 else None])
        out.update(audit_emax=r.audit_emax, trail=trail)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("--instances", type=int, default=400)
    g.add_argument("--seed", type=int, default=1)
    g.add_argument("--out", required=True)
    g.add_argument("--nmax-log2", type=int, default=18)
    g.add_argument("--cutoff", action="store_true",
                   help="also run every grid point with the distance cut-off (both radii)")
    t = sub.add_parser("train")
    t.add_argument("--data", required=True)
    t.add_argument("--out", default=WEIGHTS_PATH)
    t.add_argument("--epochs", type=int, default=300)
    t.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)
    if a.cmd == "generate":
        log = lambda m: print(m, flush=True)
        radii = (0.0, V.NEAR_RADIUS_AUTO, "tol") if a.cutoff else (0.0,)
        rows = generate(a.instances, a.seed, a.out, (2 ** 11, 2 ** a.nmax_log2), log, radii)
        print(f"[generate] wrote {rows} rows to {a.out}", flush=True)
    else:
        train(a.data, a.out, epochs=a.epochs, seed=a.seed, log=lambda m: print(m, flush=True))


if __name__ == "__main__":
    sys.exit(main())
