"""Benchmark: FMM velocity of N = 2^20 clustered vortex particles on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload clusters_1m]

A step is one pass of the whole method on device-resident float64 inputs:
quadtree rebuild (root box, keys, sort, leaf ranges) + FMM velocity (gather,
P2M, M2M, M2L + L2L, P2P, L2P), i.e. N / t particles per second.  The K timed
steps are captured into one hipGraph after the warm-up and replayed (once
untimed, then timed), so the host's launch rate does not pace the short
kernels of the rebuild; --eager issues them one call at a time instead (both
times are reported).
Two paths are timed on the same particles:

* tuned: float32 arithmetic on scaled coefficients, (p, levels) chosen by the
  learned selector to meet a max error of 1e-6 (normalised by max |u|) against
  the float64 direct sum, audited on sampled targets (selection and audit are
  reported separately and not part of a step);
* plain: everything in float64, p = 20 and the largest level with
  box side / sigma >= 8.

Accuracy of both is measured against the float64 direct sum on 4096 sampled
hold-out targets, disjoint from the 16384 targets of the selector's audit.
The P2P kernel (the dominant one) is timed with HIP events around its
launches inside the timed region; its roofline uses 15 algorithmic FLOPs
per pair (2 sub, r^2 = 3, exponent argument 1, exp 1, 1 - e 1, reciprocal 1,
2 products, 2 fused accumulations = 4) against the MI355X FP32 vector peak.
The CPU baseline is the float64 NumPy oracle on a bounded sample of targets.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "particles/s at N=1M, max rel err ≤1e-6 vs FP64 direct; tuned vs plain FP64"
FP32_PEAK_TFLOPS = 157.3
P2P_FLOPS_PER_PAIR = 15
AUDIT_TARGETS = 4096      # the metric's sample: accuracy is reported on this many hold-out targets
SELECT_AUDIT_TARGETS = 16384  # the selector's audit: the truncation error has a thin tail
HOLDOUT_SEED = 7919
CPU_MAX_WORKERS = 16


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def largest_level(side, sigma, ratio=8.0, lmax=12):
    """Largest L with (S / 2^L) / sigma >= ratio."""
    L = 0
    while L + 1 <= lmax and side / 2 ** (L + 1) / sigma >= ratio:
        L += 1
    return L


def m2l_pairs(levels):
    """(box, interaction-list box) pairs of levels 2..L: children of the
    parent's neighbours that are not adjacent, within the level's grid."""
    total = 0
    for lev in range(2, levels + 1):
        m = 1 << lev
        i = np.arange(m)
        # along one axis: count of j in [2(i//2) - 2, 2(i//2) + 3] within [0, m)
        lo = np.maximum(2 * (i // 2) - 2, 0); hi = np.minimum(2 * (i // 2) + 3, m - 1)
        span = hi - lo + 1
        near = np.minimum(i + 1, m - 1) - np.maximum(i - 1, 0) + 1
        total += int(np.sum(np.outer(span, span) - np.outer(near, near)))
    return total


def p2p_pairs(leaf_start, levels):
    """Ordered (target, source) pairs of the near field, self pairs included."""
    m = 1 << levels
    cnt = np.diff(leaf_start.astype(np.int64)).reshape(m, m)
    pad = np.pad(cnt, 1)
    nb = sum(pad[1 + dy:1 + dy + m, 1 + dx:1 + dx + m] for dy in (-1, 0, 1) for dx in (-1, 0, 1))
    return int(np.sum(cnt * nb))


def holdout_targets(n, k, exclude, seed):
    """k distinct indices in [0, n) outside ``exclude``, drawn with another seed
    (sorted int64): the sample on which the tuned accuracy is reported."""
    pool = np.setdiff1d(np.arange(n, dtype=np.int64), np.asarray(exclude, np.int64))
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(pool, size=min(k, pool.size), replace=False)).astype(np.int64)


_CPU = {}


def _cpu_chunk(idx):
    """One worker's share of the CPU baseline: the oracle's evaluation after the
    upward sweep (downward sweep, L2P, near field, cut-off) at whole leaves."""
    from threadpoolctl import threadpool_limits
    from oracle import fmm as OF
    s = _CPU
    with threadpool_limits(1):
        OF.evaluate_targets(s["x"], s["y"], s["g"], s["sigma"], s["p"], s["tree"], s["me"], idx,
                            s["radius"])
    return len(idx)


def cpu_oracle_child(spec):
    """Runs in a child process (no GPU): times the float64 NumPy oracle FMM at
    sampled targets, once on one thread and once over all usable cores (the
    tree and upward sweep in this process, then whole target leaves spread over
    forked workers), and prints the timings as one JSON line."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from oracle import fmm as OF
    P = W.config(spec["workload"])
    ts = W.sample_targets(P.n, spec["targets"], seed=99)
    p, L, radius = spec["p"], spec["levels"], spec["radius"]
    cores = max(1, min(CPU_MAX_WORKERS, len(os.sched_getaffinity(0))))
    res = {}
    for workers in (1, cores):
        with threadpool_limits(1):
            t0 = time.perf_counter()
            tree = OF.build_tree(P.x, P.y, L)
            me = OF.upward_sweep(P.x + 1j * P.y, P.gamma, tree, p) if L >= 2 else {}
            t_up = time.perf_counter() - t0
            key = tree.leaf_key()[ts]
            order = np.argsort(key, kind="stable")
            cuts = np.nonzero(np.diff(key[order]))[0] + 1
            leaves = np.split(ts[order], cuts)
            # whole leaves per chunk, about 8 chunks per worker
            nchunk = max(1, min(len(leaves), 8 * workers))
            chunks = [np.concatenate(leaves[b[0]:b[-1] + 1])
                      for b in np.array_split(np.arange(len(leaves)), nchunk) if len(b)]
            _CPU.update(x=P.x, y=P.y, g=P.gamma, sigma=P.sigma, p=p, tree=tree, me=me,
                        radius=radius)
            if workers == 1:
                for c in chunks:
                    _cpu_chunk(c)
            else:
                with mp.get_context("fork").Pool(workers) as pool:
                    pool.map(_cpu_chunk, chunks, chunksize=1)
            dt = time.perf_counter() - t0
        res[workers] = (dt, t_up)
    print(json.dumps({"n_targets": int(len(ts)), "cores": cores,
                      "one": res[1], "all": res[cores]}), flush=True)


def cpu_baseline(workload, p, levels, radius, n_targets):
    """The oracle timed in a child process (see cpu_oracle_child)."""
    import subprocess
    spec = json.dumps({"workload": workload, "p": p, "levels": levels, "radius": radius,
                       "targets": n_targets})
    r = subprocess.run([sys.executable, "-u", os.path.abspath(__file__), "--cpu-oracle-child", spec],
                       capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"CPU oracle child failed ({r.returncode}): {r.stderr[-2000:]}")
    d = json.loads(r.stdout.strip().splitlines()[-1])
    nt, cores = d["n_targets"], d["cores"]
    (t1, up1), (tc, upc) = d["one"], d["all"]
    what = (f"float64 NumPy oracle FMM (p={p}, levels={levels}, near cut-off radius {radius:.4g}) "
            f"evaluated at {nt} sampled targets of the same workload, tree and full upward sweep "
            f"included")
    return {"value": round(nt / tc, 2), "unit": "particles/s", "cores": cores, "kind": "oracle",
            "sample": f"{what}; {tc:.1f} s on {cores} cores (upward sweep {upc:.1f} s in one "
                      f"process, then whole target leaves over {cores} forked workers, one "
                      f"thread each)",
            "one_core": {"value": round(nt / t1, 2), "cores": 1,
                         "sample": f"{what}; {t1:.1f} s on 1 thread (upward sweep {up1:.1f} s)"}}


def fixed_radius(a, sigma, vf):
    if a.radius_sigma > 0:
        return a.radius_sigma * sigma
    return vf.NEAR_RADIUS_AUTO if a.cutoff else 0.0


def radius_tag(radius, sigma):
    """The near radius as recorded with measurements: "auto", 0, or in sigma (3 decimals)."""
    return "auto" if radius < 0 else (0.0 if radius == 0 else round(radius / sigma, 3))


def recorded_traffic(workload, p, levels, radius=0.0, sigma=1.0, sym=0):
    """HBM bytes per P2P launch from the committed rocprofv3 counter runs, or None
    when the kernel source or the configuration (symmetric near field included)
    differs from the measured one."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "p2p_traffic_clusters_1m.json")
    csrc = os.path.join(ROOT, "paper_0809_1810_amd", "csrc")
    try:
        rec = json.load(open(path))
        cur = hashlib.sha256(open(os.path.join(csrc, "p2p.hip"), "rb").read()).hexdigest()
        cur_math = hashlib.sha256(open(os.path.join(csrc, "p2p_math.hpp"), "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if (rec.get("p2p_source_sha256") != cur or rec.get("p2p_math_sha256") != cur_math
            or rec.get("workload") != workload
            or rec.get("p") != p or rec.get("levels") != levels
            or rec.get("near_radius_sigma", 0.0) != radius_tag(radius, sigma)
            or rec.get("sym", 0) != sym):
        return None
    return float(rec["traffic_bytes"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="clusters_1m")
    ap.add_argument("--p", type=int, default=None, help="override the tuned expansion order")
    ap.add_argument("--levels", type=int, default=None, help="override the tuned level")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--cutoff", action="store_true",
                    help="with --p/--levels: use the automatic distance cut-off of the near field")
    ap.add_argument("--radius-sigma", type=float, default=0.0,
                    help="with --p/--levels: distance cut-off radius in units of sigma")
    ap.add_argument("--cpu-targets", type=int, default=65536)
    ap.add_argument("--audit-targets", type=int, default=0,
                    help="sampled targets of the selector's FP64 direct-sum audit (default "
                         "16384); the accuracy is reported on 4096 other targets")
    ap.add_argument("--eager", action="store_true",
                    help="issue the timed steps eagerly instead of replaying them from a hipGraph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-adaptive", action="store_true",
                    help="skip the adaptive-quadtree A/B at the tuned parameters")
    ap.add_argument("--no-lattice", action="store_true",
                    help="skip the second N = 1M input (the 1024^2 lattice)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run a plain elementwise copy of this many MiB (float64), "
                         "used to scale HBM byte counters")
    ap.add_argument("--eval-lattice", type=int, default=0, metavar="M",
                    help="instead of the N=1M line, evaluate the FMM of the workload at an "
                         "M x M lattice of separate points covering the root square")
    ap.add_argument("--p2p-tile", type=int, default=0,
                    help="override the autotuned near-field tile (64, 32 or 16 targets)")
    ap.add_argument("--p2p-sym", type=int, default=-1, choices=(-1, 0, 1),
                    help="symmetric near field for the trees of this run (-1: the tuning table's)")
    ap.add_argument("--p2p-waves", type=int, default=0,
                    help="override the autotuned near-field waves per workgroup (1, 2, 4, 8)")
    ap.add_argument("--advect", type=int, default=0, metavar="K",
                    help="instead of the N=1M line, time K steps of advecting the particles with "
                         "their FMM velocity (Heun's method, two evaluations and rebuilds per step)")
    ap.add_argument("--cpu-oracle-child", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--batched", action="store_true",
                    help="instead of the N=1M line, time 256 uneven instances evaluated as one "
                         "batch (graph replay) against one call per instance")
    a = ap.parse_args()

    if a.cpu_oracle_child is not None:  # the CPU baseline's child process (no GPU)
        return cpu_oracle_child(json.loads(a.cpu_oracle_child))

    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the multi-GPU "
              "sharding of this method is a design note, not an implemented path.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_0809_1810_amd as vf

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    vf.lib()

    if a.batched:
        return bench_batched(a, torch, vf)
    if a.eval_lattice > 0:
        return bench_eval_points(a, torch, vf)
    if a.advect > 0:
        return bench_advect(a, torch, vf)

    if a.calibrate_copy_mib > 0:
        src = torch.ones(a.calibrate_copy_mib * (1 << 17), dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {a.calibrate_copy_mib} MiB read + written, 3 times")
        del src, dst

    P = W.config(a.workload)
    n = P.n
    n_audit = a.audit_targets or SELECT_AUDIT_TARGETS
    log(f"[bench] workload {P.name} n={n} sigma={P.sigma}")
    x = torch.from_numpy(P.x).cuda(); y = torch.from_numpy(P.y).cuda()
    g = torch.from_numpy(P.gamma).cuda()
    probe = vf.Tree(x, y, 0, p_max=1)        # root square of the library's tree
    side = float(probe.arrays()[0][2].item())
    probe.close()

    # ---------------- audit targets and FP64 direct reference; a second,
    # disjoint hold-out sample (another seed) on which the accuracy is reported
    tg = W.sample_targets(n, n_audit, seed=2024)
    tg_d = torch.from_numpy(tg).cuda()
    ud, vd = vf.direct_velocity(x, y, g, P.sigma, targets=tg_d)
    th = holdout_targets(n, AUDIT_TARGETS, tg, HOLDOUT_SEED)
    th_d = torch.from_numpy(th).cuda()
    uh, vh = vf.direct_velocity(x, y, g, P.sigma, targets=th_d)
    torch.cuda.synchronize()

    # ---------------- parameter choice
    L_plain = largest_level(side, P.sigma, 8.0)
    p_plain = 20
    prec_t = vf.PRECISIONS[a.precision]
    sel_info = None
    radius_t = 0.0
    if a.p is not None and a.levels is not None:
        p_t, L_t, selector = a.p, a.levels, "fixed"
        radius_t = fixed_radius(a, P.sigma, vf)
    else:
        from paper_0809_1810_amd import selector as S
        weights = S.load_weights()
        s0 = time.perf_counter()
        selection_shape(P)
        r = S.select_and_audit(x, y, g, P.sigma, 1e-6, weights=weights, targets=tg_d,
                               reference=(ud, vd))
        torch.cuda.synchronize()
        sel_ms = (time.perf_counter() - s0) * 1e3
        p_t, L_t, radius_t = r["p"], r["levels"], r["radius"]
        if r["precision"] == "fp64":
            prec_t = vf.FP64
        selector = "learned" if not r["fallback"] else "fallback"
        sel_info = {"predicted_log10_emax": r["predicted_log10"], "audit_emax": r["audit_emax"],
                    "fallback": r["fallback"], "network_choice": r["network_choice"],
                    "audit_trail": r["trail"], "select_and_audit_ms": round(sel_ms, 2)}
        log(f"[bench] selector: {json.dumps(r)} in {sel_ms:.1f} ms")


    from paper_0809_1810_amd import autotune as AT

    def run_path(L, p, prec, steps, warmup, timing=False, radius=0.0, capacity=None):
        # near-field launch shape from the autotuner's table (mean and spread of the leaf occupancy)
        AT.apply_for(n, L, cutoff=radius != 0.0, spread=AT.leaf_spread(P.x, P.y, L))
        override_tuning(a, vf)
        tree = vf.Tree(x, y, L, p_max=p)
        tree.set_near_radius(radius)
        u = torch.empty(n, dtype=torch.float64, device="cuda")
        v = torch.empty(n, dtype=torch.float64, device="cuda")

        def step():
            tree.rebuild(x, y)
            if capacity is None:
                tree.velocity(g, P.sigma, p, prec, out=(u, v))
            else:  # adaptive tree: leaves of at most `capacity` particles above level L
                tree.velocity_adaptive(g, P.sigma, p, capacity, prec, out=(u, v))
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        # the K steps issued eagerly, with the phase events (the near-field
        # kernel's launch durations, the adaptive tree's A/B); then, for the
        # uniform tree, the same K steps replayed from one hipGraph: the timed
        # result (events recorded during a capture take no replay timestamps)
        eager_ms, wall, phases = time_steps(torch, step, steps, tree if timing else None, False)
        ms = eager_ms
        if capacity is None and not a.eager:
            ms, wall, _ = time_steps(torch, step, steps, None, True)
        emax, erms, _ = vf.error_metrics(u[tg_d].contiguous(), v[tg_d].contiguous(), ud, vd)
        hmax, hrms, _ = vf.error_metrics(u[th_d].contiguous(), v[th_d].contiguous(), uh, vh)
        far_phases = []
        if timing and L >= 2 and capacity is None:
            # the expansion sweeps alone (far part only: no near field runs
            # beside them), after the timed region, for their own rooflines
            tree.enable_timing(steps)
            for _ in range(steps):
                tree.velocity(g, P.sigma, p, prec, parts=vf.PART_FAR, out=(u, v))
            far_phases = tree.read_timing()
        _, _, ls = tree.arrays()
        pairs = p2p_pairs(ls.cpu().numpy(), L)
        tw = tree.tuning()
        tree.close()
        return dict(ms=ms, eager_ms=eager_ms, wall_s=wall, phases=phases, far_phases=far_phases,
                    emax=emax, erms=erms,
                    holdout_emax=hmax, holdout_erms=hrms,
                    pairs=pairs, tile_waves=[tw["tile"], tw["waves"]], sym=tw["sym"])

    log(f"[bench] tuned: p={p_t} L={L_t} precision={a.precision} near radius={radius_t}")
    tuned = run_path(L_t, p_t, prec_t, a.steps, a.warmup, timing=True, radius=radius_t)
    log(f"[bench] tuned {tuned['ms']:.3f} ms/step emax={tuned['emax']:.3e} "
        f"(hold-out {tuned['holdout_emax']:.3e})")
    # the same method on an adaptive quadtree (A/B against the uniform tree)
    adaptive = []
    if not a.no_adaptive and L_t >= 3:
        for cap in (64, 256):
            r_ad = run_path(L_t, p_t, prec_t, a.steps, a.warmup, timing=True, radius=radius_t,
                            capacity=cap)
            adaptive.append({"leaf_capacity": cap, "levels_max": L_t,
                             "ms_per_step": round(r_ad["ms"], 4),
                             "p2p_ms": round(float(np.mean([ph["p2p"] for ph in r_ad["phases"]])), 4),
                             "holdout_emax": r_ad["holdout_emax"]})
            log(f"[bench] adaptive capacity {cap}: {r_ad['ms']:.3f} ms/step "
                f"(hold-out {r_ad['holdout_emax']:.3e})")
    plain = None
    if not a.no_plain:
        log(f"[bench] plain: p={p_plain} L={L_plain} fp64")
        plain = run_path(L_plain, p_plain, vf.FP64, a.steps, a.warmup, timing=True)
        log(f"[bench] plain {plain['ms']:.3f} ms/step emax={plain['emax']:.3e}")

    # ---------------- roofline of the dominant kernel (near field)
    p2p_ms = float(np.mean([ph["p2p"] for ph in tuned["phases"]]))
    achieved = P2P_FLOPS_PER_PAIR * tuned["pairs"] / (p2p_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                "traffic": recorded_traffic(a.workload, p_t, L_t, radius_t, P.sigma, tuned["sym"]),
                "kernel": "k_p2p<float> (symmetric near field)" if tuned["sym"] else "k_p2p<float>",
                "kernel_ms": round(p2p_ms, 4),
                "kernel_ms_from": "HIP events around the kernel's launches on its stream in the "
                                  "K timed steps issued eagerly (the same steps as the "
                                  "graph-replayed ones)",
                "pairs_per_launch": tuned["pairs"], "flops_per_pair": P2P_FLOPS_PER_PAIR,
                "work_counted": "local-list pairs only (cut-off ring pairs not counted)"
                if radius_t else "local-list pairs"}

    # ---------------- CPU baseline: the oracle on a bounded sample of targets,
    # in a child process that never touches the GPU (it forks its own workers)
    cpu = None
    if not a.no_cpu_baseline:
        r_cpu = 0.0
        if radius_t != 0.0:
            r_auto = (6.0 if prec_t != vf.FP64 else math.sqrt(76.0)) * P.sigma
            r_cpu = min(r_auto if radius_t < 0 else radius_t, vf.NEAR_RINGS_MAX * side / 2 ** L_t)
        log(f"[bench] cpu baseline: oracle FMM (p={p_t}, L={L_t}, radius={r_cpu:.4g}) "
            f"on {a.cpu_targets} targets, 1 thread and all cores")
        cpu = cpu_baseline(a.workload, p_t, L_t, r_cpu, a.cpu_targets)
        log(f"[bench] cpu {cpu['value']} particles/s ({cpu['cores']} cores), "
            f"1 thread {cpu['one_core']['value']}")

    value = n / (tuned["ms"] * 1e-3)
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(tuned["ms"], 4),
        "eager_ms_per_step": round(tuned["eager_ms"], 4),
        "timed_as": "eager calls" if a.eager else "one hipGraph replay of the K captured steps",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{P.name}: N={n}, sigma={P.sigma}, seeded synthetic",
            "p": p_t, "levels": L_t, "precision": "fp64" if prec_t == vf.FP64 else a.precision,
            "selector": selector, "selector_info": sel_info, "audit_targets": n_audit,
            "p2p_tile_waves": tuned["tile_waves"], "p2p_symmetric": bool(tuned["sym"]),
            "near_radius": ("auto: min(6 sigma, 4 w_L), distance cut-off of the near field"
                            if radius_t < 0 else radius_t),
            "near_radius_sigma": radius_tag(radius_t, P.sigma),
        },
        "accuracy": {"tuned_emax": tuned["holdout_emax"], "tuned_erms": tuned["holdout_erms"],
                     "holdout_emax": tuned["holdout_emax"], "holdout_erms": tuned["holdout_erms"],
                     "holdout_targets": int(len(th)), "holdout_seed": HOLDOUT_SEED,
                     "selection_sample_emax": tuned["emax"],
                     "selection_sample_erms": tuned["erms"],
                     "note": "tuned_emax is measured on the hold-out sample, disjoint from "
                             "the targets the selector's audit used"},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if plain is not None:
        out["plain_fp64"] = {"value": round(n / (plain["ms"] * 1e-3), 1), "ms_per_step": round(plain["ms"], 4),
                             "p": p_plain, "levels": L_plain, "emax": plain["holdout_emax"],
                             "erms": plain["holdout_erms"],
                             "p2p_ms": round(float(np.mean([ph["p2p"] for ph in plain["phases"]])), 4)}
        out["speedup_vs_plain"] = round(plain["ms"] / tuned["ms"], 3)
    out["phases_ms"] = {k: round(float(np.mean([ph[k] for ph in tuned["phases"]])), 4)
                        for k in tuned["phases"][0]}
    if prec_t != vf.FP64 and L_t >= 2:
        # M2L on the matrix cores: 8 p^2 FLOP per (box, interaction box) pair,
        # over the M2L + L2L phase (the L2L, two short launches at L = 7, is
        # part of it); sweep
        # phases from the far-only evaluations (in a full evaluation they share
        # the GPU with the near field)
        ph = {k: round(float(np.mean([f[k] for f in tuned["far_phases"]])), 4)
              for k in tuned["far_phases"][0]}
        out["sweeps_alone_ms"] = {k: ph[k] for k in ("tables", "p2m", "m2m", "m2l_l2l", "l2p")}
        m2l_flop = 8.0 * p_t * p_t * m2l_pairs(L_t)
        ach = m2l_flop / (ph["m2l_l2l"] * 1e-3) / 1e12
        out["m2l_roofline"] = {"bound": "mfma", "achieved": round(ach, 3), "peak": FP32_PEAK_TFLOPS,
                               "unit": "TFLOP/s", "frac": round(ach / FP32_PEAK_TFLOPS, 4),
                               "kernel": "k_m2l_mfma_f32 (+ k_l2l_span)", "ms": ph["m2l_l2l"],
                               "pairs": m2l_pairs(L_t), "flops_per_pair": 8 * p_t * p_t}
        # expansion sweeps: P2M reads the sorted particles (16 B) and writes the
        # leaf MEs; M2M reads 4 children and writes one parent per level (8 B / coefficient)
        nb = sum(4 ** l for l in range(2, L_t + 1))
        p2m_b = 16.0 * n + 8.0 * p_t * 4 ** L_t
        m2m_b = 8.0 * p_t * (nb - 4 ** 2 + nb - 4 ** L_t)
        sw_ms = ph["p2m"] + ph["m2m"]
        out["sweeps_hbm"] = {"bound": "hbm", "achieved": round((p2m_b + m2m_b) / (sw_ms * 1e-3) / 1e9, 1),
                             "peak": 8000.0, "unit": "GB/s",
                             "frac": round((p2m_b + m2m_b) / (sw_ms * 1e-3) / 8e12, 4),
                             "kernel": "k_p2m + k_m2m", "ms": round(sw_ms, 4),
                             "bytes": p2m_b + m2m_b}
    if adaptive:
        out["adaptive_tree"] = {
            "uniform_ms_per_step": round(tuned["eager_ms"], 4),
            "uniform_p2p_ms": out["phases_ms"]["p2p"],
            "runs": adaptive,
            "note": "the same p, deepest level and near radius on the adaptive quadtree (box "
                    "split above the leaf capacity); the step includes sorting the particles "
                    "into the adaptive leaves; both trees' steps issued eagerly"}
    if not a.no_lattice and a.workload == "clusters_1m":
        out["lattice_1m"] = second_input(a, torch, vf, "lattice_1024")
    print(json.dumps(out), flush=True)


def second_input(a, torch, vf, name):
    """The same metric on the second N = 1M input: selection with audit (and the
    cut-off comparison), then K timed rebuild + evaluation steps of the tuned
    path and of the plain FP64 path; errors against the FP64 direct sum on 4096
    sampled targets."""
    from paper_0809_1810_amd import autotune as AT
    from paper_0809_1810_amd import selector as S
    P = W.config(name)
    n = P.n
    x = torch.from_numpy(P.x).cuda(); y = torch.from_numpy(P.y).cuda()
    g = torch.from_numpy(P.gamma).cuda()
    probe = vf.Tree(x, y, 0, p_max=1)
    side = float(probe.arrays()[0][2].item())
    probe.close()
    tg_h = W.sample_targets(n, SELECT_AUDIT_TARGETS, seed=2024)
    tg = torch.from_numpy(tg_h).cuda()
    ud, vd = vf.direct_velocity(x, y, g, P.sigma, targets=tg)
    th = torch.from_numpy(holdout_targets(n, AUDIT_TARGETS, tg_h, HOLDOUT_SEED)).cuda()
    uh, vh = vf.direct_velocity(x, y, g, P.sigma, targets=th)
    selection_shape(P)
    r = S.select_and_audit(x, y, g, P.sigma, 1e-6, weights=S.load_weights(), targets=tg,
                           reference=(ud, vd))
    prec = vf.FP64 if r["precision"] == "fp64" else vf.FP32

    def run(L, p, pr, radius):
        AT.apply_for(n, L, cutoff=radius != 0.0, spread=AT.leaf_spread(P.x, P.y, L))
        override_tuning(a, vf)
        t = vf.Tree(x, y, L, p_max=p)
        t.set_near_radius(radius)
        u = torch.empty(n, dtype=torch.float64, device="cuda")
        v = torch.empty(n, dtype=torch.float64, device="cuda")
        def step():
            t.rebuild(x, y)
            t.velocity(g, P.sigma, p, pr, out=(u, v))
        for _ in range(a.warmup):
            step()
        torch.cuda.synchronize()
        ms = time_steps(torch, step, a.steps, None, not a.eager)[0]
        emax, _, _ = vf.error_metrics(u[th].contiguous(), v[th].contiguous(), uh, vh)
        t.close()
        return ms, emax

    ms_t, e_t = run(r["levels"], r["p"], prec, r["radius"])
    Lp = largest_level(side, P.sigma, 8.0)
    ms_p, e_p = run(Lp, 20, vf.FP64, 0.0)
    return {"workload": f"{name}: {int(round(n ** 0.5))}^2 cell-centred lattice in [-1,1]^2, "
                        f"Lamb-Oseen pair, sigma = h/0.8 = {P.sigma:.4g}",
            "value": round(n / (ms_t * 1e-3), 1), "unit": "particles/s",
            "ms_per_step": round(ms_t, 4), "p": r["p"], "levels": r["levels"],
            "precision": r["precision"], "near_radius": "auto" if r["radius"] < 0 else r["radius"],
            "emax": e_t, "emax_sample": "hold-out: 4096 targets disjoint from the audit's",
            "audit_emax": r["audit_emax"], "audit_trail": r["trail"],
            "plain_fp64": {"ms_per_step": round(ms_p, 4), "p": 20, "levels": Lp, "emax": e_p},
            "speedup_vs_plain": round(ms_p / ms_t, 3)}


def time_steps(torch, step, steps, tree=None, graph=True):
    """Mean ms of K steps, timed with HIP events on the current stream around
    one replay of a hipGraph that holds the K steps (captured after the warm-up
    and replayed once untimed, which uploads it), or around the K steps issued
    eagerly.  With a tree (eager steps only: its phase events take no
    timestamps inside a replayed graph), the phase times of the K steps are
    read back.  Returns (ms, wall seconds, phases)."""
    assert tree is None or not graph
    if tree is not None:
        tree.enable_timing(steps)
    graph_k = None
    if graph:
        graph_k = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph_k):
            for _ in range(steps):
                step()
        graph_k.replay()
        torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    if graph_k is not None:
        graph_k.replay()
    else:
        for _ in range(steps):
            step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phases = tree.read_timing() if tree is not None else []
    del graph_k
    return e0.elapsed_time(e1) / steps, wall, phases


def selection_shape(P):
    """The selection's trial trees take the process-wide launch shape: set the
    tuning table's shape for about 64 particles per leaf with the cut-off (and
    the input's leaf-occupancy spread there), so that every workload's
    candidates are timed the way their timed path runs."""
    from paper_0809_1810_amd import autotune as AT
    L = max(2, int(round(math.log(max(P.n, 64) / 64.0, 4))))
    AT.apply_for(P.n, L, cutoff=True, spread=AT.leaf_spread(P.x, P.y, L))


def override_tuning(a, vf):
    if a.p2p_tile or a.p2p_waves:
        vf.set_tuning(tile=a.p2p_tile or None, waves=a.p2p_waves or None)
    if a.p2p_sym >= 0:
        vf.set_tuning(sym=a.p2p_sym)



def target_pairs(leaf_start, xe, ye, root, levels):
    """Near-field (point, particle) pairs of an evaluation-point launch: points
    per leaf (floor-and-clamp rule) times the particles of the 3 x 3 list."""
    m = 1 << levels
    x0, y0, s = root
    ix = np.clip(np.floor((xe - x0) / s * m), 0, m - 1).astype(np.int64)
    iy = np.clip(np.floor((ye - y0) / s * m), 0, m - 1).astype(np.int64)
    tcnt = np.bincount(iy * m + ix, minlength=m * m).reshape(m, m)
    cnt = np.diff(leaf_start.astype(np.int64)).reshape(m, m)
    pad = np.pad(cnt, 1)
    nb = sum(pad[1 + dy:1 + dy + m, 1 + dx:1 + dx + m] for dy in (-1, 0, 1) for dx in (-1, 0, 1))
    return int(np.sum(tcnt * nb))


def bench_eval_points(a, torch, vf):
    """FMM velocity of the workload's particles at an M x M lattice of separate
    evaluation points covering the root square (the error-map set-up of
    Section 5.2 at full size): tree rebuild + evaluation at the points (their
    sort into the leaves included) per step; error against the FP64 direct
    sum at 4096 sampled points, with the quantiles of the per-point log10
    error field."""
    from paper_0809_1810_amd import autotune as AT
    from paper_0809_1810_amd import selector as S
    P = W.config(a.workload)
    n = P.n
    x = torch.from_numpy(P.x).cuda(); y = torch.from_numpy(P.y).cuda()
    g = torch.from_numpy(P.gamma).cuda()
    probe = vf.Tree(x, y, 0, p_max=1)
    root = tuple(float(r) for r in probe.arrays()[0][:3].cpu().tolist())
    probe.close()
    xe_h, ye_h = W.eval_lattice(a.eval_lattice, root)
    nt = len(xe_h)
    xe = torch.from_numpy(xe_h).cuda(); ye = torch.from_numpy(ye_h).cuda()
    sel = torch.from_numpy(W.sample_targets(nt, AUDIT_TARGETS, seed=2025)).cuda()
    xs, ys = xe[sel].contiguous(), ye[sel].contiguous()
    ud, vd = vf.direct_velocity_at(x, y, g, P.sigma, xs, ys)
    if a.p is not None and a.levels is not None:
        p, L, prec, how = a.p, a.levels, vf.PRECISIONS[a.precision], "fixed"
        radius = fixed_radius(a, P.sigma, vf)
    else:
        selection_shape(P)
        r = S.select_and_audit(x, y, g, P.sigma, 1e-6, weights=S.load_weights())
        p, L, radius = r["p"], r["levels"], r["radius"]
        prec = vf.FP64 if r["precision"] == "fp64" else vf.PRECISIONS[a.precision]
        how = "learned" if not r["fallback"] else "fallback"
    log(f"[bench] evaluation points: {nt} on the root square, p={p} L={L} ({how}), "
        f"near radius {radius}")
    AT.apply_for(n, L, cutoff=radius != 0.0, spread=AT.leaf_spread(P.x, P.y, L))
    override_tuning(a, vf)
    tree = vf.Tree(x, y, L, p_max=p)
    tree.set_near_radius(radius)
    ws = torch.empty(vf.targets_workspace_bytes(nt, L), dtype=torch.uint8, device="cuda")
    u = torch.empty(nt, dtype=torch.float64, device="cuda")
    v = torch.empty(nt, dtype=torch.float64, device="cuda")
    def step():
        tree.rebuild(x, y)
        tree.velocity_at(g, P.sigma, p, xe, ye, prec, out=(u, v), workspace=ws)
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    # eager steps with the phase events, then the same steps replayed from a graph
    eager_ms, _, phases = time_steps(torch, step, a.steps, tree, False)
    ms = eager_ms if a.eager else time_steps(torch, step, a.steps, None, True)[0]
    us, vs = u[sel].contiguous(), v[sel].contiguous()
    emax, erms, _ = vf.error_metrics(us, vs, ud, vd)
    field = vf.error_field(us, vs, ud, vd).cpu().numpy()
    pairs = target_pairs(tree.arrays()[2].cpu().numpy(), xe_h, ye_h, root, L)
    tree.close()
    p2p_ms = float(np.mean([ph["p2p"] for ph in phases]))
    achieved = P2P_FLOPS_PER_PAIR * pairs / (p2p_ms * 1e-3) / 1e12
    out = {"metric": "evaluation points/s, FMM of N=2^20 particles at an M x M lattice of points",
           "value": round(nt / (ms * 1e-3), 1), "unit": "points/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms, 4),
           "eager_ms_per_step": round(eager_ms, 4),
           "timed_as": "eager calls" if a.eager else "one hipGraph replay of the K captured steps",
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32" if prec != vf.FP64 else "f64", "data": "synthetic",
           "config": {"workload": f"{P.name}: N={n}, sigma={P.sigma}; {a.eval_lattice}^2 "
                                  "cell-centred lattice of evaluation points on the root square",
                      "p": p, "levels": L, "selector": how,
                      "near_radius": "auto: min(6 sigma, 4 w_L)" if radius < 0 else radius,
                      "p2p_tile_waves": [vf.get_tuning()["tile"], vf.get_tuning()["waves"]]},
           "accuracy": {"emax": emax, "erms": erms, "sample": AUDIT_TARGETS,
                        "log10_error_quantiles": {q: float(np.quantile(field, float(q)))
                                                  for q in ("0.5", "0.9", "0.99", "1.0")}},
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 3),
                        "traffic": None, "kernel": "k_p2p<float>",
                        "kernel_ms": round(p2p_ms, 4),
                "kernel_ms_from": "HIP events around the kernel's launches on its stream in the "
                                  "K timed steps issued eagerly (the same steps as the "
                                  "graph-replayed ones)", "pairs_per_launch": pairs,
                        "flops_per_pair": P2P_FLOPS_PER_PAIR},
           "phases_ms": {k: round(float(np.mean([ph[k] for ph in phases])), 4) for k in phases[0]}}
    print(json.dumps(out), flush=True)


def bench_advect(a, torch, vf):
    """K steps of advecting the workload's particles with their own velocity
    (eq. 5, Heun's method: per step two tree rebuilds and two evaluations),
    tuned path (selected p, L, near radius, FP32) vs the plain FP64 path;
    dt = 0.2 sigma / max|u|.  Accuracy: the tuned trajectory's final positions
    against the plain path's, relative to the largest displacement."""
    from paper_0809_1810_amd import autotune as AT
    from paper_0809_1810_amd import selector as S
    P = W.config(a.workload)
    n = P.n
    x0 = torch.from_numpy(P.x).cuda(); y0 = torch.from_numpy(P.y).cuda()
    g = torch.from_numpy(P.gamma).cuda()
    probe = vf.Tree(x0, y0, 0, p_max=1)
    side = float(probe.arrays()[0][2].item())
    probe.close()
    if a.p is not None and a.levels is not None:
        p, L = a.p, a.levels
        radius = fixed_radius(a, P.sigma, vf)
    else:
        selection_shape(P)
        r = S.select_and_audit(x0, y0, g, P.sigma, 1e-6, weights=S.load_weights())
        p, L, radius = r["p"], r["levels"], r["radius"]
    Lp = largest_level(side, P.sigma, 8.0)
    t0 = vf.Tree(x0, y0, Lp, p_max=20)
    u, v = t0.velocity(g, P.sigma, 20, vf.FP64)
    umax = float(torch.hypot(u, v).max().item())
    t0.close()
    dt = 0.2 * P.sigma / umax
    ws = None

    def run(pp, LL, prec, rad, steps):
        AT.apply_for(n, LL, cutoff=rad != 0.0, spread=AT.leaf_spread(P.x, P.y, LL))
        override_tuning(a, vf)
        x = x0.clone(); y = y0.clone()
        tree = vf.Tree(x, y, LL, p_max=pp)
        tree.set_near_radius(rad)
        xw = x0.clone(); yw = y0.clone()
        tree.advect(xw, yw, g, P.sigma, pp, dt, max(1, a.warmup // 2), prec)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        tree.advect(x, y, g, P.sigma, pp, dt, steps, prec)
        e1.record()
        torch.cuda.synchronize()
        tree.close()
        return x, y, e0.elapsed_time(e1) / steps

    K = a.advect
    log(f"[bench] advect: {K} Heun steps, dt={dt:.3e}, tuned p={p} L={L} radius={radius}")
    xt, yt, ms_t = run(p, L, vf.FP32, radius, K)
    xp, yp, ms_p = run(20, Lp, vf.FP64, 0.0, K)
    disp = float(torch.hypot(xp - x0, yp - y0).max().item())
    dev_ = float(torch.hypot(xt - xp, yt - yp).max().item())
    out = {"metric": "particle steps/s, advecting N=2^20 particles with their FMM velocity (Heun)",
           "value": round(n / (ms_t * 1e-3), 1), "unit": "particle steps/s", "n_gpus": 1,
           "steps": K, "warmup": max(1, a.warmup // 2), "ms_per_step": round(ms_t, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"{P.name}: N={n}, sigma={P.sigma}, dt = 0.2 sigma / max|u| = {dt:.4g}",
                      "p": p, "levels": L, "near_radius": "auto" if radius < 0 else radius},
           "plain_fp64": {"ms_per_step": round(ms_p, 4), "p": 20, "levels": Lp},
           "speedup_vs_plain": round(ms_p / ms_t, 3),
           "accuracy": {"max_position_difference_vs_plain": dev_, "max_displacement": disp,
                        "relative": dev_ / disp if disp > 0 else None}}
    print(json.dumps(out), flush=True)


def bench_batched(a, torch, vf):
    """256 independent instances (N log-uniform in [2048, 65536], uniform or lattice,
    p in 5..20, levels in 3..6, sigma = h / 0.8): one batched evaluation replayed
    from a hipGraph vs one single-tree call per instance; per-instance error
    against the FP64 direct sum on 64 sampled targets each."""
    insts = W.batch_instances(256, seed=4)
    dev = []
    for P, p, L in insts:
        dev.append(dict(x=torch.from_numpy(P.x).cuda(), y=torch.from_numpy(P.y).cuda(),
                        gamma=torch.from_numpy(P.gamma).cuda(), sigma=P.sigma, p=p, levels=L))
    ntot = sum(P.n for P, _, _ in insts)
    # the symmetric near field for the instances with well filled leaves
    # (--p2p-sym 0 turns it off); the single-tree comparison keeps the default
    sym = 0 if a.p2p_sym == 0 else 1
    saved = vf.get_tuning()
    vf.set_tuning(sym=sym)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = vf.Batch(dev)
        vf.set_tuning(**saved)
        for _ in range(a.warmup):
            b.run(use_graph=True)
        s.synchronize()
        e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.steps):
            b.run(use_graph=True)
        e1.record()
        s.synchronize()
        graph_ms = e0.elapsed_time(e1) / a.steps
        e0.record()
        for _ in range(a.steps):
            b.run(use_graph=False)
        e1.record()
        s.synchronize()
        eager_ms = e0.elapsed_time(e1) / a.steps
        trees = [vf.Tree(d["x"], d["y"], d["levels"], p_max=d["p"]) for d in dev]
        for t, d in zip(trees, dev):
            t.velocity(d["gamma"], d["sigma"], d["p"], vf.FP32)
        s.synchronize()
        e0.record()
        for _ in range(a.steps):
            for t, d in zip(trees, dev):
                t.rebuild(d["x"], d["y"])
                t.velocity(d["gamma"], d["sigma"], d["p"], vf.FP32)
        e1.record()
        s.synchronize()
        loop_ms = e0.elapsed_time(e1) / a.steps
        errs, errs_fmm = [], []
        for i, (t, d, (P, p, L)) in enumerate(zip(trees, dev, insts)):
            tg = torch.from_numpy(W.sample_targets(P.n, 64, seed=i)).cuda()
            ud, vd = vf.direct_velocity(d["x"], d["y"], d["gamma"], d["sigma"], targets=tg)
            ub, vb = b.u[i][tg].contiguous(), b.v[i][tg].contiguous()
            errs.append(vf.error_metrics(ub, vb, ud, vd)[0])
            t.rebuild(d["x"], d["y"])
            uf, vf64 = t.velocity(d["gamma"], d["sigma"], d["p"], vf.FP64)
            errs_fmm.append(vf.error_metrics(ub, vb, uf[tg].contiguous(), vf64[tg].contiguous())[0])
        for t in trees:
            t.close()
    errs, errs_fmm = np.array(errs), np.array(errs_fmm)
    ps = np.array([p for _, p, _ in insts])
    floors = np.array(b.substitution_bounds())
    out = {"metric": "instances/s, 256 uneven FMM instances in one batched graph replay",
           "value": round(256 / (graph_ms * 1e-3), 1), "unit": "instances/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(graph_ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"256 instances, N log-uniform [2048, 65536] (total {ntot}), "
                                  "uniform or lattice, p 5..20, levels 3..6, sigma = h/0.8, seed 4",
                      "p2p_symmetric": bool(sym)},
           "particles_per_s": round(ntot / (graph_ms * 1e-3), 1),
           "eager_batched_ms": round(eager_ms, 4), "one_call_per_instance_ms": round(loop_ms, 4),
           "speedup_vs_per_instance": round(loop_ms / graph_ms, 3),
           "per_instance_emax": {"median": float(np.median(errs)), "max": float(errs.max()),
                                 "max_p_ge_14": float(errs[ps >= 14].max()),
                                 "max_p_le_8": float(errs[ps <= 8].max()),
                                 "note": "vs the FP64 direct sum: includes the truncation and the "
                                         "kernel-substitution error of the instance's own (p, levels)"},
           "per_instance_emax_vs_fp64_fmm": {"median": float(np.median(errs_fmm)),
                                             "max": float(errs_fmm.max())},
           "substitution_floor": {"max": float(floors.max()),
                                  "instances_above_1e-6": int((floors > 1e-6).sum()),
                                  "max_emax_where_floor_le_1e-9": float(errs[floors <= 1e-9].max())
                                  if (floors <= 1e-9).any() else None,
                                  "note": "vfmm_batch_substitution_bounds: 1 / (exp(w_L^2 / 2 "
                                          "sigma^2) - 1) per instance"}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
