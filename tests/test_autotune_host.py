"""Host logic of the near-field launch-shape table (no GPU): nearest entry by
log2 of the mean particles per leaf; with the distance cut-off the entry's
fastest 64-target shape (only one lane per target culls ring sources)."""
import json

from paper_0809_1810_amd import autotune as AT


def _table(tmp_path):
    entries = [
        {"ppl_log2": 8.0, "tile": 64, "waves": 4,
         "all_ms": {"64x2": 5.1, "64x4": 4.9, "32x4": 8.5, "16x4": 12.8}},
        {"ppl_log2": 4.0, "tile": 16, "waves": 4,
         "all_ms": {"64x1": 3.3, "64x2": 3.0, "64x4": 3.1, "16x4": 2.0, "32x2": 2.4}},
        {"ppl_log2": 2.0, "tile": 32, "waves": 2},
        {"ppl_log2": 6.0, "tile": 64, "waves": 2,
         "all_ms": {"64x1": 2.2, "64x2": 2.1, "16x4": 3.0},
         "cutoff_ms": {"64x1": 2.08, "64x2": 2.11, "64x4": 2.24, "64x8": 2.5}},
    ]
    p = tmp_path / "tuning.json"
    p.write_text(json.dumps({"entries": entries}))
    return str(p)


def test_nearest_entry(tmp_path):
    path = _table(tmp_path)
    assert AT.lookup(1 << 20, 6, path) == (64, 4)   # 2^20 / 4^6 = 2^8 per leaf
    assert AT.lookup(1 << 20, 8, path) == (16, 4)   # 2^4 per leaf
    assert AT.lookup(1 << 20, 9, path) == (32, 2)   # 2^2 per leaf


def test_cutoff_takes_fastest_64_target_shape(tmp_path):
    path = _table(tmp_path)
    assert AT.lookup(1 << 20, 6, path, cutoff=True) == (64, 4)
    assert AT.lookup(1 << 20, 8, path, cutoff=True) == (64, 2)
    # an entry without timings of every shape keeps its waves or the default
    assert AT.lookup(1 << 20, 9, path, cutoff=True) == (64, 4)
    # timings taken with the cut-off take precedence over the paper split's
    assert AT.lookup(1 << 20, 7, path) == (64, 2)
    assert AT.lookup(1 << 20, 7, path, cutoff=True) == (64, 1)


def test_missing_table_defaults(tmp_path):
    assert AT.lookup(1000, 3, str(tmp_path / "absent.json")) == (64, 4)


def test_m2l_tile_lookup(tmp_path):
    entries = [{"ppl_log2": 8.0, "tile": 64, "waves": 4, "m2l_tile": 2},
               {"ppl_log2": 4.0, "tile": 16, "waves": 4}]
    p = tmp_path / "tuning.json"
    p.write_text(json.dumps({"entries": entries}))
    assert AT.lookup_m2l(1 << 20, 6, str(p)) == 2
    assert AT.lookup_m2l(1 << 20, 8, str(p)) == 0    # entry without M2L timings
    assert AT.lookup_m2l(1000, 3, str(tmp_path / "absent.json")) == 0


def test_symmetric_shapes(tmp_path):
    """Shapes timed with the symmetric near field ("64x<w>s") win when fastest,
    with and without the cut-off; entries without them keep sym = 0."""
    entries = [
        {"ppl_log2": 6.0, "tile": 64, "waves": 2,
         "all_ms": {"64x1": 2.2, "64x2": 2.1, "16x4": 3.0, "64x1s": 1.9, "64x2s": 2.0},
         "cutoff_ms": {"64x1": 2.08, "64x2": 2.11, "64x1s": 2.2, "64x2s": 1.85}},
        {"ppl_log2": 2.0, "tile": 32, "waves": 2,
         "all_ms": {"32x2": 1.0, "64x1s": 1.4}},
    ]
    p = tmp_path / "tuning.json"
    p.write_text(json.dumps({"entries": entries}))
    path = str(p)
    assert AT.lookup_shape(1 << 20, 7, path) == (64, 1, 1)
    assert AT.lookup_shape(1 << 20, 7, path, cutoff=True) == (64, 2, 1)
    assert AT.lookup(1 << 20, 7, path, cutoff=True) == (64, 2)
    assert AT.lookup_shape(1 << 20, 9, path) == (32, 2, 0)
    assert AT.lookup_shape(1000, 3, str(tmp_path / "absent.json")) == (64, 4, 0)


def test_leaf_spread():
    """The occupancy spread: 0 for even leaves, log2(1 + 1/m) in expectation
    for a Poisson population of mean m, and log2 of the pair-weighted over the
    plain mean for uneven counts."""
    import numpy as np
    assert AT.spread_from_counts([4, 4, 4, 4]) == 0.0
    assert abs(AT.spread_from_counts([8, 0, 0, 0]) - 2.0) < 1e-12   # 4 * 64 / 64 = 4
    assert abs(AT.spread_from_counts([3, 1]) - np.log2(2 * 10 / 16)) < 1e-12
    assert AT.spread_from_counts([0, 0]) == 0.0
    # a cell-centred 64 x 64 lattice has 4 points in each of the 16 x 16 leaves at L = 4
    g = (np.arange(64) + 0.5) / 64
    x, y = np.meshgrid(g, g)
    assert abs(AT.leaf_spread(x.ravel(), y.ravel(), 4)) < 1e-12
    rng = np.random.default_rng(1)
    s = AT.leaf_spread(rng.random(1 << 18), rng.random(1 << 18), 6)   # mean 64 per leaf
    assert abs(s - np.log2(1 + 1 / 64)) < 0.01


def test_lookup_with_spread(tmp_path):
    """Two entries with the same mean occupancy: without a spread the first is
    taken, with one the entry nearest in (mean, spread)."""
    entries = [
        {"ppl_log2": 6.0, "spread": 3.2, "tile": 64, "waves": 1,
         "cutoff_ms": {"64x1s": 1.7, "64x2s": 1.8}},
        {"ppl_log2": 6.0, "spread": 0.0, "tile": 64, "waves": 2,
         "cutoff_ms": {"64x1s": 0.25, "64x2s": 0.23}, "m2l_tile": 2},
    ]
    p = tmp_path / "tuning.json"
    p.write_text(json.dumps({"entries": entries}))
    path = str(p)
    assert AT.lookup_shape(1 << 20, 7, path, cutoff=True) == (64, 1, 1)
    assert AT.lookup_shape(1 << 20, 7, path, cutoff=True, spread=3.0) == (64, 1, 1)
    assert AT.lookup_shape(1 << 20, 7, path, cutoff=True, spread=0.02) == (64, 2, 1)
    assert AT.lookup_m2l(1 << 20, 7, path, spread=0.02) == 2
    assert AT.lookup_m2l(1 << 20, 7, path) == 0


def test_table_spreads():
    """Every entry of the shipped table records its workload's spread, and the
    two N = 2^20 inputs at 64 particles per leaf map to their own entries."""
    table = json.load(open(AT.TABLE_PATH))
    assert all("spread" in e for e in table["entries"])
    by = {(e["workload"], e["levels"]): e for e in table["entries"]}
    assert by[("clusters_1m", 7)]["spread"] > 2.0 and by[("lattice_1024", 7)]["spread"] == 0.0
