"""Tile-size autotuner: picks the fastest candidate and caches it per key."""
import json
import time

from paper_2609_19147_amd.tune import TileTuner


def test_picks_fastest_and_caches(tmp_path):
    calls = []
    cost = {10: 0.004, 11: 0.001, 12: 0.003}

    def run(tb):
        calls.append(tb)
        time.sleep(cost[tb])

    path = tmp_path / "tune.json"
    t = TileTuner(str(path), device="test-gpu", sync=lambda: None)
    assert t.best("qaoa", 20, "c64", run, [10, 11, 12], reps=2) == 11
    assert set(calls) == {10, 11, 12}
    saved = json.loads(path.read_text())
    assert saved == {"test-gpu|qaoa|n20|c64": 11}
    # a second tuner reads the cache and runs nothing
    calls.clear()
    t2 = TileTuner(str(path), device="test-gpu", sync=lambda: None)
    assert t2.best("qaoa", 20, "c64", run, [10, 11, 12]) == 11
    assert calls == []
    # other keys are tuned separately
    assert t2.best("qaoa", 22, "c64", run, [12]) == 12
    assert len(json.loads(path.read_text())) == 2


def test_option_grid_and_best_options(tmp_path):
    from paper_2609_19147_amd.tune import option_grid
    grid = option_grid(max_tile_bits=(12, 13), diag_low_bits=(0, -1))
    assert grid == [{"diag_low_bits": 0, "max_tile_bits": 12}, {"diag_low_bits": 0, "max_tile_bits": 13},
                    {"diag_low_bits": -1, "max_tile_bits": 12}, {"diag_low_bits": -1, "max_tile_bits": 13}]
    try:
        option_grid(tile=(1,))
        raise AssertionError("unknown option accepted")
    except ValueError:
        pass
    calls = []

    def run(opts):
        calls.append(opts)
        time.sleep(0.001 if opts == {"diag_low_bits": -1, "max_tile_bits": 12} else 0.004)

    path = tmp_path / "tune.json"
    t = TileTuner(str(path), device="test-gpu", sync=lambda: None)
    best = t.best_options("tfim", 25, "c64", run, grid, reps=2)
    assert best == {"diag_low_bits": -1, "max_tile_bits": 12}
    assert len(calls) == 4 * 3
    calls.clear()
    t2 = TileTuner(str(path), device="test-gpu", sync=lambda: None)
    assert t2.best_options("tfim", 25, "c64", run, grid) == best
    assert calls == []
    # the tile-only entry and the options entry of one workload do not collide
    assert t2.best("tfim", 25, "c64", lambda tb: None, [13]) == 13
    assert len(json.loads(path.read_text())) == 2
