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
