"""Tile-size autotuner.

The planner's one free schedule parameter is the largest tile a pass may
stage in LDS (``max_tile_bits``): larger tiles need fewer passes, smaller ones
give more workgroups per compute unit and per launch.  Which wins depends on
the workload class, the qubit count and the device, so candidates are timed
on the device and the fastest is cached in a JSON file keyed by (GPU
architecture, compute-unit count, HIP version, workload class, n, dtype).

``run(tile_bits)`` must execute one representative unit of the workload with
that tile limit (building and caching whatever it needs on first use); the
tuner calls it once to warm up and then ``reps`` times under a device
synchronisation.
"""
from __future__ import annotations

import json
import os
import time
from typing import Callable, Iterable, Optional

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "qs_tile_tune.json")


def device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "") or p.name
    return f"{arch}|cu{p.multi_processor_count}|hip{torch.version.hip}"


class TileTuner:
    def __init__(self, path: Optional[str] = None, device: Optional[str] = None,
                 sync: Optional[Callable[[], None]] = None):
        self.path = path or os.environ.get("QS_TUNE_CACHE", DEFAULT_CACHE)
        self._device = device
        self._sync = sync
        self.cache = {}
        if os.path.exists(self.path):
            with open(self.path) as fh:
                self.cache = json.load(fh)
        self.measured = {}  # key -> {tile_bits: seconds} for the calls that timed

    def _key(self, kind: str, n: int, dtype: str) -> str:
        dev = self._device if self._device is not None else device_key()
        return f"{dev}|{kind}|n{n}|{dtype}"

    def _synchronize(self) -> None:
        if self._sync is not None:
            self._sync()
        else:
            import torch
            torch.cuda.synchronize()

    def best(self, kind: str, n: int, dtype: str, run: Callable[[int], None], candidates: Iterable[int],
             reps: int = 3) -> int:
        key = self._key(kind, n, dtype)
        if key in self.cache:
            return int(self.cache[key])
        times = {}
        for tb in candidates:
            run(tb)
            self._synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                run(tb)
            self._synchronize()
            times[int(tb)] = (time.perf_counter() - t0) / reps
        if not times:
            raise ValueError("no candidate tile sizes")
        best = min(times, key=times.get)
        self.measured[key] = times
        self.cache[key] = best
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(self.cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)
        return best
