"""Plan autotuner.

The planner's schedule knobs are the largest tile a pass may stage in LDS
(``max_tile_bits``: larger tiles need fewer passes, smaller ones give more
workgroups per compute unit and per launch), the low bits of passes over high
bits (``low_bits``), the low bits kept by passes that carry diagonal layers
(``diag_low_bits``), the coset order of the workgroups (``coset_order``) and
whether ops move between a diagonal pass and the next (``balance_passes``).
Which setting wins depends on the workload class, the qubit count and the
device, so candidates are timed on the device and the fastest is cached in a
JSON file keyed by (GPU architecture, compute-unit count, HIP version,
workload class, n, dtype).

``best`` tunes the tile limit alone: ``run(tile_bits)`` must execute one
representative unit of the workload with that limit (building and caching
whatever it needs on first use); the tuner calls it once to warm up and then
``reps`` times under a device synchronisation.  ``best_options`` tunes any
set of plan options: ``run(options)`` receives a dict of ``Plan`` keyword
arguments (see ``option_grid``).
"""
from __future__ import annotations

import itertools
import json
import os
import time
from typing import Callable, Dict, Iterable, List, Optional

PLAN_KNOBS = ("max_tile_bits", "low_bits", "diag_low_bits", "coset_order", "balance_passes")


def option_grid(**axes: Iterable[int]) -> List[Dict[str, int]]:
    """Every combination of the given plan-option values, e.g.
    ``option_grid(max_tile_bits=(12, 13), diag_low_bits=(0, -1))``."""
    for k in axes:
        if k not in PLAN_KNOBS:
            raise ValueError(f"unknown plan option {k!r}")
    keys = sorted(axes)
    return [dict(zip(keys, vals)) for vals in itertools.product(*(list(axes[k]) for k in keys))]

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

    def _time(self, run: Callable, arg, reps: int) -> float:
        run(arg)
        self._synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            run(arg)
        self._synchronize()
        return (time.perf_counter() - t0) / reps

    def _save(self) -> None:
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(self.cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def best(self, kind: str, n: int, dtype: str, run: Callable[[int], None], candidates: Iterable[int],
             reps: int = 3) -> int:
        key = self._key(kind, n, dtype)
        if key in self.cache:
            return int(self.cache[key])
        times = {int(tb): self._time(run, tb, reps) for tb in candidates}
        if not times:
            raise ValueError("no candidate tile sizes")
        best = min(times, key=times.get)
        self.measured[key] = times
        self.cache[key] = best
        self._save()
        return best

    def best_options(self, kind: str, n: int, dtype: str, run: Callable[[Dict[str, int]], None],
                     candidates: Iterable[Dict[str, int]], reps: int = 3) -> Dict[str, int]:
        key = self._key(kind, n, dtype) + "|options"
        if key in self.cache:
            return dict(self.cache[key])
        cands = [dict(c) for c in candidates]
        for c in cands:
            for k in c:
                if k not in PLAN_KNOBS:
                    raise ValueError(f"unknown plan option {k!r}")
        if not cands:
            raise ValueError("no candidate options")
        times = [self._time(run, c, reps) for c in cands]
        k = min(range(len(cands)), key=times.__getitem__)
        self.measured[key] = [(c, t) for c, t in zip(cands, times)]
        self.cache[key] = cands[k]
        self._save()
        return dict(cands[k])
