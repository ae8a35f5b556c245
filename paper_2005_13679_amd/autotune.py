"""Schedule autotuner for batched H.C.

Times one batched apply for each candidate schedule (persistent grid size per
group, work order, and the size from which an instance gets a launch of its
own) on the actual batch and keeps the fastest.
Results are cached in a JSON file keyed by the batch signature (instance
shapes, which instances use a double-jump map, device name).  Set
MC_AUTOTUNE=0 to skip tuning and use the default schedule.
"""

from __future__ import annotations

import hashlib
import json
import os

import torch

from .batch import Batch

DEFAULT = {"blocks_per_cu": 2, "order": 3, "solo_tiles": 16384}
# persistent grid size x work order x size from which an instance gets a grid
# of its own (0: never)
CANDIDATES = [{"blocks_per_cu": b, "order": o, "solo_tiles": t}
              for b in (1, 2, 4) for o in (0, 2, 3) for t in (0, 16384)]


def default_cache_path() -> str:
    return os.environ.get("MC_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mc_boson", "autotune.json"))


def signature(instances) -> str:
    dev = instances[0][0].device
    name = torch.cuda.get_device_name(dev)
    shapes = sorted((t.N, t.M, t.t2 is not None, t.form) for t, _, _ in instances)
    return hashlib.sha256(json.dumps([name, shapes]).encode()).hexdigest()[:24]


def time_schedule(instances, sched, reps: int = 3) -> float:
    b = Batch(instances, sched)
    C = b.vector()
    C.real.fill_(1.0)
    C.imag.fill_(0.0)
    out = b.vector()
    b.apply_H(C, out)   # warm-up
    torch.cuda.synchronize(b.device)
    times = []
    for _ in range(reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        b.apply_H(C, out)
        e.record()
        torch.cuda.synchronize(b.device)
        times.append(s.elapsed_time(e))
    times.sort()
    return times[len(times) // 2]


def tune(instances, cache_path: str | None = None, candidates=None, reps: int = 3,
         force: bool = False) -> dict:
    """Returns {"schedule": best, "timings": [...], "cached": bool}."""
    if os.environ.get("MC_AUTOTUNE", "1") == "0":
        return {"schedule": dict(DEFAULT), "timings": [], "cached": False}
    path = cache_path or default_cache_path()
    key = signature(instances)
    cache = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if not force and key in cache:
        return {"schedule": cache[key]["schedule"], "timings": cache[key]["timings"], "cached": True}
    timings = []
    for sched in candidates or CANDIDATES:
        ms = time_schedule(instances, sched, reps)
        timings.append({"schedule": sched, "ms": ms})
    best = min(timings, key=lambda r: r["ms"])["schedule"]
    cache[key] = {"schedule": best, "timings": timings}
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, path)
    return {"schedule": best, "timings": timings, "cached": False}
