"""Autotuner for the batched launches: times candidate tile shapes
(pixels per covariance work item, tiles per projection work item) on the
batch itself and caches the fastest per batch signature in a JSON file.

The signature buckets the batch by band count (multiples of 32) and pixel
count (powers of two), so batches of similar composition share an entry.
Cache file: $PCA_TUNING_CACHE, else ~/.cache/paper_2403_18321_amd/tuning.json.
"""

from __future__ import annotations

import json
import math
import os

import torch

COV_CHUNKS = (2048, 4096, 8192, 16384)
PROJ_TILES = (4, 8, 16, 32)


def cache_path() -> str:
    p = os.environ.get("PCA_TUNING_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2403_18321_amd", "tuning.json")


def signature(batch) -> str:
    hist = {}
    for Y in batch.cubes:
        n, m = int(Y.shape[0]), int(Y.shape[1])
        key = f"m{(m + 31) // 32 * 32}n{2 ** int(math.ceil(math.log2(max(n, 1))))}"
        hist[key] = hist.get(key, 0) + 1
    parts = ",".join(f"{k}x{v}" for k, v in sorted(hist.items()))
    return f"dt{batch.dt}/mode{batch.mode}/{parts}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def time_batch(batch, reps: int = 3) -> float:
    batch.run()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        batch.run()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(batch, reps: int = 3, use_cache: bool = True, write_cache: bool = True):
    """Pick (cov_chunk, proj_tiles) for this batch; leaves it set on the batch.
    Returns (tuning dict, {candidate: ms})."""
    path = cache_path()
    sig = signature(batch)
    cache = _load(path) if use_cache else {}
    if sig in cache:
        best = cache[sig]
        batch.set_tuning(best)
        return best, {}
    times = {}
    # The two launches are independent: tune the covariance chunk with the
    # default projection, then the projection with the best chunk.
    for c in COV_CHUNKS:
        batch.set_tuning((c, 0))
        times[(c, 0)] = time_batch(batch, reps)
    best_c = min((c for c in COV_CHUNKS), key=lambda c: times[(c, 0)])
    for t in PROJ_TILES:
        batch.set_tuning((best_c, t))
        times[(best_c, t)] = time_batch(batch, reps)
    best_t = min(PROJ_TILES, key=lambda t: times[(best_c, t)])
    best = dict(cov_chunk=best_c, proj_tiles=best_t, ms=round(times[(best_c, best_t)], 4))
    batch.set_tuning(best)
    if write_cache:
        cache = _load(path)
        cache[sig] = best
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return best, times
