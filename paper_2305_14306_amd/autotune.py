"""Autotuner for the sampler's tuning fields (speculation depth and budget, search grid,
table load factor, and the binning workgroup's share of the cloud).

The tuning fields of hav_params_t never change a result, only the time it takes, so
the tuner times every candidate on the caller's own input (or a batch), checks that all
candidates return identical indices, and keeps the fastest. Results can be cached in a
JSON file keyed by the problem's shape class (log2 of N, M/N, single or batch).

    from paper_2305_14306_amd import autotune
    best, table = autotune.tune(xyz_cuda, M)             # one cloud
    best, table = autotune.tune_batch(xyz, offsets, Ms)  # a batch
    p = hav.params(**best)
"""
from __future__ import annotations

import itertools
import json
import math
import os

from . import hav

DEPTHS = (2, 4, 6)
BUDGETS = (4, 16, 64)
GRIDS = (0, 256)
TABLES = (0, 1)  # table_scale: the tables' slots are doubled per step (load factor halved)


def candidates(depths=DEPTHS, budgets=BUDGETS, grids=GRIDS, tables=TABLES):
    for d, b, g, t in itertools.product(depths, budgets, grids, tables):
        if d == 1 and b != budgets[0]:
            continue  # the budget only matters when a pass speculates
        yield dict(spec_depth=d, spec_budget=b, search_blocks=g, table_scale=t)


BINS = (0, 2048, 8192)  # bin_points: the binning workgroup's points (0 = 4,096)


def with_bins(cands, bins=BINS):
    """Each candidate once per binning workgroup shape."""
    for c in cands:
        for b in bins:
            yield dict(c, bin_points=b)


def batch_candidates():
    """A short candidate list for batches of many LiDAR-sized clouds: speculation depth,
    table load factor and the binning workgroup's points, with the default search grid."""
    return list(with_bins(candidates(depths=(2, 4), budgets=(16,), grids=(0,), tables=(0, 1))))


def _time(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _run(run_once, base: dict, reps: int, cands):
    table, ref, best = [], None, None
    for c in cands:
        kw = dict(base)
        kw.update(c)
        p = hav.params(**kw)
        out = run_once(p)
        if ref is None:
            ref = out
        elif not all((a == b).all().item() for a, b in zip(ref, out)):
            raise AssertionError(f"tuning fields {c} changed the result")
        ms = _time(lambda: run_once(p), reps)
        table.append((c, ms))
        if best is None or ms < best[1]:
            best = (c, ms)
    return best[0], table


def tune(xyz, M: int, base: dict | None = None, reps: int = 5, cands=None):
    """Fastest tuning fields for hav_sample(xyz, M) with the other parameters in base."""
    s = hav.Sampler(xyz.device)
    return _run(lambda p: [s.sample(xyz, M, p)], base or {}, reps,
                list(cands) if cands is not None else list(candidates()))


def tune_batch(xyz, offsets, Ms, base: dict | None = None, reps: int = 3, cands=None):
    """Fastest tuning fields for hav_sample_batch over the given clouds."""
    s = hav.Sampler(xyz.device)
    return _run(lambda p: s.sample_batch(xyz, offsets, Ms, p), base or {}, reps,
                list(cands) if cands is not None else list(candidates()))


def shape_key(N: int, M: int, batch: bool = False) -> str:
    return f"{'batch' if batch else 'one'}:n2^{max(0, math.ceil(math.log2(max(1, N))))}:m{round(M / N, 2)}"


def load_cache(path: str) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def save_cache(path: str, cache: dict) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def cached_or_tune(path: str, xyz, M: int, base: dict | None = None) -> dict:
    """Tuning fields from the cache at `path` for this shape class, tuning (and storing)
    them on a miss."""
    cache = load_cache(path)
    key = shape_key(xyz.shape[0], M)
    if key not in cache:
        best, _ = tune(xyz, M, base)
        cache[key] = best
        save_cache(path, cache)
    return cache[key]
