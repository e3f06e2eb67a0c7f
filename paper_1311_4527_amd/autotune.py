"""Launch-shape autotuner of the batched solver.

Candidates are (lanes per workgroup, number of workgroups) of the
persistent kernel, where instances are packed onto workgroups
longest-first by the library, and (0, 1): one launch per phase of an
iteration over all instances.  This driver times a few iterations of each
candidate on the actual batch (HIP events, through the C ABI) and keeps
the fastest.  Results are cached in a JSON file keyed
by device name and a shape signature of the batch, so a repeated batch
shape skips the search.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, List, Optional, Tuple

CACHE = os.environ.get("TWA_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "twa_tune.json"))


def shape_signature(instances) -> str:
    key = sorted((i.p, i.eta, i.dim, i.n_walls) for i in instances)
    return hashlib.sha1(json.dumps(key).encode()).hexdigest()[:16]


def candidates(n: int) -> List[Tuple[int, int]]:
    groups = sorted({max(1, n // 8), max(1, n // 4), max(1, n // 2), n})
    return [(b, g) for b in (256, 512, 1024) for g in groups] + [(0, 1)]


def _load_cache() -> Dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(c: Dict):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE + ".tmp", "w") as f:
            json.dump(c, f, indent=1)
        os.replace(CACHE + ".tmp", CACHE)
    except OSError:
        pass


def tune(batch, iters: int = 20, use_cache: bool = True, log: Optional[list] = None) -> Tuple[int, int]:
    """Pick (block, groups) for ``batch`` (a ``twa.Batch``) and apply it.

    Tuning advances the batch's instances; callers that need a fixed start
    should tune on a copy of the batch (same shapes) or reset the state."""
    import torch
    dev = torch.cuda.get_device_name(0)
    key = f"{dev}|{shape_signature(batch.instances)}|{iters}"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        b, g = cache[key]
        batch.twa_batch_config(b, g)
        return b, g
    best = None
    for b, g in candidates(len(batch)):
        batch.twa_batch_config(b, g)
        batch.twa_batch_iterate(2)          # warm (graph capture, caches)
        ms = batch.twa_batch_iterate_timed(iters)
        if log is not None:
            log.append(dict(block=b, groups=g, ms_per_iter=ms / iters))
        if best is None or ms < best[0]:
            best = (ms, b, g)
    _, b, g = best
    batch.twa_batch_config(b, g)
    if use_cache:
        cache[key] = [b, g]
        _store_cache(cache)
    return b, g
