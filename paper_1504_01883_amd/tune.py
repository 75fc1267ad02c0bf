"""Launch-shape autotuning with a persistent JSON cache.

The native tuner (lbpf_tune_batch) times every candidate launch shape of the
fused feature kernel on a batch and keeps the fastest. This module caches the
winner per shape bucket -- (crop count, mean crop area, feature dimension),
each rounded to a power of two -- so later batches of the same kind reuse it
without re-timing. Cache file: $LBPF_TUNE_CACHE, else
~/.cache/lbpf/tune.json.
"""
from __future__ import annotations

import json
import math
import os
from pathlib import Path


def cache_path() -> Path:
    p = os.environ.get("LBPF_TUNE_CACHE")
    return Path(p) if p else Path.home() / ".cache" / "lbpf" / "tune.json"


def _bucket(v: float) -> int:
    return 1 << max(0, int(math.ceil(math.log2(max(1.0, v)))))


def shape_key(n_crops: int, mean_area: float, dim: int) -> str:
    return f"features|n={_bucket(n_crops)}|area={_bucket(mean_area)}|dim={dim}"


def _load(path: Path) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tuned(ctx, batch, hist, n_crops: int, mean_area: float, reps: int = 5, path=None,
          retune: bool = False) -> dict:
    """Apply the cached launch shape for this bucket, tuning (and caching) on a miss.
    Returns {"cfg": ..., "us": ..., "cached": bool}."""
    path = Path(path) if path else cache_path()
    key = shape_key(n_crops, mean_area, ctx.dim)
    cache = _load(path)
    if not retune and key in cache:
        batch.set_launch(**cache[key]["cfg"])
        return {"cfg": cache[key]["cfg"], "us": cache[key]["us"], "cached": True}
    cfg, us = ctx.tune(batch, hist, reps)
    cache[key] = {"cfg": cfg, "us": us}
    path.parent.mkdir(parents=True, exist_ok=True)
    tmp = path.with_suffix(".tmp")
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return {"cfg": cfg, "us": us, "cached": False}
