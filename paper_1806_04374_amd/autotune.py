"""Launch-shape autotuning with a JSON cache.

The first time a (geometry, dictionary size, angle grid, K, precision, device) combination is
seen, the encoder's usable launch shapes are timed on a sample of the caller's own
coordinates (rsc_autotune_encode) and the fastest is stored; later calls apply the
cached choice without timing.  Cache file: $RSC_AUTOTUNE_CACHE, else
~/.cache/rsc_autotune.json.
"""
from __future__ import annotations

import json
import os

from . import rsc


def cache_path() -> str:
    return os.environ.get("RSC_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "rsc_autotune.json"))


def key(h: rsc.Handle, K: int) -> str:
    import torch
    name = torch.cuda.get_device_name(0).replace(" ", "_") if torch.cuda.is_available() else "cpu"
    return f"N{h.N}-S{h.S}-T{h.T}-M{h.M}-R{h.R}-K{K}-{getattr(h, 'prec', 'fp32')}-{name}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(h: rsc.Handle, xhat_sample, K: int, reps: int = 5, path: str | None = None,
         force: bool = False) -> dict:
    """Apply the cached launch shape for this handle, or time the candidates and cache the best.

    xhat_sample: device [P, B] coordinates representative of the workload (a few
    thousand patches or more, so that the launch fills the GPU).
    """
    path = path or cache_path()
    db = _load(path)
    k = key(h, K)
    if not force and k in db:
        rsc.rsc_set_launch(h, db[k]["tile"], db[k]["blocks_per_cu"])
        return dict(db[k], cached=True)
    rows = rsc.rsc_autotune_encode(h, xhat_sample, K, reps)
    tile, bpc = rsc.rsc_get_launch(h)
    entry = {"tile": tile, "blocks_per_cu": bpc, "sample_patches": int(xhat_sample.shape[0]),
             "candidates": [{"tile": t, "blocks_per_cu": b, "median_ms": m} for t, b, m in rows]}
    db[k] = entry
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1)
    os.replace(tmp, path)
    return dict(entry, cached=False)
