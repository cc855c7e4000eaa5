"""Launch-shape autotuning with an on-disk cache.

The library's nnms_autotune times, on the system's own data, the lanes per
CSR row of every level operator and of every P^T, and the persistent grid of
the triangular-solve kernel on every level, and keeps the fastest.  This
module caches the result per hierarchy shape and device in a JSON file so
that later runs reuse it without re-timing.
"""
from __future__ import annotations

import json
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuning.json")
# Revision of the tuned kernels: launch shapes measured on an older revision
# are not reused.  Raised whenever a tuned kernel changes its resource use.
KERNEL_REV = 6


def _device_name() -> str:
    """Architecture and compute-unit count (stable across tools, unlike the
    marketing name)."""
    try:
        import torch

        p = torch.cuda.get_device_properties(0)
        return f"{getattr(p, 'gcnArchName', 'gpu').split(':')[0]}-{p.multi_processor_count}cu"
    except Exception:
        return "unknown"


def tune(system, cache: Optional[str] = DEFAULT_CACHE, reps: int = 10, force: bool = False) -> dict:
    """Apply the cached tuning of system's hierarchy, or measure and cache it."""
    h = system.h
    key = f"r{KERNEL_REV}|{_device_name()}|{h.signature()}"
    db = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            db = json.load(f)
    if not force and key in db:
        h.set_tuning(db[key])
        return db[key]
    t = system.autotune(reps)
    if cache:
        db[key] = t
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return t
