"""Persistent choices of the native autotuner (msrs_autotune).

The tuner itself runs in the library (it times candidates with HIP events on
the problem's own stream); this module only keys its choices by device and
problem shape and keeps them in a JSON file, so a later process sets them
without timing again.  Cache file: $MSRS_TUNING_CACHE, else
~/.cache/msrs/tuning.json.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

from . import msrs

_KEYS = {msrs.TUNE_STAGE_OFFLINE: [msrs.TUNE_SWEEP_COLS],
         msrs.TUNE_STAGE_ONLINE: [msrs.TUNE_RECON_BATCH, msrs.TUNE_APPLY_BATCH]}


def cache_path() -> str:
    return os.environ.get("MSRS_TUNING_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "msrs", "tuning.json")


def signature(pr: "msrs.Problem", stage: int) -> str:
    import torch
    d = pr.desc
    ov = [d.overlap[i] for i in range(pr.layout().n_patches)]
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    raw = json.dumps([dev, stage, d.kind, d.n_cells, d.M, d.n_samples, d.rank, d.precision, d.n_vel, ov])
    return hashlib.sha1(raw.encode()).hexdigest()


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(pr: "msrs.Problem", stage: int, reps: int = 3, path: str | None = None, force: bool = False) -> dict:
    """Set the tuned launch shapes of `stage` on `pr`: from the cache, else by
    running the native autotuner and storing its choice.  Returns
    {"source": "cache"|"tuned", "values": {...}, "seconds": t, "trials": [...]}."""
    path = path or cache_path()
    key = signature(pr, stage)
    db = _load(path)
    t0 = time.perf_counter()
    if not force and key in db:
        vals = db[key]
        for k, v in vals.items():
            pr.set_tuning(int(k), int(v))
        return {"source": "cache", "values": {msrs.TUNE_NAMES[int(k)]: v for k, v in vals.items()},
                "seconds": time.perf_counter() - t0, "trials": []}
    trials = pr.autotune(stage, reps)
    vals = {str(k): pr.get_tuning(k) for k in _KEYS[stage]}
    db = _load(path)
    db[key] = vals
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass   # an unwritable cache only costs a re-tune next time
    return {"source": "tuned", "values": {msrs.TUNE_NAMES[int(k)]: v for k, v in vals.items()},
            "seconds": time.perf_counter() - t0, "trials": [list(t) for t in trials]}
