"""Measured choice of the launch shape (pixels per lane of the render
kernels, records per binning workgroup, persistent render kernels and their
workgroups per CU).  None of these changes results.

The search times a caller-supplied step for each candidate with HIP events
and keeps the fastest; results are cached in a JSON file keyed by device,
image size and job/record counts.  A missing or unreadable cache falls back
to the defaults.
"""
from __future__ import annotations

import json
import os

import torch

from . import native as N
from . import raster as R

DEFAULT = {"fwd_px": 1, "bwd_px": 1, "sort_chunk": 0, "persistent": False, "persist_per_cu": 0}
CANDIDATES = [
    dict(DEFAULT),
    {**DEFAULT, "fwd_px": 2},
    {**DEFAULT, "bwd_px": 2},
    {**DEFAULT, "sort_chunk": 128},
    {**DEFAULT, "sort_chunk": 256},
    {**DEFAULT, "sort_chunk": 512},
    {**DEFAULT, "persistent": True},
    {**DEFAULT, "persistent": True, "persist_per_cu": 4},
    {**DEFAULT, "persistent": True, "persist_per_cu": 8},
]


def describe(cfg: dict) -> str:
    """Short name of a launch shape, e.g. 'fwd1 bwd2 chunk256 persistent8'."""
    name = f"fwd{cfg['fwd_px']} bwd{cfg['bwd_px']} chunk{cfg['sort_chunk'] or 'auto'}"
    if cfg["persistent"]:
        name += f" persistent{cfg['persist_per_cu'] or 'occ'}"
    return name


def cache_path() -> str:
    return os.environ.get("IVRGS_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ivrgs_autotune.json"))


def key(width, height, n_jobs, n_records) -> str:
    name = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    return f"{name}|{width}x{height}|jobs{n_jobs}|rec{1 << max(int(n_records) - 1, 1).bit_length()}"


def load_cache(path=None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store(k: str, cfg: dict, path=None):
    path = path or cache_path()
    data = load_cache(path)
    data[k] = cfg
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1)
        os.replace(tmp, path)
    except OSError:
        pass


def valid(cfg) -> bool:
    try:
        return (cfg["fwd_px"] in (1, 2, 4) and cfg["bwd_px"] in (1, 2, 4) and int(cfg["sort_chunk"]) >= 0
                and isinstance(cfg["persistent"], bool) and int(cfg["persist_per_cu"]) >= 0)
    except (KeyError, TypeError, ValueError):
        return False


def apply(settings: R.Settings, cfg: dict) -> R.Settings:
    s = R.Settings(**{**settings.__dict__})
    s.fwd_px, s.bwd_px, s.sort_chunk = cfg["fwd_px"], cfg["bwd_px"], cfg["sort_chunk"]
    s.flags = (s.flags | N.FLAG_PERSISTENT) if cfg["persistent"] else (s.flags & ~N.FLAG_PERSISTENT)
    s.persist_per_cu = cfg["persist_per_cu"]
    return s


def time_ms(fn, reps: int = 5) -> float:
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(make_step, width, height, n_jobs, n_records, candidates=None, reps: int = 5,
         use_cache: bool = True, path=None):
    """make_step(cfg) -> zero-argument callable running one step with that
    launch shape.  Returns (best cfg, {index: ms})."""
    k = key(width, height, n_jobs, n_records)
    if use_cache:
        hit = load_cache(path).get(k)
        if hit is not None and valid(hit):
            return hit, {}
    times = {}
    best, best_ms = dict(DEFAULT), float("inf")
    for i, cfg in enumerate(candidates or CANDIDATES):
        ms = time_ms(make_step(cfg), reps)
        times[i] = ms
        if ms < best_ms:
            best, best_ms = cfg, ms
    if use_cache:
        store(k, best, path)
    return best, times
