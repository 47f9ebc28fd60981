"""Launch-shape selection for the fused step kernel.

The library's autotuner (lbm_axi_autotune) times every candidate shape (strip
width, rows per work item, persistent queue or one workgroup per item in one of
three orders, populations in registers or gathered again, and for batches two
stream groups) on the live state and keeps the fastest.  This module caches its
choice per architecture, precision and size class in JSON: first a file shipped
with the package (tuned_launch.json, if present), then a user cache
($LBM_AXI_TUNING_CACHE or ~/.cache/lbm_axi/tuning.json), so a known size class
is not re-tuned.
"""
from __future__ import annotations

import json
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
SHIPPED = os.path.join(_HERE, "tuned_launch.json")


def user_cache_path() -> str:
    return os.environ.get("LBM_AXI_TUNING_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "lbm_axi", "tuning.json"))


def size_class(params, precision: int) -> str:
    """arch:dtype:instances:log2(nodes):log2(max nz) -- launch shapes transfer within a class."""
    nodes = sum(p.nz * p.nr for p in params)
    maxnz = max(p.nz for p in params)
    inst = "single" if len(params) == 1 else f"batch{2 ** math.ceil(math.log2(len(params)))}"
    dtype = "f32" if precision == 1 else "f64"
    return f"gfx950:{dtype}:{inst}:n{int(math.log2(max(nodes, 1)))}:z{int(math.log2(max(maxnz, 1)))}"


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def lookup(key: str):
    for path in (SHIPPED, user_cache_path()):
        rec = _load(path).get(key)
        if rec:
            return rec
    return None


def store(key: str, launch: dict, ms: float):
    path = user_cache_path()
    data = _load(path)
    data[key] = {"launch": launch, "ms_per_step": ms}
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    except OSError:
        pass


def choose_launch(sim, wl, tune: bool = True, steps_per_trial: int = 3, log=None) -> dict:
    """Apply the cached shape for this size class, else autotune (if allowed) and cache it."""
    key = size_class(wl.params, wl.precision)
    rec = lookup(key)
    if rec:
        sim.set_launch(**rec["launch"])
        if log:
            log(f"[tuning] {key}: cached {rec['launch']}")
        return sim.get_launch()
    if tune:
        launch, ms = sim.autotune(steps_per_trial)
        store(key, launch, ms)
        if log:
            log(f"[tuning] {key}: tuned {launch} at {ms:.3f} ms/step")
        return launch
    return sim.get_launch()
