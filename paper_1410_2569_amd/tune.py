"""Autotune cache: the fastest ensemble schedule per (device architecture, ensemble shape).

The key is the device's gcnArchName and a shape class of the ensemble (instance count and the
sorted multiset of lattice sizes); the value is the lbm_tune chosen by lbm_autotune. The cache
file is LBM_AUTOTUNE_CACHE (default: ~/.cache/lbm_autotune.json).
"""
from __future__ import annotations

import hashlib
import json
import os

from .lbm import autotune

DEFAULT = os.path.join(os.path.expanduser("~"), ".cache", "lbm_autotune.json")


def cache_path() -> str:
    return os.environ.get("LBM_AUTOTUNE_CACHE", DEFAULT)


def shape_key(params_list, arch: str) -> str:
    sizes = sorted((int(p["nx"]), int(p["ny"])) for p in params_list)
    h = hashlib.sha1(json.dumps(sizes).encode()).hexdigest()[:12]
    return f"{arch}/n{len(sizes)}/{h}"


def tuned(params_list, gw_list, rho0_list, steps=200, refresh=False):
    """lbm_tune dict for the ensemble, from the cache or by running the autotuner."""
    import torch

    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = shape_key(params_list, arch)
    path = cache_path()
    cache = {}
    if os.path.exists(path):
        try:
            with open(path) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
    if not refresh and key in cache:
        return dict(cache[key], cached=True)
    best = autotune(params_list, gw_list, rho0_list, steps=steps)
    cache[key] = best
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1)
    os.replace(tmp, path)
    return dict(best, cached=False)
