"""Autotuner of the kernel variants (FFT radices per axis, columns per
workgroup of the column pass): times forward+adjoint of every variant on the
device for a grid description and caches the fastest in a JSON file keyed by
the grid and the device name.  Cache path: $HRT_TUNE_CACHE, else
~/.cache/paper_1604_07651_amd/tune.json."""
from __future__ import annotations

import json
import os

import torch

from . import _lib

VARIANTS = [f for f in range(8)]  # every combination of the three HRT_TUNE_* bits


def cache_path() -> str:
    return os.environ.get("HRT_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_1604_07651_amd", "tune.json")


def key(desc, device=None) -> str:
    name = torch.cuda.get_device_name(device)
    fields = ("nt", "nx", "dt", "x0", "dx", "ntau", "nq", "tau0", "dtau", "q0", "dq")
    grid = ",".join(f"{getattr(desc, k)!r}" for k in fields)
    return f"{name}|{grid}|{float(getattr(desc, 'oversample', 2.0))!r}"


def _load() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def tuned_flags(desc) -> int:
    """Cached best variant for `desc` on this device (0 when not tuned)."""
    entry = _load().get(key(desc))
    return int(entry["flags"]) if entry else 0


def tune(desc, reps: int = 10, variants=VARIANTS, save: bool = True) -> dict:
    """Times forward+adjoint of each variant (random input, `reps` timed
    pairs after two warm-up pairs, HIP events on the current stream) and
    returns {"flags": best, "ms": {flags: ms per pair}}, cached if `save`."""
    from .hrt import Plan
    times = {}
    gen = torch.Generator(device="cuda").manual_seed(0)
    for fl in variants:
        plan = Plan(desc, flags=fl)
        f = torch.randn(plan.data_shape, device="cuda", generator=gen)
        g = torch.empty(plan.radon_shape, device="cuda")
        fa = torch.empty(plan.data_shape, device="cuda")
        for _ in range(2):
            plan.forward(f, out=g)
            plan.adjoint(g, out=fa)
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(reps):
            plan.forward(f, out=g)
            plan.adjoint(g, out=fa)
        end.record()
        end.synchronize()
        times[fl] = start.elapsed_time(end) / reps
        plan.close()
    best = min(times, key=times.get)
    result = {"flags": int(best), "ms": {str(k): v for k, v in times.items()}}
    if save:
        data = _load()
        data[key(desc)] = result
        path = cache_path()
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1)
        os.replace(tmp, path)
    return result
