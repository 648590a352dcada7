"""Autotuner of the kernel variants (HRT_TUNE_* bits of hrt_desc.flags):
FFT radix caps per axis, columns per workgroup of the column pass, row-band
height of the spread and gather kernels, spread and gather chunk sizes.

The variants change only float32 rounding, not the operator.  The tuner
times forward+adjoint of a grid on the device and walks the variant space one
dimension at a time (coordinate search: every option of a dimension with the
others held at the best so far, then the next dimension), which covers the
48 combinations with about 15 timings.  The choice is cached in a JSON file
keyed by the grid and the device name: $HRT_TUNE_CACHE, else
~/.cache/paper_1604_07651_amd/tune.json; a cache shipped with the package
(tune_cache.json, written by this module on an MI355X) is read when the user
cache has no entry.

    python -m paper_1604_07651_amd.autotune c3 [c2 c4 c4batch ...] [--out FILE]
tunes the named grid configurations (c4: every distinct gather shape of the
64-gather uneven batch; c4batch: that batch as a whole) and writes (merges)
their entries."""
from __future__ import annotations

import json
import os

import torch

from . import _lib

# the dimensions of the search, each a list of mutually exclusive flag values
DIMENSIONS = [
    ("fft", [0, _lib.TUNE_ROW_RADIX8, _lib.TUNE_COL_RADIX8,
             _lib.TUNE_ROW_RADIX8 | _lib.TUNE_COL_RADIX8, _lib.TUNE_COL_PAIRS,
             _lib.TUNE_COL_PAIRS | _lib.TUNE_ROW_RADIX8,
             _lib.TUNE_COL_PAIRS | _lib.TUNE_COL_RADIX8,
             _lib.TUNE_COL_PAIRS | _lib.TUNE_ROW_RADIX8 | _lib.TUNE_COL_RADIX8]),
    ("band_rows", [0, _lib.TUNE_BAND4, _lib.TUNE_BAND2]),
    ("spread_chunk", [0, _lib.TUNE_SPREAD_HALF]),
    ("gather_chunk", [0, _lib.TUNE_GATHER_DOUBLE]),
]
# every combination (for callers that time the whole space)
VARIANTS = sorted({a | b | c | d for a in DIMENSIONS[0][1] for b in DIMENSIONS[1][1]
                   for c in DIMENSIONS[2][1] for d in DIMENSIONS[3][1]})
PACKAGED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


def cache_path() -> str:
    return os.environ.get("HRT_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_1604_07651_amd", "tune.json")


def key(desc, device=None) -> str:
    name = torch.cuda.get_device_name(device)
    fields = ("nt", "nx", "dt", "x0", "dx", "ntau", "nq", "tau0", "dtau", "q0", "dq")
    grid = ",".join(f"{getattr(desc, k)!r}" for k in fields)
    return f"{name}|{grid}|{float(getattr(desc, 'oversample', 2.0))!r}"


def _load(path) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def lookup(desc):
    """The cached entry for `desc` on this device (user cache first, then
    the packaged one), or None."""
    k = key(desc)
    for path in (cache_path(), PACKAGED):
        entry = _load(path).get(k)
        if entry:
            return entry
    return None


def tuned_flags(desc) -> int:
    """Cached best variant for `desc` on this device (0 when not tuned)."""
    entry = lookup(desc)
    return int(entry["flags"]) if entry else 0


def time_variant(desc, flags: int, reps: int = 10, rounds: int = 3) -> float:
    """ms per forward+adjoint of one plan with `flags` (random input, two
    warm-up pairs, then the best of `rounds` groups of `reps` timed pairs,
    HIP events on the current stream)."""
    from .hrt import Plan
    gen = torch.Generator(device="cuda").manual_seed(0)
    plan = Plan(desc, flags=flags)
    try:
        f = torch.randn(plan.data_shape, device="cuda", generator=gen)
        g = torch.empty(plan.radon_shape, device="cuda")
        fa = torch.empty(plan.data_shape, device="cuda")
        for _ in range(2):
            plan.normal(f, g=g, out=fa)
        best = float("inf")
        for _ in range(rounds):
            start = torch.cuda.Event(enable_timing=True)
            end = torch.cuda.Event(enable_timing=True)
            start.record()
            for _ in range(reps):
                plan.normal(f, g=g, out=fa)
            end.record()
            end.synchronize()
            best = min(best, start.elapsed_time(end) / reps)
        return best
    finally:
        plan.close()


def tune(desc, reps: int = 10, variants=None, save: bool = True, path: str | None = None) -> dict:
    """Finds the fastest variant for `desc`.  With `variants`, times exactly
    those; otherwise searches DIMENSIONS one at a time.  Returns {"flags":
    best, "ms": {flags: ms per forward+adjoint}}; saved to `path` (default
    the user cache) when `save`."""
    times = {}

    def t(fl):
        if fl not in times:
            times[fl] = time_variant(desc, fl, reps)
        return times[fl]

    if variants is not None:
        for fl in variants:
            t(fl)
        best = min(times, key=times.get)
    else:
        best = 0
        for _, options in DIMENSIONS:
            mask = 0
            for o in options:
                mask |= o
            base = best & ~mask
            best = min((base | o for o in options), key=t)
    result = {"flags": int(best), "ms": {str(k): round(v, 5) for k, v in sorted(times.items())}}
    if save:
        save_entry(desc, result, path)
    return result


def batch_key(descs, device=None) -> str:
    """Cache key of an uneven batch: its gathers' grid keys, in order."""
    import hashlib
    h = hashlib.sha256("\n".join(key(d, device) for d in descs).encode()).hexdigest()[:20]
    return f"batch|{torch.cuda.get_device_name(device)}|{len(descs)}|{h}"


def time_batch(descs, flags: int, reps: int = 5, rounds: int = 3) -> float:
    """ms per forward+adjoint of the whole batch, every gather with `flags`."""
    from .hrt import Batch
    gen = torch.Generator(device="cuda").manual_seed(0)
    b = Batch(descs, flags=flags)
    try:
        f = torch.randn(b.data_off[-1], device="cuda", generator=gen)
        g = b.forward(f)
        fa = b.adjoint(g)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(rounds):
            start = torch.cuda.Event(enable_timing=True)
            end = torch.cuda.Event(enable_timing=True)
            start.record()
            for _ in range(reps):
                b.forward(f, out=g)
                b.adjoint(g, out=fa)
            end.record()
            end.synchronize()
            best = min(best, start.elapsed_time(end) / reps)
        return best
    finally:
        b.close()


def tune_batch(descs, reps: int = 5, save: bool = True, path: str | None = None) -> dict:
    """The variant for a whole uneven batch (one flags value for all its
    gathers), by the same coordinate search over the batch's own timing:
    the best variant of a gather alone need not be the best inside a batch,
    where the work items of all gathers share each launch."""
    times = {}

    def t(fl):
        if fl not in times:
            times[fl] = time_batch(descs, fl, reps)
        return times[fl]

    best = 0
    for _, options in DIMENSIONS:
        mask = 0
        for o in options:
            mask |= o
        base = best & ~mask
        best = min((base | o for o in options), key=t)
    result = {"flags": int(best), "ms": {str(k): round(v, 5) for k, v in sorted(times.items())}}
    if save:
        path = path or cache_path()
        data = _load(path)
        data[batch_key(descs)] = result
        _store(path, data)
    return result


def batch_flags(descs) -> int:
    """Cached variant of the batch `descs` on this device (0 if not tuned)."""
    k = batch_key(descs)
    for path in (cache_path(), PACKAGED):
        entry = _load(path).get(k)
        if entry:
            return int(entry["flags"])
    return 0


def _store(path: str, data: dict) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def save_entry(desc, result: dict, path: str | None = None) -> None:
    path = path or cache_path()
    data = _load(path)
    data[key(desc)] = result
    _store(path, data)


def main(argv=None) -> None:
    import argparse
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import synth
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("configs", nargs="+", help="grid configurations (c1, c2, c3, ...)")
    ap.add_argument("--out", default=None, help="cache file to write (default: user cache)")
    ap.add_argument("--reps", type=int, default=10)
    args = ap.parse_args(argv)
    for name in args.configs:
        if name == "c4batch":
            res = tune_batch(synth.batch_descs(64, seed=4), path=args.out)
            print(json.dumps({"config": name, **res}), flush=True)
            continue
        if name == "c4":
            seen = {}
            for d in synth.batch_descs(64, seed=4):
                seen.setdefault((d.nt, d.nx), d)
            descs = [(f"c4 {nt}x{nx}", d) for (nt, nx), d in sorted(seen.items())]
        else:
            descs = [(name, synth.config_desc(name))]
        for label, desc in descs:
            res = tune(desc, reps=args.reps, path=args.out)
            print(json.dumps({"config": label, **res}), flush=True)


if __name__ == "__main__":
    main()
