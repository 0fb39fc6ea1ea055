"""Launch-shape autotuner for the phase kernels.

The phase kernels come in workgroup sizes of 64, 128 and 256 work-items and
with the XCD-aware or the plain workgroup order.  Every shape computes the
same bits, so the choice is a pure speed question; it depends on the lattice
size (a small lattice needs small workgroups to occupy 256 CUs, a large one
needs the XCD-aware order for L2 reuse).  The tuner times overrelaxation
steps on a clone of the field (the chain itself is never touched), keeps the
fastest shape, applies it, and remembers it in a JSON cache keyed by GPU
architecture, Nc, extents and precision (or by the chain list of a batch).
"""
import json
import os

import torch

from . import sun

CACHE = os.environ.get("SUN_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "sun_mi355x",
                                                       "tune.json"))


def _arch():
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def _load_cache():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(c):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def _time(fn, reps):
    fn()                                   # warm-up
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / reps


def lattice_key(lat):
    return f"{_arch()}:su{lat.nc}:{'x'.join(map(str, lat.L))}:{sun.DTYPE_NAMES[lat.dtype]}"


def tune_lattice(lat, reps=5, use_cache=True):
    """Picks and applies the fastest launch shape for `lat`; returns
    (block, xcd, {shape: ms per overrelaxation step})."""
    key = lattice_key(lat)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        block, xcd = cache[key]["block"], cache[key]["xcd"]
        lat.set_launch(block, xcd)
        return block, xcd, cache[key].get("ms", {})
    clone = sun.Lattice(lat.nc, lat.L, lat.dtype, device=lat.links.device)
    clone.links.copy_(lat.links)
    times = {}
    for block, xcd in sun.Lattice.LAUNCH_SHAPES:
        clone.set_launch(block, xcd)
        times[f"{block}/{xcd}"] = _time(lambda: clone.sweep(1.0, 0, 1, seed=0, reunit=False), reps)
    best = min(times, key=times.get)
    block, xcd = (int(v) for v in best.split("/"))
    lat.set_launch(block, xcd)
    cache[key] = {"block": block, "xcd": xcd, "ms": times}
    if use_cache:
        _save_cache(cache)
    return block, xcd, times


def batch_key(batch):
    parts = [f"su{l.nc}:{'x'.join(map(str, l.L))}:{sun.DTYPE_NAMES[l.dtype]}" for l in batch.lattices]
    return f"{_arch()}:batch:" + ",".join(parts)


def tune_batch(batch, reps=3, use_cache=True):
    """Picks and applies the fastest launch shape for a batch (timed on a
    clone of its chains); drops the batch's captured graph."""
    key = batch_key(batch)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        batch.set_launch(cache[key]["block"], cache[key]["xcd"])
        return cache[key]["block"], cache[key]["xcd"], cache[key].get("ms", {})
    clones = []
    for l in batch.lattices:
        c = sun.Lattice(l.nc, l.L, l.dtype, device=l.links.device)
        c.links.copy_(l.links)
        clones.append(c)
    cb = sun.Batch(clones, batch.betas, batch.seeds)
    times = {}
    for block, xcd in sun.Lattice.LAUNCH_SHAPES:
        cb.set_launch(block, xcd)
        times[f"{block}/{xcd}"] = _time(lambda: cb.sweep(0, 1, reunit=False), reps)
    best = min(times, key=times.get)
    block, xcd = (int(v) for v in best.split("/"))
    batch.set_launch(block, xcd)
    cache[key] = {"block": block, "xcd": xcd, "ms": times}
    if use_cache:
        _save_cache(cache)
    return block, xcd, times
