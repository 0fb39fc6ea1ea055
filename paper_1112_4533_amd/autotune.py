"""Launch-shape and layout autotuner for the phase kernels.

The phase kernels come in workgroup sizes of 64, 128 and 256 work-items, with
the XCD-aware or the plain workgroup order, with a cap of 8, 12, 16 or no
limit on resident waves per CU, (single lattices) with the linear or a
t-blocked tile walk of 2, 4 or 8 time slices, and with 1, 2 or 4 sites per
work-item (searched after the rest, with the chosen shape in place).  Every shape computes the same bits, so the
choice is a pure speed question, made separately for the heatbath and the
overrelaxation kernels (the heatbath draws cost arithmetic, so it prefers
more resident waves).  It depends on the lattice: a small lattice needs small
workgroups to occupy 256 CUs, a large one the XCD-aware order and a wave cap
for L2 reuse.  The tuner times heatbath-only and overrelaxation-only steps on
a clone of the field (the chain itself is never touched), applies the
fastest shape of each kind, and remembers the choice in a JSON cache keyed
by GPU architecture, Nc, extents and storage (or by the chain list of a batch).

For batches the link layout is a dimension too: the FP32 SU(3) chains can be
stored with all 18 reals or as two rows (12 reals, row 2 rebuilt on load;
paper Sec. 3).  tune_batch_layout times a heatbath and an overrelaxation
step of the whole batch in each layout (on clones) and relayout() moves the
chains into the chosen one.  Unlike the launch shape, the layout changes the
rounding of the links, so a chain keeps its layout for its whole run.
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


def _search(shapes, set_shape, step_hb, step_or, reps):
    """Times every shape for each kind; returns ({kind: best shape}, timings)."""
    best, times = {}, {}
    for kind, step in ((sun.HEATBATH, step_hb), (sun.OVERRELAX, step_or)):
        t = {}
        for shape in shapes:
            set_shape(shape, kind)
            t["/".join(map(str, shape))] = _time(step, reps)
        key = min(t, key=t.get)
        best[kind] = tuple(int(v) for v in key.split("/"))
        times["heatbath" if kind == sun.HEATBATH else "overrelax"] = t
    return best, times


def _search_spt(set_spt, step_hb, step_or, reps):
    """With the chosen shapes in place, times 1, 2 and 4 sites per
    work-item for each kind; returns ({kind: best}, timings)."""
    best, times = {}, {}
    for kind, step in ((sun.HEATBATH, step_hb), (sun.OVERRELAX, step_or)):
        t = {}
        for spt in sun.Lattice.SITES_PER_ITEM:
            set_spt(spt, kind)
            t[str(spt)] = _time(step, reps)
        best[kind] = int(min(t, key=t.get))
        set_spt(best[kind], kind)
        times[("heatbath" if kind == sun.HEATBATH else "overrelax") + "_sites_per_item"] = t
    return best, times


def lattice_key(lat):
    return f"{_arch()}:su{lat.nc}:{'x'.join(map(str, lat.L))}:{sun.DTYPE_NAMES[lat.dtype]}"


def tune_lattice(lat, reps=5, use_cache=True):
    """Picks and applies the fastest launch shape of each update kind for
    `lat`; returns ({kind: (block, xcd, waves, tblock)}, timings in ms per
    step)."""
    key = lattice_key(lat)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        best = {int(k): tuple(v) for k, v in cache[key]["shape"].items()}
        for kind, shape in best.items():
            lat.set_launch(*shape, kind=kind)
        for kind, spt in cache[key].get("sites_per_item", {}).items():
            lat.set_sites_per_item(spt, kind=int(kind))
        return best, cache[key].get("ms", {})
    clone = sun.Lattice(lat.nc, lat.L, lat.dtype, device=lat.links.device)
    clone.links.copy_(lat.links)
    shapes = []                            # distinct shapes in effect on this lattice
    for shape in sun.Lattice.LAUNCH_SHAPES:
        clone.set_launch(*shape, kind=sun.OVERRELAX)
        eff = clone.get_launch(sun.OVERRELAX)
        if eff not in shapes:
            shapes.append(eff)
    best, times = _search(shapes, lambda shape, kind: clone.set_launch(*shape, kind=kind),
                          lambda: clone.phase_step(sun.HEATBATH), lambda: clone.phase_step(sun.OVERRELAX), reps)
    for kind, shape in best.items():
        clone.set_launch(*shape, kind=kind)
        lat.set_launch(*shape, kind=kind)
    spt, t_spt = _search_spt(lambda v, kind: clone.set_sites_per_item(v, kind=kind),
                             lambda: clone.phase_step(sun.HEATBATH), lambda: clone.phase_step(sun.OVERRELAX), reps)
    times.update(t_spt)
    for kind, v in spt.items():
        lat.set_sites_per_item(v, kind=kind)
    cache[key] = {"shape": {str(k): list(v) for k, v in best.items()},
                  "sites_per_item": {str(k): v for k, v in spt.items()}, "ms": times}
    if use_cache:
        _save_cache(cache)
    return best, times


def batch_key(batch):
    parts = [f"su{l.nc}:{'x'.join(map(str, l.L))}:{sun.DTYPE_NAMES[l.dtype]}" for l in batch.lattices]
    return f"{_arch()}:batch:" + ",".join(parts)


def tune_batch(batch, reps=3, use_cache=True):
    """As tune_lattice for a batch (timed on a clone of its chains); drops
    the batch's captured graph."""
    key = batch_key(batch)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        best = {int(k): tuple(v) for k, v in cache[key]["shape"].items()}
        for kind, shape in best.items():
            batch.set_launch(*shape, kind=kind)
        for kind, spt in cache[key].get("sites_per_item", {}).items():
            batch.set_sites_per_item(spt, kind=int(kind))
        return best, cache[key].get("ms", {})
    clones = []
    for l in batch.lattices:
        c = sun.Lattice(l.nc, l.L, l.dtype, device=l.links.device)
        c.links.copy_(l.links)
        clones.append(c)
    cb = sun.Batch(clones, batch.betas, batch.seeds)
    best, times = _search(sun.Batch.LAUNCH_SHAPES, lambda shape, kind: cb.set_launch(*shape, kind=kind),
                          lambda: cb.sweep(1, 0, reunit=False), lambda: cb.sweep(0, 1, reunit=False), reps)
    for kind, shape in best.items():
        cb.set_launch(*shape, kind=kind)
        batch.set_launch(*shape, kind=kind)
    spt, t_spt = _search_spt(lambda v, kind: cb.set_sites_per_item(v, kind=kind),
                             lambda: cb.sweep(1, 0, reunit=False), lambda: cb.sweep(0, 1, reunit=False), reps)
    times.update(t_spt)
    for kind, v in spt.items():
        batch.set_sites_per_item(v, kind=kind)
    cache[key] = {"shape": {str(k): list(v) for k, v in best.items()},
                  "sites_per_item": {str(k): v for k, v in spt.items()}, "ms": times}
    if use_cache:
        _save_cache(cache)
    return best, times


def relayout(lattices, su3_f32_dtype):
    """New lattices holding the same fields, with every FP32 SU(3) chain
    stored as su3_f32_dtype ("f32" or "f32r12") and the others unchanged;
    step counters are carried over."""
    out = []
    for l in lattices:
        dt = sun.DTYPE_NAMES[l.dtype]
        if l.nc == 3 and dt in ("f32", "f32r12"):
            dt = su3_f32_dtype
        n = sun.Lattice(l.nc, l.L, dt, device=l.links.device)
        n.import_(l.export())
        n.step = l.step
        out.append(n)
    return out


LAYOUTS = ("f32", "f32r12")


def tune_batch_layout(lattices, betas, seeds, reps=3, use_cache=True):
    """Times one heatbath and one overrelaxation step of the batch with its
    FP32 SU(3) chains in each layout of LAYOUTS (on clones, default launch
    shapes); returns (fastest layout, {layout: ms per HB + OR step})."""
    key = f"{_arch()}:layout:" + ",".join(
        f"su{l.nc}:{'x'.join(map(str, l.L))}:{sun.DTYPE_NAMES[l.dtype]}" for l in lattices)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return cache[key]["layout"], cache[key]["ms"]
    times = {}
    for lay in LAYOUTS:
        clones = relayout(lattices, lay)
        cb = sun.Batch(clones, betas, seeds)
        times[lay] = _time(lambda: (cb.sweep(1, 0, reunit=False), cb.sweep(0, 1, reunit=False)), reps)
        del cb, clones
    best = min(times, key=times.get)
    cache[key] = {"layout": best, "ms": times}
    if use_cache:
        _save_cache(cache)
    return best, times
