#!/usr/bin/env python3
"""Throughput of the SU(3) Wilson-action checkerboard sweep on one MI355X.

Workload: SU(3), 32^4 periodic lattice, beta = 6.2, Haar hot start, FP32 link
storage in the two-row form (12 reals per link, row 2 rebuilt on load) with
FP64 reductions and FP64 re-unitarization.  One step is one pass
of the whole hot path over the lattice: 1 heatbath step + 4 overrelaxation
steps (each 4 directions x {even, odd} phases), re-unitarization (reporting
the unitarity drift it removed), the plaquette (FP64) and the Polyakov loop.
The same workload with 18-real FP32 links and with FP64 links is timed beside
it.  `configs` then runs every workload of the table (SU(2) 8^4 cold FP64,
SU(3) 16^4 and 32^4 hot, SU(4/6/8) 12^4, a batch of 64 small independent
chains replayed from a HIP graph) in its stated storage and in the other
precision, with throughput and the thermalized plaquette (and Polyakov loop)
means with errors from the integrated autocorrelation time, their
FP32-vs-FP64 difference in units of its error, the unitarity drift before
each re-unitarization and the relative action change of an overrelaxation
step.

Prints one JSON line.  `value` is link updates per second (one update = one
heatbath or overrelaxation visit of one link) with the field resident in HBM.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0           # MI355X HBM3E, published peak
METRIC = "link updates/sec + HBM GB/s (%roofline), SU(3) 32^4, batched FP32 vs plain FP64"


def link_bytes(nc, dtype):
    rows = 2 if dtype.endswith("r12") else nc
    reals = 4 if nc == 2 else 2 * rows * nc
    return reals * (4 if dtype.startswith("f32") else 8)


def phase_bytes(nc, V, dtype):
    """Algorithmic HBM bytes of one checkerboard phase: the whole field is
    read once (4V links: the updated U_mu of both parities and every U_nu),
    and the V/2 updated links are written: 9 link transfers per update."""
    return 9 * link_bytes(nc, dtype) * (V // 2)


def step_bytes(nc, V, dtype, n_hb, n_or):
    """Per step: 8 (n_hb + n_or) phases, re-unitarization (read + write 4V),
    plaquette (read 4V), Polyakov loop (read V)."""
    lb = link_bytes(nc, dtype)
    return 8 * (n_hb + n_or) * phase_bytes(nc, V, dtype) + (8 * V + 4 * V + V) * lb


KERNEL_SOURCES = ["sun_device.hpp", "sun_kernels.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
MALL_BYTES = 256 * 2 ** 20       # MI355X Infinity Cache (last level, in front of HBM)


def kernel_source_hash():
    """Hash of the device code, so stored byte counters are used only while
    the kernels they were taken on are unchanged."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1112_4533_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(workload):
    """Bytes per launch of the overrelaxation phase kernel that miss the L2
    (served by the Infinity Cache or HBM), from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None when the kernels changed after
    those counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(workload)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e["read_bytes"] + e["write_bytes"]


def field_bytes(run):
    return 4 * run.volume * link_bytes(run.nc, run.dtype)


def roofline(run, r, copy_gbps=None):
    """The overrelaxation phase kernel (32 of the 40 phases of a step):
    algorithmic bytes per launch over its mean launch time, against the HBM
    peak; plus the measured device-copy ceiling of the same run."""
    k = r["kernels"]["overrelax"]
    per_launch = phase_bytes(run.nc, run.volume, run.dtype)
    achieved = per_launch / (k["avg_ms"] * 1e-3) / 1e9
    fb = field_bytes(run)
    resident = fb <= MALL_BYTES
    out = {"bound": "hbm", "kernel": f"overrelaxation phase ({run.dtype} storage)", "achieved": achieved,
           "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
           "traffic": stored_traffic(run.name),
           "traffic_kind": "bytes per launch beyond L2 (Infinity Cache hits + HBM), rocprofv3 FETCH_SIZE + "
                           "WRITE_SIZE scaled by a device copy",
           "bytes_per_launch": per_launch, "avg_launch_ms": k["avg_ms"],
           "timing": r.get("timing"),
           "field_bytes": fb, "cache_resident": resident,
           "bound_note": (f"the {fb / 1e6:.0f} MB field fits the 256 MiB Infinity Cache, so part of the "
                          "re-read neighbour traffic is served there rather than by HBM" if resident else
                          f"the {fb / 1e6:.0f} MB field exceeds the 256 MiB Infinity Cache: an HBM measurement")}
    if copy_gbps:
        out["copy_ceiling_GBps"] = copy_gbps
        out["frac_of_copy_ceiling"] = achieved / copy_gbps
    return out


def copy_ceiling(nbytes=2 ** 30, reps=10):
    """Device-to-device copy rate (bytes read + written per second, GB/s) of
    an nbytes buffer, timed with events around reps copies on torch's stream:
    the practical HBM ceiling of this GPU in this run."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    gbps = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbps


def run_gpu(run, steps, warmup, tune=False):
    import torch
    from paper_1112_4533_amd import autotune, sun

    lat = sun.Lattice(run.nc, run.L, run.dtype)
    lat.init(hot=run.hot, seed=run.seed)
    if tune:
        autotune.tune_lattice(lat, reps=3, use_cache=False)
    dev = lat.links.device
    plaq = torch.zeros(3, dtype=torch.float64, device=dev)
    poly = torch.zeros(2, dtype=torch.float64, device=dev)
    drift = torch.zeros(2, dtype=torch.float64, device=dev)
    lib, stream = sun.load(), sun._stream()

    def step():
        lat.sweep(run.beta, run.n_hb, run.n_or, seed=run.seed, reunit=False)
        sun._check(lib.sun_reunitarize(lat._h, sun._ptr(drift), stream))
        lat.plaquette(plaq)
        lat.polyakov(poly)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # kernel averages from a second, separately timed pass: HIP events on
    # the launch stream bracket each run of back-to-back launches of one
    # kernel kind (the 8 heatbath and the 32 overrelaxation phases of a step,
    # each as one run; the other kernels singly), so no launch is slowed by a
    # bracket of its own, and the timed pass above carries no events at all
    lat.profile(True, every=-1)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    kernels = {}
    for name in ("heatbath", "overrelax", "reunit", "plaquette", "polyakov"):
        ms, n = lat.profile_read(name)
        kernels[name] = {"avg_ms": ms / n if n else None, "launches": n}
    lat.profile(False)
    # overrelaxation is microcanonical: the relative action change of one
    # overrelaxation step (FP64 plaquettes before and after), untimed
    p0 = lat.plaquette().cpu()
    lat.sweep(run.beta, 0, 1, seed=run.seed, reunit=False)
    p1 = lat.plaquette().cpu()
    or_ds = float((p0[0] - p1[0]) / (1.0 - p0[0]))   # S is proportional to 1 - mean plaquette
    V = run.volume
    updates = steps * (run.n_hb + run.n_or) * 4 * V
    return {
        "elapsed_s": elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "updates_per_s": updates / elapsed,
        "kernels": kernels,
        "timing": "kernel averages from a second pass of the same steps: one event pair per run of back-to-back "
                  "launches of a kernel (per step: 8 heatbath, 32 overrelaxation phases), average = run time / "
                  "launches, gaps between launches included; the step time is from a pass without events",
        "plaquette": plaq.cpu().tolist(),
        "polyakov": poly.cpu().tolist(),
        "unitarity_before_reunit": drift.cpu().tolist(),
        "step_counter": lat.step,
        "or_dS_over_S": or_ds,
        "launch": {"heatbath": lat.get_launch(sun.HEATBATH), "overrelax": lat.get_launch(sun.OVERRELAX),
                   "sites_per_item": [lat.get_sites_per_item(sun.HEATBATH), lat.get_sites_per_item(sun.OVERRELAX)]},
    }


# ---------------------------------------------------------------------------
# Every configuration of the workload table, with its precision statement
# ---------------------------------------------------------------------------
def stat_summary(series, cut):
    """Mean and error (integrated autocorrelation time) after the cut."""
    from paper_1112_4533_amd import analysis
    m, e, tau = analysis.mean_error(series[cut:])
    return {"mean": m, "err": e, "tau_int": tau}


def chain_run(run, dtype, sweeps, cut):
    """One chain of `run` with link storage `dtype`: per sweep the sweep,
    re-unitarization reporting the drift it removed, plaquette and Polyakov
    loop, all queued on the device (no host round trip inside the loop).
    Returns throughput, the thermalized plaquette and Polyakov means with
    their errors, the largest drift, and the relative action change of one
    further overrelaxation step."""
    import numpy as np
    import torch
    from paper_1112_4533_amd import sun

    lat = sun.Lattice(run.nc, run.L, dtype)
    lat.init(hot=run.hot, seed=run.seed)
    dev = lat.links.device
    plaq = torch.zeros((sweeps, 3), dtype=torch.float64, device=dev)
    poly = torch.zeros((sweeps, 2), dtype=torch.float64, device=dev)
    drift = torch.zeros((sweeps, 2), dtype=torch.float64, device=dev)
    lib, stream = sun.load(), sun._stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(sweeps):
        lat.sweep(run.beta, run.n_hb, run.n_or, seed=run.seed, reunit=False)
        sun._check(lib.sun_reunitarize(lat._h, sun._ptr(drift[k]), stream))
        lat.plaquette(plaq[k])
        lat.polyakov(poly[k])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    p0 = lat.plaquette().cpu()
    lat.sweep(run.beta, 0, 1, seed=run.seed, reunit=False)
    p1 = lat.plaquette().cpu()
    P, Pl, D = plaq.cpu().numpy(), poly.cpu().numpy(), drift.cpu().numpy()
    del lat
    torch.cuda.empty_cache()
    absL = np.hypot(Pl[:, 0], Pl[:, 1])
    return {
        "link_updates_per_s": sweeps * (run.n_hb + run.n_or) * 4 * run.volume / dt,
        "ms_per_sweep": 1e3 * dt / sweeps,
        "plaquette": stat_summary(P[:, 0], cut),
        "plaquette_spatial": stat_summary(P[:, 1], cut)["mean"],
        "plaquette_temporal": stat_summary(P[:, 2], cut)["mean"],
        "polyakov_re": stat_summary(Pl[:, 0], cut),
        "polyakov_abs": stat_summary(absL, cut),
        "max_unitarity_dev_before_reunit": float(D[:, 0].max()),
        "max_det_dev_before_reunit": float(D[:, 1].max()),
        "or_rel_action_change": float((p0[0] - p1[0]) / (1.0 - p0[0])),
        "series_first_last": [float(P[0, 0]), float(P[-1, 0])],
    }


def difference(a, b):
    """a - b of two thermalized means, its combined error and the ratio."""
    d = a["mean"] - b["mean"]
    s = (a["err"] ** 2 + b["err"] ** 2) ** 0.5
    return {"diff": d, "sigma": s, "z": d / s if s > 0 else None}


def config_entry(run, storages, sweeps, cut, reference="f64", label=None):
    out = {"workload": label or run.name, "nc": run.nc, "L": list(run.L), "beta": run.beta,
           "start": "hot" if run.hot else "cold", "n_hb": run.n_hb, "n_or": run.n_or,
           "reunit": "every sweep", "sweeps_in_config": run.sweeps, "sweeps_run": sweeps,
           "thermalization_cut": cut, "storage": {}}
    for dt in storages:
        out["storage"][dt] = chain_run(run, dt, sweeps, cut)
        print(f"config {out['workload']} {dt}: {out['storage'][dt]['ms_per_sweep']:.3f} ms/sweep, plaquette "
              f"{out['storage'][dt]['plaquette']['mean']:.6f} +- {out['storage'][dt]['plaquette']['err']:.6f}",
              file=sys.stderr, flush=True)
    ref = out["storage"][reference]["plaquette"]
    out["minus_" + reference] = {dt: difference(out["storage"][dt]["plaquette"], ref)
                                 for dt in storages if dt != reference}
    return out


def run_configs(batch_steps):
    """The five workloads: SU(2) 8^4 cold FP64, SU(3) 16^4 hot FP32, SU(3)
    32^4 hot FP32 (two-row and 18 reals) against FP64, SU(4/6/8) 12^4 FP32 and
    FP64, and the 64-chain batch.  Each runs in its stated storage and in the
    other precision from the same seed and start; chains that share seed and
    start part after a few sweeps (a heatbath decision near its threshold
    takes the other branch), after which the two are independent samples of
    the same distribution: FP32 storage is unbiased when the thermalized means
    agree within their errors (z = difference / combined error)."""
    from paper_1112_4533_amd.workloads import (SU2_8_COLD, SU3_16_HOT, SU3_32_F32_TWO_ROW, large_nc_runs)
    out = {}
    # SU(2) 8^4: the stated 20 sweeps are far too few for a mean with an
    # error, so the chains run 2000 sweeps (0.2 ms each)
    out["c1"] = config_entry(SU2_8_COLD, ["f64", "f32"], 2000, 100)
    out["c2"] = config_entry(SU3_16_HOT, ["f32", "f64"], 400, 100)
    out["c3"] = config_entry(SU3_32_F32_TWO_ROW, ["f32r12", "f32", "f64"], 200, 100,
                             label="su3_32^4_hot (two-row FP32, 18-real FP32, FP64)")
    for r32, r64 in zip(large_nc_runs("f32"), large_nc_runs("f64")):
        out[f"c4_su{r32.nc}"] = config_entry(r32, ["f32", "f64"], 200, 100, label=f"su{r32.nc}_12^4_hot")
    out["c5"] = run_batch(batch_steps, sweeps=200, cut=100)
    # the z of every FP32-vs-FP64 comparison above, as one chi-square
    import numpy as np
    from scipy.stats import chi2
    zs = []
    for k, v in out.items():
        if k == "c5":
            zs += v["per_chain_z"]
        else:
            zs += [d["z"] for d in v["minus_f64"].values()]
    zs = np.array([z for z in zs if z is not None])
    out["all_fp32_vs_fp64"] = {"comparisons": int(zs.size), "chi2": float((zs ** 2).sum()),
                               "p_value": float(chi2.sf((zs ** 2).sum(), zs.size)),
                               "max_abs_z": float(np.abs(zs).max())}
    return out


def run_batch(steps, sweeps=200, cut=100, tune=True):
    """The 64-chain batch (mixed SU(2)/SU(3), extents 8..20, per-chain beta
    and seed), hot start.  FP32 links swept together from a captured graph
    (each replay one sweep of every chain: 1 HB + 4 OR, re-unitarization,
    plaquettes), with the launch shapes and the SU(3) link layout chosen by
    the autotuner; against the same chains in FP64 swept one chain at a time
    with eager launches.  Both sets run `sweeps` sweeps with the plaquettes
    of every sweep kept; then `steps` more graph replays are timed alone."""
    import numpy as np
    import torch
    from paper_1112_4533_amd import autotune, sun
    from paper_1112_4533_amd.workloads import batch_spec

    spec = batch_spec()
    total_sites = sum(r.volume for r in spec)
    n_hb, n_or = spec[0].n_hb, spec[0].n_or
    betas, seeds = [r.beta for r in spec], [r.seed for r in spec]
    lats = []
    for r in spec:
        lat = sun.Lattice(r.nc, r.L, "f32")
        lat.init(hot=True, seed=r.seed)
        lats.append(lat)
    tuned = {}
    if tune:
        layout, t_layout = autotune.tune_batch_layout(lats, betas, seeds, reps=3, use_cache=False)
        if layout != "f32":
            lats = autotune.relayout(lats, layout)
        tuned["su3_layout"] = layout
        tuned["layout_ms_per_hb_or_step"] = t_layout
    bt = sun.Batch(lats, betas, seeds)
    if tune:
        best, _ = autotune.tune_batch(bt, reps=2, use_cache=False)
        tuned["shapes"] = {"heatbath": list(best[0]), "overrelax": list(best[1])}
    plaq32 = torch.zeros((len(spec), 3), dtype=torch.float64, device="cuda")
    series32 = torch.zeros((sweeps, len(spec)), dtype=torch.float64, device="cuda")
    bt.capture(n_sweeps=1, n_hb=n_hb, n_or=n_or, reunit=True, plaq_out=plaq32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(sweeps):
        bt.replay()
        series32[k].copy_(plaq32[:, 0])
    torch.cuda.synchronize()
    dt_stats32 = time.perf_counter() - t0
    # the drift one sweep leaves before re-unitarization
    bt.sweep(n_hb, n_or, reunit=False)
    drift32 = max(float(l.unitarity().cpu()[0]) for l in lats)
    bt.sweep(0, 0, reunit=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        bt.replay()
    torch.cuda.synchronize()
    dt32 = time.perf_counter() - t0
    upd32 = steps * (n_hb + n_or) * 4 * total_sites / dt32

    l64 = []
    for r in spec:
        lat = sun.Lattice(r.nc, r.L, "f64")
        lat.init(hot=True, seed=r.seed)
        l64.append(lat)
    series64 = torch.zeros((sweeps, len(spec)), dtype=torch.float64, device="cuda")
    plaq64 = torch.zeros((len(spec), 3), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(sweeps):
        for i, (r, lat) in enumerate(zip(spec, l64)):
            lat.sweep(r.beta, n_hb, n_or, seed=r.seed)
            lat.plaquette(plaq64[i])
        series64[k].copy_(plaq64[:, 0])
    torch.cuda.synchronize()
    dt64 = time.perf_counter() - t0
    upd64 = sweeps * (n_hb + n_or) * 4 * total_sites / dt64
    for lat, r in zip(l64, spec):
        lat.sweep(r.beta, n_hb, n_or, seed=r.seed, reunit=False)
    drift64 = max(float(l.unitarity().cpu()[0]) for l in l64)

    s32, s64 = series32.cpu().numpy(), series64.cpu().numpy()
    z = []
    for i in range(len(spec)):
        z.append(difference(stat_summary(s32[:, i], cut), stat_summary(s64[:, i], cut))["z"])
    from scipy.stats import chi2
    zz = np.array(z)
    return {
        "workload": "64 chains, SU(2) x 32 + SU(3) x 32, extents {8,12,16,20}^4, hot start, 1 HB + 4 OR, "
                    "re-unitarization every sweep",
        "chains": len(spec), "sites": total_sites, "sweeps_run": sweeps, "thermalization_cut": cut,
        "autotuned": tuned,
        "fp32_batched_graph": {"value": upd32, "unit": "link_updates/s", "ms_per_sweep": 1e3 * dt32 / steps,
                               "sweeps_timed": steps,
                               "ms_per_sweep_with_plaquette_copy": 1e3 * dt_stats32 / sweeps,
                               "max_unitarity_dev_before_reunit": drift32},
        "fp64_per_chain_eager": {"value": upd64, "unit": "link_updates/s", "ms_per_sweep": 1e3 * dt64 / sweeps,
                                 "sweeps_timed": sweeps, "max_unitarity_dev_before_reunit": drift64},
        "speedup": upd32 / upd64,
        "per_chain_z": [float(v) for v in z],
        "fp32_vs_fp64": {"chi2": float((zz ** 2).sum()), "dof": len(z), "p_value": float(chi2.sf((zz ** 2).sum(),
                                                                                                  len(z))),
                         "max_abs_z": float(np.abs(zz).max()), "mean_z": float(zz.mean())},
    }


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def run_cpu_baseline(run, sweeps, single_thread=True):
    """The FP64 CPU oracle on a bounded sample of the same workload: a few
    full sweeps (1 HB + 4 OR, re-unitarization, plaquette) of the lattice
    from the same hot start on all the threads OpenMP gives it, and on one
    thread one heatbath phase and two overrelaxation phases, weighted as the
    1 : 4 mix of a sweep."""
    import oracle as O

    U = O.new_field(run.nc, run.L, hot=run.hot, seed=run.seed)
    threads = O.num_threads()
    t0 = time.perf_counter()
    for k in range(sweeps):
        O.sweep(U, run.nc, run.L, run.beta, run.n_hb, run.n_or, run.seed, k * run.n_hb, reunit=True)
        O.plaquette(U, run.nc, run.L)
    dt = time.perf_counter() - t0
    updates = sweeps * (run.n_hb + run.n_or) * 4 * run.volume
    out = {
        "value": updates / dt,
        "unit": "link_updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{sweeps} sweeps (1 HB + 4 OR + re-unitarization + plaquette) of SU(3) {run.L[0]}^4 "
                   f"from the hot start, FP64: {updates} link updates in {dt:.2f} s on {threads} threads"),
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
    }
    if single_thread:
        O.set_num_threads(1)
        try:
            t0 = time.perf_counter()
            O.phase(U, run.nc, run.L, 0, 0, 0, run.beta, run.seed, sweeps)
            t_hb = time.perf_counter() - t0
            t0 = time.perf_counter()
            O.phase(U, run.nc, run.L, 1, 0, 0, run.beta, run.seed, 0)
            O.phase(U, run.nc, run.L, 1, 0, 1, run.beta, run.seed, 0)
            t_or = (time.perf_counter() - t0) / 2
        finally:
            O.set_num_threads(threads)
        half = run.volume // 2
        out["single_thread"] = {
            "value": (run.n_hb + run.n_or) * half / (run.n_hb * t_hb + run.n_or * t_or),
            "unit": "link_updates/s",
            "sample": f"one heatbath phase ({t_hb:.2f} s) and two overrelaxation phases ({t_or:.2f} s each) of "
                      f"{half} links on one thread, weighted {run.n_hb} : {run.n_or}",
        }
    return out


PEAK_FP32_TFLOPS = 78.6          # MI355X vector FP32 without packed instructions (= the FP64 rate)
PEAK_FP64_TFLOPS = 78.6
NC_SCAN = {"f32": (4, 5, 6, 8, 10, 12, 16, 20, 22, 24, 26, 28, 30, 32),
           "f64": (4, 5, 6, 8, 10, 12, 16, 20, 22, 24, 26, 28, 30, 32)}


def wide_update_flops(nc):
    """Algorithmic flops of one link update on the large-Nc path: 12 staple
    products and W = U A (8 Nc^3 each), and per subgroup two rows of U and W
    times a 2x2 complex matrix (32 flops per column and matrix)."""
    return 13 * 8 * nc ** 3 + (nc * (nc - 1) // 2) * 2 * 32 * nc


def run_nc_scan(reps, warmup, only=None):
    """Time per iteration (1 heatbath + 1 overrelaxation step + re-unitarization,
    the paper's large-Nc protocol) on 8^4 at beta 6.2, hot start, for the
    register path (Nc <= 4) and the workgroup-per-link path (Nc >= 4), a
    cubic fit of the latter's time in Nc (least squares in relative error),
    and the log-log slope of each kernel's time from Nc = 16 up."""
    import numpy as np
    import torch
    from paper_1112_4533_amd import sun

    L, beta = (8, 8, 8, 8), 6.2
    V = 8 ** 4
    rows, fits = [], {}
    for prec, ncs in NC_SCAN.items():
        for nc in ncs:
            if only and nc not in only:
                continue
            paths = (["register"] if nc <= sun.NC_MAX_REGISTER else []) + ["wide"]
            for path in paths:
                dtype = prec if path == "register" or nc > sun.NC_MAX_REGISTER else prec + "w"
                lat = sun.Lattice(nc, L, dtype)
                lat.init(hot=True, seed=1234)
                for _ in range(warmup):
                    lat.sweep(beta, 1, 1, seed=1234)
                torch.cuda.synchronize()
                lat.profile(True)
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                for _ in range(reps):
                    lat.sweep(beta, 1, 1, seed=1234)
                b.record()
                b.synchronize()
                ms = a.elapsed_time(b) / reps
                kern = {k: lat.profile_read(k) for k in ("heatbath", "overrelax", "reunit")}
                lat.profile(False)
                row = {"nc": nc, "precision": prec, "path": path, "ms_per_iteration": ms,
                       "link_updates_per_s": 2 * 4 * V / (ms * 1e-3),
                       "kernel_avg_ms": {k: (t / n if n else None) for k, (t, n) in kern.items()}}
                if path == "wide":
                    t_or = row["kernel_avg_ms"]["overrelax"]
                    fl = wide_update_flops(nc) * V / 2
                    peak = PEAK_FP32_TFLOPS if prec == "f32" else PEAK_FP64_TFLOPS
                    row["overrelax_tflops"] = fl / (t_or * 1e-3) / 1e12
                    row["overrelax_frac_of_peak"] = row["overrelax_tflops"] / peak
                rows.append(row)
                print(json.dumps(row), flush=True)
                del lat
        w = [r for r in rows if r["precision"] == prec and r["path"] == "wide"]
        if len(w) < 5 or w[-1]["nc"] <= 16:   # too few sizes for the fit
            continue
        x = np.array([r["nc"] for r in w], dtype=float)
        y = np.array([r["ms_per_iteration"] for r in w])
        c = np.polyfit(x, y, 3, w=1.0 / y)          # least squares in relative error
        slopes = {}
        for k in ("heatbath", "overrelax", "reunit"):
            t = np.array([r["kernel_avg_ms"][k] for r in w])
            lo = int(np.searchsorted(x, 16))
            slopes[k] = float(np.log(t[-1] / t[lo]) / np.log(x[-1] / x[lo]))
        fits[prec] = {"ms_cubic_coeffs_high_to_low": c.tolist(),
                      "max_rel_residual": float(np.max(np.abs(np.polyval(c, x) - y) / y)),
                      "cubic_share_at_max_nc": float(c[0] * x[-1] ** 3 / y[-1]),
                      "loglog_slope_nc16_to_max": slopes}
    return {"nc_scan": {"lattice": "8^4", "beta": beta, "iteration": "1 HB + 1 OR + re-unitarization",
                        "rows": rows, "fit": fits}}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=8, help="oracle sweeps in the CPU-baseline sample")
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the run of every workload with its FP32-vs-FP64 statement")
    ap.add_argument("--head", choices=["two_row", "eighteen"], default="two_row",
                    help="SU(3) storage of the headline line (the other is reported beside it)")
    ap.add_argument("--no-second", action="store_true", help="skip the other storage's leg")
    ap.add_argument("--tune", action="store_true", help="autotune launch shapes before timing")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GB",
                    help="only copy a GB-sized device buffer 5 times (the reference kernel for "
                         "scaling HBM byte counters), then exit")
    ap.add_argument("--nc-scan", action="store_true",
                    help="only time one iteration against Nc (4..32) on 8^4 and fit a cubic, then exit")
    ap.add_argument("--nc-list", type=int, nargs="+", default=None,
                    help="with --nc-scan: only these Nc (no fit below five sizes)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the 64-chain batch with its default launch shapes and link layout (no tuner), "
                         "then exit")
    args = ap.parse_args()
    if args.batch_only:
        b = run_batch(max(4, args.steps), sweeps=max(8, args.steps), cut=max(8, args.steps) // 2, tune=False)
        print(json.dumps({"batch": {k: b[k] for k in ("chains", "sites", "fp32_batched_graph",
                                                      "fp64_per_chain_eager", "speedup")}}), flush=True)
        return
    if args.nc_scan:
        print(json.dumps(run_nc_scan(max(1, args.steps // 10), max(1, args.warmup // 3), only=args.nc_list)),
              flush=True)
        return
    if args.copy_calibration > 0:
        import torch
        n = int(args.copy_calibration * 1e9) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent chains shard without communication; one lattice needs a halo exchange per phase)",
              file=sys.stderr)
        sys.exit(2)

    from paper_1112_4533_amd.workloads import SU3_32_F32, SU3_32_F32_TWO_ROW, SU3_32_F64

    # the headline is the faster FP32 storage of the same workload (two-row);
    # --head eighteen makes the 18-real form the headline
    head, other = ((SU3_32_F32_TWO_ROW, SU3_32_F32) if args.head == "two_row" else (SU3_32_F32, SU3_32_F32_TWO_ROW))
    copy_gbps = copy_ceiling()
    r_head = run_gpu(head, args.steps, args.warmup, tune=args.tune)
    r18 = None if args.no_second else run_gpu(other, args.steps, args.warmup, tune=args.tune)
    r64 = None if args.no_f64 else run_gpu(SU3_32_F64, max(2, args.steps // 2), max(1, args.warmup // 2))

    V = head.volume
    line = {
        "metric": METRIC,
        "value": r_head["updates_per_s"],
        "unit": "link_updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r_head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (Haar hot start from Philox, seed 1234)",
        "config": {
            "workload": head.name, "nc": head.nc, "L": list(head.L), "beta": head.beta,
            "n_hb": head.n_hb, "n_or": head.n_or, "reunit": "every sweep",
            "storage": ("FP32, SU(3) two-row (12 reals per link, row 2 rebuilt on load)"
                        if head.dtype.endswith("r12") else "FP32, full 3x3 (18 reals per link)"),
            "step": "sweep + reunitarize(drift) + plaquette + polyakov",
        },
        "roofline": roofline(head, r_head, copy_gbps),
        "effective_GBps_whole_step": step_bytes(head.nc, V, head.dtype, head.n_hb, head.n_or)
        / (r_head["ms_per_step"] * 1e-3) / 1e9,
        "kernels": r_head["kernels"],
        "launch": r_head["launch"],
        "accuracy": {
            "plaquette": r_head["plaquette"],
            "polyakov": r_head["polyakov"],
            "max_unitarity_dev_before_reunit": r_head["unitarity_before_reunit"],
            "overrelaxation_rel_action_change": r_head["or_dS_over_S"],
        },
    }
    if r18:
        line["eighteen_real" if args.head == "two_row" else "two_row"] = {
            "workload": other.name, "value": r18["updates_per_s"], "unit": "link_updates/s",
            "ms_per_step": r18["ms_per_step"], "roofline": roofline(other, r18, copy_gbps), "kernels": r18["kernels"],
            "launch": r18["launch"], "plaquette": r18["plaquette"],
            "max_unitarity_dev_before_reunit": r18["unitarity_before_reunit"],
            "overrelaxation_rel_action_change": r18["or_dS_over_S"],
            "headline_over_this": r_head["updates_per_s"] / r18["updates_per_s"],
        }
    if r64:
        line["fp64"] = {
            "workload": SU3_32_F64.name, "value": r64["updates_per_s"], "unit": "link_updates/s",
            "ms_per_step": r64["ms_per_step"], "steps": max(2, args.steps // 2), "kernels": r64["kernels"],
            "plaquette": r64["plaquette"], "max_unitarity_dev_before_reunit": r64["unitarity_before_reunit"],
            "overrelaxation_rel_action_change": r64["or_dS_over_S"],
            "fp32_over_fp64": r_head["updates_per_s"] / r64["updates_per_s"],
        }
    if not args.no_configs:
        line["configs"] = run_configs(max(4, args.steps))
        if not args.no_batch:
            c5 = line["configs"]["c5"]
            line["batch"] = {k: c5[k] for k in ("chains", "sites", "autotuned", "fp32_batched_graph",
                                                "fp64_per_chain_eager", "speedup")}
    elif not args.no_batch:
        b = run_batch(max(4, args.steps), sweeps=max(8, args.steps), cut=max(8, args.steps) // 2)
        line["batch"] = {k: b[k] for k in ("chains", "sites", "autotuned", "fp32_batched_graph",
                                           "fp64_per_chain_eager", "speedup")}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = run_cpu_baseline(SU3_32_F32, args.cpu_sweeps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
