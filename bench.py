#!/usr/bin/env python3
"""Throughput of the SU(3) Wilson-action checkerboard sweep on one MI355X.

Workload: SU(3), 32^4 periodic lattice, beta = 6.2, Haar hot start, FP32 link
storage with FP64 reductions and FP64 re-unitarization.  One step is one pass
of the whole hot path over the lattice: 1 heatbath step + 4 overrelaxation
steps (each 4 directions x {even, odd} phases), re-unitarization (reporting
the unitarity drift it removed), the plaquette (FP64) and the Polyakov loop.
The same workload with FP64 link storage is timed beside it.

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


def run_gpu(run, steps, warmup, tune=True):
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
    lat.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernels = {}
    for name in ("heatbath", "overrelax", "reunit", "plaquette", "polyakov"):
        ms, n = lat.profile_read(name)
        kernels[name] = {"avg_ms": ms / n if n else None, "launches": n}
    lat.profile(False)
    V = run.volume
    updates = steps * (run.n_hb + run.n_or) * 4 * V
    return {
        "elapsed_s": elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "updates_per_s": updates / elapsed,
        "kernels": kernels,
        "plaquette": plaq.cpu().tolist(),
        "polyakov": poly.cpu().tolist(),
        "unitarity_before_reunit": drift.cpu().tolist(),
        "step_counter": lat.step,
        "launch": {"heatbath": lat.get_launch(sun.HEATBATH), "overrelax": lat.get_launch(sun.OVERRELAX)},
    }


def run_batch(steps, warmup, f64_sweeps):
    """The 64-chain batch (mixed SU(2)/SU(3), extents 8..20, per-chain beta
    and seed): FP32 links swept together from a captured graph (each replay
    is one sweep of every chain: 1 HB + 4 OR, re-unitarization, plaquettes),
    against the same chains in FP64 swept one chain at a time with eager
    launches."""
    import torch
    from paper_1112_4533_amd import sun
    from paper_1112_4533_amd.workloads import batch_spec

    spec = batch_spec()
    total_sites = sum(r.volume for r in spec)
    n_hb, n_or = spec[0].n_hb, spec[0].n_or
    lats = []
    for r in spec:
        lat = sun.Lattice(r.nc, r.L, "f32")
        lat.init(hot=True, seed=r.seed)
        lats.append(lat)
    bt = sun.Batch(lats, [r.beta for r in spec], [r.seed for r in spec])
    from paper_1112_4533_amd import autotune
    autotune.tune_batch(bt, reps=2, use_cache=False)
    plaq32 = torch.zeros((len(spec), 3), dtype=torch.float64, device="cuda")
    bt.capture(n_sweeps=1, n_hb=n_hb, n_or=n_or, reunit=True, plaq_out=plaq32)
    for _ in range(warmup):
        bt.replay()
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
    plaq64 = torch.zeros((len(spec), 3), dtype=torch.float64, device="cuda")

    def sweep64():
        for i, (r, lat) in enumerate(zip(spec, l64)):
            lat.sweep(r.beta, n_hb, n_or, seed=r.seed)
            lat.plaquette(plaq64[i])

    for _ in range(warmup):
        sweep64()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(f64_sweeps):
        sweep64()
    torch.cuda.synchronize()
    dt64 = time.perf_counter() - t0
    upd64 = f64_sweeps * (n_hb + n_or) * 4 * total_sites / dt64
    # both chains sets have now run warmup + timed sweeps; compare their plaquettes
    # after catching the FP64 set up to the same sweep count
    for _ in range(steps - f64_sweeps):
        sweep64()
    d = (plaq32[:, 0] - plaq64[:, 0]).cpu()
    return {
        "chains": len(spec), "sites": total_sites,
        "fp32_batched_graph": {"value": upd32, "unit": "link_updates/s", "ms_per_sweep": 1e3 * dt32 / steps,
                               "sweeps": steps, "launch": {"heatbath": bt.launch[0], "overrelax": bt.launch[1]}},
        "fp64_per_chain_eager": {"value": upd64, "unit": "link_updates/s", "ms_per_sweep": 1e3 * dt64 / f64_sweeps,
                                 "sweeps": f64_sweeps},
        "speedup": upd32 / upd64,
        "plaquette_f32_minus_f64": {"mean": float(d.mean()), "std": float(d.std()),
                                    "after_sweeps": warmup + steps},
    }


def run_cpu_baseline(run, sweeps):
    """The FP64 CPU oracle on a bounded sample of the same workload: a few
    full sweeps (1 HB + 4 OR, re-unitarization, plaquette) of the 32^4 lattice
    from the same hot start."""
    import oracle as O

    U = O.new_field(run.nc, run.L, hot=run.hot, seed=run.seed)
    t0 = time.perf_counter()
    for k in range(sweeps):
        O.sweep(U, run.nc, run.L, run.beta, run.n_hb, run.n_or, run.seed, k * run.n_hb, reunit=True)
        O.plaquette(U, run.nc, run.L)
    dt = time.perf_counter() - t0
    updates = sweeps * (run.n_hb + run.n_or) * 4 * run.volume
    return {
        "value": updates / dt,
        "unit": "link_updates/s",
        "cores": O.num_threads(),
        "kind": "oracle",
        "sample": (f"{sweeps} sweeps (1 HB + 4 OR + re-unitarization + plaquette) of SU(3) {run.L[0]}^4 "
                   f"from the hot start, FP64: {updates} link updates in {dt:.2f} s"),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=8, help="oracle sweeps in the CPU-baseline sample")
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-two-row", action="store_true")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GB",
                    help="only copy a GB-sized device buffer 5 times (the reference kernel for "
                         "scaling HBM byte counters), then exit")
    args = ap.parse_args()
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

    run = SU3_32_F32
    r32 = run_gpu(run, args.steps, args.warmup)
    r64 = None if args.no_f64 else run_gpu(SU3_32_F64, max(2, args.steps // 2), max(1, args.warmup // 2))
    r12 = None if args.no_two_row else run_gpu(SU3_32_F32_TWO_ROW, args.steps, args.warmup)

    V = run.volume
    k_or = r32["kernels"]["overrelax"]
    per_launch = phase_bytes(run.nc, V, run.dtype)
    achieved = per_launch / (k_or["avg_ms"] * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": r32["updates_per_s"],
        "unit": "link_updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (Haar hot start from Philox, seed 1234)",
        "config": {
            "workload": run.name, "nc": run.nc, "L": list(run.L), "beta": run.beta,
            "n_hb": run.n_hb, "n_or": run.n_or, "reunit": "every sweep",
            "step": "sweep + reunitarize(drift) + plaquette + polyakov",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "overrelaxation phase (k_update<3,float,OR>)",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": None,
            "bytes_per_launch": per_launch,
            "avg_launch_ms": k_or["avg_ms"],
        },
        "effective_GBps_whole_step": step_bytes(run.nc, V, run.dtype, run.n_hb, run.n_or) / (r32["ms_per_step"] * 1e-3) / 1e9,
        "kernels": r32["kernels"],
        "launch": r32["launch"],
        "accuracy": {
            "plaquette": r32["plaquette"],
            "polyakov": r32["polyakov"],
            "max_unitarity_dev_before_reunit": r32["unitarity_before_reunit"],
        },
    }
    if r64:
        line["fp64"] = {
            "value": r64["updates_per_s"], "unit": "link_updates/s", "ms_per_step": r64["ms_per_step"],
            "steps": max(2, args.steps // 2), "kernels": r64["kernels"], "plaquette": r64["plaquette"],
            "max_unitarity_dev_before_reunit": r64["unitarity_before_reunit"],
            "f32_over_f64": r32["updates_per_s"] / r64["updates_per_s"],
        }
    if r12:
        k12 = r12["kernels"]["overrelax"]
        pb12 = phase_bytes(run.nc, V, SU3_32_F32_TWO_ROW.dtype)
        a12 = pb12 / (k12["avg_ms"] * 1e-3) / 1e9
        line["two_row"] = {
            "workload": SU3_32_F32_TWO_ROW.name, "value": r12["updates_per_s"], "unit": "link_updates/s",
            "ms_per_step": r12["ms_per_step"],
            "roofline": {"bound": "hbm", "kernel": "overrelaxation phase, two-row storage", "achieved": a12,
                         "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": a12 / PEAK_HBM_GBS,
                         "bytes_per_launch": pb12, "avg_launch_ms": k12["avg_ms"]},
            "kernels": r12["kernels"], "plaquette": r12["plaquette"],
            "max_unitarity_dev_before_reunit": r12["unitarity_before_reunit"],
            "speedup_over_18_real": r12["updates_per_s"] / r32["updates_per_s"],
        }
    if not args.no_batch:
        line["batch"] = run_batch(max(4, args.steps), args.warmup, max(2, args.steps // 4))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = run_cpu_baseline(run, args.cpu_sweeps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
