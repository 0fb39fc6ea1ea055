"""Generates a chain of SU(Nc) configurations on one GPU (paper Sec. 4
protocol: per sweep n_hb heatbath and n_or overrelaxation steps, then
re-unitarization and the plaquette), with periodic configuration files,
a per-sweep history and resume.

    python -m paper_1112_4533_amd.run --nc 3 --L 16 16 16 16 --beta 6.0 \\
        --sweeps 200 --save-every 50 --out runs/su3_16 [--resume]

Writes into --out:
  history.jsonl   one line per sweep: plaquette {total, spatial, temporal},
                  Polyakov loop {re, im}, the unitarity drift removed by that
                  sweep's re-unitarization, and the sweep's wall time
  cfg_NNNNNN.sun  the configuration after sweep NNNNNN (configio format)
  summary.json    the mean plaquette after the thermalization cut, its error
                  from the integrated autocorrelation time, and throughput
--resume continues from the newest configuration file in --out (the field,
the RNG step counter and the sweep count), after checking that it belongs to
the same run; the continued chain is bitwise the chain that was never
interrupted.

The library's watchdog checks the field in every re-unitarization (a NaN or
infinite entry, or a unitarity or determinant deviation above --watchdog
before the projection).  When it trips the run stops without writing that
sweep, records the failure in summary.json and exits with an error; the
newest configuration file is then the last good state to --resume from.
"""
import argparse
import glob
import json
import os
import sys
import time

from . import analysis, configio


def _latest_config(out):
    files = sorted(glob.glob(os.path.join(out, "cfg_*.sun")))
    return files[-1] if files else None


def _read_history(path, upto):
    rows = []
    if os.path.exists(path):
        with open(path) as f:
            for line in f:
                r = json.loads(line)
                if r["sweep"] <= upto:
                    rows.append(r)
    return rows


def run(args):
    import torch
    from . import sun

    os.makedirs(args.out, exist_ok=True)
    hist_path = os.path.join(args.out, "history.jsonl")
    params = {"nc": args.nc, "L": list(args.L), "beta": args.beta, "seed": args.seed, "n_hb": args.n_hb,
              "n_or": args.n_or, "storage": args.dtype}
    done = 0
    if args.resume and _latest_config(args.out):
        path = _latest_config(args.out)
        head = configio.read_header(path)
        for k, v in params.items():
            if head.get(k) != v:
                raise SystemExit(f"{path}: {k} = {head.get(k)!r}, this run has {v!r}")
        lat, head = configio.load_lattice(path)
        done = int(head["sweeps"])
        history = _read_history(hist_path, done)
        print(f"resuming {args.out} at sweep {done} from {os.path.basename(path)}", flush=True)
    else:
        lat = sun.Lattice(args.nc, args.L, args.dtype)
        lat.init(hot=(args.start == "hot"), seed=args.seed)
        history = []
    with open(hist_path, "w") as f:          # the history up to the restart point
        for r in history:
            f.write(json.dumps(r) + "\n")

    watch = args.watchdog if args.watchdog is not None else (1e-4 if args.dtype.startswith("f32") else 1e-10)
    lat.watchdog(watch)
    dev = lat.links.device
    plaq = torch.zeros(3, dtype=torch.float64, device=dev)
    poly = torch.zeros(2, dtype=torch.float64, device=dev)
    drift = torch.zeros(2, dtype=torch.float64, device=dev)
    lib, stream = sun.load(), sun._stream()
    t_run = time.perf_counter()
    n_new = 0
    with open(hist_path, "a") as hf:
        for sweep in range(done + 1, args.sweeps + 1):
            t0 = time.perf_counter()
            lat.sweep(args.beta, args.n_hb, args.n_or, seed=args.seed, reunit=False)
            sun._check(lib.sun_reunitarize(lat._h, sun._ptr(drift), stream))
            lat.plaquette(plaq)
            lat.polyakov(poly)
            if watch > 0:
                try:
                    lat.check()
                except sun.SunNumericError as e:
                    last = _latest_config(args.out)
                    fail = {"params": params, "failed_at_sweep": sweep, "error": str(e),
                            "resume_from": os.path.basename(last) if last else None}
                    with open(os.path.join(args.out, "summary.json"), "w") as f:
                        json.dump(fail, f, indent=1)
                    raise SystemExit(f"sweep {sweep}: {e}; last good configuration: {fail['resume_from']}")
            row = {"sweep": sweep, "plaquette": plaq.cpu().tolist(), "polyakov": poly.cpu().tolist(),
                   "drift": drift.cpu().tolist(), "seconds": time.perf_counter() - t0}
            hf.write(json.dumps(row) + "\n")
            hf.flush()
            history.append(row)
            n_new += 1
            if args.save_every and (sweep % args.save_every == 0 or sweep == args.sweeps):
                configio.save_lattice(os.path.join(args.out, f"cfg_{sweep:06d}.sun"), lat, args.beta, args.seed,
                                      sweep, n_hb=args.n_hb, n_or=args.n_or, plaquette=row["plaquette"][0])
            if args.progress and sweep % args.progress == 0:
                print(f"sweep {sweep}: plaquette {row['plaquette'][0]:.6f}", flush=True)
    wall = time.perf_counter() - t_run

    therm = args.therm if args.therm is not None else args.sweeps // 5
    series = [r["plaquette"][0] for r in history if r["sweep"] > therm]
    mean, err, tau = analysis.mean_error(series) if series else (float("nan"),) * 3
    V = 1
    for v in args.L:
        V *= v
    summary = {"params": params, "sweeps": args.sweeps, "thermalization_cut": therm,
               "plaquette_mean": mean, "plaquette_error": err, "tau_int_sweeps": tau,
               "max_drift": max((r["drift"][0] for r in history), default=0.0),
               "sweeps_this_call": n_new, "wall_s": wall,
               "link_updates_per_s": (n_new * (args.n_hb + args.n_or) * 4 * V / wall) if n_new else None}
    with open(os.path.join(args.out, "summary.json"), "w") as f:
        json.dump(summary, f, indent=1)
    print(json.dumps(summary), flush=True)
    return summary


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--nc", type=int, required=True)
    ap.add_argument("--L", type=int, nargs=4, required=True)
    ap.add_argument("--beta", type=float, required=True)
    ap.add_argument("--dtype", default="f32", help="link storage: f32, f64, f32r12, f64r12 (SU(3)), f32w, f64w")
    ap.add_argument("--start", choices=["hot", "cold"], default="hot")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--sweeps", type=int, required=True, help="total sweeps of the chain")
    ap.add_argument("--n-hb", type=int, default=1)
    ap.add_argument("--n-or", type=int, default=4)
    ap.add_argument("--save-every", type=int, default=0, help="write a configuration every this many sweeps")
    ap.add_argument("--therm", type=int, default=None, help="sweeps left out of the summary (default sweeps / 5)")
    ap.add_argument("--out", required=True)
    ap.add_argument("--resume", action="store_true")
    ap.add_argument("--progress", type=int, default=0, help="print the plaquette every this many sweeps")
    ap.add_argument("--watchdog", type=float, default=None,
                    help="largest unitarity or determinant deviation a re-unitarization may find (default 1e-4 "
                         "for FP32 storage, 1e-10 for FP64; 0 turns the check off)")
    args = ap.parse_args(argv)
    run(args)
    return 0


if __name__ == "__main__":
    sys.exit(main())
