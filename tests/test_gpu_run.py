"""The run tool on the GPU: a chain interrupted and resumed from its
configuration file is bitwise the chain that ran straight through."""
import json
import os

import numpy as np
import pytest

from paper_1112_4533_amd import configio, run

pytestmark = pytest.mark.gpu


def _history(d):
    with open(os.path.join(d, "history.jsonl")) as f:
        rows = [json.loads(l) for l in f]
    for r in rows:
        r.pop("seconds")
    return rows


@pytest.mark.parametrize("dtype", ["f32r12", "f64"])
def test_resume_is_bitwise(gpu, tmp_path, dtype):
    common = ["--nc", "3", "--L", "8", "8", "4", "8", "--beta", "5.9", "--dtype", dtype, "--seed", "5",
              "--n-or", "2", "--save-every", "3"]
    a, b = str(tmp_path / "a"), str(tmp_path / "b")
    run.main(common + ["--sweeps", "8", "--out", a])
    run.main(common + ["--sweeps", "3", "--out", b])
    run.main(common + ["--sweeps", "8", "--out", b, "--resume"])
    fa, ha = configio.load(os.path.join(a, "cfg_000008.sun"))
    fb, hb = configio.load(os.path.join(b, "cfg_000008.sun"))
    assert np.array_equal(fa, fb) and ha["sha256"] == hb["sha256"]
    assert ha["rng_step"] == hb["rng_step"] == 8
    assert _history(a) == _history(b) and len(_history(a)) == 8
    s = json.load(open(os.path.join(b, "summary.json")))
    assert s["sweeps_this_call"] == 5 and 0.3 < s["plaquette_mean"] < 0.7


def test_resume_refuses_another_run(gpu, tmp_path):
    d = str(tmp_path / "c")
    run.main(["--nc", "2", "--L", "4", "4", "4", "4", "--beta", "2.3", "--sweeps", "2", "--save-every", "2",
              "--out", d])
    with pytest.raises(SystemExit):
        run.main(["--nc", "2", "--L", "4", "4", "4", "4", "--beta", "2.4", "--sweeps", "4", "--out", d,
                  "--resume"])


def test_load_lattice_continues_the_chain(gpu, tmp_path):
    sun = gpu
    lat = sun.Lattice(4, (4, 4, 4, 4), "f32")
    lat.init(hot=True, seed=2)
    lat.sweep(11.1, 1, 1, seed=2)
    p = str(tmp_path / "x.sun")
    configio.save_lattice(p, lat, 11.1, 2, 1)
    twin, head = configio.load_lattice(p)
    assert head["storage"] == "f32" and twin.step == lat.step == 1
    lat.sweep(11.1, 1, 1, seed=2)
    twin.sweep(11.1, 1, 1, seed=2)
    assert np.array_equal(lat.export().cpu().numpy(), twin.export().cpu().numpy())


# ---------------------------------------------------------------------------
# The watchdog: a non-finite or non-unitary field is reported by the next
# check, and the chain resumes from its last good configuration
# ---------------------------------------------------------------------------
def test_watchdog_trips_on_an_imported_nan_and_the_chain_resumes_bitwise(gpu, tmp_path):
    sun = gpu
    import torch
    nc, L, beta, seed = 3, (8, 8, 4, 8), 5.9, 5
    ref = sun.Lattice(nc, L, "f32")
    ref.init(hot=True, seed=seed)
    ref.watchdog(1e-4)
    for _ in range(4):
        ref.sweep(beta, 1, 2, seed=seed)
    assert ref.check() == 0.0                      # a healthy FP32 chain stays far below 1e-4

    lat = sun.Lattice(nc, L, "f32")
    lat.init(hot=True, seed=seed)
    lat.watchdog(1e-4)
    for _ in range(2):
        lat.sweep(beta, 1, 2, seed=seed)
    assert lat.check() == 0.0
    p = str(tmp_path / "good.sun")
    configio.save_lattice(p, lat, beta, seed, 2, n_hb=1, n_or=2)
    # the failure is forced from the host: one link of the imported field is NaN
    f = lat.export().cpu().numpy()
    f[1, 37, 0, 1] = np.nan
    lat.import_(torch.from_numpy(f))
    lat.sweep(beta, 1, 2, seed=seed)
    with pytest.raises(sun.SunNumericError) as e:
        lat.check()
    assert e.value.code == sun.SUN_ENUMERIC and "infinite" in str(e.value)
    lat.watchdog(1e-4)                             # re-arming clears the state
    # resume from the last good file: bitwise the uninterrupted chain
    c, head = configio.load_lattice(p)
    assert head["rng_step"] == 2
    c.watchdog(1e-4)
    for _ in range(2):
        c.sweep(beta, 1, 2, seed=seed)
    assert c.check() == 0.0
    torch.cuda.synchronize()
    assert torch.equal(ref.links, c.links) and ref.step == c.step == 4


@pytest.mark.parametrize("dtype,ok,trip", [("f32", 1e-4, 1e-9), ("f64", 1e-10, 1e-17), ("f32r12", 1e-4, 1e-9)])
def test_watchdog_threshold_and_paths(gpu, dtype, ok, trip):
    """The check rides on every re-unitarization (of a sweep, or called
    alone); FP32 storage drifts ~1e-7..1e-5 between them, FP64 ~1e-15.  A
    sweep without re-unitarization makes no check."""
    sun = gpu
    lat = sun.Lattice(3, (6, 4, 4, 8), dtype)
    lat.init(hot=True, seed=8)
    lat.watchdog(ok)
    lat.sweep(6.0, 1, 2, seed=8)
    lat.sweep(6.0, 1, 2, seed=8, reunit=False)
    lat.reunitarize()
    assert lat.check() == 0.0
    lat.watchdog(trip)
    lat.sweep(6.0, 1, 2, seed=8, reunit=False)     # no re-unitarization: no check
    assert lat.check() == 0.0
    drift = lat.reunitarize(report=True)
    with pytest.raises(sun.SunNumericError):
        lat.check()
    # the largest tripped deviation is the drift the re-unitarization reported
    lat.watchdog(trip)
    lat.sweep(6.0, 1, 2, seed=8, reunit=False)
    drift = lat.reunitarize(report=True)
    try:
        lat.check()
        assert False, "the watchdog did not trip"
    except sun.SunNumericError:
        pass
    import ctypes
    d = ctypes.c_double()
    assert sun.load().sun_check(lat._h, ctypes.byref(d), sun._stream()) == sun.SUN_ENUMERIC
    assert d.value == float(drift.max().cpu())


def test_watchdog_on_the_workgroup_path(gpu):
    sun = gpu
    import torch
    lat = sun.Lattice(6, (4, 4, 2, 4), "f32")
    lat.init(hot=True, seed=3)
    lat.watchdog(1e-4)
    lat.sweep(24.98, 1, 1, seed=3)
    assert lat.check() == 0.0
    f = lat.export().cpu().numpy()
    f[2, 5, 3, 3] = np.inf
    lat.import_(torch.from_numpy(f))
    lat.reunitarize()
    with pytest.raises(sun.SunNumericError):
        lat.check()


def test_run_tool_stops_on_the_watchdog_and_resumes(gpu, tmp_path):
    """An absurd threshold trips the run tool's check on its first sweep
    after a save; the run stops with the failure in summary.json, and a
    resume with the default threshold continues bitwise."""
    common = ["--nc", "3", "--L", "8", "4", "4", "8", "--beta", "5.9", "--dtype", "f32", "--seed", "9",
              "--n-or", "2", "--save-every", "2"]
    a, b = str(tmp_path / "a"), str(tmp_path / "b")
    run.main(common + ["--sweeps", "4", "--out", a])
    run.main(common + ["--sweeps", "2", "--out", b])
    with pytest.raises(SystemExit) as e:
        run.main(common + ["--sweeps", "4", "--out", b, "--resume", "--watchdog", "1e-12"])
    assert "sweep 3" in str(e.value) and "cfg_000002.sun" in str(e.value)
    s = json.load(open(os.path.join(b, "summary.json")))
    assert s["failed_at_sweep"] == 3 and s["resume_from"] == "cfg_000002.sun"
    run.main(common + ["--sweeps", "4", "--out", b, "--resume"])
    fa, _ = configio.load(os.path.join(a, "cfg_000004.sun"))
    fb, _ = configio.load(os.path.join(b, "cfg_000004.sun"))
    assert np.array_equal(fa, fb)
    assert _history(a) == _history(b)
