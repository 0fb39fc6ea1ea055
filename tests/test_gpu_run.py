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
