"""Configuration files and the autocorrelation analysis of the run tool
(CPU only)."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_1112_4533_amd import analysis, configio


def _meta(nc, L):
    return {"nc": nc, "L": list(L), "storage": "f64", "beta": 6.0, "seed": 7, "rng_step": 11, "sweeps": 3}


def test_config_round_trip_is_exact(tmp_path):
    nc, L = 3, (4, 2, 2, 4)
    U = O.new_field(nc, L, hot=True, seed=3)
    p = str(tmp_path / "a.sun")
    configio.save(p, U, dict(_meta(nc, L), plaquette=0.5))
    V, head = configio.load(p)
    assert V.dtype == np.complex128 and np.array_equal(V, U)
    assert head["rng_step"] == 11 and head["L"] == list(L) and head["plaquette"] == 0.5
    assert configio.read_header(p)["sha256"] == head["sha256"]
    assert not [f for f in os.listdir(tmp_path) if ".tmp" in f]


def test_config_rejects_damage(tmp_path):
    nc, L = 2, (2, 2, 2, 2)
    U = O.new_field(nc, L, hot=True, seed=1)
    p = str(tmp_path / "b.sun")
    configio.save(p, U, _meta(nc, L))
    raw = bytearray(open(p, "rb").read())
    raw[-5] ^= 0x01                                     # one flipped payload bit
    open(p, "wb").write(bytes(raw))
    with pytest.raises(ValueError, match="checksum"):
        configio.load(p)
    open(p, "wb").write(b"NOTACFG!" + bytes(raw[8:]))
    with pytest.raises(ValueError, match="not a configuration"):
        configio.load(p)
    open(p, "wb").write(bytes(raw[:-16]))               # truncated
    with pytest.raises(ValueError):
        configio.load(p)
    with pytest.raises(ValueError, match="lacks"):
        configio.save(p, U, {"nc": nc, "L": list(L)})
    with pytest.raises(ValueError, match="shape"):
        configio.save(p, U[:, :-1], _meta(nc, L))


def test_tau_int_of_white_noise_and_ar1():
    """AR(1), x_t = phi x_{t-1} + e_t, has rho(t) = phi^t and
    tau_int = (1 + phi) / (2 (1 - phi)); white noise has tau_int = 1/2."""
    rng = np.random.default_rng(0)
    tau, _ = analysis.tau_int(rng.standard_normal(100000))
    assert abs(tau - 0.5) < 0.03
    for phi in (0.5, 0.8):
        e = rng.standard_normal(200000)
        x = np.empty_like(e)
        x[0] = e[0]
        for t in range(1, len(e)):
            x[t] = phi * x[t - 1] + e[t]
        tau, w = analysis.tau_int(x)
        want = (1 + phi) / (2 * (1 - phi))
        assert abs(tau - want) / want < 0.08, (phi, tau, want)
        rho = analysis.autocorrelation(x)
        assert abs(rho[1] - phi) < 0.01 and abs(rho[2] - phi ** 2) < 0.02


def test_mean_error_covers_the_true_mean():
    """The autocorrelation-corrected error of AR(1) means covers the true
    mean (0) about as often as a normal error bar should."""
    rng = np.random.default_rng(1)
    hits = 0
    for _ in range(200):
        e = rng.standard_normal(2000)
        x = np.empty_like(e)
        x[0] = e[0]
        for t in range(1, len(e)):
            x[t] = 0.7 * x[t - 1] + e[t]
        m, err, _ = analysis.mean_error(x)
        hits += abs(m) < err
    assert 0.58 < hits / 200 < 0.78


def test_run_cli_parses(tmp_path):
    from paper_1112_4533_amd import run
    with pytest.raises(SystemExit):
        run.main(["--nc", "3"])                        # missing required arguments
