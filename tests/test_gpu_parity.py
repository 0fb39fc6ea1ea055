"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Both sides draw the same Philox words, so one chain is one sample path.

Tolerances (an error model, not fitted constants).  Within one checkerboard
phase every updated link depends only on links the phase does not touch, so a
phase is compared link by link without cascades.  The rounding of W = U A is
of order eps |A| (eps the storage precision's unit roundoff), and the
subgroup direction V = P / k divides it by k, so a link whose update has
conditioning c = |A|_F / k_min (reported by the oracle) lands within
K eps (1 + c) of the oracle.  Counting the operations gives a worst case of a
few hundred for K (staple: six triple products of 3 x 3 matrices summed;
W = U A; three subgroup steps, each dividing by its k); the test uses
K = 64 (gpu_common.K_LINK), above the largest K measured over every
comparison (19 in FP64, 14 in FP32 on fresh fields, 34 in FP32 on fields
drifted by 6e-6 across a sweep without re-unitarization, where the staple's
SU(3) row-2 shortcut adds an error of order the drift).  FP32 decisions
(Creutz/KP switch, accept test) depend on alpha = 2 beta k / Nc and so move
by about the same relative amount; a link may differ by O(1) only where the
oracle's margin of one of its decisions lies within K_FLIP eps (1 + c),
K_FLIP = 2 K_LINK, and no more links may do so than three times the
expected number (or 3).  Over several sweeps the chain is chaotic (the
oracle itself, perturbed at 1e-16, drifts by orders of magnitude per sweep),
so free-running sweeps are compared against that measured sensitivity, and
whole-sweep parity is instead checked phase by phase along the trajectory,
plus bitwise equality of a sweep with its documented sequence of phases.
Every comparison records how close it ran to its bound (gpu_common.record).
"""
import numpy as np
import pytest
import torch

import oracle as O
from stats import binned_mean_err

pytestmark = pytest.mark.gpu

from gpu_common import (BETA, EPS, K_FLIP, K_TYP, SPREAD_FACTOR, TOL, compare_links, gpu_lattice,
                        oracle_phase_diag, record, rounded, thermal_field, to_np)


def record_draws(what, dtype, alpha, d, bad, margin):
    """Evidence of a sampler comparison: the largest deviation of the draws
    that agree, in units of the tolerance and of eps (1 + alpha) (alpha
    enters through the logarithms and the division by alpha), and the
    margins of the draws whose decision flipped."""
    ok = ~bad
    record(what=what, dtype=dtype, links=int(d.size), max_dU=float(d[ok].max()),
           max_dU_over_tol=float(d[ok].max() / TOL[dtype]),
           max_K_alpha=float((d[ok] / (EPS[dtype[:3]] * (1.0 + alpha[ok]))).max()),
           flips=int(bad.sum()), flip_margins=[float(m) for m in margin[bad][:50]],
           flip_alphas=[float(a) for a in alpha[bad][:50]])


def check_draw_flips(dtype, alpha, bad, margin):
    """FP64 draws agree everywhere.  An FP32 draw may take the other branch
    of a decision only where the oracle's margin lies within the decision
    window K_FLIP eps (1 + alpha) (alpha rounded to FP32 moves every
    decision input by about eps alpha), and no more draws may do so than
    three times the expected count (two decisions per draw, each flipping
    with probability at most 2 K_TYP eps (1 + alpha)), or 3."""
    if dtype.startswith("f64"):
        assert not bad.any(), int(bad.sum())
        return
    eps = EPS["f32"]
    assert np.all(margin[bad] < K_FLIP * eps * (1.0 + alpha[bad])), margin[bad]
    expected = float((2 * 2 * K_TYP * eps * (1.0 + alpha)).sum())
    assert bad.sum() <= max(3.0, 3.0 * expected), (int(bad.sum()), expected)


# ---------------------------------------------------------------------------
# The SU(2) draw
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sampler_parity(gpu, dtype):
    sun = gpu
    alpha = np.concatenate([np.zeros(64), np.linspace(0.01, 60.0, 40000), np.full(64, 1.7)])
    xg, ag = sun.sample_su2(torch.from_numpy(alpha).cuda(), seed=31, step=5, mu_sg=(2 << 16) | 1, dtype=dtype)
    xg, ag = to_np(xg), to_np(ag)
    xo, ao, margin = O.sample_su2(alpha, seed=31, step=5, mu_sg=(2 << 16) | 1)
    d = np.abs(xg - xo).max(axis=1)
    bad = (d > TOL[dtype]) | (ag != ao)
    record_draws("sampler alpha 0..60", dtype, alpha, d, bad, margin)
    check_draw_flips(dtype, alpha, bad, margin)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sampler_parity_large_alpha(gpu, dtype):
    # the couplings of the large-Nc runs (beta ~ Nc^2) reach the hundreds
    sun = gpu
    alpha = np.geomspace(60.0, 5000.0, 8192)
    xg, ag = sun.sample_su2(torch.from_numpy(alpha).cuda(), seed=77, step=3, mu_sg=(1 << 16) | 5, dtype=dtype)
    xg, ag = to_np(xg), to_np(ag)
    xo, ao, margin = O.sample_su2(alpha, seed=77, step=3, mu_sg=(1 << 16) | 5)
    d = np.abs(xg - xo).max(axis=1)
    bad = (d > TOL[dtype]) | (ag != ao)
    record_draws("sampler alpha 60..5000", dtype, alpha, d, bad, margin)
    check_draw_flips(dtype, alpha, bad, margin)
    assert np.all(ag > 0)                        # no draw runs out of attempts
    assert np.all(np.abs(np.linalg.norm(xg, axis=1) - 1) < 1e-5)


def test_sampler_empty_input(gpu):
    x, a = gpu.sample_su2(torch.zeros(0, dtype=torch.float64, device="cuda"), seed=1)
    assert x.shape == (0, 4) and a.shape == (0,)


# ---------------------------------------------------------------------------
# Start configurations and the field round trip
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nc,dtype", [(n, d) for n in (2, 3, 4, 5, 6, 8) for d in ("f64", "f32")]
                         + [(3, "f64r12"), (3, "f32r12")])
def test_hot_start_parity(gpu, nc, dtype):
    L = (4, 4, 2, 6)
    lat = gpu_lattice(gpu, nc, L, dtype, hot=True, seed=1234)
    got = to_np(lat.export())
    want = O.new_field(nc, L, hot=True, seed=1234)
    # one Gram-Schmidt pass over a Gaussian matrix: rounding ~ cond(M) * eps
    tol = 1e-12 if dtype.startswith("f64") else 1e-6
    assert np.abs(got - want).max() < tol


@pytest.mark.parametrize("nc", [2, 3, 4])
def test_cold_start_exact(gpu, nc):
    lat = gpu_lattice(gpu, nc, (4, 4, 4, 4), "f32", hot=False)
    assert np.array_equal(to_np(lat.plaquette()), [1.0, 1.0, 1.0])
    assert np.array_equal(to_np(lat.polyakov()), [1.0, 0.0])
    assert np.array_equal(to_np(lat.unitarity()), [0.0, 0.0])


@pytest.mark.parametrize("nc", [2, 3, 6])
def test_export_import_roundtrip(gpu, nc):
    L = (6, 4, 4, 2)
    U = thermal_field(nc, L, BETA[nc], sweeps=1)
    lat = gpu_lattice(gpu, nc, L, "f64", field=U)
    if nc == 2:   # the quaternion form keeps row 0 and rebuilds row 1
        assert np.abs(to_np(lat.export()) - U).max() < 1e-15
    else:
        assert np.array_equal(to_np(lat.export()), U)


# ---------------------------------------------------------------------------
# Observables on one and the same field
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nc,dtype", [(n, d) for n in (2, 3, 4, 6, 8) for d in ("f64", "f32")]
                         + [(3, "f64r12"), (3, "f32r12")])
def test_observables_parity(gpu, nc, dtype):
    L = (6, 4, 4, 8)      # V/2 = 384: a ragged second block
    lat = gpu_lattice(gpu, nc, L, dtype, field=thermal_field(nc, L, BETA[nc]))
    U = to_np(lat.export())                 # the field as the GPU stores it
    np.testing.assert_allclose(to_np(lat.plaquette()), O.plaquette(U, nc, L), rtol=1e-13, atol=1e-15)
    pg = to_np(lat.polyakov())
    po = O.polyakov(U, nc, L)
    assert abs(complex(pg[0], pg[1]) - po) < 1e-13
    ug, uo = to_np(lat.unitarity()), O.unitarity(U, nc, L)
    np.testing.assert_allclose(ug, uo, rtol=1e-6, atol=1e-15)


@pytest.mark.parametrize("nc,dtype,L", [
    (3, "f32r12", (4, 4, 4, 2)),    # fewer time slices than stretches: most stretches empty
    (3, "f64", (4, 4, 2, 12)),      # stretches of one and two links
    (2, "f32", (2, 2, 4, 10)),
    (4, "f64", (2, 4, 2, 18)),      # four stretches for SU(4), lengths 4 and 5
    (3, "f32", (4, 4, 4, 1)),       # no time direction: the loop is the identity
    (6, "f32", (2, 2, 2, 6)),       # one work-item per site (large Nc)
])
def test_polyakov_every_time_extent(gpu, nc, dtype, L):
    """The product along t is split into stretches combined as an ordered
    tree; every extent, including ones shorter than the stretch count, must
    give the ordered product of the oracle."""
    lat = gpu_lattice(gpu, nc, L, dtype, hot=True, seed=99)
    U = to_np(lat.export())
    pg = to_np(lat.polyakov())
    po = O.polyakov(U, nc, L)
    assert abs(complex(pg[0], pg[1]) - po) < 1e-12, (complex(pg[0], pg[1]), po)
    if L[3] == 1:
        assert abs(po - 1.0) < 1e-12


@pytest.mark.parametrize("nc", [2, 3, 4, 6, 8])
def test_reunitarize_parity(gpu, nc):
    L = (4, 4, 4, 4)
    rng = np.random.default_rng(nc)
    U = thermal_field(nc, L, BETA[nc], sweeps=1)
    U = U + 1e-3 * (rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape))
    if nc == 2:   # SU(2) is stored as a quaternion: keep the matrix in a0 + i a.sigma form
        U[..., 1, 0] = -np.conj(U[..., 0, 1])
        U[..., 1, 1] = np.conj(U[..., 0, 0])
    lat = gpu_lattice(gpu, nc, L, "f64", field=U)
    before = to_np(lat.reunitarize(report=True))
    after = to_np(lat.export())
    np.testing.assert_allclose(before, O.unitarity(U, nc, L), rtol=1e-10)
    O.reunitarize(U, nc, L)
    assert np.abs(after - U).max() < 1e-13
    assert to_np(lat.unitarity()).max() < 1e-13


# ---------------------------------------------------------------------------
# Single checkerboard phases (links within a phase are independent, so a
# phase compares every link without cascades)
# ---------------------------------------------------------------------------
PHASE_CASES = [(nc, dt) for nc in (2, 3, 4, 6) for dt in ("f64", "f32")] + [(3, "f64r12"), (3, "f32r12")]


@pytest.mark.parametrize("nc,dtype,L", [(3, "f32r12", (6, 4, 1, 4)), (2, "f64", (4, 1, 4, 4)), (4, "f32", (4, 4, 4, 1))])
def test_phase_parity_3d(gpu, nc, dtype, L):
    """3D lattices (one absent direction): every phase of both kinds."""
    beta = BETA[nc]
    base = O.new_field(nc, L, hot=True, seed=17)
    for kind in (0, 1):
        for mu in range(4):
            lat = gpu_lattice(gpu, nc, L, dtype, field=base)
            want = to_np(lat.export())
            lat.phase(kind, mu, 1, beta, seed=5, step=1)
            got = to_np(lat.export())
            if L[mu] == 1:      # absent direction: nothing to update
                assert np.array_equal(got, want)
                continue
            m, k = oracle_phase_diag(want, nc, L, kind, mu, 1, beta, 5, 1)
            compare_links(got, want, dtype, m, k, f"3D nc={nc} {dtype} kind={kind} mu={mu}")


@pytest.mark.parametrize("nc,dtype", PHASE_CASES)
@pytest.mark.parametrize("kind", [0, 1])
def test_phase_parity(gpu, nc, dtype, kind):
    L = (6, 4, 4, 8)
    beta = BETA[nc]
    base = thermal_field(nc, L, beta)
    flips = 0
    for mu in range(4):
        for par in range(2):
            lat = gpu_lattice(gpu, nc, L, dtype, field=base)
            want = to_np(lat.export())          # the field as the GPU stores it
            lat.phase(kind, mu, par, beta, seed=99, step=7)
            got = to_np(lat.export())
            m, k = oracle_phase_diag(want, nc, L, kind, mu, par, beta, 99, 7)
            flips += compare_links(got, want, dtype, m, k, f"nc={nc} {dtype} kind={kind} mu={mu} p={par}")
    print(f"flips: {flips}")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_phase_parity_beta_zero_and_two_site_extent(gpu, dtype):
    """beta = 0 (alpha = 0 Creutz limit) and extents of 2, where x+nu and
    x-nu are the same site."""
    nc, L = 3, (2, 2, 2, 2)
    base = rounded(thermal_field(nc, L, 6.0), dtype)
    for beta in (0.0, 6.0):
        lat = gpu_lattice(gpu, nc, L, dtype, field=base)
        lat.phase(0, 1, 1, beta, seed=5, step=3)
        got = to_np(lat.export())
        want = base.copy()
        m, k = oracle_phase_diag(want, nc, L, 0, 1, 1, beta, 5, 3)
        compare_links(got, want, dtype, m, k, f"beta={beta}")


# ---------------------------------------------------------------------------
# Whole sweeps
# ---------------------------------------------------------------------------
def run_phases_like_a_sweep(lat, beta, n_hb, n_or, seed):
    """The documented sweep: n_hb heatbath steps (RNG steps counter + h), then
    n_or overrelaxation steps, each over mu = 0..3, even then odd; then
    re-unitarization; the counter advances by n_hb."""
    step0 = lat.step
    for h in range(n_hb):
        for mu in range(4):
            for p in range(2):
                lat.phase(0, mu, p, beta, seed, step0 + h)
    for _ in range(n_or):
        for mu in range(4):
            for p in range(2):
                lat.phase(1, mu, p, beta, seed, 0)
    lat.reunitarize()
    lat.step = step0 + n_hb


@pytest.mark.parametrize("nc,dtype,n_hb,n_or", [(2, "f64", 1, 3), (3, "f32", 1, 4), (3, "f64", 2, 1),
                                                (4, "f32", 1, 1)])
def test_sweep_is_its_phase_sequence_bitwise(gpu, nc, dtype, n_hb, n_or):
    L = (6, 4, 4, 8)
    a = gpu_lattice(gpu, nc, L, dtype, hot=True, seed=21)
    b = gpu_lattice(gpu, nc, L, dtype, hot=True, seed=21)
    for _ in range(2):
        a.sweep(BETA[nc], n_hb, n_or, seed=21)
        run_phases_like_a_sweep(b, BETA[nc], n_hb, n_or, 21)
    torch.cuda.synchronize()
    assert torch.equal(a.links, b.links)
    assert a.step == b.step == 2 * n_hb


@pytest.mark.parametrize("nc,dtype,hot", [(2, "f64", False), (3, "f64", True), (4, "f64", True),
                                          (3, "f32", True), (2, "f32", True), (3, "f32r12", True),
                                          (3, "f64r12", True)])
def test_sweep_trajectory_parity_phase_by_phase(gpu, nc, dtype, hot):
    """Two sweeps (1 HB + 2 OR) from a start configuration, every phase and
    the re-unitarization compared with the oracle applied to the GPU's own
    state before that phase."""
    L, beta, seed = (6, 4, 4, 8), BETA[nc], 1234
    lat = gpu_lattice(gpu, nc, L, dtype, hot=hot, seed=seed)
    flips = 0
    for sweep in range(2):
        for kind, step in [(0, sweep)] + [(1, 0)] * 2:
            for mu in range(4):
                for p in range(2):
                    before = to_np(lat.export())
                    lat.phase(kind, mu, p, beta, seed, step)
                    m, k = oracle_phase_diag(before, nc, L, kind, mu, p, beta, seed, step)
                    flips += compare_links(to_np(lat.export()), before, dtype, m, k,
                                           f"sweep {sweep} kind {kind} mu {mu} p {p}")
        before = to_np(lat.export())
        lat.reunitarize()
        O.reunitarize(before, nc, L)
        compare_links(to_np(lat.export()), before, dtype, what=f"reunit after sweep {sweep}")
    print(f"FP32 decision flips along the trajectory: {flips}")


@pytest.mark.parametrize("dtype,L,sweeps", [("f32", (8, 8, 8, 8), 2), ("f32r12", (8, 8, 8, 8), 2),
                                            ("f32", (16, 16, 16, 16), 1), ("f32r12", (16, 16, 16, 16), 1)])
def test_bench_schedule_trajectory_phase_by_phase(gpu, dtype, L, sweeps):
    """The benchmark's schedule on 8^4 and 16^4 from a hot start: 1 HB + 4 OR with no
    re-unitarization until the end of the sweep, so the FP32 links drift
    away from unitarity (~1e-6) across the 40 phases while the SU(3) staple
    terms are built with row 2 = conj(row0 x row1), which is exact only for
    unitary links.  Every phase is compared with the oracle (full 3 x 3
    products) applied to the GPU's own state before it."""
    nc, beta, seed = 3, 6.2, 1234
    lat = gpu_lattice(gpu, nc, L, dtype, hot=True, seed=seed)
    flips = 0
    for sweep in range(sweeps):
        for kind, step in [(0, sweep)] + [(1, 0)] * 4:
            for mu in range(4):
                for p in range(2):
                    before = to_np(lat.export())
                    lat.phase(kind, mu, p, beta, seed, step)
                    m, k = oracle_phase_diag(before, nc, L, kind, mu, p, beta, seed, step)
                    flips += compare_links(to_np(lat.export()), before, dtype, m, k,
                                           f"bench schedule sweep {sweep} kind {kind} mu {mu} p {p}")
        drift = to_np(lat.reunitarize(report=True))
        record(what=f"drift before reunit, sweep {sweep}", dtype=dtype, drift=float(drift[0]))
        assert 1e-8 < drift[0] < 1e-4
    print(f"FP32 decision flips along the bench schedule: {flips}")


def sensitivity(U0, nc, L, beta, n_hb, n_or, seed, nsweeps, eps, twins=3):
    """Max |U - U'| per sweep between an oracle chain and twins whose start
    differs by eps-sized noise (the largest over `twins` twins): how far
    rounding alone can move this trajectory."""
    rng = np.random.default_rng(0)
    a = U0.copy()
    bs = [U0 + eps * (rng.standard_normal(U0.shape) + 1j * rng.standard_normal(U0.shape)) for _ in range(twins)]
    out = []
    for k in range(nsweeps):
        O.sweep(a, nc, L, beta, n_hb, n_or, seed, k * n_hb)
        for b in bs:
            O.sweep(b, nc, L, beta, n_hb, n_or, seed, k * n_hb)
        out.append(max(np.abs(a - b).max() for b in bs))
    return out


@pytest.mark.parametrize("nc,L,beta,start,n_hb,n_or", [
    (2, (8, 8, 8, 8), 2.3, "cold", 1, 3),        # SU(2) 8^4 cold start, 1 HB + 3 OR
    (3, (8, 8, 8, 8), 6.0, "thermal", 1, 4),     # SU(3), 1 HB + 4 OR
    (3, (8, 8, 8, 8), 6.0, "hot", 1, 4),
    (4, (6, 6, 6, 6), 11.1, "thermal", 1, 1),    # SU(4), 1 HB + 1 OR
    (3, (10, 6, 4, 6), 5.7, "hot", 2, 1),        # ragged volume, 2 HB steps per sweep
    (3, (8, 8, 1, 1), 3.0, "hot", 1, 2),         # 2D lattice
])
def test_free_running_sweeps_f64(gpu, nc, L, beta, start, n_hb, n_or):
    """Three free-running FP64 sweeps: the GPU chain stays within the
    rounding sensitivity of the oracle chain (1e-12 + SPREAD_FACTOR x the
    largest spread of three 1e-15-perturbed oracle twins), and the
    plaquettes agree to the same bound.  The chain is chaotic, so the bound
    grows about a hundredfold per sweep from a hot start and this test
    checks little after the first sweep; the phase-by-phase trajectory
    tests carry the weight there."""
    seed = 1234
    if start == "thermal":
        U = O.new_field(nc, L, hot=False, seed=seed)
        for k in range(10):
            O.sweep(U, nc, L, beta, 1, 2, 99, k)
    else:
        U = O.new_field(nc, L, hot=(start == "hot"), seed=seed)
    sens = sensitivity(U, nc, L, beta, n_hb, n_or, seed, 3, 1e-15)
    bound = [1e-12 + SPREAD_FACTOR["f64"] * s for s in sens]
    lat = gpu_lattice(gpu, nc, L, "f64", field=U)
    lat.step = 0
    for k in range(3):
        lat.sweep(beta, n_hb, n_or, seed=seed)
        O.sweep(U, nc, L, beta, n_hb, n_or, seed, k * n_hb)
        assert lat.step == (k + 1) * n_hb
        dev = np.abs(to_np(lat.export()) - U).max()
        print(f"sweep {k}: max |dU| = {dev:.2e}, bound {bound[k]:.2e}")
        record(what=f"free-running sweep {k}", dtype="f64", max_dU=float(dev), max_dU_over_tol=float(dev / bound[k]),
               max_dU_over_spread=float(dev / sens[k]) if sens[k] > 0 else None)
        assert dev <= bound[k], (k, dev, bound[k])
        if bound[k] < 1e-6:
            assert np.abs(to_np(lat.plaquette()) - O.plaquette(U, nc, L)).max() <= bound[k]


def test_f32_chain_matches_f64_oracle_statistically(gpu):
    """FP32 links with FP64 reductions against the FP64 oracle chain: the
    long-run plaquette agrees within the combined statistical error."""
    nc, L, beta = 3, (6, 6, 6, 6), 5.7
    lat = gpu_lattice(gpu, nc, L, "f32", hot=True, seed=11)
    U = O.new_field(nc, L, hot=True, seed=12)
    pg, po = [], []
    out = torch.empty(3, dtype=torch.float64, device="cuda")
    series = torch.empty(300, dtype=torch.float64, device="cuda")
    for k in range(350):
        lat.sweep(beta, 1, 2, seed=11)
        O.sweep(U, nc, L, beta, 1, 2, 12, k)
        if k >= 50:
            lat.plaquette(out)
            series[k - 50] = out[0]
            po.append(O.plaquette(U, nc, L)[0])
    pg = to_np(series)
    mg, eg = binned_mean_err(pg)
    mo, eo = binned_mean_err(po)
    print(f"plaquette FP32 GPU {mg:.5f} +- {eg:.5f}, FP64 oracle {mo:.5f} +- {eo:.5f}")
    assert abs(mg - mo) < 4 * np.hypot(eg, eo)


def test_2d_su2_exact_plaquette_on_gpu(gpu):
    """The GPU chain alone against the exact 2D SU(2) torus result."""
    from closed_forms import su2_torus_plaquette
    L, beta = (16, 16, 1, 1), 2.3
    lat = gpu_lattice(gpu, 2, L, "f32", hot=True, seed=5)
    out = torch.empty(3, dtype=torch.float64, device="cuda")
    n = 4000
    series = torch.empty(n, dtype=torch.float64, device="cuda")
    for k in range(100 + n):
        lat.sweep(beta, 1, 3, seed=5)
        if k >= 100:
            lat.plaquette(out)
            series[k - 100] = out[0]
    m, e = binned_mean_err(to_np(series))
    exact = su2_torus_plaquette(beta, 256)
    print(f"2D SU(2) GPU {m:.5f} +- {e:.5f}, exact {exact:.5f}")
    assert abs(m - exact) < 4 * e


@pytest.mark.parametrize("nc,dtype,beta", [(3, "f32r12", 6.0), (3, "f64", 3.0), (4, "f32", 11.1),
                                           (4, "f64w", 11.1), (8, "f32", 44.4)])
def test_2d_sun_one_link_plaquette_on_gpu(gpu, nc, dtype, beta):
    """The GPU chain alone against the exact 2D SU(Nc) result (the
    plaquettes of a 2D lattice are independent up to the torus constraint,
    so the mean of (1/Nc) ReTr P is d ln z / d beta of the one-link
    integral z = sum_k det I_{k+j-i}(beta/Nc)): the register path in FP32
    (two-row and 18 reals) and FP64, and the workgroup-per-link path at
    Nc = 4 and 8."""
    from closed_forms import one_link_plaquette
    L = (32, 32, 1, 1)
    lat = gpu_lattice(gpu, nc, L, dtype, hot=True, seed=7)
    out = torch.empty(3, dtype=torch.float64, device="cuda")
    n = 3000
    series = torch.empty(n, dtype=torch.float64, device="cuda")
    for k in range(200 + n):
        lat.sweep(beta, 1, 3, seed=7)
        if k >= 200:
            lat.plaquette(out)
            series[k - 200] = out[0]
    m, e = binned_mean_err(to_np(series))
    exact = one_link_plaquette(nc, beta)
    record(what=f"2D SU({nc}) beta {beta} plaquette", dtype=dtype, mean=m, err=e, exact=float(exact),
           z=float((m - exact) / e))
    print(f"2D SU({nc}) {dtype} beta {beta}: GPU {m:.5f} +- {e:.5f}, exact {exact:.5f}")
    assert abs(m - exact) < 4 * e


# ---------------------------------------------------------------------------
# Full size, launch configuration of the benchmark (SU(3) 32^4; FP32 two-row
# is the headline, FP32 18-real and FP64 the precision comparison)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["f32", "f32r12", "f64"])
def test_full_size_su3_32_phase_parity(gpu, dtype):
    """Every direction at the benchmark's shape and launch configuration: a
    heatbath phase and an overrelaxation phase for each mu (the heatbath on
    one parity, the overrelaxation on the other), each checked link by link
    from the GPU's own input field (a phase's staples contain links the
    previous phases updated, so an allowed FP32 decision flip would
    otherwise cascade), then the plaquette of the final field."""
    nc, L, beta = 3, (32, 32, 32, 32), 6.2
    lat = gpu_lattice(gpu, nc, L, dtype, hot=True, seed=1234)
    before = to_np(lat.export())
    want = O.new_field(nc, L, hot=True, seed=1234)
    assert np.abs(before - want).max() < 1e-6
    del want
    flips = 0
    for mu in range(4):
        for kind, par in ((0, mu & 1), (1, (mu & 1) ^ 1)):
            lat.phase(kind, mu, par, beta, seed=1234, step=0)
            got = to_np(lat.export())
            m, k = oracle_phase_diag(before, nc, L, kind, mu, par, beta, 1234, 0)
            flips += compare_links(got, before, dtype, m, k, f"32^4 kind {kind} mu {mu} p {par}")
            before = got
    print(f"32^4 flips: {flips}")
    np.testing.assert_allclose(to_np(lat.plaquette()), O.plaquette(before, nc, L), rtol=0, atol=1e-12)


@pytest.mark.parametrize("dtype", ["f32r12", "f64"])
def test_field_past_4_gib_phase_parity(gpu, dtype):
    """A field larger than 4 GiB (SU(3) on 64^3 x 96: 4.8 GB two-row FP32,
    14.5 GB FP64), so that link addresses pass 2^32 bytes: a heatbath and an
    overrelaxation phase of direction 3, whose links lie at the top of the
    field, checked link by link against the oracle, the other directions
    unchanged bit for bit, then the plaquette of the final field."""
    nc, L, beta, seed = 3, (64, 64, 64, 96), 6.2, 4242
    lat = gpu_lattice(gpu, nc, L, dtype, hot=True, seed=seed)
    assert lat.links.numel() * lat.links.element_size() > 2 ** 32
    before = to_np(lat.export())
    for kind, par in ((0, 1), (1, 0)):
        lat.phase(kind, 3, par, beta, seed=seed, step=0)
        got = to_np(lat.export())
        for mu in range(3):
            assert np.array_equal(got[mu], before[mu]), mu
        m, k = oracle_phase_diag(before, nc, L, kind, 3, par, beta, seed, 0)   # before -> the oracle's field
        compare_links(got[3:], before[3:], dtype, m[3:], k[3:], f"64^3x96 kind {kind} mu 3 p {par}")
        del before
        before = got
    np.testing.assert_allclose(to_np(lat.plaquette()), O.plaquette(before, nc, L), rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# Chain state, determinism, timing hooks
# ---------------------------------------------------------------------------
def test_resume_is_bitwise(gpu):
    nc, L = 3, (8, 8, 8, 8)
    a = gpu_lattice(gpu, nc, L, "f32", hot=True, seed=3)
    for _ in range(4):
        a.sweep(6.0, 1, 2, seed=3)
    b = gpu_lattice(gpu, nc, L, "f32", hot=True, seed=3)
    for _ in range(2):
        b.sweep(6.0, 1, 2, seed=3)
    ckpt, step = b.export(), b.step
    c = gpu_lattice(gpu, nc, L, "f32", field=to_np(ckpt))
    c.step = step
    for _ in range(2):
        c.sweep(6.0, 1, 2, seed=3)
    assert torch.equal(a.links, c.links)
    assert a.step == c.step == 4


def test_profile_counts_launches(gpu):
    lat = gpu_lattice(gpu, 3, (8, 8, 8, 8), "f32")
    lat.profile(True)
    lat.sweep(6.0, 1, 4, seed=1)
    lat.plaquette()
    ms_hb, n_hb = lat.profile_read("heatbath")
    ms_or, n_or = lat.profile_read("overrelax")
    assert (n_hb, n_or) == (8, 32) and ms_hb > 0 and ms_or > 0
    assert lat.profile_read("reunit")[1] == 1 and lat.profile_read("plaquette")[1] == 1
    # sampled: launches 0, 5, 10, ... of each kind are timed
    lat.profile(True, every=5)
    lat.sweep(6.0, 1, 4, seed=1)
    lat.sweep(6.0, 1, 4, seed=1)
    assert lat.profile_read("heatbath")[1] == 4 and lat.profile_read("overrelax")[1] == 13
    assert lat.profile_read("reunit")[1] == 1
    lat.profile(False)
    lat.sweep(6.0, 1, 4, seed=1)
    assert lat.profile_read("overrelax")[1] == 0
    # run mode: one event pair per run of back-to-back launches of a kind,
    # counted as that many launches; single phases are runs of one
    lat.profile(True, every=-1)
    lat.sweep(6.0, 1, 4, seed=1)
    lat.sweep(6.0, 2, 1, seed=1)
    lat.phase(1, 0, 0, 6.0, 1, 0)
    ms_or, n_or = lat.profile_read("overrelax")
    assert lat.profile_read("heatbath")[1] == 24 and n_or == 41 and ms_or > 0
    assert lat.profile_read("reunit")[1] == 2
    lat.profile(False)


def test_rejects_bad_arguments(gpu):
    sun = gpu
    with pytest.raises(sun.SunError):
        sun.Lattice(3, (8, 7, 8, 8))
    with pytest.raises(sun.SunError):
        sun.Lattice(33, (8, 8, 8, 8))
    lat = gpu_lattice(sun, 3, (4, 4, 4, 4), "f32")
    with pytest.raises(sun.SunError):
        lat.phase(0, 4, 0, 6.0, 1, 0)
    with pytest.raises(sun.SunError):
        lat.sweep(6.0, -1, 0)


# ---------------------------------------------------------------------------
# Batches of independent chains
# ---------------------------------------------------------------------------
BATCH = [  # (nc, L, dtype, beta, seed)
    (2, (6, 6, 6, 6), "f32", 2.3, 11),
    (3, (8, 8, 8, 8), "f32", 5.9, 12),
    (3, (4, 4, 4, 6), "f64", 6.1, 13),
    (2, (8, 8, 1, 1), "f64", 2.5, 14),
    (4, (4, 4, 4, 4), "f32", 11.1, 15),
    (3, (10, 6, 4, 6), "f32", 5.7, 16),
]


def test_batch_is_bitwise_the_chains_alone(gpu):
    sun = gpu
    alone = [gpu_lattice(sun, nc, L, dt, hot=True, seed=sd) for nc, L, dt, b, sd in BATCH]
    batched = [gpu_lattice(sun, nc, L, dt, hot=True, seed=sd) for nc, L, dt, b, sd in BATCH]
    for lat, (nc, L, dt, beta, sd) in zip(alone, BATCH):
        for _ in range(5):
            lat.sweep(beta, 1, 2, seed=sd)
    bt = sun.Batch(batched, [c[3] for c in BATCH], [c[4] for c in BATCH])
    bt.sweep(1, 2)
    bt.sweep(1, 2)
    plaq = torch.zeros((len(BATCH), 3), dtype=torch.float64, device="cuda")
    bt.capture(n_sweeps=1, n_hb=1, n_or=2, plaq_out=plaq)
    for _ in range(3):       # replays with eager work and synchronisation between them
        bt.replay()
        torch.cuda.synchronize()
        _ = bt.plaquette()
        torch.cuda.synchronize()
    bt.sync()
    for i, (a, b) in enumerate(zip(alone, batched)):
        assert torch.equal(a.links, b.links), f"chain {i} differs"
        assert a.step == b.step == 5
        assert torch.equal(a.plaquette(), plaq[i]), f"plaquette of chain {i}"


def test_batch_couplings_from_a_device_array(gpu):
    """A coupling scan without a new batch: sweeps given a device array of
    couplings, eager and from a graph whose replays read the array's
    contents at that time, equal the chains run alone with those couplings
    (bitwise); sweeps given no array keep the last couplings."""
    sun = gpu
    cfg = BATCH[:3] + BATCH[4:]
    b1 = torch.tensor([c[3] + 0.3 for c in cfg], dtype=torch.float64, device="cuda")
    b2 = torch.tensor([c[3] - 0.2 for c in cfg], dtype=torch.float64, device="cuda")
    alone = [gpu_lattice(sun, nc, L, dt, hot=True, seed=sd) for nc, L, dt, b, sd in cfg]
    batched = [gpu_lattice(sun, nc, L, dt, hot=True, seed=sd) for nc, L, dt, b, sd in cfg]
    for i, (lat, (nc, L, dt, beta, sd)) in enumerate(zip(alone, cfg)):
        lat.sweep(float(b1[i]), 1, 2, seed=sd)          # eager, array b1
        lat.sweep(float(b1[i]), 1, 2, seed=sd)          # no array: b1 stays
        lat.sweep(float(b2[i]), 1, 2, seed=sd)          # graph replay with b2 in the array
        lat.sweep(float(b1[i]), 1, 2, seed=sd)          # same graph, b1 written back
    bt = sun.Batch(batched, [c[3] for c in cfg], [c[4] for c in cfg])
    bt.sweep(1, 2, beta=b1)
    bt.sweep(1, 2)
    arr = b2.clone()
    bt.capture(n_sweeps=1, n_hb=1, n_or=2, beta=arr)
    bt.replay()
    torch.cuda.synchronize()
    arr.copy_(b1)
    torch.cuda.synchronize()
    bt.replay()
    torch.cuda.synchronize()
    bt.sync()
    for i, (a, b) in enumerate(zip(alone, batched)):
        assert torch.equal(a.links, b.links), f"chain {i} differs"


@pytest.mark.parametrize("nc,L,dt", [(3, (6, 4, 2, 4), "f32r12"), (2, (4, 2, 2, 6), "f64")])
def test_one_chain_batch_is_the_chain_alone(gpu, nc, L, dt):
    """The degenerate batch: one chain, ragged extents (V/2 not a multiple
    of the workgroup size)."""
    sun = gpu
    beta, sd = BETA[nc], 4321
    alone = gpu_lattice(sun, nc, L, dt, hot=True, seed=sd)
    batched = gpu_lattice(sun, nc, L, dt, hot=True, seed=sd)
    for _ in range(3):
        alone.sweep(beta, 1, 3, seed=sd)
    bt = sun.Batch([batched], [beta], [sd])
    for _ in range(3):
        bt.sweep(1, 3)
    bt.sync()
    assert torch.equal(alone.links, batched.links)
    assert alone.step == batched.step == 3
    assert torch.equal(alone.plaquette(), bt.plaquette()[0])


def test_batch_eager_and_graph_agree_over_many_replays(gpu):
    sun = gpu
    spec = BATCH[:3]
    a = [gpu_lattice(sun, nc, L, dt, hot=True, seed=sd) for nc, L, dt, b, sd in spec]
    g = [gpu_lattice(sun, nc, L, dt, hot=True, seed=sd) for nc, L, dt, b, sd in spec]
    ba = sun.Batch(a, [c[3] for c in spec], [c[4] for c in spec])
    bg = sun.Batch(g, [c[3] for c in spec], [c[4] for c in spec])
    bg.capture(n_sweeps=2, n_hb=1, n_or=1)
    for _ in range(4):
        ba.sweep(1, 1)
        ba.sweep(1, 1)
        bg.replay()
        torch.cuda.synchronize()
        for x, y in zip(a, g):
            assert torch.equal(x.links, y.links)


# ---------------------------------------------------------------------------
# Launch shapes and the autotuner
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nc,dtype", [(2, "f32"), (3, "f32"), (3, "f64"), (4, "f32")])
def test_every_launch_shape_gives_the_same_bits(gpu, nc, dtype):
    """Every launch shape, including the t-blocked walks (which apply at
    blocks of 64 and 128 on this lattice: an (x, y) plane holds 128
    checkerboard sites), updates every link exactly once per phase."""
    sun = gpu
    L = (16, 16, 4, 8)
    ref = None
    for shape in sun.Lattice.LAUNCH_SHAPES:
        lat = gpu_lattice(sun, nc, L, dtype, hot=True, seed=8)
        lat.set_launch(*shape)
        block, _, _, tb = shape
        eff = shape[:3] + ((tb if tb > 1 and 128 % block == 0 else 0),)
        assert lat.launch == (eff, eff)
        lat.sweep(BETA[nc], 1, 2, seed=8)
        lat.sweep(BETA[nc], 1, 2, seed=8)
        torch.cuda.synchronize()
        if ref is None:
            ref = lat.links.clone()
        else:
            assert torch.equal(ref, lat.links), shape
    # several sites per work-item: a workgroup takes 2 or 4 tiles of its walk
    for shape in [(256, 1, 12, 4), (64, 0, 0, 4), (128, 1, 16, 0)]:
        for spt in (2, 4):
            lat = gpu_lattice(sun, nc, L, dtype, hot=True, seed=8)
            lat.set_launch(*shape)
            lat.set_sites_per_item(spt)
            lat.set_launch(*shape)   # keeps the sites per work-item
            assert lat.get_sites_per_item(0) == lat.get_sites_per_item(1) == spt
            lat.sweep(BETA[nc], 1, 2, seed=8)
            lat.sweep(BETA[nc], 1, 2, seed=8)
            torch.cuda.synchronize()
            assert torch.equal(ref, lat.links), (shape, spt)


@pytest.mark.parametrize("nc,dtype,L", [(3, "f32r12", (16, 16, 4, 8)), (3, "f64", (6, 4, 2, 6)),
                                         (2, "f32", (8, 8, 8, 8)), (4, "f32", (4, 4, 4, 4))])
def test_random_tile_orders_give_the_same_bits(gpu, nc, dtype, L):
    """Race canary: every phase takes its tiles in a random order of its own
    (a random affine permutation of the walk positions), with several
    seeds, launch shapes and sites per work-item; the field after two
    sweeps must equal the default order's bitwise.  A phase whose updates
    depended on one another -- a link read after another workgroup wrote
    it -- would change with the order."""
    sun = gpu
    ref = gpu_lattice(sun, nc, L, dtype, hot=True, seed=8)
    for _ in range(2):
        ref.sweep(BETA[nc], 1, 2, seed=8)
    torch.cuda.synchronize()
    for seed, shape, spt in [(1, (256, 1, 12, 4), 1), (2, (64, 0, 0, 0), 1), (3, (128, 1, 16, 4), 2),
                             (0xDEADBEEF, (256, 1, 0, 0), 4)]:
        lat = gpu_lattice(sun, nc, L, dtype, hot=True, seed=8)
        lat.set_launch(*shape)
        lat.set_sites_per_item(spt)
        lat.set_tile_order(seed)
        for _ in range(2):
            lat.sweep(BETA[nc], 1, 2, seed=8)
        torch.cuda.synchronize()
        assert torch.equal(ref.links, lat.links), (seed, shape, spt)
    lat.set_tile_order(0)


def test_batch_launch_shapes_and_tuner(gpu, tmp_path, monkeypatch):
    sun = gpu
    from paper_1112_4533_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    spec = BATCH
    ref = [gpu_lattice(sun, nc, L, dt, hot=True, seed=sd) for nc, L, dt, b, sd in spec]
    rb = sun.Batch(ref, [c[3] for c in spec], [c[4] for c in spec])
    rb.sweep(1, 2)
    rb.sweep(1, 2)
    for hb, orx, spt in [((64, 0, 0), (128, 1, 12), (1, 1)), ((256, 1, 16), (64, 1, 8), (2, 4)),
                         ((128, 0, 8), (256, 0, 0), (4, 2))]:
        shape = (hb, orx, spt)
        lats = [gpu_lattice(sun, nc, L, dt, hot=True, seed=sd) for nc, L, dt, b, sd in spec]
        bt = sun.Batch(lats, [c[3] for c in spec], [c[4] for c in spec])
        bt.set_launch(*hb, kind=0)
        bt.set_launch(*orx, kind=1)
        bt.set_sites_per_item(spt[0], kind=0)
        bt.set_sites_per_item(spt[1], kind=1)
        bt.sweep(1, 2)
        bt.capture(n_sweeps=1, n_hb=1, n_or=2)
        bt.replay()
        torch.cuda.synchronize()
        for a, b in zip(ref, lats):
            assert torch.equal(a.links, b.links), shape
    # the tuner works on clones: the chains' fields are unchanged by tuning
    before = [l.links.clone() for l in ref]
    best, times = autotune.tune_batch(rb, reps=1)
    assert all(best[k] in sun.Batch.LAUNCH_SHAPES for k in (0, 1))
    assert len(times["heatbath"]) == len(times["overrelax"]) == len(sun.Batch.LAUNCH_SHAPES)
    for a, b in zip(before, ref):
        assert torch.equal(a, b.links)
    lat = ref[1]
    before = lat.links.clone()
    best, times = autotune.tune_lattice(lat, reps=1)
    assert lat.launch == (best[0], best[1])
    assert all(lat.get_sites_per_item(k) in sun.Lattice.SITES_PER_ITEM for k in (0, 1))
    assert len(times["overrelax_sites_per_item"]) == len(sun.Lattice.SITES_PER_ITEM)
    assert all(tuple(map(int, k.split("/"))) in sun.Lattice.LAUNCH_SHAPES for k in times["overrelax"])
    assert torch.equal(before, lat.links)
    # a second call comes from the cache
    assert autotune.tune_lattice(lat)[0] == best
