"""GPU parity of the large-Nc path (one workgroup per link, link-major
storage) against the FP64 oracle, for 4 <= Nc <= 32.

The tolerances are those of test_gpu_parity (K_LINK eps (1 + c) per link,
FP32 decision flips inside K_FLIP eps (1 + c) counted), widened where the
oracle itself is sensitive: one link update is a chain of Nc (Nc - 1) / 2
subgroup steps (496 at Nc = 32), each dividing by its own k, so rounding
compounds along the chain.  The oracle's phase is run three more times with
its input perturbed at the storage precision's rounding level (1e-7 FP32,
1e-15 FP64), and a link may differ by up to SPREAD_FACTOR times the largest
change those perturbations make to it (10 in FP64, 100 in FP32: the FP32
arithmetic along the chain adds rounding at every step, which an input
perturbation does not model)."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_common import (EPS, K_FLIP, K_TYP, TOL, beta_for, compare_links, gpu_lattice, oracle_phase_diag,
                        record, rounded, thermal_field, to_np, twin_spread)

pytestmark = pytest.mark.gpu

SMALL = (4, 4, 2, 2)      # V/2 = 32 links per phase
REL = {"f32": 1e-7, "f64": 1e-15}   # input perturbation of the oracle twin


@pytest.mark.parametrize("nc,dtype", [(4, "f64w"), (4, "f32w"), (5, "f32"), (9, "f64"), (9, "f32"), (16, "f64"),
                                      (16, "f32"), (28, "f64"), (32, "f64"), (32, "f32")])
def test_wide_hot_start_parity(gpu, nc, dtype):
    L = (4, 2, 2, 2)
    lat = gpu_lattice(gpu, nc, L, dtype, hot=True, seed=1234)
    got = to_np(lat.export())
    want = O.new_field(nc, L, hot=True, seed=1234)
    # Gram-Schmidt of an Nc x Nc Gaussian matrix: rounding ~ cond(M) eps
    tol = 1e-11 if dtype.startswith("f64") else 1e-6
    assert np.abs(got - want).max() < tol


@pytest.mark.parametrize("nc", [4, 10])
def test_wide_cold_start_exact(gpu, nc):
    lat = gpu_lattice(gpu, nc, (4, 4, 2, 2), "f32w", hot=False)
    assert np.array_equal(to_np(lat.plaquette()), [1.0, 1.0, 1.0])
    assert np.array_equal(to_np(lat.polyakov()), [1.0, 0.0])
    assert np.array_equal(to_np(lat.unitarity()), [0.0, 0.0])


@pytest.mark.parametrize("nc,dtype", [(5, "f64w"), (12, "f32"), (12, "f64")])
def test_wide_roundtrip(gpu, nc, dtype):
    L = (4, 2, 2, 2)
    U = O.new_field(nc, L, hot=True, seed=5)
    lat = gpu_lattice(gpu, nc, L, dtype, field=U)
    assert np.array_equal(to_np(lat.export()), rounded(U, dtype))


@pytest.mark.parametrize("nc,dtype", [(4, "f64w"), (9, "f64"), (9, "f32"), (13, "f64"), (16, "f64"), (32, "f32")])
def test_wide_observables_parity(gpu, nc, dtype):
    L = (4, 2, 2, 4)
    lat = gpu_lattice(gpu, nc, L, dtype, field=thermal_field(nc, L, beta_for(nc), sweeps=1))
    U = to_np(lat.export())
    np.testing.assert_allclose(to_np(lat.plaquette()), O.plaquette(U, nc, L), rtol=1e-13, atol=1e-15)
    pg = to_np(lat.polyakov())
    assert abs(complex(pg[0], pg[1]) - O.polyakov(U, nc, L)) < 1e-13
    np.testing.assert_allclose(to_np(lat.unitarity()), O.unitarity(U, nc, L), rtol=1e-6, atol=1e-14)


@pytest.mark.parametrize("nc,noise,tol", [(4, 1e-3, 1e-12), (9, 1e-3, 1e-12), (16, 1e-3, 1e-12), (32, 1e-3, 1e-12),
                                          (9, 1.0, 1e-10), (16, 1.0, 1e-10), (32, 1.0, 1e-10)])
def test_wide_reunitarize_parity(gpu, nc, noise, tol):
    """Near-unitary links (noise 1e-3: one Gram-Schmidt pass per row) and
    general ones (noise 1: the later rows lose more than half their norm to
    the projection and take the second pass); the latter agree with the
    oracle to the conditioning of a random matrix times the unit roundoff."""
    L = (4, 2, 2, 2)
    rng = np.random.default_rng(nc)
    U = O.new_field(nc, L, hot=True, seed=9)
    U = U + noise * (rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape))
    lat = gpu_lattice(gpu, nc, L, "f64" if nc > 8 else "f64w", field=U)
    before = to_np(lat.reunitarize(report=True))
    after = to_np(lat.export())
    np.testing.assert_allclose(before, O.unitarity(U, nc, L), rtol=1e-10)
    O.reunitarize(U, nc, L)
    assert np.abs(after - U).max() < tol
    assert to_np(lat.unitarity()).max() < 1e-13


PHASES = [(0, 0, 0), (0, 3, 1), (1, 1, 1), (1, 2, 0)]   # (kind, mu, parity)


@pytest.mark.parametrize("nc,dtype", [(4, "f64w"), (4, "f32w"), (5, "f64w"), (9, "f64"), (9, "f32"),
                                      (16, "f64"), (16, "f32"), (24, "f64"), (32, "f64"), (32, "f32"),
                                      (21, "f32"), (27, "f32"),    # matrix-core products on ragged tiles
                                      (30, "f32")])                # with the staple sum in registers
def test_wide_phase_parity(gpu, nc, dtype):
    beta = beta_for(nc)
    base = thermal_field(nc, SMALL, beta, sweeps=1) if nc <= 16 else O.new_field(nc, SMALL, hot=True, seed=21)
    lat = gpu_lattice(gpu, nc, SMALL, dtype, field=base)
    flips = 0
    for kind, mu, par in PHASES:
        before = to_np(lat.export())               # the GPU's own input field
        lat.phase(kind, mu, par, beta, seed=77, step=3)
        got = to_np(lat.export())
        sp = twin_spread(before, nc, SMALL, kind, mu, par, beta, 77, 3, rel=REL[dtype[:3]])
        want = before.copy()
        m, k = oracle_phase_diag(want, nc, SMALL, kind, mu, par, beta, 77, 3)
        dec = (np.prod(SMALL) // 2) * nc * (nc - 1) // 2 if kind == 0 else None
        flips += compare_links(got, want, dtype, m, k, f"nc={nc} {dtype} kind={kind} mu={mu} p={par}", spread=sp,
                               decisions=dec)
    print(f"flips: {flips}")


def test_wide_su32_8x4_phase_parity(gpu):
    """The paper's largest single-precision case: SU(32) on 8^4."""
    nc, L, beta = 32, (8, 8, 8, 8), 6.2
    lat = gpu_lattice(gpu, nc, L, "f32", hot=True, seed=1234)
    base = to_np(lat.export())
    lat.phase(0, 1, 0, beta, seed=1234, step=0)
    got = to_np(lat.export())
    sp = twin_spread(base, nc, L, 0, 1, 0, beta, 1234, 0, rel=REL["f32"])
    m, k = oracle_phase_diag(base, nc, L, 0, 1, 0, beta, 1234, 0)
    flips = compare_links(got, base, "f32", m, k, "SU(32) 8^4 heatbath", spread=sp,
                          decisions=(8 ** 4 // 2) * nc * (nc - 1) // 2)
    print(f"flips: {flips}")


@pytest.mark.parametrize("dtype", ["f64w", "f32w"])
def test_wide_batched_sampler_parity(gpu, dtype):
    """The large-Nc draw, batched over eight subgroups with the fall-back to
    attempts 8..63, against the oracle's sequential sampler on the same
    counters (element i: subgroup mu_sg + i mod 8 of site i / 8).  Near
    alpha = 1.7, the hybrid's lowest acceptance, some draws need more than
    eight attempts on either side of the switch and so take the fall-back."""
    sun = gpu
    alpha = np.concatenate([np.zeros(64), np.linspace(0.01, 60.0, 40000), np.full(160000, 1.7),
                            np.full(160000, 1.69)])
    mu_sg = (2 << 16) | 8
    xg, ag = sun.sample_su2(torch.from_numpy(alpha).cuda(), seed=31, step=5, mu_sg=mu_sg, dtype=dtype)
    xg, ag = to_np(xg), to_np(ag)
    xo, ao, margin = np.zeros((alpha.size, 4)), np.zeros(alpha.size, dtype=np.int32), np.zeros(alpha.size)
    for s in range(8):
        xo[s::8], ao[s::8], margin[s::8] = O.sample_su2(alpha[s::8], seed=31, step=5, mu_sg=mu_sg + s)
    assert (ao[alpha == 1.7] > 8).sum() > 0 and (ao[alpha == 1.69] > 8).sum() > 0
    d = np.abs(xg - xo).max(axis=1)
    bad = (d > TOL[dtype]) | (ag != ao)
    ok = ~bad
    record(what="batched sampler", dtype=dtype, links=int(d.size), max_dU=float(d[ok].max()),
           max_dU_over_tol=float(d[ok].max() / TOL[dtype]), flips=int(bad.sum()),
           flip_margins=[float(m) for m in margin[bad][:50]])
    if dtype == "f64w":
        assert not bad.any(), (d.max(), int((ag != ao).sum()))
    else:
        # as check_draw_flips of the register-path sampler test
        eps = EPS["f32"]
        assert np.all(margin[bad] < K_FLIP * eps * (1.0 + alpha[bad]))
        expected = float((2 * 2 * K_TYP * eps * (1.0 + alpha)).sum())
        assert bad.sum() <= max(3.0, 3.0 * expected), (int(bad.sum()), expected)


@pytest.mark.parametrize("nc", [4])
def test_wide_agrees_with_register_path(gpu, nc):
    """The two implementations of SU(4) draw the same random numbers: a
    heatbath and an overrelaxation phase agree to FP64 rounding."""
    L = (4, 4, 2, 2)
    U = thermal_field(nc, L, beta_for(nc), sweeps=1)
    a = gpu_lattice(gpu, nc, L, "f64", field=U)
    b = gpu_lattice(gpu, nc, L, "f64w", field=U)
    for lat in (a, b):
        lat.phase(0, 2, 1, beta_for(nc), seed=5, step=1)
        lat.phase(1, 0, 0, beta_for(nc), seed=5, step=1)
    assert np.abs(to_np(a.export()) - to_np(b.export())).max() < 1e-11
    np.testing.assert_allclose(to_np(a.plaquette()), to_np(b.plaquette()), rtol=1e-13)


def test_wide_sweep_is_its_phase_sequence(gpu):
    nc, L = 10, (4, 4, 2, 2)
    beta = beta_for(nc)
    a = gpu_lattice(gpu, nc, L, "f32", hot=True, seed=4)
    b = gpu_lattice(gpu, nc, L, "f32", hot=True, seed=4)
    a.sweep(beta, 1, 2, seed=4)
    for kind, steps in ((0, 1), (1, 2)):
        for _ in range(steps):
            for mu in range(4):
                for par in range(2):
                    b.phase(kind, mu, par, beta, seed=4, step=0)
    b.reunitarize()
    assert torch.equal(a.links, b.links)
    assert a.step == 1


@pytest.mark.parametrize("nc,dtype", [(9, "f32"), (16, "f32"), (20, "f32"), (12, "f64"), (26, "f64"), (32, "f64"),
                                      (24, "f32")])
def test_wide_one_or_two_wavefronts_give_the_same_bits(gpu, nc, dtype):
    """A link's update on one wavefront (launch block 64), on two (block
    128: loads and vector-unit products shared by row groups) and with the
    default choice give the same field bit for bit, heatbath and
    overrelaxation (at Nc = 24 in FP32 the matrix-core products stay on the
    first wavefront and the second shares the loads)."""
    sun = gpu
    L, beta = (4, 4, 2, 2), beta_for(nc)
    base = O.new_field(nc, L, hot=True, seed=41)
    fields = []
    for block in (64, 128, 256):
        lat = gpu_lattice(sun, nc, L, dtype, field=base)
        lat.set_launch(block)
        for kind, mu, par in [(0, 1, 0), (1, 2, 1), (0, 3, 1), (1, 0, 0)]:
            lat.phase(kind, mu, par, beta, seed=5, step=3)
        torch.cuda.synchronize()
        fields.append(lat.links.clone())
    assert torch.equal(fields[0], fields[1])
    assert torch.equal(fields[0], fields[2])


def test_wide_field_past_4_gib_phase_parity(gpu):
    """The workgroup-per-link path on a field larger than 4 GiB (SU(8) FP64
    on 32^3 x 34: 4.6 GB), so that link addresses pass 2^32 bytes: a heatbath
    phase of direction 3 (the top of the field) link by link against the
    oracle, the other directions unchanged bit for bit."""
    nc, L, dtype, seed = 8, (32, 32, 32, 34), "f64", 99
    beta = beta_for(nc)
    lat = gpu_lattice(gpu, nc, L, dtype, hot=True, seed=seed)
    assert lat.links.numel() * lat.links.element_size() > 2 ** 32
    before = to_np(lat.export())
    lat.phase(0, 3, 1, beta, seed=seed, step=0)
    got = to_np(lat.export())
    for mu in range(3):
        assert np.array_equal(got[mu], before[mu]), mu
    sp = twin_spread(before, nc, L, 0, 3, 1, beta, seed, 0, rel=REL["f64"], twins=1)
    m, k = oracle_phase_diag(before, nc, L, 0, 3, 1, beta, seed, 0)
    compare_links(got[3:], before[3:], dtype, m[3:], k[3:], "SU(8) 32^3x34 kind 0 mu 3 p 1", spread=sp[3:])


WIDE_BATCH = [  # (nc, L, dtype, beta, seed)
    (5, (4, 4, 2, 2), "f32", beta_for(5), 21),
    (5, (4, 2, 4, 2), "f32", beta_for(5) + 0.7, 22),    # same group, other extents and coupling
    (8, (4, 4, 2, 2), "f64", beta_for(8), 23),
    (4, (4, 4, 2, 2), "f32w", 11.1, 24),                # SU(4) on the workgroup-per-link path
    (3, (4, 4, 4, 4), "f32", 6.0, 25),                  # a register-path chain in the same batch
    (6, (4, 4, 1, 4), "f64", beta_for(6), 26),          # 3D: an absent direction
    (24, (4, 2, 2, 2), "f32", beta_for(24), 27),        # matrix-core products
    (22, (2, 2, 4, 2), "f64", beta_for(22), 28),        # staple sum in registers
    (12, (4, 2, 2, 4), "f32", beta_for(12), 29),        # two wavefronts per link
    (26, (2, 2, 2, 4), "f64", beta_for(26), 30),        # two wavefronts for the overrelaxation
]


def test_wide_chains_in_a_batch_are_bitwise_the_chains_alone(gpu):
    """Large-Nc chains join a batch (one launch per phase for each Nc and
    precision): two eager sweeps, then a captured sweep replayed three times
    with eager work between the replays, give bitwise the fields and
    plaquettes of the chains swept alone, and the step counters advance
    alike."""
    sun = gpu
    alone = [gpu_lattice(sun, nc, L, dt, hot=True, seed=sd) for nc, L, dt, b, sd in WIDE_BATCH]
    batched = [gpu_lattice(sun, nc, L, dt, hot=True, seed=sd) for nc, L, dt, b, sd in WIDE_BATCH]
    for lat, (nc, L, dt, beta, sd) in zip(alone, WIDE_BATCH):
        for _ in range(5):
            lat.sweep(beta, 1, 2, seed=sd)
    bt = sun.Batch(batched, [c[3] for c in WIDE_BATCH], [c[4] for c in WIDE_BATCH])
    bt.sweep(1, 2)
    bt.sweep(1, 2)
    plaq = torch.zeros((len(WIDE_BATCH), 3), dtype=torch.float64, device="cuda")
    bt.capture(n_sweeps=1, n_hb=1, n_or=2, plaq_out=plaq)
    for _ in range(3):
        bt.replay()
        torch.cuda.synchronize()
        _ = bt.plaquette()
        torch.cuda.synchronize()
    bt.sync()
    for i, (a, b) in enumerate(zip(alone, batched)):
        assert torch.equal(a.links, b.links), f"chain {i} {WIDE_BATCH[i][:3]} differs"
        assert a.step == b.step == 5
        assert torch.equal(a.plaquette(), plaq[i]), f"plaquette of chain {i}"
        assert torch.equal(a.plaquette(), bt.plaquette()[i]), f"eager batch plaquette of chain {i}"
    # the batch's launch block reaches its large-Nc groups too (64: one
    # wavefront per link, 128: two), with the same bits
    for block in (64, 128):
        again = [gpu_lattice(sun, nc, L, dt, hot=True, seed=sd) for nc, L, dt, b, sd in WIDE_BATCH]
        bb = sun.Batch(again, [c[3] for c in WIDE_BATCH], [c[4] for c in WIDE_BATCH])
        bb.set_launch(block)
        for _ in range(5):
            bb.sweep(1, 2)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(zip(alone, again)):
            assert torch.equal(a.links, b.links), f"block {block}: chain {i} {WIDE_BATCH[i][:3]} differs"


def test_wide_batch_couplings_from_a_device_array(gpu):
    """As the register path's coupling-array test, for a batch of large-Nc
    chains: a graph replay reads the coupling array's contents at that
    time."""
    sun = gpu
    cfg = WIDE_BATCH[:4]
    b1 = torch.tensor([c[3] + 0.3 for c in cfg], dtype=torch.float64, device="cuda")
    b2 = torch.tensor([c[3] - 0.2 for c in cfg], dtype=torch.float64, device="cuda")
    alone = [gpu_lattice(sun, nc, L, dt, hot=True, seed=sd) for nc, L, dt, b, sd in cfg]
    batched = [gpu_lattice(sun, nc, L, dt, hot=True, seed=sd) for nc, L, dt, b, sd in cfg]
    for i, (lat, (nc, L, dt, beta, sd)) in enumerate(zip(alone, cfg)):
        for bb in (b1, b2, b1):
            lat.sweep(float(bb[i]), 1, 1, seed=sd)
    bt = sun.Batch(batched, [c[3] for c in cfg], [c[4] for c in cfg])
    bt.sweep(1, 1, beta=b1)
    arr = b2.clone()
    bt.capture(n_sweeps=1, n_hb=1, n_or=1, beta=arr)
    bt.replay()
    torch.cuda.synchronize()
    arr.copy_(b1)
    torch.cuda.synchronize()
    bt.replay()
    torch.cuda.synchronize()
    bt.sync()
    for i, (a, b) in enumerate(zip(alone, batched)):
        assert torch.equal(a.links, b.links), f"chain {i} differs"


@pytest.mark.parametrize("nc,dtype,L", [(5, "f64", (4, 4, 1, 4)), (9, "f32", (4, 2, 4, 1)), (6, "f64", (4, 1, 4, 1))])
def test_wide_absent_direction(gpu, nc, dtype, L):
    """3D and 2D lattices: links of an absent direction stay the identity,
    the staple has 2(d-1) terms, and the observables normalise over the
    planes that exist."""
    beta = beta_for(nc)
    base = O.new_field(nc, L, hot=True, seed=31)
    lat = gpu_lattice(gpu, nc, L, dtype, field=base)
    for kind, mu, par in [(0, 0, 1), (1, 1, 0), (0, 3 if L[3] > 1 else 2, 0)]:
        before = to_np(lat.export())
        lat.phase(kind, mu, par, beta, seed=3, step=2)
        got = to_np(lat.export())
        sp = twin_spread(before, nc, L, kind, mu, par, beta, 3, 2, rel=REL[dtype[:3]])
        want = before.copy()
        m, k = oracle_phase_diag(want, nc, L, kind, mu, par, beta, 3, 2)
        compare_links(got, want, dtype, m, k, f"3D nc={nc} kind={kind} mu={mu}", spread=sp)
    U = to_np(lat.export())
    absent = [d for d in range(4) if L[d] == 1][0]
    assert np.array_equal(U[absent], np.broadcast_to(np.eye(nc), U[absent].shape))
    np.testing.assert_allclose(to_np(lat.plaquette()), O.plaquette(U, nc, L), rtol=1e-13, atol=1e-15)
    pg = to_np(lat.polyakov())
    assert abs(complex(pg[0], pg[1]) - O.polyakov(U, nc, L)) < 1e-13


@pytest.mark.parametrize("nc,dtype", [(4, "f64"), (4, "f64w"), (6, "f64"), (12, "f64"), (32, "f64")])
def test_wide_permutation_links_need_pivoting(gpu, nc, dtype):
    """Links that are permutation matrices times phases: every column of the
    LU elimination has a single nonzero below the pivot row, so the
    determinant depends on the row exchanges (and on the first largest pivot
    among zeros).  Re-unitarization and the unitarity report must match the
    oracle (SU(4) also on the register path, whose determinant pivots the
    same way)."""
    L = (4, 2, 2, 2)
    rng = np.random.default_rng(nc)
    V = int(np.prod(L))
    U = np.zeros((4, V, nc, nc), dtype=np.complex128)
    for mu in range(4):
        for s in range(V):
            perm = rng.permutation(nc)
            U[mu, s, np.arange(nc), perm] = np.exp(1j * rng.uniform(-np.pi, np.pi, nc))
    lat = gpu_lattice(gpu, nc, L, dtype, field=U)
    np.testing.assert_allclose(to_np(lat.unitarity()), O.unitarity(U, nc, L), rtol=1e-10, atol=1e-14)
    lat.reunitarize()
    O.reunitarize(U, nc, L)
    assert np.abs(to_np(lat.export()) - U).max() < 1e-13
    assert to_np(lat.unitarity()).max() < 1e-13
