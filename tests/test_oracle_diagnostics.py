"""Oracle pins for the diagnostics the GPU comparison rests on.

* the plaquette's split into planes without and with direction 3 (paper
  Sec. 2, plaquette), against per-plane plaquette maps computed in numpy;
* the unitarity deviation max_ij |(U^dag U - 1)_ij| and max |det U - 1|,
  against numpy on fields that are deliberately not unitary;
* the decision margin of the SU(2) draw (paper Sec. 2, SU(2) heatbath: the
  Creutz / Kennedy-Pendleton switch and each accept test), recomputed by
  brute force in numpy from the pinned Philox words;
* the per-link decision margin and conditioning |A|_F / k_min of a heatbath
  phase, recomputed in numpy from the pinned staple, the subgroup projection
  of the Cabibbo-Marinari step and the brute-force draw.
"""
import numpy as np
import pytest

import oracle as O
from lattice_np import plaquette_map

SWITCH = 1.7
CAP = 64


# ---------------------------------------------------------------------------
# Plaquette split
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nc", [2, 3, 4])
@pytest.mark.parametrize("L", [(4, 6, 2, 8), (4, 6, 1, 8), (4, 6, 2, 1), (2, 1, 1, 6)])
def test_plaquette_split_against_numpy(nc, L):
    """out = {all planes, planes without direction 3, planes with it}, each
    the mean of ReTr P / Nc over the present planes of its class."""
    U = O.new_field(nc, L, hot=True, seed=7 + nc)
    present = [m for m in range(4) if L[m] > 1]
    V = O.volume(L)
    spatial, temporal = [], []
    for a in present:
        for b in present:
            if a < b:
                (temporal if b == 3 else spatial).append(plaquette_map(U, L, a, b).sum())
    want_sp = sum(spatial) / (nc * V * len(spatial)) if spatial else 0.0
    want_tm = sum(temporal) / (nc * V * len(temporal)) if temporal else 0.0
    n = len(spatial) + len(temporal)
    want_all = (sum(spatial) + sum(temporal)) / (nc * V * n) if n else 0.0
    got = O.plaquette(U, nc, L)
    np.testing.assert_allclose(got, [want_all, want_sp, want_tm], rtol=0, atol=1e-14)
    # a hot field's two classes differ well beyond that tolerance, so a
    # swapped or misclassified plane would show
    if spatial and temporal:
        assert abs(want_sp - want_tm) > 1e-4


def test_plaquette_split_sees_one_changed_plane():
    """Multiplying the time links of one time slice by a centre-free phase
    changes only the temporal planes that contain them."""
    nc, L = 3, (4, 4, 4, 6)
    U = O.new_field(nc, L, hot=True, seed=3)
    before = O.plaquette(U, nc, L)
    W = U.copy()
    G = W.reshape(4, L[3], L[2], L[1], L[0], nc, nc)
    G[3, 2] = G[3, 2] @ np.diag(np.exp(1j * np.array([0.3, -0.1, -0.2])))
    after = O.plaquette(W, nc, L)
    assert after[1] == before[1]                       # spatial planes untouched
    assert abs(after[2] - before[2]) > 1e-6            # temporal planes moved


# ---------------------------------------------------------------------------
# Unitarity deviation
# ---------------------------------------------------------------------------
def numpy_unitarity(U):
    nc = U.shape[-1]
    M = np.conj(np.swapaxes(U, -1, -2)) @ U - np.eye(nc)
    return np.abs(M).max(), np.abs(np.linalg.det(U) - 1).max()


@pytest.mark.parametrize("nc", [2, 3, 4, 6])
def test_unitarity_against_numpy_on_non_unitary_fields(nc):
    L = (4, 2, 2, 4)
    rng = np.random.default_rng(40 + nc)
    U = O.new_field(nc, L, hot=True, seed=nc)
    # non-normal perturbations: U^dag U and U U^dag differ, so the order of
    # the product is tested too
    X = U + 0.05 * (rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape))
    got = O.unitarity(X, nc, L)
    want = numpy_unitarity(X)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=0)
    other = np.abs(X @ np.conj(np.swapaxes(X, -1, -2)) - np.eye(nc)).max()
    assert abs(other - want[0]) > 1e-3 * want[0]


@pytest.mark.parametrize("nc", [2, 3, 5])
def test_unitarity_of_scaled_identity_and_one_bad_link(nc):
    """Deviation on the diagonal only (U = (1 + e) 1): max |U^dag U - 1| =
    (1 + e)^2 - 1 and |det - 1| = (1 + e)^Nc - 1; and a single bad link
    among unitary ones sets the maximum."""
    L = (2, 2, 2, 2)
    e = 1e-3
    U = O.new_field(nc, L)
    U *= 1 + e
    got = O.unitarity(U, nc, L)
    np.testing.assert_allclose(got, [(1 + e) ** 2 - 1, (1 + e) ** nc - 1], rtol=1e-10)
    U = O.new_field(nc, L, hot=True, seed=5)
    M = np.eye(nc, dtype=np.complex128)
    M[0, nc - 1] = 0.02j                    # (U^dag U - 1) has 0.02 off the diagonal
    U[2, 9] = U[2, 9] @ M
    got = O.unitarity(U, nc, L)
    np.testing.assert_allclose(got, numpy_unitarity(U), rtol=1e-10, atol=1e-15)
    assert got[0] > 0.019


# ---------------------------------------------------------------------------
# Decision margin of the SU(2) draw, by brute force
# ---------------------------------------------------------------------------
def uniforms(seed, site, step, mu_sg, word3):
    w = O.philox((site, step, mu_sg, word3), (seed & 0xFFFFFFFF, seed >> 32))
    return [((x >> 8) + 1) * 2.0 ** -24 for x in w]


def brute_draw(alpha, seed, site, step, mu_sg):
    """The hybrid draw written out: returns (x0, attempts, margin), with the
    margin the smallest |alpha - 1.7| and |r^2 - (1 - x0^2)| (Creutz) or
    |r^2 - (1 - lambda^2)| (Kennedy-Pendleton) over the attempts taken."""
    m = abs(alpha - SWITCH)
    for hit in range(CAP):
        r = uniforms(seed, site, step, mu_sg, hit)
        if alpha < SWITCH:
            x0 = 2 * r[0] - 1 if alpha == 0 else 1 + np.log1p((1 - r[0]) * np.expm1(-2 * alpha)) / alpha
            lhs, rhs = r[1] ** 2, 1 - x0 * x0
        else:
            lam2 = -(np.log(r[0]) + np.cos(2 * np.pi * r[1]) ** 2 * np.log(r[2])) / (2 * alpha)
            lhs, rhs = r[3] ** 2, 1 - lam2
            x0 = 1 - 2 * lam2
        m = min(m, abs(lhs - rhs))
        if lhs <= rhs:
            return x0, hit + 1, m
    return 1.0, 0, m


def test_sampler_margin_brute_force():
    alpha = np.array([0.0, 0.02, 0.3, 1.0, 1.6999, 1.7, 1.7001, 2.5, 8.0, 50.0, 0.7, 3.3])
    seed, step, mu_sg = 2024, 9, (3 << 16) | 2
    x, att, margin = O.sample_su2(alpha, seed=seed, step=step, mu_sg=mu_sg)
    for i, a in enumerate(alpha):
        x0, n, m = brute_draw(float(a), seed, i, step, mu_sg)
        assert att[i] == n, (a, att[i], n)
        assert abs(x[i, 0] - x0) < 1e-13, (a, x[i, 0], x0)
        assert abs(margin[i] - m) <= 1e-14 * max(1.0, m), (a, margin[i], m)
    # at alpha = 1.7 +- 1e-4 the switch itself is the closest decision
    assert margin[4] <= 1.0000001e-4 and margin[6] <= 1.0000001e-4 and margin[5] == 0.0


def test_sampler_margin_over_many_draws():
    """Across 2000 draws the oracle's margin and attempt count equal the brute
    force, including rejected attempts (the margin looks at every attempt up
    to the accepted one)."""
    rng = np.random.default_rng(5)
    alpha = np.concatenate([rng.uniform(0, 3.5, 1000), rng.uniform(3.5, 40, 1000)])
    x, att, margin = O.sample_su2(alpha, seed=77, step=1, mu_sg=1)
    rejected_somewhere = 0
    for i, a in enumerate(alpha):
        x0, n, m = brute_draw(float(a), 77, i, 1, 1)
        assert att[i] == n and abs(margin[i] - m) <= 1e-14 * max(1.0, m) and abs(x[i, 0] - x0) < 1e-13
        rejected_somewhere += n > 1
    assert rejected_somewhere > 100


# ---------------------------------------------------------------------------
# Per-link margin and conditioning of a heatbath phase
# ---------------------------------------------------------------------------
def su2_matrix(x):
    return np.array([[x[0] + 1j * x[3], x[2] + 1j * x[1]], [-x[2] + 1j * x[1], x[0] - 1j * x[3]]])


def brute_direction(seed, site, step, mu_sg):
    u = uniforms(seed, site, step, mu_sg, 1 << 24)
    cos_t = 1 - 2 * u[0]
    return cos_t, np.sqrt(1 - cos_t * cos_t), 2 * np.pi * u[1]


def brute_heatbath_link(U, nc, L, s, mu, beta, seed, step):
    """Cabibbo-Marinari step written out in numpy from the (pinned) staple:
    returns (new link, margin, |A|_F / k_min)."""
    A = O.staple(U, nc, L, s, mu)
    Ul = U[mu, s].copy()
    W = Ul @ A
    margin, kmin, sg = np.inf, np.inf, 0
    for i in range(nc):
        for j in range(i + 1, nc):
            w = W[np.ix_([i, j], [i, j])]
            P = 0.5 * (w + np.array([[np.conj(w[1, 1]), -np.conj(w[1, 0])], [-np.conj(w[0, 1]), np.conj(w[0, 0])]]))
            k = np.sqrt(max(np.linalg.det(P).real, 0.0))
            kmin = min(kmin, k)
            Vm = P / k if k > 0 else np.eye(2)
            mu_sg = (mu << 16) | sg
            x0, n, m = brute_draw(2 * beta * k / nc, seed, s, step, mu_sg)
            margin = min(margin, m)
            sg += 1
            if n == 0:
                continue
            cos_t, sin_t, phi = brute_direction(seed, s, step, mu_sg)
            if 2 * beta * k / nc < SWITCH:
                rad = np.sqrt(1 - x0 * x0)
            else:
                lam2 = (1 - x0) / 2
                rad = 2 * np.sqrt(lam2) * np.sqrt(1 - lam2)
            X = su2_matrix([x0, rad * sin_t * np.cos(phi), rad * sin_t * np.sin(phi), rad * cos_t])
            a = X @ np.conj(Vm.T)
            for M in (Ul, W):
                M[[i, j], :] = a @ M[[i, j], :]
    return Ul, margin, np.linalg.norm(A) / kmin


@pytest.mark.parametrize("nc,beta", [(2, 2.3), (3, 6.0), (3, 0.9), (4, 11.1)])
def test_phase_margin_and_conditioning_brute_force(nc, beta):
    L, mu, par, seed, step = (4, 4, 2, 4), 1, 1, 31, 4
    U = O.new_field(nc, L, hot=True, seed=60 + nc)
    for k in range(2):
        O.sweep(U, nc, L, beta, 1, 1, 61, k)
    before = U.copy()
    margin, _, cond = O.phase(U, nc, L, 0, mu, par, beta, seed, step, want_margin=True)
    coords = [(s % 4, (s // 4) % 4, (s // 16) % 2, s // 32) for s in range(O.volume(L))]
    odd = [s for s, c in enumerate(coords) if sum(c) % 2 == par]
    assert np.all(margin[[s for s in range(O.volume(L)) if s not in odd]] == -1)
    for s in odd[::5]:
        Ul, m, c = brute_heatbath_link(before, nc, L, s, mu, beta, seed, step)
        assert abs(margin[s] - m) <= 1e-12 * max(1.0, m), (s, margin[s], m)
        assert abs(cond[s] - c) <= 1e-10 * c, (s, cond[s], c)
        assert np.abs(U[mu, s] - Ul).max() < 1e-12, s
