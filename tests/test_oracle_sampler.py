"""Oracle pins: the SU(2) heatbath draw (paper Sec. 2, SU(2) heatbath).

x0 must have density sqrt(1 - x0^2) exp(alpha x0) on [-1, 1] (both sides of
the Creutz / Kennedy-Pendleton switch at alpha = 1.7), and (x1, x2, x3) must
be isotropic on the sphere of radius sqrt(1 - x0^2).
"""
import numpy as np
import pytest
from scipy import stats

import oracle as O
from closed_forms import su2_x0_bin_probs, su2_x0_mean, su2_x0_moment

ALPHAS = [0.0, 0.05, 0.5, 1.69, 1.71, 3.0, 10.0, 50.0]
N = 200_000


@pytest.mark.parametrize("alpha", ALPHAS)
def test_x0_distribution(alpha):
    x, att, _ = O.sample_su2(np.full(N, alpha), seed=4321 + int(alpha * 100))
    assert np.all(att > 0)
    x0 = x[:, 0]
    # unit norm
    assert np.abs(np.sum(x * x, axis=1) - 1).max() < 1e-13
    # mean against I2/I1 within 4 sigma
    m, sd = x0.mean(), x0.std()
    assert abs(m - su2_x0_mean(alpha)) < 4 * sd / np.sqrt(N)
    # chi^2 on 40 bins, equal width on [-1, 1] (narrow tail bins merged away)
    edges = np.linspace(-1, 1, 41)
    probs = su2_x0_bin_probs(edges, alpha)
    h, _ = np.histogram(x0, bins=edges)
    keep = probs * N > 20
    e = probs[keep] * N
    chi2 = ((h[keep] - e) ** 2 / e).sum() + ((h[~keep].sum() - probs[~keep].sum() * N) ** 2
                                             / max(probs[~keep].sum() * N, 1.0))
    assert stats.chi2.sf(chi2, keep.sum()) > 1e-3


@pytest.mark.parametrize("alpha", [0.5, 3.0, 10.0])
def test_direction_isotropic(alpha):
    x, _, _ = O.sample_su2(np.full(N, alpha), seed=77)
    v = x[:, 1:]
    m2 = su2_x0_moment(alpha, 2)
    for c in range(3):
        assert abs(v[:, c].mean()) < 4 * v[:, c].std() / np.sqrt(N)
        assert abs((v[:, c] ** 2).mean() - (1 - m2) / 3) < 4 * (v[:, c] ** 2).std() / np.sqrt(N)
    # off-diagonal second moments vanish
    assert abs((v[:, 0] * v[:, 1]).mean()) < 4 * (v[:, 0] * v[:, 1]).std() / np.sqrt(N)


def test_acceptance_rates():
    # Creutz acceptance is pi I1(alpha) / (2 sinh alpha); KP's rises with alpha
    from scipy import special
    for alpha in [0.5, 1.5]:
        _, att, _ = O.sample_su2(np.full(N, alpha), seed=5)
        acc = N / att.sum()
        want = np.pi * special.iv(1, alpha) / (2 * np.sinh(alpha))
        assert abs(acc - want) < 0.01
    _, att, _ = O.sample_su2(np.full(N, 50.0), seed=5)
    assert N / att.sum() > 0.98


def test_counters_select_the_stream():
    a = np.full(1000, 2.0)
    x1, _, _ = O.sample_su2(a, seed=1, step=0)
    x2, _, _ = O.sample_su2(a, seed=1, step=0)
    x3, _, _ = O.sample_su2(a, seed=1, step=1)
    x4, _, _ = O.sample_su2(a, seed=2, step=0)
    x5, _, _ = O.sample_su2(a, seed=1, step=0, mu_sg=1)
    assert np.array_equal(x1, x2)
    for other in (x3, x4, x5):
        assert np.abs(other - x1).max() > 0.5


def test_heatbath_link_conditional_distribution():
    """One SU(2) link redrawn many times with its staple held fixed: with
    k = sqrt(det A), x0 = ReTr(U' A) / (2k) must follow
    sqrt(1 - x0^2) exp(beta k x0) (paper Sec. 2)."""
    L = (4, 4, 4, 4)
    beta = 2.3
    U = O.new_field(2, L, hot=True, seed=9)
    s, mu = 37, 1
    A = O.staple(U, 2, L, s, mu)
    k = np.sqrt(np.linalg.det(A).real)
    n = 40_000
    x0 = np.empty(n)
    for step in range(n):
        W = U.copy()
        O.heatbath_link(W, 2, L, s, mu, beta, seed=1, step=step)
        x0[step] = np.real(np.trace(W[mu, s] @ A)) / (2 * k)
    edges = np.linspace(-1, 1, 21)
    probs = su2_x0_bin_probs(edges, beta * k)
    h, _ = np.histogram(x0, bins=edges)
    keep = probs * n > 20
    e = probs[keep] * n
    chi2 = ((h[keep] - e) ** 2 / e).sum()
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-3
    assert abs(x0.mean() - su2_x0_mean(beta * k)) < 4 * x0.std() / np.sqrt(n)
