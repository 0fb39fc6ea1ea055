"""Oracle pins: Markov-chain averages against exact results.

2D lattices (L = {L, L, 1, 1}) with the Wilson action have exactly known
plaquette averages (see closed_forms.py).  These runs pin the whole update
chain: staple orientation, subgroup projection and coupling alpha = 2 beta k/Nc,
embedding, the sampler, and the chessboard schedule (paper Sec. 2 and Sec. 3).
A wrong orientation, a wrong factor in alpha, or a transposed embedding moves
the average far outside the error bars.
"""
import numpy as np
import pytest

import oracle as O
from closed_forms import one_link_plaquette, su2_torus_plaquette
from stats import binned_mean_err


def run_chain(nc, L, beta, n_therm, n_meas, n_or, seed, hot=True):
    U = O.new_field(nc, L, hot=hot, seed=seed)
    step = 0
    series = []
    for k in range(n_therm + n_meas):
        O.sweep(U, nc, L, beta, 1, n_or, seed, step)
        step += 1
        if k >= n_therm:
            series.append(O.plaquette(U, nc, L)[0])
    return U, np.array(series)


@pytest.mark.parametrize("beta", [1.0, 2.3, 4.0])
def test_2d_su2_exact_plaquette(beta):
    L = (8, 8, 1, 1)
    _, series = run_chain(2, L, beta, 50, 3000, 3, seed=1234)
    m, e = binned_mean_err(series)
    exact = su2_torus_plaquette(beta, 64)
    assert abs(m - exact) < 4 * e, (m, e, exact)
    assert e < 0.003


@pytest.mark.parametrize("nc,beta", [(3, 3.0), (3, 6.0), (4, 11.1)])
def test_2d_sun_one_link_plaquette(nc, beta):
    L = (16, 16, 1, 1)
    _, series = run_chain(nc, L, beta, 50, 1200, 2, seed=99)
    m, e = binned_mean_err(series)
    exact = one_link_plaquette(nc, beta)
    assert abs(m - exact) < 4 * e, (m, e, exact)
    assert e < 0.004


@pytest.mark.parametrize("nc", [2, 3])
def test_beta_zero_heatbath_gives_haar(nc):
    L = (4, 4, 4, 4)
    U, series = run_chain(nc, L, 0.0, 2, 200, 0, seed=3, hot=False)
    var = 0.25 if nc == 2 else 1.0 / (2 * nc * nc)
    m = series.mean()
    # sweeps at beta = 0 are independent: plain standard error
    assert abs(m) < 5 * np.sqrt(var / (6 * U.shape[1] * series.size))
    links = U.reshape(-1, nc, nc)
    tr = np.trace(links, axis1=1, axis2=2)
    assert abs(np.mean(np.abs(tr) ** 2) - 1.0) < 0.1


@pytest.mark.parametrize("nc,beta", [(2, 0.5), (3, 0.9)])
def test_4d_strong_coupling(nc, beta):
    """In 4D the plaquette differs from the one-link value only at order
    beta^4 relative (smallest closed surface: a cube of 6 plaquettes)."""
    L = (4, 4, 4, 4)
    _, series = run_chain(nc, L, beta, 20, 400, 1, seed=5)
    m, e = binned_mean_err(series)
    exact = one_link_plaquette(nc, beta)
    assert abs(m - exact) < 4 * e + 0.02 * exact, (m, e, exact)


@pytest.mark.parametrize("nc,beta", [(2, 100.0), (3, 300.0)])
def test_4d_weak_coupling_equipartition(nc, beta):
    """At large beta each of the Nc^2 - 1 modes per link carries 1/2 of
    the Gaussian weight: 1 - P = (Nc^2 - 1) / (4 beta) to leading order in 4D."""
    L = (4, 4, 4, 4)
    _, series = run_chain(nc, L, beta, 30, 100, 1, seed=8, hot=False)
    m = series.mean()
    lead = (nc * nc - 1) / (4.0 * beta)
    assert abs((1 - m) - lead) < 0.1 * lead, (1 - m, lead)
