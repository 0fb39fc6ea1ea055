"""Oracle pins: re-unitarization, staple, overrelaxation, observables.

Each pin compares the oracle with something other than itself: a library QR,
plaquettes computed independently in numpy, exact invariances of the Wilson
action (paper Sec. 2), or closed-form Haar moments.
"""
import numpy as np
import pytest

import oracle as O
from lattice_np import centre_transform, gauge_transform, haar_su, plaquette_map

NCS = [2, 3, 4, 6]


def qr_reunit(M):
    """Row Gram-Schmidt of M via a library QR of M^dag (positive-diagonal
    normalisation), then the last row multiplied by conj(det)/|det|."""
    Q, R = np.linalg.qr(M.conj().T)
    d = np.diag(R)
    Q = Q * (d / np.abs(d))[None, :]
    G = Q.conj().T
    det = np.linalg.det(G)
    G[-1] *= np.conj(det) / abs(det)
    return G


@pytest.mark.parametrize("nc", [2, 3, 4, 5, 6, 8])
def test_reunit_matches_library_qr(nc):
    rng = np.random.default_rng(nc)
    for _ in range(20):
        M = rng.standard_normal((nc, nc)) + 1j * rng.standard_normal((nc, nc))
        R = O.reunit_matrix(M)
        np.testing.assert_allclose(R, qr_reunit(M), atol=1e-13, rtol=0)


@pytest.mark.parametrize("nc", [2, 3, 4, 6, 8])
def test_reunit_unitary_det_one_idempotent(nc):
    rng = np.random.default_rng(100 + nc)
    for _ in range(20):
        M = rng.standard_normal((nc, nc)) + 1j * rng.standard_normal((nc, nc))
        R = O.reunit_matrix(M)
        assert np.abs(R.conj().T @ R - np.eye(nc)).max() < 1e-14
        assert abs(np.linalg.det(R) - 1) < 1e-14
        np.testing.assert_allclose(O.reunit_matrix(R), R, atol=5e-15, rtol=0)


@pytest.mark.parametrize("nc", [2, 3, 4])
def test_cold_start_is_trivial(nc):
    L = (4, 4, 4, 4)
    U = O.new_field(nc, L)
    assert np.array_equal(O.plaquette(U, nc, L), [1.0, 1.0, 1.0])
    assert O.polyakov(U, nc, L) == 1.0
    assert np.array_equal(O.unitarity(U, nc, L), [0.0, 0.0])
    # staple of the cold field: 2(d-1) identity matrices
    np.testing.assert_array_equal(O.staple(U, nc, L, 17, 2), 6 * np.eye(nc))


@pytest.mark.parametrize("nc", NCS)
def test_staple_closes_the_plaquettes(nc):
    """ReTr(U_mu(x) A_mu(x)) equals the sum of ReTr P over the 2(d-1)
    plaquettes containing the link, computed in numpy from the definition."""
    L = (4, 4, 2, 6)
    U = O.new_field(nc, L, hot=True, seed=7)
    V = U.shape[1]
    pm = {(m, n): plaquette_map(U, L, m, n).reshape(V) for m in range(4) for n in range(4) if m != n}
    rng = np.random.default_rng(0)
    for s in rng.integers(0, V, 12):
        x = [s % L[0], (s // L[0]) % L[1], (s // (L[0] * L[1])) % L[2], s // (L[0] * L[1] * L[2])]
        for mu in range(4):
            A = O.staple(U, nc, L, s, mu)
            lhs = np.real(np.trace(U[mu, s] @ A))
            rhs = 0.0
            for nu in range(4):
                if nu == mu:
                    continue
                xm = list(x)
                xm[nu] = (xm[nu] - 1) % L[nu]
                sm = xm[0] + L[0] * (xm[1] + L[1] * (xm[2] + L[2] * xm[3]))
                rhs += pm[(mu, nu)][s] + pm[(mu, nu)][sm]
            assert abs(lhs - rhs) < 1e-12


def _thermalised(nc, L, beta, sweeps=3, seed=11):
    U = O.new_field(nc, L, hot=True, seed=seed)
    for k in range(sweeps):
        O.sweep(U, nc, L, beta, 1, 1, seed, k)
    return U


def test_su2_overrelaxation_is_an_involution():
    L = (4, 4, 4, 4)
    U = _thermalised(2, L, 2.3)
    for s, mu in [(0, 0), (77, 1), (200, 3)]:
        W = U.copy()
        O.overrelax_link(W, 2, L, s, mu)
        assert np.abs(W[mu, s] - U[mu, s]).max() > 1e-3   # it moved
        O.overrelax_link(W, 2, L, s, mu)
        np.testing.assert_allclose(W, U, atol=1e-13, rtol=0)


@pytest.mark.parametrize("nc", [3, 4, 6])
def test_overrelaxation_reverse_order_undoes_forward(nc):
    L = (4, 4, 4, 4)
    U = _thermalised(nc, L, 2.0 * nc)
    for s, mu in [(3, 0), (101, 2)]:
        W = U.copy()
        O.overrelax_link(W, nc, L, s, mu)
        assert np.abs(W[mu, s] - U[mu, s]).max() > 1e-3
        O.overrelax_link(W, nc, L, s, mu, reverse=True)
        np.testing.assert_allclose(W, U, atol=1e-12, rtol=0)


@pytest.mark.parametrize("nc", [2, 3, 4])
def test_overrelaxation_conserves_action(nc):
    L = (4, 4, 4, 4)
    beta = {2: 2.3, 3: 6.0, 4: 11.1}[nc]
    U = _thermalised(nc, L, beta)
    S0 = O.action(U, nc, L, beta)
    p0 = O.plaquette(U, nc, L)[0]
    for mu in range(4):
        for p in range(2):
            O.phase(U, nc, L, 1, mu, p, beta, 0, 0)
    S1 = O.action(U, nc, L, beta)
    assert abs(S1 - S0) / S0 < 1e-12
    # and the field did change
    assert O.unitarity(U, nc, L)[0] < 1e-13
    assert abs(O.plaquette(U, nc, L)[0] - p0) < 1e-12


@pytest.mark.parametrize("nc", [2, 3])
def test_cold_start_is_overrelaxation_fixed_point(nc):
    L = (4, 4, 4, 4)
    U = O.new_field(nc, L)
    V0 = U.copy()
    O.sweep(U, nc, L, 5.0, 0, 2, 0, 0, reunit=False)
    np.testing.assert_array_equal(U, V0)


@pytest.mark.parametrize("nc", [2, 3, 4])
def test_gauge_invariance(nc):
    L = (4, 4, 4, 6)
    U = _thermalised(nc, L, 2.0 * nc, sweeps=2)
    rng = np.random.default_rng(5)
    g = haar_su(nc, U.shape[1], rng)
    Ug = gauge_transform(U, L, g)
    assert np.abs(Ug - U).max() > 0.1
    np.testing.assert_allclose(O.plaquette(Ug, nc, L), O.plaquette(U, nc, L), atol=1e-13, rtol=0)
    assert abs(O.polyakov(Ug, nc, L) - O.polyakov(U, nc, L)) < 1e-13
    assert abs(O.action(Ug, nc, L, 1.0) - O.action(U, nc, L, 1.0)) < 1e-9


@pytest.mark.parametrize("nc", [2, 3, 4])
def test_centre_symmetry(nc):
    L = (4, 4, 4, 6)
    U = _thermalised(nc, L, 2.0 * nc, sweeps=2)
    Uz = centre_transform(U, L, t0=2)
    np.testing.assert_allclose(O.plaquette(Uz, nc, L), O.plaquette(U, nc, L), atol=1e-13, rtol=0)
    z = np.exp(2j * np.pi / nc)
    assert abs(O.polyakov(Uz, nc, L) - z * O.polyakov(U, nc, L)) < 1e-13


@pytest.mark.parametrize("nc", [2, 3, 4, 6])
def test_hot_start_haar_moments(nc):
    L = (8, 8, 8, 8)
    U = O.new_field(nc, L, hot=True, seed=1234)
    links = U.reshape(-1, nc, nc)
    n = links.shape[0]
    # one Gram-Schmidt pass over a Gaussian matrix: error ~ cond(M) * eps
    assert O.unitarity(U, nc, L).max() < 1e-12
    tr = np.trace(links, axis1=1, axis2=2)
    # E Tr U = 0, E |Tr U|^2 = 1, E |U_ij|^2 = 1/N  (Haar on SU(N))
    assert abs(tr.mean()) < 5 * np.sqrt(1.0 / n)
    m2 = np.abs(tr) ** 2
    assert abs(m2.mean() - 1.0) < 5 * m2.std() / np.sqrt(n)
    e2 = np.abs(links) ** 2
    assert np.all(np.abs(e2.mean(axis=0) - 1.0 / nc) < 5 * e2.std(axis=0) / np.sqrt(n))
    # mean plaquette of independent Haar links: 0 with var(ReTr P / N) known
    var = 0.25 if nc == 2 else 1.0 / (2 * nc * nc)
    p = O.plaquette(U, nc, L)[0]
    assert abs(p) < 5 * np.sqrt(var / (6 * U.shape[1]))
    # different seeds give different fields; same seed the same field
    np.testing.assert_array_equal(O.new_field(nc, L, hot=True, seed=1234), U)
    assert np.abs(O.new_field(nc, L, hot=True, seed=1235) - U).max() > 0.1


def test_absent_directions_stay_identity():
    L = (8, 8, 1, 1)
    U = O.new_field(3, L, hot=True, seed=3)
    O.sweep(U, 3, L, 3.0, 1, 1, 3, 0)
    eye = np.broadcast_to(np.eye(3), U[2].shape)
    np.testing.assert_array_equal(U[2], eye)
    np.testing.assert_array_equal(U[3], eye)


def test_argument_checks():
    assert not O.valid(3, (7, 8, 8, 8))      # odd extent breaks the chessboard
    assert not O.valid(3, (1, 8, 8, 8))      # direction 0 must be present
    assert not O.valid(1, (8, 8, 8, 8))
    assert O.valid(3, (8, 8, 1, 1))
    with pytest.raises(ValueError):
        O.new_field(3, (6, 5, 4, 4))
