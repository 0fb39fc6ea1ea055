"""Oracle pins at large Nc (the reference of the workgroup-per-link path,
Nc up to 32): the same independent checks as at small Nc -- a library QR,
plaquettes from the definition in numpy, exact invariances of the action,
Haar moments, and the 2D one-link closed form for the whole update chain."""
import numpy as np
import pytest

import oracle as O
from closed_forms import one_link_plaquette
from lattice_np import centre_transform, gauge_transform, haar_su, plaquette_map
from stats import binned_mean_err
from test_oracle_algebra import qr_reunit


@pytest.mark.parametrize("nc", [10, 16, 32])
def test_reunit_matches_library_qr_large(nc):
    rng = np.random.default_rng(nc)
    for _ in range(5):
        M = rng.standard_normal((nc, nc)) + 1j * rng.standard_normal((nc, nc))
        R = O.reunit_matrix(M)
        # both are rounding away from the same Q; the gap grows with cond(M)
        np.testing.assert_allclose(R, qr_reunit(M), atol=1e-12 * np.linalg.cond(M), rtol=0)
        assert np.abs(R.conj().T @ R - np.eye(nc)).max() < 1e-13
        assert abs(np.linalg.det(R) - 1) < 1e-13
        np.testing.assert_allclose(O.reunit_matrix(R), R, atol=1e-14, rtol=0)


def test_staple_closes_the_plaquettes_nc10():
    nc, L = 10, (2, 2, 2, 4)
    U = O.new_field(nc, L, hot=True, seed=3)
    V = U.shape[1]
    pm = {(m, n): plaquette_map(U, L, m, n).reshape(V) for m in range(4) for n in range(4) if m != n}
    for s in (0, 5, 17, 31):
        x = [s % L[0], (s // L[0]) % L[1], (s // (L[0] * L[1])) % L[2], s // (L[0] * L[1] * L[2])]
        for mu in range(4):
            lhs = np.real(np.trace(U[mu, s] @ O.staple(U, nc, L, s, mu)))
            rhs = 0.0
            for nu in range(4):
                if nu == mu:
                    continue
                xm = list(x)
                xm[nu] = (xm[nu] - 1) % L[nu]
                rhs += pm[(mu, nu)][s] + pm[(mu, nu)][xm[0] + L[0] * (xm[1] + L[1] * (xm[2] + L[2] * xm[3]))]
            assert abs(lhs - rhs) < 1e-11


@pytest.mark.parametrize("nc", [12, 16])
def test_overrelaxation_reverse_order_undoes_forward_large(nc):
    L = (4, 4, 2, 2)
    U = O.new_field(nc, L, hot=True, seed=nc)
    for s, mu in [(3, 0), (21, 3)]:
        W = U.copy()
        O.overrelax_link(W, nc, L, s, mu)
        assert np.abs(W[mu, s] - U[mu, s]).max() > 1e-3
        O.overrelax_link(W, nc, L, s, mu, reverse=True)
        # the chain of Nc (Nc - 1) / 2 subgroup steps amplifies rounding
        np.testing.assert_allclose(W, U, atol=1e-9, rtol=0)


def test_overrelaxation_conserves_action_nc10():
    nc, L, beta = 10, (4, 4, 2, 2), 86.7
    U = O.new_field(nc, L, hot=True, seed=2)
    for k in range(2):
        O.sweep(U, nc, L, beta, 1, 0, 2, k)
    S0 = O.action(U, nc, L, beta)
    before = U.copy()
    for mu in range(4):
        for p in range(2):
            O.phase(U, nc, L, 1, mu, p, beta, 0, 0)
    assert np.abs(U - before).max() > 1e-3
    assert abs(O.action(U, nc, L, beta) - S0) / S0 < 1e-11


def test_gauge_and_centre_symmetry_nc10():
    nc, L = 10, (4, 2, 2, 4)
    U = O.new_field(nc, L, hot=True, seed=8)
    g = haar_su(nc, U.shape[1], np.random.default_rng(6))
    Ug = gauge_transform(U, L, g)
    assert np.abs(Ug - U).max() > 0.1
    np.testing.assert_allclose(O.plaquette(Ug, nc, L), O.plaquette(U, nc, L), atol=1e-13, rtol=0)
    assert abs(O.polyakov(Ug, nc, L) - O.polyakov(U, nc, L)) < 1e-13
    Uz = centre_transform(U, L, t0=1)
    np.testing.assert_allclose(O.plaquette(Uz, nc, L), O.plaquette(U, nc, L), atol=1e-13, rtol=0)
    assert abs(O.polyakov(Uz, nc, L) - np.exp(2j * np.pi / nc) * O.polyakov(U, nc, L)) < 1e-13


@pytest.mark.parametrize("nc", [16, 32])
def test_hot_start_haar_moments_large(nc):
    L = (4, 4, 4, 4) if nc == 16 else (4, 4, 2, 2)
    U = O.new_field(nc, L, hot=True, seed=1234)
    links = U.reshape(-1, nc, nc)
    n = links.shape[0]
    assert O.unitarity(U, nc, L).max() < 1e-12
    tr = np.trace(links, axis1=1, axis2=2)
    assert abs(tr.mean()) < 5 * np.sqrt(1.0 / n)
    m2 = np.abs(tr) ** 2
    assert abs(m2.mean() - 1.0) < 5 * m2.std() / np.sqrt(n)
    e2 = np.abs(links) ** 2
    assert abs(e2.mean() - 1.0 / nc) < 5 * e2.std() / np.sqrt(e2.size)


def test_2d_su8_one_link_plaquette():
    """SU(8) on a 2D torus at beta = 44.4: the whole update chain (28
    subgroups per link) against the one-link closed form."""
    nc, L, beta = 8, (8, 8, 1, 1), 44.4
    U = O.new_field(nc, L, hot=True, seed=21)
    series = []
    for k in range(700):
        O.sweep(U, nc, L, beta, 1, 2, 21, k)
        if k >= 50:
            series.append(O.plaquette(U, nc, L)[0])
    m, e = binned_mean_err(np.array(series))
    exact = one_link_plaquette(nc, beta)
    assert abs(m - exact) < 4 * e, (m, e, exact)
    assert e < 0.004


def _perm_sign(perm):
    """Sign of a permutation from its cycle decomposition."""
    seen, sign = np.zeros(len(perm), dtype=bool), 1
    for i in range(len(perm)):
        if not seen[i]:
            j, length = i, 0
            while not seen[j]:
                seen[j] = True
                j = perm[j]
                length += 1
            sign *= -1 if length % 2 == 0 else 1
    return sign


@pytest.mark.parametrize("nc", [4, 7, 12])
def test_determinant_of_phased_permutations(nc):
    """Links P D (a permutation matrix times unit phases) have the closed-form
    determinant sign(P) prod(phases), reached by the LU elimination only
    through its row exchanges; re-unitarization keeps the rows and multiplies
    the last one by the conjugate of that determinant."""
    L = (2, 2, 2, 2)
    rng = np.random.default_rng(5 + nc)
    V = int(np.prod(L))
    U = np.zeros((4, V, nc, nc), dtype=np.complex128)
    dets = np.zeros((4, V), dtype=np.complex128)
    for mu in range(4):
        for s in range(V):
            perm = rng.permutation(nc)
            ph = np.exp(1j * rng.uniform(-np.pi, np.pi, nc))
            U[mu, s, np.arange(nc), perm] = ph
            dets[mu, s] = _perm_sign(perm) * np.prod(ph)
    dev = O.unitarity(U, nc, L)
    assert dev[0] < 1e-15
    assert abs(dev[1] - np.abs(dets - 1).max()) < 1e-13
    want = U.copy()
    want[:, :, nc - 1, :] *= np.conj(dets)[:, :, None]
    O.reunitarize(U, nc, L)
    assert np.abs(U - want).max() < 1e-14
