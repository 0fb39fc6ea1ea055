"""numpy helpers the tests use to transform fields independently of the
oracle: Haar matrices (QR of complex Gaussians, Mezzadri's phase fix),
gauge transformations, centre transformations and per-plane plaquette maps.
"""
import numpy as np


def grid(U, L):
    """(4, V, N, N) -> (4, Lt, Lz, Ly, Lx, N, N); direction mu is axis 4 - mu."""
    N = U.shape[-1]
    return U.reshape(4, L[3], L[2], L[1], L[0], N, N)


def shift(a, mu, n=+1):
    """a(x + n mu) for arrays laid out (Lt, Lz, Ly, Lx, ...)."""
    return np.roll(a, -n, axis=3 - mu)


def dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def plaquette_map(U, L, mu, nu):
    """ReTr P_mu_nu(x) on every site, P = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag."""
    G = grid(U, L)
    Um, Un = G[mu], G[nu]
    P = Um @ shift(Un, mu) @ dag(shift(Um, nu)) @ dag(Un)
    return np.real(np.trace(P, axis1=-2, axis2=-1))


def haar_su(N, n, rng):
    """n Haar-random SU(N) matrices: QR of complex Gaussians with the
    diagonal phases of R moved into Q, then the determinant divided out."""
    Z = (rng.standard_normal((n, N, N)) + 1j * rng.standard_normal((n, N, N))) / np.sqrt(2)
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(Q)
    Q[:, :, 0] *= np.conj(det)[:, None] / np.abs(det)[:, None]
    return Q


def gauge_transform(U, L, g):
    """U_mu(x) -> g(x) U_mu(x) g(x+mu)^dag; g has shape (V, N, N)."""
    N = U.shape[-1]
    G = grid(U, L).copy()
    gg = g.reshape(L[3], L[2], L[1], L[0], N, N)
    for mu in range(4):
        G[mu] = gg @ G[mu] @ dag(shift(gg, mu))
    return G.reshape(U.shape)


def centre_transform(U, L, t0, k=1):
    """Multiplies every U_3(xvec, t0) by exp(2 pi i k / N)."""
    N = U.shape[-1]
    G = grid(U, L).copy()
    G[3, t0] *= np.exp(2j * np.pi * k / N)
    return G.reshape(U.shape)
