"""Closed-form values the oracle is pinned to (independent of its code).

* SU(2) heatbath draw: density of x0 is sqrt(1 - x0^2) exp(alpha x0) on
  [-1, 1] (paper Sec. 2, SU(2) heatbath).  Its normaliser is pi I1(alpha)/alpha
  and its mean is I2(alpha)/I1(alpha).
* One-link integral of SU(N) (Bars-Green / Brower-Rossi-Tan):
  z(beta) = int dU exp((beta/N) ReTr U) = sum_k det[I_{k+j-i}(beta/N)]_{i,j}.
  On a 2D lattice with the Wilson action (paper Sec. 2) the plaquettes are
  independent up to a global torus constraint, so the mean of (1/N) ReTr P is
  d ln z / d beta.  For SU(2) this is I2(beta)/I1(beta).
* SU(2) on an L x L torus, exactly (character expansion, genus 1):
  <(1/2) Tr P> = (1/Np) d/dbeta ln sum_{n>=1} (2 I_n(beta)/beta)^Np.
"""
import numpy as np
from scipy import integrate, special


def su2_x0_mean(alpha):
    if alpha == 0:
        return 0.0
    return float(special.ive(2, alpha) / special.ive(1, alpha))


def su2_x0_density(x, alpha):
    return np.sqrt(np.clip(1.0 - x * x, 0.0, None)) * np.exp(alpha * (x - 1.0))


def su2_x0_moment(alpha, k):
    num = integrate.quad(lambda x: x ** k * su2_x0_density(x, alpha), -1, 1, limit=200,
                         epsabs=0, epsrel=1e-12)[0]
    den = integrate.quad(lambda x: su2_x0_density(x, alpha), -1, 1, limit=200,
                         epsabs=0, epsrel=1e-12)[0]
    return num / den


def su2_x0_bin_probs(edges, alpha):
    den = integrate.quad(lambda x: su2_x0_density(x, alpha), -1, 1, limit=200,
                         epsabs=0, epsrel=1e-12)[0]
    return np.array([integrate.quad(lambda x: su2_x0_density(x, alpha), a, b, limit=100,
                                    epsabs=0, epsrel=1e-10)[0] for a, b in zip(edges[:-1], edges[1:])]) / den


def one_link_z(N, beta, kmax=40):
    x = beta / N
    tot = 0.0
    for k in range(-kmax, kmax + 1):
        M = np.empty((N, N))
        for i in range(N):
            for j in range(N):
                M[i, j] = special.iv(k + j - i, x)
        tot += np.linalg.det(M)
    return tot


def one_link_plaquette(N, beta, h=1e-4):
    """d ln z / d beta by a 4th-order central difference."""
    f = lambda b: np.log(one_link_z(N, b))
    return (-f(beta + 2 * h) + 8 * f(beta + h) - 8 * f(beta - h) + f(beta - 2 * h)) / (12 * h)


def su2_torus_plaquette(beta, n_plaq, nmax=60, h=1e-4):
    def lnZ(b):
        # sum_n (2 I_n(b)/b)^Np, factored by the n = 1 term for range
        r = np.array([special.ive(n, b) / special.ive(1, b) for n in range(1, nmax)])
        return n_plaq * np.log(2 * special.iv(1, b) / b) + np.log(np.sum(r ** n_plaq))
    return (-lnZ(beta + 2 * h) + 8 * lnZ(beta + h) - 8 * lnZ(beta - h) + lnZ(beta - 2 * h)) / (12 * h) / n_plaq
