"""Time-series analysis of a Markov chain's measurements: autocorrelation,
the integrated autocorrelation time with automatic windowing (Madras and
Sokal, J. Stat. Phys. 50 (1988) 109), and the error of a mean that accounts
for it.  Used by the run tool on the plaquette history."""
import numpy as np


def autocorrelation(x):
    """Normalized autocorrelation rho(t), t = 0 .. n - 1, of a series (FFT,
    zero-padded so that the estimate is the plain lagged sum / n)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    if n < 2:
        return np.ones(n)
    d = x - x.mean()
    f = np.fft.rfft(d, 2 * n)
    acov = np.fft.irfft(f * np.conj(f))[:n] / n
    if acov[0] == 0.0:
        return np.concatenate([[1.0], np.zeros(n - 1)])
    return acov / acov[0]


def tau_int(x, c=6.0):
    """(tau, window): tau(W) = 1/2 + sum_{t=1}^{W} rho(t), with W the first
    lag at which W >= c tau(W)."""
    rho = autocorrelation(x)
    n = len(rho)
    tau = 0.5
    for w in range(1, n):
        tau += rho[w]
        if w >= c * tau:
            return float(tau), w
    return float(tau), n - 1


def mean_error(x, c=6.0):
    """(mean, error, tau): error^2 = 2 tau var / n."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    if n < 2:
        return float(x.mean()) if n else float("nan"), float("nan"), float("nan")
    tau, _ = tau_int(x, c)
    tau = max(tau, 0.5)
    return float(x.mean()), float(np.sqrt(2.0 * tau * x.var() / n)), tau
