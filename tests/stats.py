"""Small statistics helpers for the Monte Carlo pins (binned errors)."""
import numpy as np


def binned_mean_err(series, nbins=20):
    """Mean and standard error from nbins equal bins (autocorrelation-safe
    when a bin is much longer than the integrated autocorrelation time)."""
    x = np.asarray(series, dtype=np.float64)
    n = (x.size // nbins) * nbins
    bins = x[x.size - n:].reshape(nbins, -1).mean(axis=1)
    return float(bins.mean()), float(bins.std(ddof=1) / np.sqrt(nbins))
