"""Batch statistics of an ensemble of histories (Sec. 4.1, eq. ErrorCLT; Sec. 4.2).

Oracle (test infrastructure).

The stochastic unravellings estimate an expectation by the average over n_conf independent
histories, and the paper attaches to it the statistical error of the central limit theorem,
sqrt(Delta^2 / n_conf), with Delta^2 the variance of the quantity over the histories.  The
paper does not say which variance estimator it takes; here Delta^2 is the unbiased sample
variance, with divisor n_conf - 1, around the arithmetic batch mean.  For complex entries
(off-diagonal correlations) the variance is that of the complex value, E|X - mean|^2, the
sum of the variances of its real and imaginary parts.

All functions take the per-history values stacked along axis 0 and work entry by entry.
"""
import numpy as np


def batch_mean(values):
    """(1/B) sum_b X_b, entry by entry."""
    X = np.asarray(values)
    B = X.shape[0]
    total = np.zeros(X.shape[1:], dtype=X.dtype)
    for b in range(B):
        total = total + X[b]
    return total / B


def batch_variance(values):
    """sum_b |X_b - mean|^2 / (B - 1), entry by entry (0 for a batch of one history)."""
    X = np.asarray(values)
    B = X.shape[0]
    m = batch_mean(X)
    acc = np.zeros(X.shape[1:], dtype=np.float64)
    for b in range(B):
        acc = acc + np.abs(X[b] - m) ** 2
    if B < 2:
        return np.zeros(X.shape[1:], dtype=np.float64)
    return acc / (B - 1)


def clt_error(values):
    """Statistical error of the batch mean, sqrt(Delta^2 / n_conf) (eq. ErrorCLT)."""
    X = np.asarray(values)
    return np.sqrt(batch_variance(X) / X.shape[0])


def ratio_mean(values, norms):
    """sum_b X_b / sum_b n_b: the ratio estimator of the linear unravelling (Sec. 4.2), which
    divides out the fluctuation of the histories' norms n_b = <psi_b|psi_b>."""
    X = np.asarray(values)
    n = np.asarray(norms, dtype=np.float64)
    total = np.zeros(X.shape[1:], dtype=X.dtype)
    for b in range(X.shape[0]):
        total = total + X[b]
    return total / np.sum(n)
