"""FP64 references of the two background models the paper compares ERX with.

TEST INFRASTRUCTURE ONLY: imported by the tests.  The GPU library never imports or
calls anything here, and nothing here imports the GPU library.

* IMC ("No EMAs", Sec. IV-D, ablation): the moving averages of Sec. III-C are
  replaced by incremental mean and covariance updates that weigh every pixel of
  every line seen so far equally.  Reading: the background of line t is the sample
  mean and the sample covariance (divisor N - 1) of all N = t p pixels of lines
  1..t, which is what the batch Welford update the paper cites maintains; line t
  is scored with it after its own update, with the ridge eps I as in ERX.  For
  t = 1 this is ERX's initial background.
* RX Baseline (Sec. IV-B): a rolling buffer holds the most recent W = 99 lines; the
  mean and the covariance of all pixels in the buffer (divisor n, as in the RX
  definition of Sec. II-A) score the centre line of the buffer.  Reading: the
  window of the lines t - W + 1 .. t scores line t - (W - 1) / 2 (W odd), so the
  first scored line is the (W + 1) / 2-th, once W lines have arrived; the ridge is
  a parameter, 0 by default (the RX definition has none).

Both are written as the plain definitions: the statistics of the stacked pixels,
then a Cholesky solve per pixel.
"""
from __future__ import annotations

import numpy as np


def _scores(Xline, mu, K, ridge):
    b = K.shape[0]
    L = np.linalg.cholesky(K + ridge * np.eye(b))
    R = (np.asarray(Xline, np.float64) - mu).T          # b x p
    M = np.linalg.solve(L, R)                           # forward substitution's result
    return np.sqrt(np.sum(M * M, axis=0))


def imc_background(X, t):
    """Mean and sample covariance of all pixels of lines 0..t (0-based)."""
    P = np.asarray(X[: t + 1], np.float64).reshape(-1, X.shape[2])
    mu = P.mean(axis=0)
    C = P - mu
    return mu, C.T @ C / (P.shape[0] - 1)


def imc_run(X, ridge: float = 1e-5) -> np.ndarray:
    """Scores [T][p] of every line under the IMC background."""
    X = np.asarray(X, np.float64)
    out = np.empty(X.shape[:2])
    for t in range(X.shape[0]):
        mu, K = imc_background(X, t)
        out[t] = _scores(X[t], mu, K, ridge)
    return out


def rx_window_background(X, t, window: int):
    """Mean and population covariance of all pixels of lines t-window+1..t."""
    P = np.asarray(X[t - window + 1: t + 1], np.float64).reshape(-1, X.shape[2])
    mu = P.mean(axis=0)
    C = P - mu
    return mu, C.T @ C / P.shape[0]


def rx_baseline_run(X, window: int = 99, ridge: float = 0.0):
    """(first scored line, scores [T - window + 1][p]): the window ending at line t
    scores line t - (window - 1) // 2."""
    X = np.asarray(X, np.float64)
    T = X.shape[0]
    half = (window - 1) // 2
    rows = []
    for t in range(window - 1, T):
        mu, K = rx_window_background(X, t, window)
        rows.append(_scores(X[t - half], mu, K, ridge))
    return half, np.array(rows).reshape(-1, X.shape[1])
