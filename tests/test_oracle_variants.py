"""Pins of the IMC and RX Baseline references (oracle/variants.py) against what the
paper and mathematics fix: the batch Welford update the paper cites for IMC, the
first-line case, trace identities of the sample statistics, invariances, equal
weighting of past lines (IMC) and the window's locality (RX Baseline)."""
import numpy as np
import pytest

import oracle
from oracle import variants as V


def welford_batches(X):
    """Batch Welford (Schubert and Gertz, 2018): merge each line's mean and sum of
    squared deviations into the running ones; returns the sample covariance after
    every line."""
    out = []
    nA, muA, CA = 0, None, None
    for line in np.asarray(X, np.float64):
        nB = line.shape[0]
        muB = line.mean(0)
        D = line - muB
        CB = D.T @ D
        if nA == 0:
            nA, muA, CA = nB, muB, CB
        else:
            n = nA + nB
            d = muB - muA
            muA = muA + d * nB / n
            CA = CA + CB + np.outer(d, d) * nA * nB / n
            nA = n
        out.append((muA.copy(), CA / (nA - 1)))
    return out


def test_imc_equals_batch_welford():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((9, 13, 6)) + np.linspace(0, 3, 9)[:, None, None]
    for t, (mu, K) in enumerate(welford_batches(X)):
        m2, K2 = V.imc_background(X, t)
        assert np.allclose(mu, m2, rtol=0, atol=1e-12) and np.allclose(K, K2, rtol=0, atol=1e-12)


def test_imc_first_line_is_erx_initialisation():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((5, 30, 7))
    assert np.allclose(V.imc_run(X)[0], oracle.run(X, 1.0, 1e-5)["delta"][0], rtol=1e-12, atol=0)


def test_imc_trace_identity():
    """With the sample statistics of the N pooled pixels and eps = 0, the squared
    distances of those pixels sum to (N - 1) b."""
    rng = np.random.default_rng(2)
    X = rng.standard_normal((6, 20, 5))
    t = 4
    mu, K = V.imc_background(X, t)
    P = X[: t + 1].reshape(-1, 5)
    d2 = V._scores(P, mu, K, 0.0) ** 2
    assert abs(d2.sum() - (P.shape[0] - 1) * 5) < 1e-9


def test_imc_weighs_past_lines_equally():
    """Permuting the lines before t leaves line t's scores unchanged (not so for EMAs)."""
    rng = np.random.default_rng(3)
    X = rng.standard_normal((7, 25, 4)) * np.linspace(1, 2, 7)[:, None, None]
    Y = X.copy()
    Y[:6] = X[[3, 0, 5, 1, 4, 2]]
    assert np.allclose(V.imc_run(X)[6], V.imc_run(Y)[6], rtol=1e-12, atol=0)
    assert not np.allclose(oracle.run(X, 0.1)["delta"][6], oracle.run(Y, 0.1)["delta"][6], rtol=1e-6)


def test_imc_affine_invariance():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((5, 30, 4))
    A = rng.standard_normal((4, 4)) + 3 * np.eye(4)
    Y = X @ A.T + rng.standard_normal(4)
    assert np.allclose(V.imc_run(X, 0.0), V.imc_run(Y, 0.0), rtol=1e-9, atol=0)


def test_rx_window_trace_identity():
    """The window's own (divisor n) statistics: squared distances of its n pixels sum to n b."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((12, 15, 4))
    mu, K = V.rx_window_background(X, 10, 5)
    P = X[6:11].reshape(-1, 4)
    d2 = V._scores(P, mu, K, 0.0) ** 2
    assert abs(d2.sum() - P.shape[0] * 4) < 1e-9


def test_rx_window_one_line_is_scaled_erx():
    """A one-line window is per-line RX with divisor p: delta^2 = p / (p - 1) times ERX's
    (momentum 1, ridge 0), whose line covariance divides by p - 1."""
    rng = np.random.default_rng(6)
    X = rng.standard_normal((4, 20, 3))
    first, S = V.rx_baseline_run(X, window=1)
    erx = oracle.run(X, 1.0, 0.0)["delta"]
    assert first == 0 and np.allclose(S ** 2, erx ** 2 * 20 / 19, rtol=1e-12, atol=0)


def test_rx_window_over_all_lines_is_global_rx():
    rng = np.random.default_rng(7)
    X = rng.standard_normal((5, 12, 3))
    first, S = V.rx_baseline_run(X, window=5)
    P = X.reshape(-1, 3)
    mu = P.mean(0)
    K = np.cov(P.T, ddof=0)
    want = np.sqrt(np.einsum("pi,ij,pj->p", X[2] - mu, np.linalg.inv(K), X[2] - mu))
    assert first == 2 and S.shape == (1, 12) and np.allclose(S[0], want, rtol=1e-10, atol=0)


def test_rx_window_locality_and_invariance():
    rng = np.random.default_rng(8)
    X = rng.standard_normal((11, 16, 3))
    _, S = V.rx_baseline_run(X, window=5)
    Y = X.copy()
    Y[0] += 5.0  # only the first window sees line 0
    _, S2 = V.rx_baseline_run(Y, window=5)
    assert not np.allclose(S[0], S2[0]) and np.allclose(S[1:], S2[1:], rtol=1e-12, atol=0)
    A = rng.standard_normal((3, 3)) + 2 * np.eye(3)
    _, S3 = V.rx_baseline_run(X @ A.T + 1.0, window=5)
    assert np.allclose(S, S3, rtol=1e-9, atol=0)
