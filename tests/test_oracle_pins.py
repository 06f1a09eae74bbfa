"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than its own formulas:
an exact rational brute force, a library solve of the plain definition,
closed forms, invariances and identities.  The mutation tests in
test_oracle_mutants.py show that plausible slips in the oracle fail these pins.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# helpers that are NOT the oracle's algorithm
# --------------------------------------------------------------------------
def frac_solve(A, r):
    """Exact Gauss-Jordan solve A y = r over the rationals."""
    n = len(r)
    M = [list(A[i]) + [r[i]] for i in range(n)]
    for c in range(n):
        piv = next(i for i in range(c, n) if M[i][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for i in range(n):
            if i != c and M[i][c] != 0:
                f = M[i][c] / M[c][c]
                M[i] = [a - f * b for a, b in zip(M[i], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


def frac_erx(X, alpha, eps):
    """delta^2 of every pixel from the plain definition, exactly.

    X: list of lines, each a list of pixels (lists of ints).  Uses the
    definition delta^2 = r^T (K_t + eps I)^{-1} r with the EMA background
    (Sec. III-C, Eqs. (18)-(21); Sec. III-D), solved by Gauss-Jordan.
    """
    out = []
    mu = K = None
    for t, line in enumerate(X):
        p, b = len(line), len(line[0])
        mh = [sum(Fraction(px[j]) for px in line) / p for j in range(b)]
        Kh = [[sum((px[i] - mh[i]) * (px[j] - mh[j]) for px in line) / (p - 1)
               for j in range(b)] for i in range(b)]
        if t == 0:
            mu, K = mh, Kh
        else:
            mu = [(1 - alpha) * mu[j] + alpha * mh[j] for j in range(b)]
            K = [[(1 - alpha) * K[i][j] + alpha * Kh[i][j] for j in range(b)] for i in range(b)]
        A = [[K[i][j] + (eps if i == j else 0) for j in range(b)] for i in range(b)]
        row = []
        for px in line:
            r = [px[j] - mu[j] for j in range(b)]
            y = frac_solve(A, r)
            row.append(sum(ri * yi for ri, yi in zip(r, y)))
        out.append(row)
    return out


def numpy_erx(X, alpha, eps):
    """Literal recurrence with np.cov(ddof=1) and np.linalg.solve."""
    T, p, b = X.shape
    mu = K = None
    out = np.empty((T, p))
    for t in range(T):
        mh = X[t].mean(0)
        Kh = np.atleast_2d(np.cov(X[t], rowvar=False, ddof=1))
        if t == 0:
            mu, K = mh, Kh
        else:
            mu = (1 - alpha) * mu + alpha * mh
            K = (1 - alpha) * K + alpha * Kh
        R = X[t] - mu
        Y = np.linalg.solve(K + eps * np.eye(b), R.T)
        out[t] = np.sqrt(np.einsum("ij,ji->i", R, Y))
    return out


def rel(a, b):
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


# --------------------------------------------------------------------------
# P1: exact rational brute force on tiny integer inputs
# --------------------------------------------------------------------------
@pytest.mark.parametrize("alpha", [Fraction(1), Fraction(1, 2), Fraction(1, 10)])
@pytest.mark.parametrize("eps", [Fraction(0), Fraction(1, 100000)])
@pytest.mark.parametrize("b,p,T", [(1, 3, 4), (2, 4, 5), (3, 5, 6)])
def test_p1_exact_bruteforce(alpha, eps, b, p, T):
    rng = np.random.default_rng(1000 * b + 10 * p + T)
    while True:
        Xi = rng.integers(-6, 7, size=(T, p, b))
        # skip rank-deficient draws when there is no ridge
        if all(np.linalg.matrix_rank(Xi[t] - Xi[t].mean(0)) == b for t in range(T)):
            break
    exact = frac_erx(Xi.tolist(), alpha, eps)
    got = oracle.run(Xi.astype(np.float64), float(alpha), float(eps))["delta"]
    for t in range(T):
        for i in range(p):
            e = float(exact[t][i])
            assert abs(got[t, i] ** 2 - e) <= 1e-12 * max(e, 1e-3), (t, i, got[t, i] ** 2, e)


def test_golden_worked_example():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "worked_2band.txt"))
            if l.strip() and not l.startswith("#")]
    X = np.zeros((2, 4, 2))
    want = np.zeros((2, 4))
    for t, i, x0, x1, d2 in rows:
        X[int(t) - 1, int(i)] = [float(x0), float(x1)]
        want[int(t) - 1, int(i)] = float(Fraction(d2))
    got = oracle.run(X, 0.5, 0.0)["delta"] ** 2
    np.testing.assert_allclose(got, want, rtol=1e-14)


# --------------------------------------------------------------------------
# P2: NumPy brute force of the plain definition
# --------------------------------------------------------------------------
@pytest.mark.parametrize("b,p,T,alpha,eps", [(1, 7, 9, 0.1, 1e-5), (5, 16, 20, 0.1, 1e-5),
                                             (16, 64, 50, 0.3, 1e-3), (8, 9, 12, 1.0, 0.0),
                                             (12, 40, 30, 0.01, 1e-5)])
def test_p2_numpy_bruteforce(b, p, T, alpha, eps):
    rng = np.random.default_rng(b * 7 + p)
    X = rng.standard_normal((T, p, b)) @ rng.standard_normal((b, b)) + rng.uniform(0, 1, b)
    want = numpy_erx(X, alpha, eps)
    got = oracle.run(X, alpha, eps)["delta"]
    assert rel(got, want) < 1e-10


# --------------------------------------------------------------------------
# P3: momentum 1 is per-line RX with the (p-1) covariance of that line alone
# --------------------------------------------------------------------------
def test_p3_momentum_one_is_per_line_rx():
    rng = np.random.default_rng(3)
    T, p, b, eps = 6, 30, 5, 1e-5
    X = rng.standard_normal((T, p, b)) * rng.uniform(0.5, 2, b)
    got = oracle.run(X, 1.0, eps)["delta"]
    for t in range(T):
        alone = oracle.run(X[t:t + 1], 0.37, eps)["delta"][0]   # a fresh stream: first line only
        np.testing.assert_allclose(got[t], alone, rtol=1e-12)
        # line t's scores do not depend on the lines before it
        Y = X.copy()
        Y[:t] = rng.standard_normal((t, p, b))
        np.testing.assert_allclose(oracle.run(Y, 1.0, eps)["delta"][t], got[t], rtol=1e-12)


# --------------------------------------------------------------------------
# P4: trace identities for delta^2 (not delta)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("b,p", [(1, 2), (3, 10), (10, 40), (32, 100)])
def test_p4_trace_identity(b, p):
    rng = np.random.default_rng(b + p)
    X = rng.standard_normal((1, p, b)) @ rng.standard_normal((b, b))
    d2 = oracle.run(X, 1.0, 0.0)["delta"][0] ** 2
    # sum_i r_i^T K^-1 r_i = tr(K^-1 (p-1) K) = (p-1) b
    assert abs(d2.sum() - (p - 1) * b) < 1e-9 * p * b
    # with the population (1/n) statistics of the scored set the mean score is b
    assert abs(d2.mean() * p / (p - 1) - b) < 1e-9 * b


# --------------------------------------------------------------------------
# P5/P6: invariances
# --------------------------------------------------------------------------
def _stream(seed, T=12, p=25, b=6):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((T, p, b)) @ rng.standard_normal((b, b)) + rng.uniform(0, 3, b)


@pytest.mark.parametrize("alpha", [1.0, 0.5, 0.1, 0.01])
def test_p5_affine_invariance_without_ridge(alpha):
    X = _stream(5)
    rng = np.random.default_rng(55)
    A = rng.standard_normal((6, 6)) + 3 * np.eye(6)
    c = rng.standard_normal(6)
    d0 = oracle.run(X, alpha, 0.0)["delta"]
    d1 = oracle.run(X @ A.T + c, alpha, 0.0)["delta"]
    assert rel(d1, d0) < 1e-8
    # per-band scaling is a special (diagonal) case
    s = rng.uniform(0.1, 10, 6)
    assert rel(oracle.run(X * s, alpha, 0.0)["delta"], d0) < 1e-9


def test_p5_orthogonal_invariance_with_ridge():
    X = _stream(6)
    rng = np.random.default_rng(66)
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    d0 = oracle.run(X, 0.1, 1e-2)["delta"]
    assert rel(oracle.run(X @ Q.T, 0.1, 1e-2)["delta"], d0) < 1e-10
    perm = rng.permutation(6)
    assert rel(oracle.run(X[..., perm], 0.1, 1e-2)["delta"], d0) < 1e-12
    # a non-orthogonal scaling with a ridge does change the scores
    assert rel(oracle.run(X * 10.0, 0.1, 1e-2)["delta"], d0) > 1e-6


def test_p6_shift_invariance_with_ridge():
    X = _stream(7)
    c = np.random.default_rng(77).standard_normal(6) * 100
    d0 = oracle.run(X, 0.1, 1e-5)["delta"]
    assert rel(oracle.run(X + c, 0.1, 1e-5)["delta"], d0) < 1e-9


# --------------------------------------------------------------------------
# P7: stationarity
# --------------------------------------------------------------------------
def test_p7_identical_lines():
    rng = np.random.default_rng(8)
    line = rng.standard_normal((20, 4)) @ rng.standard_normal((4, 4))
    X = np.repeat(line[None], 9, axis=0)
    r = oracle.run(X, 0.1, 1e-5, history=True)
    for t in range(1, 9):
        np.testing.assert_allclose(r["delta"][t], r["delta"][0], rtol=1e-12)
    np.testing.assert_allclose(r["K_hist"][-1], np.cov(line, rowvar=False, ddof=1), rtol=1e-12)
    np.testing.assert_allclose(r["mu_hist"][-1], line.mean(0), rtol=1e-12)


# --------------------------------------------------------------------------
# P8: one band, closed form
# --------------------------------------------------------------------------
def test_p8_single_band_closed_form():
    rng = np.random.default_rng(9)
    X = rng.uniform(0, 1, (7, 11, 1))
    alpha, eps = 0.25, 1e-3
    mu = var = None
    got = oracle.run(X, alpha, eps)["delta"]
    for t in range(7):
        x = X[t, :, 0]
        m, v = x.mean(), ((x - x.mean()) ** 2).sum() / 10
        mu, var = (m, v) if t == 0 else ((1 - alpha) * mu + alpha * m, (1 - alpha) * var + alpha * v)
        np.testing.assert_allclose(got[t], np.abs(x - mu) / math.sqrt(var + eps), rtol=1e-13)


# --------------------------------------------------------------------------
# P9: EMA closed-form weights
# --------------------------------------------------------------------------
def test_p9_ema_closed_form():
    rng = np.random.default_rng(10)
    T, p, b, a = 15, 12, 3, 0.3
    X = rng.standard_normal((T, p, b))
    r = oracle.run(X, a, 1e-5, history=True)
    for t in range(T):
        w = np.array([(1 - a) ** t] + [a * (1 - a) ** (t - j) for j in range(1, t + 1)])
        assert abs(w.sum() - 1) < 1e-12
        Kc = sum(w[j] * np.cov(X[j], rowvar=False, ddof=1) for j in range(t + 1))
        mc = sum(w[j] * X[j].mean(0) for j in range(t + 1))
        np.testing.assert_allclose(r["K_hist"][t], Kc, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(r["mu_hist"][t], mc, rtol=1e-12, atol=1e-15)


# --------------------------------------------------------------------------
# P10: pixel-permutation equivariance, line-order sensitivity
# --------------------------------------------------------------------------
def test_p10_equivariance_and_order():
    X = _stream(11)
    rng = np.random.default_rng(111)
    perm = rng.permutation(X.shape[1])
    d0 = oracle.run(X, 0.1, 1e-5)["delta"]
    np.testing.assert_allclose(oracle.run(X[:, perm], 0.1, 1e-5)["delta"], d0[:, perm], rtol=1e-11)
    # reversing the line order (a "flipped" scan) changes scores unless momentum is 1
    drev = oracle.run(X[::-1].copy(), 0.1, 1e-5)["delta"][::-1]
    assert rel(drev, d0) > 1e-3
    np.testing.assert_allclose(oracle.run(X[::-1].copy(), 1.0, 1e-5)["delta"][::-1],
                               oracle.run(X, 1.0, 1e-5)["delta"], rtol=1e-12)


# --------------------------------------------------------------------------
# P11: push granularity does not change results
# --------------------------------------------------------------------------
def test_p11_chunking():
    X = _stream(12, T=23)
    d0 = oracle.run(X, 0.1, 1e-5)["delta"]
    s = oracle.Stream(6, 25, 0.1, 1e-5)
    parts = [s.push(X[a:b])["delta"] for a, b in [(0, 1), (1, 8), (8, 9), (9, 23)]]
    np.testing.assert_array_equal(np.concatenate(parts), d0)
    # state save / restore
    s2 = oracle.Stream(6, 25, 0.1, 1e-5)
    s2.push(X[:10])
    t, mu, K = s2.state()
    s3 = oracle.Stream(6, 25, 0.1, 1e-5)
    s3.set_state(t, mu, K)
    np.testing.assert_array_equal(s3.push(X[10:])["delta"], d0[10:])


# --------------------------------------------------------------------------
# line normalisation (Sec. III-E, Eq. (24))
# --------------------------------------------------------------------------
def test_normalisation():
    X = _stream(13)
    r = oracle.run(X, 0.1, 1e-5, normalise=True)
    dn = r["delta_n"]
    np.testing.assert_allclose(dn.mean(1), 0, atol=1e-12)
    np.testing.assert_allclose(dn.std(1), 1, rtol=1e-12)   # numpy std is the population std
    np.testing.assert_allclose(dn, (r["delta"] - r["delta"].mean(1, keepdims=True))
                               / r["delta"].std(1, keepdims=True), rtol=1e-10, atol=1e-12)
    np.testing.assert_array_equal(oracle.normalise(np.full(5, 3.0)), np.zeros(5))


# --------------------------------------------------------------------------
# degenerate cases: not positive definite, NaN, invalid arguments
# --------------------------------------------------------------------------
def test_not_pd_without_ridge():
    X = _stream(14, T=5)
    X[2:, :, 3] = 0.5          # constant band (exact in binary) from line 3 on
    r = oracle.run(X, 1.0, 0.0)   # momentum 1: K_t is the singular line covariance
    assert list(r["notpd"]) == [0, 0, 1, 1, 1]
    assert np.isnan(r["delta"][2:]).all() and np.isfinite(r["delta"][:2]).all()
    r2 = oracle.run(X, 1.0, 1e-5)   # the ridge restores positive definiteness
    assert not r2["notpd"].any() and np.isfinite(r2["delta"]).all()


def test_rank_deficient_line_with_ridge_scores():
    rng = np.random.default_rng(15)
    X = rng.standard_normal((3, 4, 10))   # p <= b: every line covariance is singular
    r = oracle.run(X, 0.1, 1e-5)
    assert not r["notpd"].any() and np.isfinite(r["delta"]).all()


def test_nan_propagates_forward_only():
    X = _stream(16, T=6)
    X[3, 5, 2] = np.nan
    d = oracle.run(X, 0.1, 1e-5)["delta"]
    assert np.isfinite(d[:3]).all() and np.isnan(d[3:]).all()


@pytest.mark.parametrize("b,p,a,e", [(0, 5, 0.1, 0), (3, 1, 0.1, 0), (3, 5, 0.0, 0),
                                     (3, 5, 1.5, 0), (3, 5, 0.1, -1e-3), (3, 5, float("nan"), 0)])
def test_invalid_arguments(b, p, a, e):
    with pytest.raises(ValueError):
        oracle.Stream(b, p, a, e).push(np.zeros((1, p, b)))


def test_cholesky_helpers():
    rng = np.random.default_rng(17)
    M = rng.standard_normal((7, 7))
    A = M @ M.T + np.eye(7)
    L, info = oracle.cholesky(A)
    assert info == 0
    np.testing.assert_allclose(L @ L.T, A, rtol=1e-12, atol=1e-12)
    assert np.all(np.diag(L) > 0) and np.allclose(np.triu(L, 1), 0)
    r = rng.standard_normal(7)
    d, m = oracle.mahalanobis(L, r)
    np.testing.assert_allclose(d ** 2, r @ np.linalg.solve(A, r), rtol=1e-12)
    _, info = oracle.cholesky(np.diag([1.0, 0.0, 2.0]))
    assert info == 2
