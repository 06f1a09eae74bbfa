"""Pins of the FP64 surrogate reference (oracle/surrogate.py) against facts that
do not come from it: reductions to plain ERX, invariance of ERX under an
orthogonal projection (with a ridge), and central finite differences of its own
forward pass for every gradient (the line statistics held fixed, as defined)."""
import numpy as np
import pytest

import oracle
from oracle import surrogate as S


def data(n, p, b, seed):
    rng = np.random.default_rng(seed)
    F = rng.normal(0, 0.3, (b, b))
    return rng.normal(0.5, 1.0, (n, p, b)) @ F.T + rng.normal(0, 1.0, b)


def test_identity_projection_without_network_is_plain_erx():
    X = data(6, 40, 16, 1)
    P = S.init_params(16, seed=2)
    P["W"], P["c"], P["w2"], P["c2"] = np.eye(16), np.zeros(16), np.zeros(S.HIDDEN), np.zeros(1)
    got = S.forward(P, X, 0.3, 1e-5)["score"]
    want = oracle.run(X, 0.3, 1e-5)["delta"]
    np.testing.assert_allclose(got, want, rtol=1e-10)


def test_constant_output_scales_the_score():
    X = data(5, 30, 9, 3)
    P = S.init_params(9, seed=4)
    P["w2"] = np.zeros(S.HIDDEN)
    base = S.forward(P, X, 0.2)["score"]
    P["c2"] = np.array([np.log(2.0)])
    np.testing.assert_allclose(S.forward(P, X, 0.2)["score"], 2.0 * base, rtol=1e-12)


def test_orthogonal_projection_keeps_erx():
    """ERX is invariant under x -> Q x + c with Q orthogonal, for any ridge, so
    a 16-band stream projected by an orthogonal W scores as plain ERX."""
    X = data(5, 50, 16, 5)
    Q, _ = np.linalg.qr(np.random.default_rng(6).normal(size=(16, 16)))
    P = S.init_params(16)
    P["W"], P["c"], P["w2"], P["c2"] = Q, np.arange(16.0), np.zeros(S.HIDDEN), np.zeros(1)
    got = S.forward(P, X, 0.1, 1e-5)["score"]
    np.testing.assert_allclose(got, oracle.run(X, 0.1, 1e-5)["delta"], rtol=1e-8)


@pytest.mark.parametrize("name", S.PARAM_NAMES)
def test_gradients_match_central_differences(name):
    n, p, b = 4, 12, 7
    X = data(n, p, b, 7)
    P = S.init_params(b, seed=8)
    P["w2"] = np.random.default_rng(9).normal(0, 0.5, S.HIDDEN)
    P["a1"] = np.random.default_rng(10).normal(0, 0.5, S.HIDDEN)
    target = np.exp(np.random.default_rng(11).normal(0.5, 0.3, (n, p)))
    loss, g, f = S.loss_and_grads(P, X, target, 0.3)
    stats = (f["mu"], f["M"])  # held fixed, as in the definition
    flat = np.asarray(P[name], np.float64).reshape(-1)
    rng = np.random.default_rng(12)
    idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
    h = 1e-7  # small enough that no ReLU kink is crossed (the smallest |pre-activation| is ~4e-5)
    for k in idx:
        Pp = {kk: np.array(v, np.float64, copy=True) for kk, v in P.items()}
        Pm = {kk: np.array(v, np.float64, copy=True) for kk, v in P.items()}
        Pp[name].reshape(-1)[k] += h
        Pm[name].reshape(-1)[k] -= h
        lp, _, _ = S.loss_and_grads(Pp, X, target, 0.3, stats=stats)
        lm, _, _ = S.loss_and_grads(Pm, X, target, 0.3, stats=stats)
        fd = (lp - lm) / (2 * h)
        an = np.asarray(g[name]).reshape(-1)[k]
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (name, k, fd, an)


def test_golden_worked_surrogate():
    """The hand-worked example in tests/golden/surrogate_worked.txt: the projection's
    orientation, the whitening, the hidden layer (orientation of A1, ReLU, bias), the
    output layer and the composition score = ||u|| exp(o)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "surrogate_worked.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    s = np.sqrt(31.0 / 2.0)
    val = {"S": s * np.exp(s - 0.2), "R": s * np.exp(-0.2)}
    want = np.array([val[r[1]] for r in rows])
    b = 16
    X = np.zeros((1, 32, b))
    for i in range(b):
        X[0, 2 * i, i] = s
        X[0, 2 * i + 1, i] = -s
    P = {"W": np.zeros((S.K, b)), "c": 0.1 * np.arange(1, S.K + 1), "A1": np.zeros((S.HIDDEN, S.K)),
         "a1": np.zeros(S.HIDDEN), "w2": np.zeros(S.HIDDEN), "c2": np.array([-0.1])}
    for j in range(S.K):
        P["W"][j, (j + 1) % b] = 1.0
    P["A1"][0, 0], P["A1"][1, 0], P["A1"][2, 1] = 1.0, 2.0, -1.0
    P["a1"][3] = 0.5
    P["w2"][:4] = [0.5, 0.25, 1.0, -0.2]
    got = S.forward(P, X, 0.1, ridge=0.0)["score"][0]
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=0)


def test_loss_weights_pixels_scored_above_the_background():
    """Special cases of the weighted loss: targets below sqrt(b) weigh 1 (the plain mean
    squared log error); a pixel whose target is 2 sqrt(b) counts four times; the weight
    stops at 100 (targets of 10 sqrt(b) and beyond)."""
    b = 16
    X = data(1, 40, b, 5)
    P = S.init_params(b, seed=3)
    logs = np.log(S.forward(P, X, 0.2)["score"])
    for scale, w in ((1.0, 1.0), (2.0, 4.0), (10.0, 100.0), (30.0, 100.0)):
        target = np.full(logs.shape, 0.5 * np.sqrt(b))
        target[0, 0] = scale * np.sqrt(b)
        e2 = (logs - np.log(target)) ** 2
        want = (e2.sum() + (w - 1.0) * e2[0, 0]) / e2.size
        loss, _, _ = S.loss_and_grads(P, X, target, 0.2)
        assert abs(loss - want) < 1e-12 * max(1.0, want), (scale, loss, want)
