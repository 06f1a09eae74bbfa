"""Pins of the sparse random projection reference (oracle/srp.py, Sec. III-B) against
what the paper and mathematics fix: the published SplitMix64 output sequence, the
weight values and their law (non-zero with probability 1/s, E[w^2] = 1/d, about
d sqrt(b) active weights), norm preservation in expectation, and the projected
ERX reducing to plain ERX on Z = X W."""
import math

import numpy as np
import pytest

import oracle
from oracle import srp


def test_splitmix64_published_outputs():
    """The first outputs of SplitMix64 from state 0 (Steele, Lea and Flood 2014; Vigna's
    reference splitmix64.c)."""
    assert [srp.splitmix64(0, k) for k in (1, 2, 3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                        0x06C45D188009454F]


@pytest.mark.parametrize("b,d", [(108, 5), (224, 5), (13, 3), (90, 16)])
def test_weight_values_and_law(b, d):
    s = math.sqrt(b)
    Ws = [srp.srp_matrix(b, d, seed) for seed in range(40)]
    vals = np.unique(np.concatenate([W.ravel() for W in Ws]))
    assert set(np.round(vals / math.sqrt(s / d), 12)) <= {-1.0, 0.0, 1.0}
    counts = np.array([(W != 0).sum() for W in Ws], np.float64)
    # n_aw = (b d) / s = d sqrt(b) in expectation; binomial spread over 40 draws
    n_aw = d * math.sqrt(b)
    sd = math.sqrt(b * d * (1 / s) * (1 - 1 / s) / len(Ws))
    assert abs(counts.mean() - n_aw) < 5 * sd
    # E[w^2] = (s / d) (1 / s) = 1 / d; w^2 has variance (s / d)^2 (1 / s)(1 - 1 / s) per weight
    w2 = np.mean([np.mean(W ** 2) for W in Ws])
    assert abs(w2 - 1.0 / d) < 5 * math.sqrt((s / d) ** 2 / s * (1 - 1 / s) / (b * d * len(Ws)))
    signs = np.concatenate([np.sign(W[W != 0]) for W in Ws])
    assert abs(signs.mean()) < 5 / math.sqrt(signs.size)


def test_norm_preserved_in_expectation():
    """E ||W^T x||^2 = ||x||^2 since the weights are independent with E[w^2] = 1/d."""
    rng = np.random.default_rng(0)
    x = rng.standard_normal(108)
    sq = [np.sum((x @ srp.srp_matrix(108, 5, seed)) ** 2) for seed in range(400)]
    assert abs(np.mean(sq) / np.sum(x ** 2) - 1.0) < 0.15


def test_seeds_give_different_matrices():
    assert not np.array_equal(srp.srp_matrix(64, 5, 1), srp.srp_matrix(64, 5, 2))
    assert np.array_equal(srp.srp_matrix(64, 5, 7), srp.srp_matrix(64, 5, 7))


def test_projected_erx_is_erx_of_projection():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((12, 40, 30))
    W = srp.srp_matrix(30, 5, 3)
    Z = np.einsum("tpb,bd->tpd", X, W)
    a = srp.run(X, 5, 3, 0.1)["delta"]
    b = oracle.run(Z, 0.1, 1e-5)["delta"]
    assert np.allclose(a, b, rtol=1e-13, atol=0)
