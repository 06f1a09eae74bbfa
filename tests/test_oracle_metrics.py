"""Pins of the FP64 detection-metric reference (oracle/metrics.py, Sec. IV-C) against
values fixed by the definitions, not against the reference itself: pair counting
(the Mann-Whitney statistic equals the trapezoid ROC area), closed forms of
separable and constant scores, the symmetry AUC(-s) = 1 - AUC(s), and a fine
Riemann sum of the threshold curves."""
import numpy as np
import pytest

from oracle import metrics as M


def pair_count_auc(s, y):
    """Fraction of (anomaly, background) pairs ranked correctly, ties counting 1/2."""
    pos, neg = s[y], s[~y]
    gt = (pos[:, None] > neg[None, :]).sum()
    eq = (pos[:, None] == neg[None, :]).sum()
    return (gt + 0.5 * eq) / (pos.size * neg.size)


@pytest.mark.parametrize("seed", range(6))
def test_auc_equals_pair_counting_with_ties(seed):
    rng = np.random.default_rng(seed)
    n = 60 + 20 * seed
    s = rng.integers(0, 12, n).astype(np.float64)  # many ties
    y = rng.random(n) < 0.3
    y[0], y[1] = True, False
    assert abs(M.auc(s, y) - pair_count_auc(s, y)) < 1e-12


def test_auc_closed_forms():
    s = np.arange(10.0)
    y = s >= 7
    assert abs(M.auc(s, y) - 1.0) < 1e-12
    assert abs(M.auc(-s, y)) < 1e-12
    assert abs(M.auc(np.ones(10), y) - 0.5) < 1e-12
    rng = np.random.default_rng(3)
    s = rng.standard_normal(200)
    y = rng.random(200) < 0.2
    assert abs(M.auc(-s, y) - (1.0 - M.auc(s, y))) < 1e-12


def test_roc_curve_endpoints():
    rng = np.random.default_rng(4)
    s = rng.standard_normal(50)
    y = rng.random(50) < 0.4
    fpr, tpr, thr = M.roc_curve(s, y)
    assert (fpr[0], tpr[0]) == (0.0, 0.0) and (fpr[-1], tpr[-1]) == (1.0, 1.0)
    assert np.all(np.diff(fpr) >= 0) and np.all(np.diff(tpr) >= 0)
    assert thr.size == np.unique(s).size


@pytest.mark.parametrize("positive", [True, False])
def test_threshold_area_by_riemann_sum(positive):
    """The exact step integral against a midpoint sum over 200000 thresholds."""
    rng = np.random.default_rng(5)
    s = np.round(rng.gamma(2.0, 1.0, 300), 2)
    y = rng.random(300) < 0.25
    v = (s - s.min()) / (s.max() - s.min())
    cls = v[y] if positive else v[~y]
    K = 200000
    taus = (np.arange(K) + 0.5) / K
    sv = np.sort(cls)
    rate = (cls.size - np.searchsorted(sv, taus, side="left")) / cls.size  # #(cls >= tau) / #cls
    riemann = rate.mean()
    assert abs(M.rate_tau_area(s, y, positive) - riemann) < 2e-4
    # the area under P(V >= tau) over [0, 1] is E[V]
    assert abs(M.rate_tau_area(s, y, positive) - cls.mean()) < 1e-12


def test_metric_combinations_and_exclusion():
    rng = np.random.default_rng(6)
    s = rng.standard_normal(400)
    y = rng.random(400) < 0.1
    s[[3, 77]] = np.nan
    s[100] = np.inf
    m = M.detection_metrics(s, y)
    assert m["excluded"] == 3 and m["positives"] + m["negatives"] == 397
    assert abs(m["auc_td"] - (m["auc"] + m["auc_tpr_tau"]) / 2) < 1e-15
    assert abs(m["auc_bs"] - (m["auc"] - m["auc_fpr_tau"] + 1) / 2) < 1e-15
    const = M.detection_metrics(np.full(20, 2.5), np.arange(20) < 5)
    assert abs(const["auc"] - 0.5) < 1e-12 and const["auc_tpr_tau"] == 0.0 and const["auc_fpr_tau"] == 0.0


def test_perfect_detector_metrics():
    """Anomalies at the top score, background at the bottom: every metric is at its best."""
    s = np.array([0.0] * 8 + [1.0] * 2)
    y = s > 0.5
    m = M.detection_metrics(s, y)
    assert abs(m["auc"] - 1.0) < 1e-12 and m["auc_tpr_tau"] == 1.0 and m["auc_fpr_tau"] == 0.0
    assert abs(m["auc_td"] - 1.0) < 1e-12 and abs(m["auc_bs"] - 1.0) < 1e-12
