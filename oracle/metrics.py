"""FP64 reference of the detection metrics of Sec. IV-C (ROC AUC, AUC_TD, AUC_BS).

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's checks.
The GPU library never imports or calls anything here.

The functions follow the definitions of Sec. IV-C step by step:

* The ROC curve pairs, for every threshold tau, the true positive rate
  TPR(tau) = #(anomalies with score >= tau) / #anomalies with the false positive
  rate FPR(tau) = #(background pixels with score >= tau) / #background pixels
  (Eqs. (26)-(27)).  "All potential thresholds" are the distinct scores; the
  curve runs from (0, 0) (tau above every score) to (1, 1).
* AUC is the area under that curve, taken by the trapezoid rule between the
  points of consecutive thresholds (the curve is straight between them: pixels
  with equal scores change class together).
* AUC_TPR,tau and AUC_FPR,tau are the areas under TPR(tau) and FPR(tau) as
  functions of the threshold.  The thresholds are taken on the scores
  min-max normalised over the evaluated pixels, so tau runs over [0, 1] and
  both areas lie in [0, 1] (reading: the paper rescales the metrics of its
  reference to [0, 1]; all scores equal gives normalised scores 0).  TPR(tau) is
  a step function of tau, integrated exactly over its steps.
* AUC_TD = (AUC + AUC_TPR,tau) / 2 and AUC_BS = (AUC - AUC_FPR,tau + 1) / 2
  (Eqs. (28)-(29)).

Pixels with a non-finite score are left out of every metric and counted.
"""
from __future__ import annotations

import numpy as np


def _split(scores, truth):
    s = np.asarray(scores, np.float64).ravel()
    y = np.asarray(truth).ravel().astype(bool)
    fin = np.isfinite(s)
    return s[fin], y[fin], int((~fin).sum())


def roc_curve(scores, truth):
    """(FPR, TPR, thresholds): one point per distinct score (descending), plus (0, 0)."""
    s, y, _ = _split(scores, truth)
    P, N = int(y.sum()), int((~y).sum())
    thr, inv = np.unique(s, return_inverse=True)      # ascending distinct scores
    pos_at = np.bincount(inv, weights=y, minlength=thr.size)
    neg_at = np.bincount(inv, weights=~y, minlength=thr.size)
    # pixels with score >= thr[i]: counts from the top threshold down
    tp = np.cumsum(pos_at[::-1])
    fp = np.cumsum(neg_at[::-1])
    tpr = np.concatenate([[0.0], tp / P])
    fpr = np.concatenate([[0.0], fp / N])
    return fpr, tpr, thr[::-1]


def auc(scores, truth) -> float:
    """Area under the ROC curve by the trapezoid rule over all distinct thresholds."""
    fpr, tpr, _ = roc_curve(scores, truth)
    return float(np.sum((fpr[1:] - fpr[:-1]) * (tpr[1:] + tpr[:-1]) / 2.0))


def _normalised(s):
    lo, hi = s.min(), s.max()
    return (s - lo) / (hi - lo) if hi > lo else np.zeros_like(s)


def rate_tau_area(scores, truth, positive: bool) -> float:
    """Area under TPR(tau) (positive=True) or FPR(tau) over tau in [0, 1], the scores
    min-max normalised: the rate is constant on each interval (v_{i-1}, v_i] between
    consecutive distinct normalised scores, where it equals #(class >= v_i) / #class."""
    s, y, _ = _split(scores, truth)
    v = _normalised(s)
    cls = np.sort(v[y] if positive else v[~y])
    steps = np.unique(v)
    steps = steps[steps > 0.0]
    prev = np.concatenate([[0.0], steps[:-1]])
    at_least = cls.size - np.searchsorted(cls, steps, side="left")  # #(class >= v_i)
    return float(np.sum((steps - prev) * at_least / cls.size))


def detection_metrics(scores, truth) -> dict:
    s, y, excluded = _split(scores, truth)
    a = auc(scores, truth)
    atp = rate_tau_area(scores, truth, True)
    afp = rate_tau_area(scores, truth, False)
    return dict(auc=a, auc_tpr_tau=atp, auc_fpr_tau=afp, auc_td=(a + atp) / 2.0,
                auc_bs=(a - afp + 1.0) / 2.0, positives=int(y.sum()), negatives=int((~y).sum()),
                excluded=excluded)
