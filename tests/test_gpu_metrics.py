"""erx_detection_metrics (Sec. IV-C) on the GPU against the FP64 reference of
oracle/metrics.py: AUC exactly (an integer pair count divided once), the threshold
areas to FP64 summation order."""
import sys

import numpy as np
import pytest
import torch

import datagen
import oracle
from oracle import metrics as M

pytestmark = pytest.mark.gpu


def log(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def erx():
    import paper_2408_14947_amd as m
    m.load()
    return m


def check(erx, s, y, tol_area=1e-9):
    got = erx.detection_metrics(torch.as_tensor(s, dtype=torch.float32).cuda(),
                                torch.as_tensor(y.astype(np.uint8)).cuda())
    want = M.detection_metrics(np.asarray(s, np.float32), y)
    log(f"  n={s.size} P={want['positives']} auc gpu {got['auc']:.12f} ref {want['auc']:.12f}")
    for k in ("positives", "negatives", "excluded"):
        assert got[k] == want[k], k
    assert abs(got["auc"] - want["auc"]) <= 1e-12
    for k in ("auc_tpr_tau", "auc_fpr_tau", "auc_td", "auc_bs"):
        assert abs(got[k] - want[k]) <= tol_area, (k, got[k], want[k])
    return got


@pytest.mark.parametrize("n,frac,levels", [(10, 0.3, 4), (2047, 0.1, 50), (2049, 0.5, 0), (100000, 0.01, 1000),
                                           (300001, 0.7, 0), (1 << 20, 0.002, 0)])
def test_metrics_random(erx, n, frac, levels):
    """Random scores, with many ties when levels > 0; frac > 0.5 sorts the background."""
    log(f"metrics random n={n} anomaly fraction {frac} levels {levels}")
    rng = np.random.default_rng(n)
    s = rng.standard_normal(n)
    if levels:
        s = np.floor(s * levels / 4.0)
    y = rng.random(n) < frac
    y[0], y[-1] = True, False
    s = s + 0.8 * y  # anomalies tend to score higher
    check(erx, s.astype(np.float32), y)


def test_metrics_on_erx_scores(erx):
    """The detector's own scores of a synthetic scene against its anomaly mask."""
    log("metrics of ERX scores (108 bands, 200 lines x 640 px)")
    scene = datagen.make_scene(1, 0, 108, 640, 200)
    X, mask = datagen.lines(scene, 0, 200)
    det = erx.Detector(108, 640, 0.1)
    det.push(X.cuda())
    sc = det.scores().reshape(-1)
    torch.cuda.synchronize()
    got = check(erx, sc.cpu().numpy(), mask.numpy().reshape(-1).astype(bool))
    assert got["auc"] > 0.9


def test_metrics_exclusion_and_errors(erx):
    log("metrics: non-finite scores, one-class input")
    rng = np.random.default_rng(7)
    s = rng.standard_normal(5000).astype(np.float32)
    y = rng.random(5000) < 0.2
    s[[1, 10, 100]] = np.nan
    s[[2, 20]] = np.inf
    s[3] = -np.inf
    got = check(erx, s, y)
    assert got["excluded"] == 6
    check(erx, np.full(3000, 1.5, np.float32), np.arange(3000) < 100)  # all equal: auc 1/2, areas 0
    with pytest.raises(erx.ErxError):
        erx.detection_metrics(torch.zeros(100, device="cuda"), torch.zeros(100, dtype=torch.uint8, device="cuda"))
