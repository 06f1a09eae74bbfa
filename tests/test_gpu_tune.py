"""Autotuner of the launch settings: it times its candidates, caches the winner, and
its choice does not change the scores."""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import datagen  # noqa: E402

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def erx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2408_14947_amd as m
    m.load()
    return m


def test_autotune_single_stream_caches_and_keeps_results(erx, tmp_path):
    b, p, a = 40, 200, 0.1
    cache = str(tmp_path / "tune.json")
    log(f"autotune one stream b={b} p={p}")
    r = erx.autotune(b, p, a, cache=cache)
    assert r["candidates"] > 0 and r["us_per_line"] > 0
    assert r["block_lines"] in (512, 1024, 2048, 4096, 8192) and r["scan_lines"] in (32, 64, 128)
    again = erx.autotune(b, p, a, cache=cache)
    assert again["candidates"] == 0
    assert {k: again[k] for k in ("block_lines", "scan_lines", "small_path")} == \
        {k: r[k] for k in ("block_lines", "scan_lines", "small_path")}
    assert erx.tune_lookup(b, p, cache)["block_lines"] == r["block_lines"]
    # scores of a handle with the tuned setting against the defaults, same lines
    sc = datagen.make_scene(2, 3, b, p, 300, drift=True, patches=True)
    X = datagen.lines(sc, 0, 300, device="cuda")[0]
    outs = []
    for kw in ({}, {"block_lines": r["block_lines"], "scan_lines": r["scan_lines"]},
               {"block_lines": 128, "scan_lines": 32}):
        d = erx.Detector(b, p, a, **kw)
        d.push(X)
        outs.append(d.scores().cpu().numpy().astype(np.float64))
        d.close()
    for o in outs[1:]:
        assert (np.abs(o - outs[0]) / np.maximum(np.abs(outs[0]), 1.0)).max() <= 1e-6


def test_autotune_batch_of_small_band_streams(erx, tmp_path):
    b, p, ns = 8, 256, 40
    log(f"autotune batch of {ns} streams b={b} p={p}")
    r = erx.autotune(b, p, 0.2, dtype="f16", nstreams=ns, cache=str(tmp_path / "t.json"))
    assert r["candidates"] == 5 and r["small_path"] in (0, 1, 2)
    assert r["block_lines"] in (1024, 4096, 16384)
