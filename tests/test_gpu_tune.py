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
    assert r["score_tiles"] in (1, 2) and r["candidates"] == 5 * 3 * 2 and r["gram_macro"] == 0
    again = erx.autotune(b, p, a, cache=cache)
    assert again["candidates"] == 0
    assert {k: again[k] for k in ("block_lines", "scan_lines", "small_path", "score_tiles", "gram_macro")} == \
        {k: r[k] for k in ("block_lines", "scan_lines", "small_path", "score_tiles", "gram_macro")}
    assert erx.tune_lookup(b, p, cache)["block_lines"] == r["block_lines"]
    # scores of a handle with the tuned setting against the defaults, same lines
    sc = datagen.make_scene(2, 3, b, p, 300, drift=True, patches=True)
    X = datagen.lines(sc, 0, 300, device="cuda")[0]
    outs = []
    for kw in ({}, {"block_lines": r["block_lines"], "scan_lines": r["scan_lines"], "score_tiles": r["score_tiles"]},
               {"block_lines": 128, "scan_lines": 32}):
        d = erx.Detector(b, p, a, **kw)
        d.push(X)
        outs.append(d.scores().cpu().numpy().astype(np.float64))
        d.close()
    for o in outs[1:]:
        assert (np.abs(o - outs[0]) / np.maximum(np.abs(outs[0]), 1.0)).max() <= 1e-6


def test_autotune_chooses_the_gram_blocking(erx, tmp_path):
    """Above 64 bands the split-FP16 Gram's macro tile (64 or 128 bands) is a candidate too;
    both write the same statistics, so the choice is a matter of time only."""
    b, p = 108, 640
    log(f"autotune one stream b={b} p={p} with the Gram blocking")
    r = erx.autotune(b, p, 0.1, cache=str(tmp_path / "g.json"))
    log(f"  {r}")
    assert r["gram_macro"] in (64, 128) and r["candidates"] == 5 * 3 * 2 * 2


def test_autotune_batch_of_small_band_streams(erx, tmp_path):
    b, p, ns = 8, 256, 40
    log(f"autotune batch of {ns} streams b={b} p={p}")
    r = erx.autotune(b, p, 0.2, dtype="f16", nstreams=ns, cache=str(tmp_path / "t.json"))
    assert r["candidates"] == 8 and r["small_path"] in (0, 1, 2) and r["score_tiles"] in (1, 2)
    assert r["block_lines"] in (1024, 4096, 16384)


@pytest.mark.parametrize("b,p,dtype", [(5, 300, "f32"), (40, 201, "u16"), (108, 640, "f32"), (224, 1024, "f16"),
                                       (304, 130, "f32")])
def test_score_tile_shapes_give_identical_scores(erx, b, p, dtype):
    """The score kernel's tile shapes (one or two 16-pixel tiles per wave) run the same
    products for every pixel: the scores are bit-identical, for one stream and a batch."""
    log(f"score tile shapes b={b} p={p} {dtype}")
    T = 40
    sc = datagen.make_scene(2, 7, b, p, T, storage=dtype)
    X = datagen.lines(sc, 0, T, device="cuda")[0]
    outs = []
    for pt in (1, 2):
        d = erx.Detector(b, p, 0.1, dtype=dtype, score_tiles=pt, block_lines=16)
        d.push(X)
        outs.append(d.scores().cpu().numpy())
        d.close()
    np.testing.assert_array_equal(outs[0], outs[1])
    bouts = []
    for pt in (1, 2):
        bt = erx.Batch([b, b], [p, p], [0.1, 0.3], dtype=dtype, score_tiles=pt, block_lines=32)
        bt.push([X, X])
        bouts.append([o.cpu().numpy() for o in bt.scores()])
    for s_ in range(2):
        np.testing.assert_array_equal(bouts[0][s_], bouts[1][s_])
    # the batch cuts passes differently from the single handle: equal up to the rounding
    # of the FP64 moving averages
    np.testing.assert_allclose(bouts[0][0], outs[0], rtol=1e-6, atol=1e-6)
