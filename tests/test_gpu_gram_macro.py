"""The split-FP16 Gram on 128-band macro tiles (k_gram8) against the one on 64-band
macro tiles (k_gram4) and the FP64 oracle.

Both kernels run the same operations in the same order for every output value (band
shift and scale from the first 64 pixels, the three FP16 products of each 32-pixel
step, FP32 partials over 64 pixels added into FP64, FP64 band sums reduced in the
same grouping); only the assignment of tiles to workgroups differs.  So the per-line
statistics, and everything computed from them, must agree bit for bit, on full and
ragged pixel chunks, band counts that are not a multiple of 4 (element loads), every
storage type, and the last macro column that is partly empty.
"""
import numpy as np
import pytest
import torch

import datagen
import oracle

pytestmark = pytest.mark.gpu


def log(msg):
    print(f"[gpu-gram-macro] {msg}", flush=True)


@pytest.fixture(scope="module")
def erx():
    import paper_2408_14947_amd as m
    m.load()
    return m


def run(erx, X, b, p, storage, gram_macro, **kw):
    det = erx.Detector(b, p, 0.1, dtype=storage, gram_macro=gram_macro, block_lines=16, scan_lines=8, **kw)
    det.push(X.cuda())
    got = det.scores().cpu().numpy()
    t, mu, K = det.state()
    return got, mu, K


@pytest.mark.parametrize("b,p,T,storage", [(65, 100, 20, "f32"), (70, 257, 18, "u16"), (100, 77, 20, "f32"),
                                           (128, 64, 12, "f16"), (129, 1000, 10, "f32"), (203, 130, 12, "f32"),
                                           (224, 1024, 8, "f32"), (226, 130, 10, "u16"), (300, 33, 10, "f32"),
                                           (304, 200, 9, "f16")])
def test_macro_tile_sizes_agree_bit_for_bit(erx, b, p, T, storage):
    log(f"b={b} p={p} T={T} {storage}")
    kind = "gauss" if storage == "f16" else "mixture"
    sc = datagen.make_scene(91, b % 7, b, p, T, kind=kind, storage=storage, drift=True)
    X, _ = datagen.lines(sc, 0, T)
    s64, mu64, K64 = run(erx, X, b, p, storage, 64)
    s128, mu128, K128 = run(erx, X, b, p, storage, 128)
    log(f"  max |score diff| {np.abs(s64 - s128).max():.3e}")
    assert np.array_equal(mu64, mu128) and np.array_equal(K64, K128)
    assert np.array_equal(s64, s128)
    if p <= b:
        # fewer pixels than bands: the first lines' backgrounds are singular up to the
        # ridge, so only the agreement of the two tilings is checked here
        return
    want = oracle.run(datagen.storage_to_float64(X, storage), 0.1, 1e-5)["delta"]
    err = np.abs(s128 - want) / np.maximum(np.abs(want), 1.0)
    log(f"  max err vs oracle {err.max():.3e}")
    assert err.max() <= 1e-4


def test_default_choice_is_exact_too(erx):
    """gram_macro 0 picks 128-band macro tiles from 65 bands on: same values."""
    b, p, T = 160, 300, 10
    sc = datagen.make_scene(92, 0, b, p, T)
    X, _ = datagen.lines(sc, 0, T)
    s0, _, K0 = run(erx, X, b, p, "f32", 0)
    s64, _, K64 = run(erx, X, b, p, "f32", 64)
    assert np.array_equal(s0, s64) and np.array_equal(K0, K64)


def test_batch_with_both_macro_tile_sizes(erx):
    """Streams of several band counts in one batch: the pass descriptors carry the choice."""
    bands, pixels = [70, 140, 224, 33], [130, 200, 96, 64]
    T = 12
    Xs = []
    for i, (b, p) in enumerate(zip(bands, pixels)):
        sc = datagen.make_scene(93, i, b, p, T)
        Xs.append(datagen.lines(sc, 0, T)[0].cuda())
    out = {}
    for gm in (64, 128):
        bt = erx.Batch(bands, pixels, [0.1] * 4, gram_macro=gm, small_path=0)
        bt.push(Xs)
        out[gm] = [s.cpu().numpy() for s in bt.scores()]
    for a, c in zip(out[64], out[128]):
        assert np.array_equal(a, c)
