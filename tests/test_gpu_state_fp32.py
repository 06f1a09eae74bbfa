"""FP32 storage of the moving-average state, the per-line statistics and the scan
carries (state_fp32), against the FP64 oracle.

Storing a value in FP32 perturbs each covariance entry by at most one rounding,
|dK_ij| <= 2^-24 |K_ij|, after the local scan, in the segment carry and in the
stream's state (the recurrence itself runs in FP64).  That is a componentwise
relative perturbation, of the size of the one the FP32 (or split-FP16) Gram already
makes by summing p products in FP32, so the FP32-class configurations are held to
the plain path's 1e-4 of the oracle, scaled like the other reduced-precision
reports by max(1, kappa_max / 2e5) (the first-order error is linear in the
condition number; the FP64 state reaches 5e-5 at kappa 3.5e5 on these scenes).
With a 16-bit Gram the Gram's input rounding dominates: the whole pattern is held
to the reduced-precision Gram's max bound, and what the FP32 storage adds is
checked against an FP64-state run of the same input (at most the FP32-class bound).
"""
import numpy as np
import pytest
import torch

import datagen
import oracle

pytestmark = pytest.mark.gpu

BOUNDS = {"bf16": (1e-2, 3e-3), "fp16": (1e-3, 5e-4)}
KAPPA_REF = 2e5


def log(msg):
    print(f"[gpu-state-fp32] {msg}", flush=True)


@pytest.fixture(scope="module")
def erx():
    import paper_2408_14947_amd as m
    m.load()
    return m


def rel_err(got, want):
    return np.abs(np.asarray(got, np.float64) - want) / np.maximum(np.abs(want), 1.0)


def report(got, want):
    e = rel_err(got, want)
    return {"max": float(e.max()), "p99": float(np.quantile(e, 0.99)), "median": float(np.median(e))}


def kappa_max(out, ridge=1e-5):
    K = out["K_hist"]
    b = K.shape[-1]
    return float(max(np.linalg.cond(k + ridge * np.eye(b)) for k in K))


@pytest.mark.parametrize("prec", ["split16", "fp32"])
@pytest.mark.parametrize("b,p,T,blk,seg", [(1, 40, 30, 8, 4), (16, 300, 70, 24, 8), (37, 301, 70, 33, 8),
                                           (108, 640, 90, 40, 16), (224, 1024, 40, 2048, 64),
                                           (304, 200, 20, 8, 4)])
def test_state_fp32_parity(erx, prec, b, p, T, blk, seg):
    """Several passes per push (block_lines < T) so the FP32 state is written and read
    back between passes, and ragged segments."""
    log(f"b={b} p={p} T={T} blk={blk} seg={seg} prec={prec}")
    sc = datagen.make_scene(71, b, b, p, T, drift=True)
    X, _ = datagen.lines(sc, 0, T)
    det = erx.Detector(b, p, 0.1, precision=prec, state_fp32=True, block_lines=blk, scan_lines=seg)
    det.push(X.cuda())
    got = det.scores().cpu().numpy()
    want = oracle.run(X.numpy(), 0.1, 1e-5)["delta"]
    e = rel_err(got, want)
    log(f"  max err {e.max():.3e} median {np.median(e):.3e}")
    assert np.isfinite(got).all() and e.max() <= 1e-4


def test_state_fp32_differs_from_fp64_state_by_rounding(erx):
    """The two storage types give scores that differ (the FP32 path really runs) by far
    less than the parity bound."""
    b, p, T = 108, 640, 60
    sc = datagen.make_scene(72, 0, b, p, T)
    X = datagen.lines(sc, 0, T)[0].cuda()
    out = {}
    for f32 in (False, True):
        det = erx.Detector(b, p, 0.1, precision="fp32", state_fp32=f32, block_lines=16)
        det.push(X)
        out[f32] = det.scores().cpu().numpy().astype(np.float64)
    d = rel_err(out[True], out[False])
    log(f"fp32 vs fp64 state: max {d.max():.3e}")
    assert 0.0 < d.max() <= 1e-4


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_mixed_pattern_error_report(erx, prec):
    """The whole precision pattern: 16-bit Gram, FP32 state, FP32 Cholesky with an FP64
    re-factor above a condition estimate of 1e6; error per stream against the oracle."""
    specs = [(108, 640, 80, "f32", 0.1), (224, 1024, 40, "f32", 0.1), (300, 520, 24, "u16", 0.1),
             (37, 301, 70, "u16", 0.3)]
    for i, (b, p, T, storage, a) in enumerate(specs):
        sc = datagen.make_scene(73, i, b, p, T, storage=storage, momentum=a)
        X, _ = datagen.lines(sc, 0, T)
        det = erx.Detector(b, p, a, dtype=storage, precision=prec, state_fp32=True, fp64_cond_threshold=1e6,
                           block_lines=32, scan_lines=16)
        det.push(X.cuda())
        got = det.scores().cpu().numpy()
        ref = oracle.run(datagen.storage_to_float64(X, storage), a, 1e-5, history=True)
        rep = report(got, ref["delta"])
        kap = kappa_max(ref)
        st = det.stats()
        log(f"  {prec} b={b} p={p} T={T} {storage}: max {rep['max']:.2e} p99 {rep['p99']:.2e} "
            f"median {rep['median']:.2e} kappa_max {kap:.3g} fp64 re-factors {st['fp64_refactors']}")
        scale = max(1.0, kap / KAPPA_REF)
        mx, p99 = BOUNDS[prec]
        assert rep["max"] <= mx * scale and rep["p99"] <= p99 * scale, (b, rep, kap)


def test_batch_state_fp32(erx):
    """Uneven streams (two of at most 16 bands, which take the general path with FP32
    storage), pushed in two halves, with FP32 and with FP64 state: split-FP16 Gram with
    every line factored in FP64, and the BF16 pattern with the FP32 Cholesky and its
    FP64 re-factor above 1e6.  Per-stream error report against the oracle."""
    specs = [(37, 300, 40, 0.1), (100, 130, 25, 0.3), (16, 640, 60, 0.2), (5, 256, 50, 0.05),
             (224, 256, 12, 0.1)]
    data = []
    for i, (b, p, T, a) in enumerate(specs):
        sc = datagen.make_scene(74, i, b, p, T, storage="u16", momentum=a)
        data.append(datagen.lines(sc, 0, T)[0])
    refs = [oracle.run(datagen.storage_to_float64(data[s], "u16"), specs[s][3], 1e-5, history=True)
            for s in range(len(specs))]
    kaps = [kappa_max(r) for r in refs]
    for prec, thr in (("split16", 0.0), ("bf16", 1e6)):
        rep = {}
        for f32 in (False, True):
            bt = erx.Batch([s[0] for s in specs], [s[1] for s in specs], [s[3] for s in specs], dtype="u16",
                           precision=prec, fp64_cond_threshold=thr, state_fp32=f32, block_lines=64,
                           scan_lines=16, small_path=1 if f32 else 0)  # both runs on the general path
            half = [x[: x.shape[0] // 2] for x in data]
            rest = [x[x.shape[0] // 2:] for x in data]
            bt.push([x.cuda() for x in half])
            first = [o.cpu().numpy() for o in bt.scores()]
            bt.push([x.cuda() for x in rest])
            second = [o.cpu().numpy() for o in bt.scores()]
            rep[f32] = [report(np.concatenate([first[s], second[s]]), refs[s]["delta"]) for s in range(len(specs))]
            if f32:
                for s, (b, p, T, a) in enumerate(specs):
                    t, mu, K = bt.state(s)
                    assert t == T
                    np.testing.assert_allclose(mu, refs[s]["mu_hist"][-1], rtol=1e-5, atol=1e-7)
        for s, (b, p, T, a) in enumerate(specs):
            r32, r64 = rep[True][s], rep[False][s]
            scale = max(1.0, kaps[s] / KAPPA_REF)
            log(f"  batch {prec} stream {s} b={b} p={p}: FP32 state max {r32['max']:.2e} p99 {r32['p99']:.2e} | "
                f"FP64 state max {r64['max']:.2e} p99 {r64['p99']:.2e} | kappa_max {kaps[s]:.3g}")
            assert r32["max"] <= r64["max"] + 1e-4 * scale, (prec, s, r32, r64)
            if prec == "split16":
                assert r32["max"] <= 1e-4 * scale, (s, r32)
            else:
                assert r32["max"] <= BOUNDS["bf16"][0] * scale, (s, r32)


def test_state_fp32_get_set_round_trip(erx):
    """set_state rounds the given background to FP32 once; get_state returns it; pushing
    on from it matches the oracle started from the same background."""
    b, p, T = 40, 200, 30
    sc = datagen.make_scene(75, 0, b, p, 2 * T)
    X = datagen.lines(sc, 0, 2 * T)[0].numpy()
    st = oracle.Stream(b, p, 0.1)
    st.push(X[:T])
    t0, mu, K = st.state()
    det = erx.Detector(b, p, 0.1, state_fp32=True)
    det.set_state(t0, mu, K)
    t1, mu1, K1 = det.state()
    assert t1 == t0
    np.testing.assert_array_equal(mu1, mu.astype(np.float32).astype(np.float64))
    Ku = np.triu(K) + np.triu(K, 1).T  # the library keeps the upper triangle
    np.testing.assert_array_equal(K1, Ku.astype(np.float32).astype(np.float64))
    det.push(torch.from_numpy(X[T:]).cuda())
    got = det.scores().cpu().numpy()
    want = st.push(X[T:])["delta"]
    e = rel_err(got, want)
    log(f"resume from FP32 state: max err {e.max():.3e}")
    assert e.max() <= 1e-4
