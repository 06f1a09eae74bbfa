"""Many uneven streams in shared device passes, against the FP64 oracle and
against single-stream handles."""
import sys

import numpy as np
import pytest
import torch

import datagen
import oracle

pytestmark = pytest.mark.gpu
TOL = 1e-4


def log(msg):
    print(f"[gpu-batch] {msg}", flush=True)


@pytest.fixture(scope="module")
def erx():
    import paper_2408_14947_amd as m
    m.load()
    return m


def rel_err(got, want):
    return np.abs(np.asarray(got, np.float64) - want) / np.maximum(np.abs(want), 1.0)


def make_streams(specs, cfg=21):
    scenes, data = [], []
    for i, (b, p, T, a, kind, storage) in enumerate(specs):
        sc = datagen.make_scene(cfg, i, b, p, T, kind=kind, storage=storage, momentum=a)
        X, _ = datagen.lines(sc, 0, T)
        scenes.append(sc)
        data.append(X)
    return scenes, data


SPECS = [  # bands, pixels, lines, momentum, kind, storage
    (37, 300, 70, 0.1, "mixture", "f32"),
    (100, 130, 45, 0.3, "mixture", "f32"),
    (48, 257, 90, 0.05, "mixture", "f32"),
    (16, 640, 120, 0.2, "gauss", "f32"),
    (5, 96, 33, 1.0, "gauss", "f32"),
    (224, 300, 20, 0.1, "mixture", "f32"),
    (40, 64, 150, 0.1, "mixture", "f32"),
]


@pytest.mark.parametrize("graphs", [False, True])
def test_batch_uneven_streams_match_oracle(erx, graphs):
    log(f"uneven streams, graphs={graphs}")
    scenes, data = make_streams(SPECS)
    bt = erx.Batch([s[0] for s in SPECS], [s[1] for s in SPECS], [s[3] for s in SPECS],
                   block_lines=96, scan_lines=16, graphs=graphs)
    oras = [oracle.Stream(s[0], s[1], s[3], 1e-5) for s in SPECS]
    dev = [X.cuda() for X in data]
    # three pushes of uneven sizes per stream, some empty
    cuts = [[0, 10, 10, 70], [0, 5, 30, 45], [0, 90, 90, 90], [0, 1, 60, 120], [0, 33, 33, 33],
            [0, 7, 13, 20], [0, 64, 100, 150]]
    for k in range(3):
        chunk = [dev[s][cuts[s][k]:cuts[s][k + 1]] for s in range(len(SPECS))]
        bt.push([x if x.shape[0] else None for x in chunk])
        outs = bt.scores()
        for s in range(len(SPECS)):
            n = cuts[s][k + 1] - cuts[s][k]
            if n == 0:
                assert outs[s] is None
                continue
            want = oras[s].push(data[s][cuts[s][k]:cuts[s][k + 1]].numpy())["delta"]
            err = rel_err(outs[s].cpu().numpy(), want).max()
            assert err <= TOL, (k, s, err)
    for s in range(len(SPECS)):
        t, mu, K = bt.state(s)
        assert t == SPECS[s][2]


def test_batch_equals_single_stream_handles(erx):
    log("batch vs single handles")
    specs = SPECS[:4]
    scenes, data = make_streams(specs)
    bt = erx.Batch([s[0] for s in specs], [s[1] for s in specs], [s[3] for s in specs],
                   block_lines=128, scan_lines=16)
    bt.push([X.cuda() for X in data])
    outs = bt.scores()
    for s, (b, p, T, a, _, _) in enumerate(specs):
        det = erx.Detector(b, p, a, block_lines=128, scan_lines=16)
        det.push(data[s].cuda())
        single = det.scores().cpu().numpy()
        assert rel_err(outs[s].cpu().numpy(), single.astype(np.float64)).max() <= 1e-6


def test_graph_replays_match_eager(erx):
    """Passes of identical shape replay one captured graph; eager work and
    synchronisations run between the replays, and every replay is checked."""
    log("graph replay vs eager")
    specs = [(12, 320, 128, 0.15, "gauss", "f32")] * 6
    scenes, data = make_streams(specs, cfg=22)
    dev = [X.cuda() for X in data]
    g = erx.Batch([s[0] for s in specs], [s[1] for s in specs], [s[3] for s in specs],
                  block_lines=96, scan_lines=16, graphs=True)
    e = erx.Batch([s[0] for s in specs], [s[1] for s in specs], [s[3] for s in specs],
                  block_lines=96, scan_lines=16, graphs=False)
    for k in range(4):
        part = [x[32 * k:32 * (k + 1)] for x in dev]
        g.push(part)
        og = g.scores()
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work
        torch.cuda.synchronize()
        e.push(part)
        oe = e.scores()
        for a, b in zip(og, oe):
            assert torch.equal(a, b), k
        del junk


def test_batch_multispectral_f16(erx):
    """Small-band streams stored in FP16 (4..16 bands, per-stream momentum)."""
    log("multispectral f16")
    scs = datagen.config_scenes(4, scale_lines=60, streams=24)
    data = [datagen.lines(sc, 0, sc.lines)[0] for sc in scs]
    bt = erx.Batch([sc.bands for sc in scs], [sc.pixels for sc in scs], [sc.momentum for sc in scs],
                   dtype="f16", block_lines=512, scan_lines=32)
    bt.push([X.cuda() for X in data])
    outs = bt.scores()
    for sc, X, o in zip(scs, data, outs):
        want = oracle.run(datagen.storage_to_float64(X, "f16"), sc.momentum, 1e-5)["delta"]
        assert rel_err(o.cpu().numpy(), want).max() <= TOL


def test_batch_uneven_u16(erx):
    """Uneven band/pixel counts, uint16 counts scaled by 2^-16."""
    log("uneven u16")
    scs = datagen.config_scenes(3, scale_lines=24, streams=6)
    data = [datagen.lines(sc, 0, sc.lines)[0] for sc in scs]
    bt = erx.Batch([sc.bands for sc in scs], [sc.pixels for sc in scs], [sc.momentum for sc in scs],
                   dtype="u16", block_lines=64, scan_lines=8)
    bt.push([X.cuda() for X in data])
    outs = bt.scores()
    for sc, X, o in zip(scs, data, outs):
        want = oracle.run(datagen.storage_to_float64(X, "u16"), sc.momentum, 1e-5)["delta"]
        err = rel_err(o.cpu().numpy(), want).max()
        log(f"  b={sc.bands} p={sc.pixels}: max err {err:.2e}")
        assert err <= TOL


def small_specs(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        b = int(rng.integers(1, 17))
        p = int(rng.choice([2, 17, 96, 300, 1280]))
        T = int(rng.integers(1, 70))
        a = float(rng.choice([1.0, 0.3, 0.05]))
        out.append((b, p, T, a))
    return out


@pytest.mark.parametrize("storage", ["f32", "f16", "u16"])
def test_small_band_fused_path_matches_oracle(erx, storage):
    """Streams of 1..16 bands through the fused one-workgroup-per-stream path,
    pushed in two uneven parts, against the FP64 oracle; state after the pushes."""
    specs = small_specs(40, {"f32": 1, "f16": 2, "u16": 3}[storage])
    log(f"fused small-band path, {storage}, {len(specs)} streams")
    data = []
    for i, (b, p, T, a) in enumerate(specs):
        sc = datagen.make_scene(51, i, b, p, T, kind="gauss", storage=storage, momentum=a)
        data.append(datagen.lines(sc, 0, T)[0])
    bt = erx.Batch([s[0] for s in specs], [s[1] for s in specs], [s[3] for s in specs], dtype=storage,
                   small_path=1)
    dev = [x.cuda() for x in data]
    cut = [T // 3 for (_, _, T, _) in specs]
    oras = [oracle.Stream(b, p, a, 1e-5) for (b, p, T, a) in specs]
    for part in range(2):
        chunk = [x[:k] if part == 0 else x[k:] for x, k in zip(dev, cut)]
        bt.push([c if c.shape[0] else None for c in chunk])
        outs = bt.scores()
        for s, (b, p, T, a) in enumerate(specs):
            lo, hi = (0, cut[s]) if part == 0 else (cut[s], T)
            if hi == lo:
                assert outs[s] is None
                continue
            want = oras[s].push(datagen.storage_to_float64(data[s][lo:hi], storage))["delta"]
            err = rel_err(outs[s].cpu().numpy(), want).max()
            assert err <= TOL, (part, s, b, p, err)
    for s, (b, p, T, a) in enumerate(specs):
        t, mu, K = bt.state(s)
        t_o, mu_o, K_o = oras[s].state()
        assert t == T == t_o
        np.testing.assert_allclose(mu, mu_o, rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(K, K_o, rtol=1e-4, atol=1e-6 * max(1.0, np.abs(K_o).max()))
    assert bt.stats()["fp64_refactors"] == sum(s[2] for s in specs)


def lds_specs(n, seed, esz):
    """Streams whose every line fits the fused path's LDS buffer (at most 40960 bytes, a
    multiple of 16 bytes, so each line of a fresh allocation starts 16-byte aligned)."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        b = int(rng.integers(1, 17))
        p = int(rng.choice([2, 8, 16, 96, 304, 640, 1280]))
        if (p * b * esz) % 16 or p * b * esz > 40960:
            continue
        out.append((b, p, int(rng.integers(1, 60)), float(rng.choice([1.0, 0.3, 0.05]))))
    return out


@pytest.mark.parametrize("storage", ["f32", "f16", "u16"])
def test_small_band_lds_variant_matches_oracle(erx, storage):
    """The fused path with each line held in LDS (lines of at most 40960 bytes on 16-byte
    boundaries), pushed in two uneven parts, against the FP64 oracle and against the
    variant that streams every tile from device memory."""
    esz = 4 if storage == "f32" else 2
    specs = lds_specs(36, {"f32": 11, "f16": 12, "u16": 13}[storage], esz)
    specs[0] = (16, 40960 // (16 * esz), 9, 0.1)  # the largest line the buffer takes
    log(f"fused small-band path, line in LDS, {storage}, {len(specs)} streams")
    data = []
    for i, (b, p, T, a) in enumerate(specs):
        sc = datagen.make_scene(53, i, b, p, T, kind="gauss", storage=storage, momentum=a)
        data.append(datagen.lines(sc, 0, T)[0])
    dev = [x.cuda() for x in data]
    cut = [T // 3 for (_, _, T, _) in specs]
    outs_by_mode = {}
    for mode in (1, 2):
        bt = erx.Batch([s[0] for s in specs], [s[1] for s in specs], [s[3] for s in specs], dtype=storage,
                       small_path=mode)
        got = [[], []]
        for part in range(2):
            chunk = [x[:k] if part == 0 else x[k:] for x, k in zip(dev, cut)]
            bt.push([c if c.shape[0] else None for c in chunk])
            got[part] = [None if o is None else o.cpu().numpy() for o in bt.scores()]
        outs_by_mode[mode] = got
        if mode == 1:
            for s, (b, p, T, a) in enumerate(specs):
                t, mu, K = bt.state(s)
                o = oracle.run(datagen.storage_to_float64(data[s], storage), a, 1e-5, history=True)
                assert t == T
                np.testing.assert_allclose(mu, o["mu_hist"][-1], rtol=1e-5, atol=1e-6)
                np.testing.assert_allclose(K, o["K_hist"][-1], rtol=1e-4,
                                           atol=1e-6 * max(1.0, np.abs(o["K_hist"][-1]).max()))
            assert bt.stats()["fp64_refactors"] == sum(s[2] for s in specs)
    oras = [oracle.Stream(b, p, a, 1e-5) for (b, p, T, a) in specs]
    for part in range(2):
        for s, (b, p, T, a) in enumerate(specs):
            lo, hi = (0, cut[s]) if part == 0 else (cut[s], T)
            o1, o2 = outs_by_mode[1][part][s], outs_by_mode[2][part][s]
            if hi == lo:
                assert o1 is None and o2 is None
                continue
            want = oras[s].push(datagen.storage_to_float64(data[s][lo:hi], storage))["delta"]
            err = rel_err(o1, want).max()
            assert err <= TOL, (part, s, b, p, err)
            assert rel_err(o1, o2.astype(np.float64)).max() <= 2 * TOL, (part, s, b, p)


def test_small_band_fused_path_equals_general_path(erx):
    specs = [(b, 640, 50, 0.1) for b in (3, 8, 12, 16)] * 3
    data = []
    for i, (b, p, T, a) in enumerate(specs):
        sc = datagen.make_scene(52, i, b, p, T, kind="gauss", momentum=a)
        data.append(datagen.lines(sc, 0, T)[0].cuda())
    res = {}
    for mode in (0, 1):
        bt = erx.Batch([s[0] for s in specs], [s[1] for s in specs], [s[3] for s in specs], small_path=mode)
        bt.push(data)
        res[mode] = [o.cpu().numpy().astype(np.float64) for o in bt.scores()]
    for a, b in zip(res[0], res[1]):
        assert rel_err(b, a).max() <= 2 * TOL


def test_small_band_fused_path_not_pd(erx):
    """Ridge 0 and a constant band: every line's covariance is singular; the
    fused path flags the same lines as the oracle and scores them NaN."""
    b, p, T = 6, 64, 5
    rng = np.random.default_rng(7)
    X = rng.normal(0.5, 0.1, size=(T, p, b)).astype(np.float32)
    X[:, :, 2] = 0.25
    bt = erx.Batch([b] * 33, [p] * 33, [0.2] * 33, ridge=0.0, small_path=1)
    dev = torch.from_numpy(X).cuda()
    bt.push([dev] * 33)
    with pytest.raises(erx.ErxError):
        bt.scores(allow_notpd=False)
    outs = bt.scores()
    want = oracle.run(X, 0.2, 0.0)
    assert np.all(want["notpd"])
    assert np.all(np.isnan(outs[0].cpu().numpy()))
    assert bt.stats()["notpd"] == 33 * T
