"""The paper's comparison backgrounds through the C ABI against their FP64 references
(oracle/variants.py): IMC ("No EMAs", equal weights over all lines so far) per pixel
within 1e-4, its exported state against the pooled sample statistics, chunked pushes
and a state round trip."""
import sys

import numpy as np
import pytest
import torch

import datagen
from oracle import srp as oracle_srp
from oracle import variants as V

pytestmark = pytest.mark.gpu
TOL = 1e-4


def log(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def erx():
    import paper_2408_14947_amd as m
    m.load()
    return m


def rel_err(got, want):
    return np.abs(np.asarray(got, np.float64) - want) / np.maximum(np.abs(want), 1.0)


@pytest.mark.parametrize("b,p,T,blk,seg,chunks", [(16, 100, 50, 2048, 64, 1), (40, 200, 90, 32, 8, 3),
                                                  (108, 640, 60, 2048, 16, 2), (224, 300, 40, 24, 7, 1)])
def test_imc_matches_reference(erx, b, p, T, blk, seg, chunks):
    log(f"IMC b={b} p={p} T={T} block_lines={blk} scan_lines={seg} pushes={chunks}")
    scene = datagen.make_scene(51, b, b, p, T, drift=True)
    X, _ = datagen.lines(scene, 0, T)
    det = erx.Detector(b, p, 0.1, background="imc", block_lines=blk, scan_lines=seg)
    Xd = X.cuda()
    cuts = np.linspace(0, T, chunks + 1).astype(int)
    got = []
    for a, c in zip(cuts[:-1], cuts[1:]):
        det.push(Xd[a:c])
        got.append(det.scores().cpu().numpy())
    got = np.concatenate(got)
    want = V.imc_run(X.numpy())
    err = rel_err(got, want)
    t, mu, K = det.state()
    mu_r, K_r = V.imc_background(X.numpy(), T - 1)
    kerr = np.abs(K - K_r).max() / np.abs(K_r).max()
    log(f"  max err {err.max():.3e}  state: mean {np.abs(mu - mu_r).max():.2e}  cov {kerr:.2e}")
    assert err.max() <= TOL
    assert t == T and np.abs(mu - mu_r).max() <= 1e-6 and kerr <= 1e-6


def test_imc_state_round_trip_and_srp(erx):
    """Setting the exported IMC state on a fresh detector continues the stream; IMC also
    runs behind the projection of Sec. III-B (the paper's ablation configuration)."""
    log("IMC state round trip; IMC with a 5-dimensional projection")
    b, p, T = 32, 150, 40
    scene = datagen.make_scene(52, 0, b, p, T)
    X, _ = datagen.lines(scene, 0, T)
    Xd = X.cuda()
    a = erx.Detector(b, p, 0.1, background="imc")
    a.push(Xd[:25])
    t, mu, K = a.state()
    c = erx.Detector(b, p, 0.1, background="imc")
    c.set_state(t, mu, K)
    c.push(Xd[25:])
    got = c.scores().cpu().numpy()
    want = V.imc_run(X.numpy())[25:]
    log(f"  continued after set_state: max err {rel_err(got, want).max():.3e}")
    assert rel_err(got, want).max() <= TOL
    d = erx.Detector(b, p, 0.1, background="imc", srp_dims=5, srp_seed=9)
    d.push(Xd)
    got = d.scores().cpu().numpy()
    Z = oracle_srp.project(X.numpy(), oracle_srp.srp_matrix(b, 5, 9))
    want = V.imc_run(Z)
    log(f"  IMC + SRP d=5: max err {rel_err(got, want).max():.3e}")
    assert rel_err(got, want).max() <= TOL


@pytest.mark.parametrize("b,p,T,W,ridge,blk,pushes", [(8, 64, 40, 9, 0.0, 2048, 1), (40, 200, 70, 15, 1e-5, 16, 3),
                                                      (108, 200, 150, 99, 0.0, 64, 2), (224, 160, 120, 99, 0.0, 2048, 1),
                                                      (30, 100, 12, 1, 0.0, 5, 1), (20, 50, 30, 5, 0.0, 3, 4)])
def test_rx_baseline_matches_reference(erx, b, p, T, W, ridge, blk, pushes):
    log(f"RX Baseline b={b} p={p} T={T} window={W} ridge={ridge} block_lines={blk} pushes={pushes}")
    scene = datagen.make_scene(53, b, b, p, T, drift=True)
    X, _ = datagen.lines(scene, 0, T)
    det = erx.RXBaseline(b, p, window=W, ridge=ridge, block_lines=blk, scan_lines=8)
    Xd = X.cuda()
    cuts = np.linspace(0, T, pushes + 1).astype(int)
    firsts, outs = [], []
    for a, c in zip(cuts[:-1], cuts[1:]):
        det.push(Xd[a:c])
        f, s = det.scores()
        if s.shape[0]:
            firsts.append(f)
            outs.append(s)
    got = np.concatenate(outs)
    first, want = V.rx_baseline_run(X.numpy(), window=W, ridge=ridge)
    err = rel_err(got, want)
    log(f"  first scored line {firsts[0]} (ref {first}), {got.shape[0]} lines, max err {err.max():.3e}")
    assert firsts[0] == first and got.shape == want.shape
    assert err.max() <= TOL
