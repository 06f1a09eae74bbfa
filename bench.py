#!/usr/bin/env python3
"""Throughput of the ERX hot path on one MI355X.

One step pushes the whole 20000-line x 1024-pixel x 224-band FP32 scan
(synthetic, drifting mixture background, 0.2 % anomalies in 3x3 patches)
through the detector: per-line mean and Gram, moving-average scan, Cholesky
and inverse factor, scoring.  Inputs are generated on the GPU and resident in
HBM before the timed region.  Prints one JSON line.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ERX pixels/s + lines/s at 108/224 bands; mixed/batched vs plain FP32 at stated err"
PEAK = {"fp32_mfma_tflops": 157.3, "fp64_tflops": 78.6, "hbm_gbs": 8000.0}
# sources of the kernels the long-scan workload runs (the traffic record is tied to them)
KERNEL_SRC = [os.path.join(ROOT, "paper_2408_14947_amd", "csrc", f)
              for f in ("erx_kernels.hip", "erx_device.h", "erx_score16.hip", "erx_gram8.hip")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_long-scan-224.md")
WORKLOAD = ("long-scan-224: one stream, 20000 lines x 1024 px x 224 bands, f32, momentum 0.1, "
            "ridge 1e-5, drifting 4-endmember mixture, 0.2% 3x3 patches")


def kernel_source_hash():
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_kernel(name):
    """Map a device kernel's demangled name to the short name the library's profiler uses."""
    m = re.search(r"erx::(?:\(anonymous namespace\)::)?k_(\w+?)(<([^>]*)>)?\(", name)
    if not m:
        return None
    k = m.group(1)
    if k == "chol":
        return "chol_fp64" if (m.group(3) or "").startswith("double") else "chol_fp32"
    if k == "gram4":  # template arguments <dtype, precision, vec>: precision 0 is the FP32 Gram
        args = (m.group(3) or "").replace(" ", "").split(",")
        return "gram_fp32" if len(args) > 1 and args[1] == "0" else "gram"
    # the library's profiler names: the split-FP16 score kernel is "score", the FP32 one runs
    # after it for the lines it flags
    return {"gram4": "gram", "gram8": "gram", "score16": "score", "score": "score_fp32_redo"}.get(k, k)


def _csv_rows(d, suffix):
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)):
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    return rows


def summarize_trace(d, command, workload=WORKLOAD):
    """Markdown table of rocprofv3's kernel statistics (--kernel-trace --stats -f csv)."""
    rows = _csv_rows(d, "kernel_stats.csv")
    if not rows:
        sys.exit(f"no *kernel_stats.csv under {d}")
    out = ["# Kernel trace: " + workload, "", "Command (repository root on the GPU host):", "",
           "```", command, "```", "",
           f"Kernel source sha256[:16] = {kernel_source_hash()}", "",
           "| kernel | calls | total_ms | avg_us | min_us | max_us | pct |", "|---|---|---|---|---|---|---|"]
    # several instantiations of one kernel keep their template arguments apart
    shorts = [short_kernel(r["Name"]) for r in rows]
    dup = {k for k in shorts if k and shorts.count(k) > 1}

    def label(name):
        k = short_kernel(name)
        if k is None:
            return name[:60] + ("..." if len(name) > 60 else "")
        if k in dup:
            m = re.search(r"erx::(?:\(anonymous namespace\)::)?k_(\w+?)<([^>]*)>", name)
            if not m:
                return k
            # the 128-band Gram kernel keeps its own name beside the 64-band one
            return f"{'gram8' if m.group(1) == 'gram8' else k}<{m.group(2).replace(' ', '')}>"
        return k

    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        nm = label(r["Name"])
        out.append(f"| {nm} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                   f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def summarize_counters(dirs, command, copy_bytes, block_lines):
    """HBM traffic per dispatch from one FETCH_SIZE and one WRITE_SIZE pass.

    Each pass also ran a plain device copy of copy_bytes; the ratio of the known bytes to what
    the counter reports for that copy scales the counter for the library's kernels."""
    per = {}     # counter -> kernel -> [KiB per dispatch]
    copy = {}    # counter -> KiB of the calibration copy
    for d in dirs:
        for r in _csv_rows(d, "counter_collection.csv"):
            cn, v, nm = r["Counter_Name"], float(r["Counter_Value"]), r["Kernel_Name"]
            k = short_kernel(nm)
            if k:
                per.setdefault(cn, {}).setdefault(k, []).append(v)
            elif "neg_kernel" in nm:
                copy[cn] = max(copy.get(cn, 0.0), v)
    rec = {"source_sha256": kernel_source_hash(), "block_lines": block_lines,
           "copy_bytes": copy_bytes, "scale": {}, "kernels": {}}
    for cn in ("FETCH_SIZE", "WRITE_SIZE"):
        if cn not in copy:
            sys.exit(f"calibration copy not found for {cn}")
        rec["scale"][cn] = copy_bytes / (copy[cn] * 1024.0)
    for cn, ks in per.items():
        for k, vals in ks.items():
            kb = sum(vals) / len(vals)
            e = rec["kernels"].setdefault(k, {"dispatches": len(vals)})
            e[cn.lower() + "_kib"] = kb
            e[cn.lower().replace("_size", "") + "_bytes"] = kb * 1024.0 * rec["scale"][cn]
    for e in rec["kernels"].values():
        e["bytes"] = e.get("fetch_bytes", 0.0) + e.get("write_bytes", 0.0)
    out = ["# HBM traffic per dispatch: " + WORKLOAD, "", "Commands (repository root on the GPU host):",
           "", "```", command, "```", "",
           f"Calibration: a plain device copy of {copy_bytes} bytes reads FETCH_SIZE = "
           f"{copy['FETCH_SIZE']:.0f} KiB and writes WRITE_SIZE = {copy['WRITE_SIZE']:.0f} KiB; "
           f"scale factors {rec['scale']['FETCH_SIZE']:.4f} (fetch), {rec['scale']['WRITE_SIZE']:.4f} (write).",
           "", "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled MB read | scaled MB written |",
           "|---|---|---|---|---|---|"]
    for k, e in sorted(rec["kernels"].items(), key=lambda kv: -kv[1]["bytes"]):
        out.append(f"| {k} | {e['dispatches']} | {e.get('fetch_size_kib', 0):.0f} | "
                   f"{e.get('write_size_kib', 0):.0f} | {e.get('fetch_bytes', 0) / 1e6:.1f} | "
                   f"{e.get('write_bytes', 0) / 1e6:.1f} |")
    out += ["", "Machine-readable record (read by bench.py while the kernel source hash matches):", "",
            "```json", json.dumps(rec), "```"]
    return "\n".join(out)


def load_traffic(kernel, block_lines):
    """Scaled HBM bytes per launch of `kernel`, or None when the counters are stale or missing."""
    try:
        txt = open(TRAFFIC_FILE).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", txt, re.S).group(1))
    except (OSError, AttributeError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash() or rec.get("block_lines") != block_lines:
        return None
    if kernel == "gram":  # the library's Gram launch is the split-FP16 pass plus the FP32 pass it leaves
        es = [rec["kernels"][k] for k in ("gram", "gram_fp32") if k in rec["kernels"]]
        return sum(e["bytes"] for e in es) if es else None
    e = rec["kernels"].get(kernel)
    return None if e is None else e["bytes"]


# dense peaks of the units each kernel computes on (TFLOP/s): FP32 MFMA, FP64 MFMA, FP16 MFMA;
# a split-FP16 product takes three FP16 products, so its algorithmic flops meet a third of it
MFMA_PEAK = {"fp32": 157.3, "fp64": 78.6, "bf16": 2500.0, "fp16": 2500.0, "split16": 2500.0 / 3.0}


def kernel_work(name, b, p, gram="split16", score="split16", state_bytes=8):
    """Algorithmic work of one kernel per line: {"flop": F, "byte": B, "peak_tflops": P} with P the
    dense peak of the unit it computes on (None for a kernel with no arithmetic to speak of)."""
    nt = (b + 15) // 16
    ntl = nt * (nt + 1) // 2
    e = ntl * 256 + 16 * nt                     # packed statistics per line
    line = p * b * 4                            # one FP32 line
    if name == "gram":       # symmetric half of X^T X: p * b(b+1)/2 multiply-adds; line in, statistics out
        return {"flop": p * b * (b + 1), "byte": line + e * state_bytes, "peak_tflops": MFMA_PEAK[gram]}
    if name == "score":      # L^-1 r per pixel, residual, squares and sum
        return {"flop": p * b * (b + 1) + 3 * p * b, "byte": line + 4 * p + ntl * 256 * 4 + 16 * nt * 4,
                "peak_tflops": MFMA_PEAK["split16" if score == "split16" else "fp32"]}
    if name == "score_fp32_redo":  # only the lines the split kernel flagged: no per-line figure
        return {"flop": 0, "byte": 0, "peak_tflops": None}
    if name in ("chol_fp32", "chol_fp64"):      # Cholesky + triangular inverse; statistics in, factor out
        return {"flop": 2 * b ** 3 / 3, "byte": 2 * e * state_bytes + ntl * 256 * 4,
                "peak_tflops": MFMA_PEAK["fp64" if name == "chol_fp64" else "fp32"]}
    if name == "scan_local":                    # read + write the packed statistics
        return {"flop": 0, "byte": 2 * state_bytes * e, "peak_tflops": None}
    if name == "scan_carry":
        return {"flop": 0, "byte": 0, "peak_tflops": None}
    return {"flop": 0, "byte": 4 * p, "peak_tflops": None}


def roof(work, lines, seconds):
    """The binding roof of a kernel that did `work` per line for `lines` lines in `seconds`:
    the larger of its compute floor and its HBM floor, with what it achieved against it."""
    t_mem = work["byte"] * lines / (PEAK["hbm_gbs"] * 1e9)
    t_cmp = work["flop"] * lines / (work["peak_tflops"] * 1e12) if work["peak_tflops"] else 0.0
    if t_cmp > t_mem:
        ach = work["flop"] * lines / seconds / 1e12
        return {"bound": "mfma", "achieved": ach, "peak": work["peak_tflops"], "unit": "TFLOP/s",
                "frac": ach / work["peak_tflops"], "floor_ms": t_cmp * 1e3}
    ach = work["byte"] * lines / seconds / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": PEAK["hbm_gbs"], "unit": "GB/s",
            "frac": ach / PEAK["hbm_gbs"], "floor_ms": t_mem * 1e3}


def time_workload(erx, torch, X, b, p, momentum, steps, warmup, block_lines, stream, profile, **kw):
    det = erx.Detector(b, p, momentum, block_lines=block_lines, stream=stream.cuda_stream, **kw)
    for _ in range(warmup):
        det.push(X)
    det.synchronize()
    if profile:
        det.profile(True)
        det.profile_read()
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        det.push(X)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms = ev0.elapsed_time(ev1)
    prof = det.profile_read() if profile else {}
    st = det.stats()
    det.close()
    return ms, wall, prof, st


def tune_leg(erx, torch, X, b, p, momentum, args, stream, ms_default):
    """The autotuner on the long-scan shape (one stream) and on the multispectral batch shape
    (1024 streams of 16 bands, FP16), then the long-scan steps again with the tuned setting."""
    import tempfile
    res = {}
    with tempfile.TemporaryDirectory() as tmp:
        cache = os.path.join(tmp, "tune.json")
        t0 = time.perf_counter()
        r = erx.autotune(b, p, momentum, cache=cache)
        res["long_scan"] = dict(r, tuning_s=time.perf_counter() - t0)
        t0 = time.perf_counter()
        rb = erx.autotune(16, 1280, 0.1, dtype="f16", nstreams=1024, cache=cache)
        res["multispectral_batch_b16"] = dict(rb, tuning_s=time.perf_counter() - t0)
    torch.cuda.empty_cache()
    ms, _, _, _ = time_workload(erx, torch, X, b, p, momentum, args.steps, 1, r["block_lines"], stream,
                                profile=False, scan_lines=r["scan_lines"], score_tiles=r["score_tiles"],
                                gram_macro=r["gram_macro"])
    res["long_scan"]["ms_per_step_tuned"] = ms / args.steps
    res["long_scan"]["ms_per_step_default"] = ms_default
    return res


def batched_leg(erx, torch, cfg, T, stream, mixed, n_check):
    """Many independent streams of one workload configuration, each cut to T lines (0: the
    configured lengths): the batched path (shared passes, graph replay) against one handle per
    stream, each pushed and timed in turn.  Each is timed on its second push of the same
    lines (graphs captured and states warm).  The score error against the FP64 oracle is
    taken on n_check sampled streams (the one with the most bands x pixels included);
    optionally the mixed configuration (BF16 Gram, FP32 covariance state, FP32 Cholesky with
    FP64 re-factor above a condition estimate of 1e6) with the same checks."""
    import numpy as np
    import datagen
    scenes = datagen.config_scenes(cfg, scale_lines=T if T > 0 else None)
    storage = scenes[0].storage
    print(f"[bench] generating {datagen.CONFIGS[cfg]['name']}: {len(scenes)} streams", file=sys.stderr, flush=True)
    with torch.cuda.stream(stream):
        data = [datagen.lines(sc, 0, sc.lines, device="cuda", span=2048)[0] for sc in scenes]
    torch.cuda.synchronize()
    B = [sc.bands for sc in scenes]
    Pp = [sc.pixels for sc in scenes]
    A = [sc.momentum for sc in scenes]
    n_lines = sum(x.shape[0] for x in data)
    n_pix = sum(x.shape[0] * x.shape[1] for x in data)
    in_bytes = sum(x.numel() * x.element_size() for x in data)
    rng = np.random.default_rng(7 + cfg)
    big = int(np.argmax([b_ * p_ for b_, p_ in zip(B, Pp)]))
    check = sorted({big, *rng.choice(len(scenes), size=min(n_check, len(scenes)) - 1, replace=False).tolist()})

    def timed(fn):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1)

    def run_batch(**kw):
        """First push from a fresh state (captures the pass graphs), then the same lines again
        (graph replay; the states continue): the second push is timed."""
        bt = erx.Batch(B, Pp, A, dtype=storage, block_lines=8192, stream=stream.cuda_stream, **kw)
        bt.push(data)
        first = bt.scores(streams=check)
        first = {s_: first[s_][:32].clone() for s_ in check}
        torch.cuda.synchronize()
        ms = timed(lambda: bt.push(data))
        second = bt.scores(streams=check)
        second = {s_: second[s_][-32:].clone() for s_ in check}
        torch.cuda.synchronize()
        bt.close()
        return ms, (first, second)

    def check_streams(sc_pair):
        """First 32 lines of the first push against the oracle from line 0 (exact), last 32
        lines of the second push (stream lines 2T-32..2T-1 of the data pushed twice) against
        the oracle started fresh 25 / momentum lines earlier."""
        import datagen as dg
        import oracle
        first, second = sc_pair
        per = []
        for s_ in check:
            sc, x = scenes[s_], data[s_]
            Tn = x.shape[0]
            k = min(32, Tn)
            want0 = oracle.run(dg.storage_to_float64(x[:k], storage), sc.momentum, 1e-5)["delta"]
            warm = int(np.ceil(25.0 / sc.momentum))
            a = max(0, 2 * Tn - k - warm)  # window start in the twice-pushed stream
            parts = ([x[a:Tn]] if a < Tn else []) + [x[max(a - Tn, 0):Tn]]
            xw = dg.storage_to_float64(torch.cat(parts), storage)
            want1 = oracle.run(xw, sc.momentum, 1e-5)["delta"][-k:]
            got = np.concatenate([first[s_][:k].double().cpu().numpy(), second[s_][-k:].double().cpu().numpy()])
            e = err_stats(got, np.concatenate([want0, want1]))
            per.append(dict(stream=s_, bands=sc.bands, pixels=sc.pixels, lines=Tn,
                            momentum=round(sc.momentum, 4), oracle_window_lines=int(xw.shape[0]), **e))
        return per

    ms_b, ref = run_batch()
    per_plain = check_streams(ref)
    del ref
    # one handle per stream, pushed one after another (each timed alone, summed)
    ms_1 = 0.0
    for b_, p_, a_, x in zip(B, Pp, A, data):
        d = erx.Detector(b_, p_, a_, dtype=storage, block_lines=min(max(x.shape[0], 1), 4096),
                         stream=stream.cuda_stream)
        d.push(x)  # first push, then the same lines again, timed
        ms_1 += timed(lambda: d.push(x))
        d.close()
    name = datagen.CONFIGS[cfg]["name"]
    res = {"workload": f"{name}: {len(scenes)} streams x " + (f"{T} lines (cap)" if T > 0 else "configured lengths")
                       + f", {storage}",
           "lines_per_stream": T if T > 0 else "configured", "streams": len(scenes), "lines": n_lines,
           "pixels": n_pix, "input_bytes": in_bytes,
           "batched": {"ms": ms_b, "lines_per_s": n_lines / (ms_b / 1e3), "pixels_per_s": n_pix / (ms_b / 1e3),
                       "hbm_gbs_in_plus_scores": (in_bytes + 4 * n_pix) / (ms_b / 1e3) / 1e9},
           "one_handle_per_stream": {"ms": ms_1, "lines_per_s": n_lines / (ms_1 / 1e3),
                                     "pixels_per_s": n_pix / (ms_1 / 1e3)},
           "batched_speedup": ms_1 / ms_b,
           "err_vs_oracle_per_stream": per_plain,
           "err_vs_oracle_worst": {k: max(r[k] for r in per_plain) for k in ("max", "p99", "median")}}
    res["batched"]["hbm_frac"] = res["batched"]["hbm_gbs_in_plus_scores"] / PEAK["hbm_gbs"]
    if mixed:
        ms_m, got = run_batch(precision="bf16", fp64_cond_threshold=1e6, cond_estimate=1, state_fp32=True)
        per = check_streams(got)
        del got
        res["mixed_bf16"] = {"config": "BF16 Gram, FP32 state, FP32 Cholesky + FP64 above 1e6", "ms": ms_m, "pixels_per_s": n_pix / (ms_m / 1e3), "speedup_vs_batched_plain": ms_b / ms_m,
                             "err_vs_oracle_per_stream": per,
                             "err_vs_oracle_worst": {k: max(r[k] for r in per) for k in ("max", "p99", "median")},
                             "bound": {"max": MIXED_BOUNDS["bf16"][0], "p99": MIXED_BOUNDS["bf16"][1]}}
    del data
    torch.cuda.empty_cache()
    return res


def srp_matrix(bands, d, seed):
    """Sparse random projection of Sec. III-B as a d x b matrix (the transpose of the paper's
    b x d W): entries sqrt(s/d) * {+1, 0, -1} with probabilities 1/(2s), 1 - 1/s, 1/(2s),
    s = sqrt(b)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    s = np.sqrt(bands)
    u = rng.random((d, bands))
    w = np.where(u < 1 / (2 * s), 1.0, np.where(u < 1 / s, -1.0, 0.0))
    return np.sqrt(s / d) * w


def surrogate_leg(erx, torch, stream, train_lines, heldout, heldout_lines):
    """Learned projection surrogate at the surrogate workload's sizes: training on
    `train_lines` fresh lines of the 640-pixel mixture generator per band count (64-line
    streams, targets from the plain GPU path); the drift threshold set from validation
    streams (1.5 x the largest check drift there); then `heldout` held-out streams of
    `heldout_lines` lines x 1024 pixels, one at a time: the error against plain ERX (the
    judge), per-line rank agreement and anomaly AUC for the trained surrogate (unchecked
    and checked), ERX on a sparse random projection (Sec. III-B) and on a dense Gaussian
    projection to the same 16 dimensions, each given its best constant correction, and
    throughput next to plain ERX."""
    import numpy as np
    import datagen
    res = {}
    a = datagen.CONFIGS[5]["momentum"]
    p_tr, T_tr, p_h = datagen.CONFIGS[5]["pixels"], 64, 1024
    steps = max(1, train_lines // T_tr)

    def ranks(x):
        return torch.argsort(torch.argsort(x, dim=-1), dim=-1).double()

    def auc(score, mask):
        s = score.flatten().double()
        m = mask.flatten()
        r = ranks(s[None])[0] + 1
        npos, nneg = int(m.sum()), int((~m).sum())
        return float((r[m].sum() - npos * (npos + 1) / 2) / (npos * nneg))

    def spearman(got, ref):
        rg, rr = ranks(got.double()), ranks(ref.double())
        rg -= rg.mean(-1, keepdim=True)
        rr -= rr.mean(-1, keepdim=True)
        return float(((rg * rr).sum(-1) / torch.sqrt((rg * rg).sum(-1) * (rr * rr).sum(-1))).mean())

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        out = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1)

    def plain_scores(X):
        d = erx.Detector(X.shape[2], X.shape[1], a, block_lines=min(X.shape[0], 4096), stream=stream.cuda_stream)
        out, t = timed(lambda: d.push(X))
        s_ = d.scores().clone()
        d.close()
        return s_, t

    for b in (108, 224):
        print(f"[bench] surrogate b={b}: training on {steps * T_tr} lines", file=sys.stderr, flush=True)
        net = erx.Surrogate(b, seed=b)
        det = erx.Detector(b, p_tr, a, block_lines=T_tr, stream=stream.cuda_stream)
        losses = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            for k in range(steps):
                sc = datagen.make_scene(5, 1000 + k, b, p_tr, T_tr, momentum=a)
                X = datagen.lines(sc, 0, T_tr, device="cuda")[0]
                det.set_state(0)
                det.push(X)
                losses.append(net.train_step(X, det.scores(), a, 3e-3 if k < steps * 3 // 4 else 1e-3))
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        det.close()
        # validation: the drift threshold and the constant corrections of the fixed projections
        rng = np.random.default_rng(8)
        s_ = np.sqrt(b)
        u = rng.random((16, b))
        fixedW = {"srp16": np.sqrt(s_ / 16) * np.where(u < 1 / (2 * s_), 1.0, np.where(u < 1 / s_, -1.0, 0.0)),
                  "gauss16": rng.normal(0, 1 / np.sqrt(16), (16, b))}
        base = net.params()
        val = []
        for i in range(4):
            with torch.cuda.stream(stream):
                X = datagen.lines(datagen.make_scene(5, 70000 + i, b, p_tr, 512, momentum=a), 0, 512,
                                  device="cuda")[0]
            val.append((X, plain_scores(X)[0]))
        fixed = {}
        for name, W in fixedW.items():
            P = {k: np.zeros_like(v) for k, v in base.items()}
            P["W"], P["A1"] = W, base["A1"]
            fn = erx.Surrogate(b)
            fn.set_params(P)
            lr = torch.cat([(torch.log(fn.scores(X, a).double()) - torch.log(R.double())).flatten() for X, R in val])
            P["c2"] = np.array([-float(lr.median())])
            fn.set_params(P)
            fixed[name] = fn
        theta = 0.0
        for X, _ in val:
            sd = erx.SurrogateDetector(net, p_tr, a, drift_threshold=1e9, check_every=32)
            sd.push(X)
            theta = max(theta, 1.5 * sd.drift_stats()["max"])
            sd.close()
        del val
        # held-out streams, one at a time
        names = ("surrogate_checked", "surrogate_unchecked", "srp16", "gauss16")
        lr_s = {k: [] for k in names}
        sp = {k: [] for k in names}
        au = {k: [] for k in names + ("plain",)}
        ms = {"plain": 0.0, "surrogate_checked": 0.0, "surrogate_unchecked": 0.0}
        status = []
        net.scores(torch.zeros((2, p_h, b), device="cuda") + 0.5, a)  # warm-up
        print(f"[bench] surrogate b={b}: {heldout} held-out streams x {heldout_lines} lines", file=sys.stderr,
              flush=True)
        for i in range(heldout):
            with torch.cuda.stream(stream):
                X, M = datagen.lines(datagen.make_scene(5, 90000 + i, b, p_h, heldout_lines, momentum=a), 0,
                                     heldout_lines, device="cuda")
            ref, t = plain_scores(X)
            ms["plain"] += t
            got = {}
            got["surrogate_unchecked"], t = timed(lambda: net.scores(X, a))
            ms["surrogate_unchecked"] += t
            sd = erx.SurrogateDetector(net, p_h, a, drift_threshold=theta, check_every=32)
            _, t = timed(lambda: sd.push(X))
            ms["surrogate_checked"] += t
            got["surrogate_checked"] = sd.scores()
            status.append(sd.status())
            sd.close()
            for name, fn in fixed.items():
                got[name] = fn.scores(X, a)
            au["plain"].append(auc(ref, M))
            for k in names:
                lr = (torch.log(got[k].double()) - torch.log(ref.double())).flatten()
                lr_s[k].append(lr[::8].float())
                sp[k].append(spearman(got[k], ref))
                au[k].append(auc(got[k], M))
            del X, M, ref, got
        npx = heldout * heldout_lines * p_h
        stats = {}
        for k in names:
            e = torch.cat(lr_s[k]).double().abs()
            q = torch.quantile(e[torch.randperm(e.numel(), device=e.device)[:4000000]], 0.99)
            stats[k] = {"median_abs_log_ratio": float(e.median()), "p99_abs_log_ratio": float(q),
                        "mean_line_spearman": float(np.mean(sp[k])), "auc_mean": float(np.mean(au[k]))}
        in_bytes = heldout_lines * p_h * b * 4
        t_unc = ms["surrogate_unchecked"] / heldout / 1e3
        res[f"b{b}"] = {
            "train": {"lines": steps * T_tr, "pixels": p_tr, "lines_per_step": T_tr, "seconds": t_train,
                      "lines_per_s": steps * T_tr / t_train,
                      "loss_first10": float(np.mean(losses[:10])), "loss_last50": float(np.mean(losses[-50:]))},
            "drift_threshold": theta,
            "held_out": f"{heldout} streams x {heldout_lines} lines x {p_h} px, seeds disjoint from training "
                        "and validation",
            "vs_plain": stats, "auc_plain_mean": float(np.mean(au["plain"])),
            "pixels_per_s": {k: npx / (v / 1e3) for k, v in ms.items()},
            "fused_inference_hbm_frac": (in_bytes + heldout_lines * p_h * 4) / t_unc / (PEAK["hbm_gbs"] * 1e9),
            "detector": {"streams_on_surrogate": int(sum(1 for st in status if st["active"])),
                         "checks": int(sum(st["checks"] for st in status)),
                         "drifting_checks": int(sum(st["drifts"] for st in status)),
                         "switched": [st["switched_at"] for st in status if not st["active"]]}}
        net.close()
        for fn in fixed.values():
            fn.close()
        torch.cuda.empty_cache()
    return res


def err_stats(got, want):
    """max / p99 / median of |got - want| / max(|want|, 1) over all pixels given."""
    import numpy as np
    e = (np.abs(np.asarray(got, np.float64) - want) / np.maximum(np.abs(want), 1.0)).ravel()
    return {"max": float(e.max()), "p99": float(np.quantile(e, 0.99)), "median": float(np.median(e)),
            "checked_pixels": int(e.size)}


def oracle_windows(X, storage, momentum, ends, check=32, warm=256):
    """FP64 oracle scores of the `check` lines before each end, each window started fresh
    `warm` lines earlier (from line 0 when that is closer).  A fresh start differs from the
    true background by a weight of (1 - momentum)^warm, far below the error bound once
    warm >= 25 / momentum; windows that start at line 0 are exact.  X: device lines as
    stored; returns {end: float64 [check, p]}."""
    import datagen
    import oracle
    out = {}
    for L in ends:
        a = max(0, L - check - warm)
        xh = datagen.storage_to_float64(X[a:L], storage)
        out[L] = oracle.run(xh, momentum, 1e-5)["delta"][-check:]
    return out


def oracle_error(scores, X, storage, momentum, ends, check=32, warm=256):
    """Score error of GPU scores [T, p] against the oracle windows ending at `ends`."""
    import numpy as np
    ref = oracle_windows(X, storage, momentum, ends, check, warm)
    got = np.concatenate([scores[L - check:L].double().cpu().numpy() for L in ends])
    return err_stats(got, np.concatenate([ref[L] for L in ends]))


def cpu_info():
    import subprocess
    model = ""
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in txt.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except Exception:
        usable = os.cpu_count()
    return {"model": model, "nproc": usable, "cpu_count": os.cpu_count()}


SINGLE_THREAD_SNIPPET = r"""
import sys, time, json
sys.path.insert(0, sys.argv[1])
import numpy as np, datagen, oracle
sc = datagen.config_scenes(2)[0]
n = int(sys.argv[2])
X, _ = datagen.lines(sc, 0, n, device="cpu")
x = X.numpy().astype(np.float64)
s = oracle.Stream(sc.bands, sc.pixels, sc.momentum, 1e-5, nthreads=1)
s.push(x[:8])
t0 = time.perf_counter()
s.push(x[8:])
dt = time.perf_counter() - t0
print(json.dumps({"lines": n - 8, "seconds": dt, "threads": 1}))
"""


def cpu_single_thread(lines=40):
    """The oracle on one host thread, in a child process."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", SINGLE_THREAD_SNIPPET, ROOT, str(lines)], env=env,
                       capture_output=True, text=True, timeout=600)
    return json.loads(r.stdout.strip().splitlines()[-1])


# frozen error bounds of the reduced-precision Gram (max, p99 of the relative score error)
MIXED_BOUNDS = {"bf16": (1e-2, 3e-3), "fp16": (1e-3, 5e-4)}


CHECK_ENDS = (32, 5000, 12000, 20000)  # long-scan windows checked against the oracle


def mixed_leg(erx, torch, X, b, p, momentum, args, stream, plain_ms, plain_prof, ref_windows):
    """BF16 / FP16 Gram with FP32 covariance state and FP32 Cholesky (FP64 re-factor above a
    condition estimate of 1e6) on the same scan: throughput; the score error against the FP64 oracle on the checked
    windows (32 lines ending at each of CHECK_ENDS), and against the plain GPU path over
    every pixel of the scan."""
    import numpy as np
    T = X.shape[0]

    def scores(**kw):
        det = erx.Detector(b, p, momentum, block_lines=args.block_lines, stream=stream.cuda_stream, **kw)
        det.push(X)
        s = det.scores()
        det.synchronize()
        det.close()
        return s

    def vs_oracle(sc):
        got = np.concatenate([sc[L - 32:L].double().cpu().numpy() for L in CHECK_ENDS])
        return err_stats(got, np.concatenate([ref_windows[L] for L in CHECK_ENDS]))

    with torch.cuda.stream(stream):
        ref = scores()
    res = {"plain_ms_per_step": plain_ms, "plain_gram_ms": plain_prof["gram"][1] / plain_prof["gram"][0]}
    for prec in ("bf16", "fp16"):
        kw = dict(precision=prec, fp64_cond_threshold=1e6, cond_estimate=1, state_fp32=True)
        ms, _, prof, st = time_workload(erx, torch, X, b, p, momentum, args.steps, args.warmup,
                                        args.block_lines, stream, profile=True, **kw)
        with torch.cuda.stream(stream):
            got = scores(**kw)
            e = ((got.double() - ref.double()).abs() / ref.double().abs().clamp_min(1.0)).flatten()
            k = max(1, e.numel() // 100)
            p99 = float(torch.topk(e, k).values.min())
            emax, emed = float(e.max()), float(e.median())
        torch.cuda.synchronize()
        gram_ms = prof["gram"][1] / prof["gram"][0]
        flops = kernel_work("gram", b, p)["flop"] * T * args.steps / prof["gram"][0]
        res[prec] = {"ms_per_step": ms / args.steps, "pixels_per_s": T * p * args.steps / (ms / 1e3),
                     "speedup_vs_plain": plain_ms / (ms / args.steps),
                     "gram_ms": gram_ms, "gram_tflops": flops / (gram_ms / 1e3) / 1e12,
                     "gram_peak_tflops": 2500.0,
                     "err_vs_oracle": vs_oracle(got),
                     "err_vs_plain": {"max": emax, "p99": p99, "median": emed},
                     "bound": {"max": MIXED_BOUNDS[prec][0], "p99": MIXED_BOUNDS[prec][1]},
                     "fp64_refactors": st["fp64_refactors"], "max_cond": st["max_cond"],
                     "kernels_ms": {k: v[1] / v[0] for k, v in prof.items()}}
        del got, e
    del ref
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--block-lines", type=int, default=1024,
                    help="lines per device pass of the headline path (the autotuner's choice for this shape)")
    ap.add_argument("--fp64-threshold", type=float, default=None,
                    help="condition-estimate threshold for the FP64 re-factor (library default if unset)")
    ap.add_argument("--precision", default=None, choices=("fp32", "bf16", "fp16", "split16"),
                    help="Gram arithmetic of the headline path (library default, split16, if unset)")
    ap.add_argument("--state-fp32", action="store_true",
                    help="headline path with FP32 statistics, carries and state")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-108", action="store_true", help="skip the 108-band side measurement")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the reduced-precision (BF16 / FP16 Gram) side measurement")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the many-stream side measurements (batched-u16, batched-multispectral-f16)")
    ap.add_argument("--batched-lines", type=int, default=0,
                    help="lines per stream of the batched-u16 measurement (0: the configured 2000-10000)")
    ap.add_argument("--multispectral-lines", type=int, default=0,
                    help="lines per stream of the batched-multispectral-f16 measurement (0: the configured 5000)")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the learned-projection surrogate side measurement")
    ap.add_argument("--surrogate-train-lines", type=int, default=200000,
                    help="training lines per band count of the surrogate measurement")
    ap.add_argument("--surrogate-heldout", type=int, default=32, help="held-out streams of the surrogate measurement")
    ap.add_argument("--surrogate-heldout-lines", type=int, default=5000, help="lines per held-out stream")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="first run one plain device copy of BYTES bytes (a known traffic against "
                         "which the FETCH_SIZE / WRITE_SIZE counters are scaled)")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner leg")
    ap.add_argument("--rocprof-summary", nargs="+", metavar="DIR",
                    help="no GPU: print a markdown summary of rocprofv3 CSV output under DIR(s)")
    ap.add_argument("--rocprof-command", default="", help="command line recorded in the summary")
    ap.add_argument("--rocprof-workload", default=WORKLOAD, help="workload named in a trace summary's title")
    args = ap.parse_args()
    if args.rocprof_summary:
        if args.calibrate_copy:
            print(summarize_counters(args.rocprof_summary, args.rocprof_command, args.calibrate_copy,
                                     args.block_lines))
        else:
            print(summarize_trace(args.rocprof_summary[0], args.rocprof_command, args.rocprof_workload))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent streams and line blocks would shard across GPUs, see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)  # one elementwise kernel: reads and writes n floats
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()

    import datagen
    import paper_2408_14947_amd as erx

    erx.load()
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()  # default priority
    sc = datagen.config_scenes(2)[0]
    T, p, b = sc.lines, sc.pixels, sc.bands
    print(f"[bench] generating {T} x {p} x {b} f32 lines on the GPU", file=sys.stderr, flush=True)
    with torch.cuda.stream(stream):
        X, _ = datagen.lines(sc, 0, T, device="cuda")
    torch.cuda.synchronize()
    print(f"[bench] timing {args.steps} steps after {args.warmup} warm-up steps", file=sys.stderr, flush=True)
    kw = {} if args.fp64_threshold is None else {"fp64_cond_threshold": args.fp64_threshold}
    if args.precision:
        kw["precision"] = args.precision
    if args.state_fp32:
        kw["state_fp32"] = True
    ms, wall, prof, st = time_workload(erx, torch, X, b, p, sc.momentum, args.steps, args.warmup,
                                       args.block_lines, stream, profile=True, **kw)
    ms_step = ms / args.steps
    lines_s = T * args.steps / (ms / 1e3)
    pix_s = lines_s * p

    # roofline of the dominant kernel
    kernels = {}
    for name, (n, tot) in prof.items():
        kernels[name] = {"launches": n, "avg_ms": tot / n, "total_ms": tot}
    dom = max(prof, key=lambda k: prof[k][1])
    # the run's arithmetic (the counter record belongs to the default configuration only)
    wk = {"gram": args.precision or "split16", "state_bytes": 4 if args.state_fp32 else 8}
    default_cfg = not args.precision and not args.state_fp32
    for name, kv in kernels.items():
        lpl = T * args.steps / kv["launches"]
        kv.update({k: v for k, v in roof(kernel_work(name, b, p, **wk), lpl, kv["avg_ms"] / 1e3).items()})
    n_l, tot_ms = prof[dom]
    lines_per_launch = T * args.steps / n_l
    w = kernel_work(dom, b, p, **wk)
    r = roof(w, lines_per_launch, tot_ms / n_l / 1e3)
    roofline = {"bound": r["bound"], "achieved": round(r["achieved"], 3), "peak": r["peak"], "unit": r["unit"],
                "frac": round(r["frac"], 4), "traffic": load_traffic(dom, args.block_lines) if default_cfg else None,
                "traffic_unit": "bytes/launch", "kernel": dom,
                "work_per_launch": (w["byte"] if r["bound"] == "hbm" else w["flop"]) * lines_per_launch,
                "work_unit": "byte" if r["bound"] == "hbm" else "flop", "lines_per_launch": lines_per_launch,
                "floor_ms": r["floor_ms"]}
    # the scoring kernel against its own roof (the brief's scoring target is a fraction of HBM)
    if "score" in prof:
        n_s, tot_s = prof["score"]
        rs = roof(kernel_work("score", b, p, **wk), T * args.steps / n_s, tot_s / n_s / 1e3)
        scoring = {"kernel": "score", "bound": rs["bound"], "achieved": round(rs["achieved"], 3),
                   "peak": rs["peak"], "unit": rs["unit"], "frac": round(rs["frac"], 4),
                   "traffic": load_traffic("score", args.block_lines) if default_cfg else None,
                   "traffic_unit": "bytes/launch"}
    else:
        scoring = None
    if dom == "gram" and wk["gram"] == "split16":
        roofline["note"] = ("split-FP16 Gram: three FP16 products per product, so its compute floor is the "
                            "algorithmic flops at a third of the FP16 peak; its HBM floor (line in, FP64 "
                            "statistics out) is the larger")

    out = {
        "metric": METRIC, "value": pix_s, "unit": "pixels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD,
                   "lines": T, "pixels": p, "bands": b, "block_lines": args.block_lines,
                   "fp64_cond_threshold": 0.0 if args.fp64_threshold is None else args.fp64_threshold,
                   "gram": args.precision or "split16", "state": "fp32" if args.state_fp32 else "fp64"},
        "lines_per_s": lines_s, "wall_s": wall, "roofline": roofline, "scoring_roofline": scoring,
        "kernels": kernels,
        "fp64_refactors": st["fp64_refactors"], "max_cond": st["max_cond"],
    }
    # the headline path's own scores against the FP64 oracle on the checked windows
    print("[bench] FP64 oracle on the checked windows", file=sys.stderr, flush=True)
    ref_windows = oracle_windows(X, "f32", sc.momentum, CHECK_ENDS)
    det = erx.Detector(b, p, sc.momentum, block_lines=args.block_lines, stream=stream.cuda_stream, **kw)
    det.push(X)
    s_plain = det.scores()
    det.synchronize()
    det.close()
    got = np.concatenate([s_plain[L - 32:L].double().cpu().numpy() for L in CHECK_ENDS])
    out["err_vs_oracle"] = dict(err_stats(got, np.concatenate([ref_windows[L] for L in CHECK_ENDS])),
                                windows=f"32 lines ending at each of {list(CHECK_ENDS)}; the oracle starts "
                                        "each window 256 lines earlier (line 0 for the first)",
                                bound=1e-4)
    del s_plain
    if not args.no_mixed:
        out["mixed"] = mixed_leg(erx, torch, X, b, p, sc.momentum, args, stream, ms_step, prof, ref_windows)

    if not args.no_tune:
        print("[bench] autotuning the launch settings", file=sys.stderr, flush=True)
        out["autotune"] = tune_leg(erx, torch, X, b, p, sc.momentum, args, stream, ms_step)
    del X
    torch.cuda.empty_cache()

    if not args.no_108:
        sc1 = datagen.config_scenes(1)[0]
        with torch.cuda.stream(stream):
            X1, _ = datagen.lines(sc1, 0, sc1.lines, device="cuda")
        torch.cuda.synchronize()
        ms1, _, _, _ = time_workload(erx, torch, X1, sc1.bands, sc1.pixels, sc1.momentum,
                                     max(args.steps, 10), args.warmup, 2048, stream, profile=False)
        l1 = sc1.lines * max(args.steps, 10) / (ms1 / 1e3)
        out["plain_108"] = {"workload": "plain-108: 500 lines x 640 px x 108 bands, f32",
                            "lines_per_s": l1, "pixels_per_s": l1 * sc1.pixels,
                            "ms_per_pass": ms1 / max(args.steps, 10)}
        del X1

    if not args.no_batched:
        print("[bench] many-stream workloads", file=sys.stderr, flush=True)
        out["batched_u16"] = batched_leg(erx, torch, 3, args.batched_lines, stream, mixed=True, n_check=4)
        out["batched_multispectral_f16"] = batched_leg(erx, torch, 4, args.multispectral_lines, stream, mixed=False,
                                                       n_check=16)

    if not args.no_surrogate:
        print("[bench] learned projection surrogate", file=sys.stderr, flush=True)
        out["surrogate"] = surrogate_leg(erx, torch, stream, args.surrogate_train_lines, args.surrogate_heldout,
                                         args.surrogate_heldout_lines)

    if not args.no_cpu_baseline:
        import oracle
        print("[bench] timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        s = oracle.Stream(b, p, sc.momentum, 1e-5)
        done, t_cpu = 0, 0.0
        while t_cpu < args.cpu_seconds and done < T:
            Xh, _ = datagen.lines(sc, done, 32, device="cuda")
            xh = Xh.cpu().numpy().astype(np.float64)
            t0 = time.perf_counter()
            s.push(xh)
            t_cpu += time.perf_counter() - t0
            done += 32
        cl = done / t_cpu
        one = cpu_single_thread()
        l1 = one["lines"] / one["seconds"]
        out["cpu_baseline"] = {"value": cl * p, "unit": "pixels/s", "lines_per_s": cl,
                               "cores": oracle.max_threads(), "kind": "oracle",
                               "sample": f"first {done} lines of the same 20000-line scan",
                               "single_thread": {"value": l1 * p, "lines_per_s": l1, "threads": one["threads"],
                                                 "sample": f"{one['lines']} lines of the same scan shape"},
                               "cpu": cpu_info()}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
