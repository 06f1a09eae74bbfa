#!/usr/bin/env python3
"""Throughput of the ERX hot path on one MI355X.

One step pushes the whole 20000-line x 1024-pixel x 224-band FP32 scan
(synthetic, drifting mixture background, 0.2 % anomalies in 3x3 patches)
through the detector: per-line mean and Gram, moving-average scan, Cholesky
and inverse factor, scoring.  Inputs are generated on the GPU and resident in
HBM before the timed region.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ERX pixels/s + lines/s at 108/224 bands; mixed/batched vs plain FP32 at stated err"
PEAK = {"fp32_mfma_tflops": 157.3, "fp64_tflops": 78.6, "hbm_gbs": 8000.0}


def kernel_work(name, b, p):
    """(bound, algorithmic amount per line, unit) of one kernel."""
    if name == "gram":       # symmetric half of X^T X: p * b(b+1)/2 multiply-adds
        return "mfma", p * b * (b + 1), "flop"
    if name == "score":      # lower-triangular L^-1 r per pixel, residual, squares and sum
        return "mfma", p * b * (b + 1) + 3 * p * b, "flop"
    if name in ("chol_fp32", "chol_fp64"):  # Cholesky + triangular inverse
        return "mfma", 2 * b ** 3 / 3, "flop"
    if name in ("scan_local",):             # read + write the FP64 packed statistics
        e = ((b + 15) // 16) * ((b + 15) // 16 + 1) // 2 * 256 + 16 * ((b + 15) // 16)
        return "hbm", 2 * 8 * e, "byte"
    if name == "scan_carry":
        return "hbm", 0, "byte"
    return "hbm", 4 * p, "byte"


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--block-lines", type=int, default=4096)
    ap.add_argument("--fp64-threshold", type=float, default=None,
                    help="condition-estimate threshold for the FP64 re-factor (library default if unset)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-108", action="store_true", help="skip the 108-band side measurement")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one device-to-device copy of BYTES bytes (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters against a known traffic) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent streams and line blocks would shard across GPUs, see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n}))
        return

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
    bound, per_line, unit = kernel_work(dom, b, p)
    n_l, tot_ms = prof[dom]
    lines_per_launch = T * args.steps / n_l
    work_launch = per_line * lines_per_launch
    avg_s = tot_ms / n_l / 1e3
    if unit == "flop":
        achieved = work_launch / avg_s / 1e12
        peak = PEAK["fp32_mfma_tflops"]
        runit = "TFLOP/s"
    else:
        achieved = work_launch / avg_s / 1e9
        peak = PEAK["hbm_gbs"]
        runit = "GB/s"
    for name, kv in kernels.items():
        bd, pl, un = kernel_work(name, b, p)
        lpl = T * args.steps / kv["launches"]
        rate = pl * lpl / (kv["avg_ms"] / 1e3)
        kv["achieved"] = rate / (1e12 if un == "flop" else 1e9)
        kv["unit"] = "TFLOP/s" if un == "flop" else "GB/s"
    roofline = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": runit,
                "frac": round(achieved / peak, 4), "traffic": None, "kernel": dom,
                "work_per_launch": work_launch, "lines_per_launch": lines_per_launch}

    out = {
        "metric": METRIC, "value": pix_s, "unit": "pixels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "long-scan-224: one stream, 20000 lines x 1024 px x 224 bands, f32, "
                               "momentum 0.1, ridge 1e-5, drifting 4-endmember mixture, 0.2% 3x3 patches",
                   "lines": T, "pixels": p, "bands": b, "block_lines": args.block_lines,
                   "fp64_cond_threshold": 0.0 if args.fp64_threshold is None else args.fp64_threshold},
        "lines_per_s": lines_s, "wall_s": wall, "roofline": roofline, "kernels": kernels,
        "fp64_refactors": st["fp64_refactors"], "max_cond": st["max_cond"],
    }
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
        out["cpu_baseline"] = {"value": cl * p, "unit": "pixels/s", "lines_per_s": cl,
                               "cores": oracle.max_threads(), "kind": "oracle",
                               "sample": f"first {done} lines of the same 20000-line scan"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
