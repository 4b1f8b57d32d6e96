#!/usr/bin/env python3
"""Benchmark of the CFOG + 3-D-FFT SSD matching hot path on one MI355X.

One step = the whole hot path on one synthetic pair: CFOG extraction of A and B
(volume + FP64 summed-area table each) and SSD matching of every control point
(FFT correlation, FP64 energies, argmin).  Inputs are resident in HBM before the
timed region starts.

Default workload (plain_2048): one 2048^2 fp32 pair (800 blobs sigma 3-40,
300 rectangles, |sin(3A)| x Gamma(4) speckle, |shift| <= 20), 400 control
points on a 20x20 grid, template 100, search radius 20.

Prints ONE JSON line (rank 0).  `--gpus N` with N > 1 is refused: this build
runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def algorithmic_bytes_per_cp(N: int, r: int, m: int = 9, surfaces: bool = False) -> int:
    """HBM bytes one control point must move at minimum: the template and
    search-window volumes (fp32, m channels), the four SAT corner blocks of the
    (2r+1)^2 window energies (fp64), the CP and the 24-byte result."""
    Ws, K = N + 2 * r, 2 * r + 1
    b = 4 * m * (N * N + Ws * Ws) + 4 * 8 * K * K + 16 + 24
    if surfaces:
        b += 4 * K * K
    return b


def fft_flops_per_cp(N: int, r: int, P: int, m: int = 9) -> float:
    """Flops of the FFT matcher per control point with the 5 n log2 n model per
    complex FFT of length n: per channel, ceil(N/2) + ceil(Ws/2) packed row
    FFTs and 2 (P/2+1) column FFTs, a complex multiply-add per half-spectrum
    point; then (P/2+1) + ceil(K/2) inverse FFTs."""
    Ws, K, PH = N + 2 * r, 2 * r + 1, P // 2 + 1
    f = 5.0 * P * np.log2(P)
    per_ch = ((N + 1) // 2 + (Ws + 1) // 2 + 2 * PH) * f + 8.0 * P * PH
    return m * per_ch + (PH + (K + 1) // 2) * f


def extract_bytes_per_px(m: int = 9) -> int:
    """Image read (4) + volume write (4m) + FP64 SAT write (8)."""
    return 4 + 4 * m + 8


def cpu_baseline(A, B, cps, N, r, budget_s: float = 20.0):
    """The FP64 oracle (CFOG of both images + brute-force SSD) on a bounded
    sample of control points; scaled to CP matches/s of the whole workload."""
    import oracle as O
    t0 = time.perf_counter()
    D1 = O.cfog(A.astype(np.float64))
    D2 = O.cfog(B.astype(np.float64))
    t_ext = time.perf_counter() - t0
    t1 = time.perf_counter()
    n = 0
    for cp in cps:
        O.ssd_surface_direct(D1, D2, cp, N, r)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    t_cp = (time.perf_counter() - t1) / n
    total = t_ext + len(cps) * t_cp
    return dict(value=len(cps) / total, unit="CP matches/s", cores=1, kind="oracle",
                sample=f"FP64 CFOG of both {A.shape[0]}x{A.shape[1]} images ({t_ext:.1f} s) + direct SSD of "
                       f"{n} of {len(cps)} CPs ({t_cp:.3f} s/CP), extrapolated to all {len(cps)} CPs",
                seconds=round(time.perf_counter() - t0, 2))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--path", choices=["plain", "batched"], default="plain")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the timed steps, run one plain device-to-device copy of this many MiB "
                         "(a counter calibration point for HBM traffic)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on exactly one GPU (asked for --gpus {args.gpus}); "
              "the matching path shards by control point and needs no collectives", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1808_06194_amd import cfog, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = synth.PLAIN_2048
    A, B, shift, cps, N, r = synth.plain_workload(w)
    m = 9
    H, W = A.shape
    K = 2 * r + 1
    dA = torch.from_numpy(A).to(dev)
    dB = torch.from_numpy(B).to(dev)
    dcps = torch.from_numpy(cps).to(dev)
    volA = torch.empty((m, H, W), dtype=torch.float32, device=dev)
    volB = torch.empty_like(volA)
    satA = torch.empty((H + 1, W + 1), dtype=torch.float64, device=dev)
    satB = torch.empty_like(satA)
    job = cfog.Job(volA, satA, volB, satB, dcps, N, r)
    flags = cfog.PATH_PLAIN_FFT if args.path == "plain" else cfog.PATH_BATCHED_FFT
    stream = torch.cuda.current_stream()

    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def step(evs=None):
        if evs:
            evs[0].record(stream)
        cfog.cfog_extract(dA, m=m, vol=volA, sat=satA, stream=stream)
        cfog.cfog_extract(dB, m=m, vol=volB, sat=satB, stream=stream)
        if evs:
            evs[1].record(stream)
        cfog.match_batch([job], m=m, flags=flags, stream=stream)
        if evs:
            evs[2].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[ev(), ev(), ev()] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    step_ms = np.array([e[0].elapsed_time(e[2]) for e in evs])
    ext_ms = np.array([e[0].elapsed_time(e[1]) for e in evs])
    match_ms = np.array([e[1].elapsed_time(e[2]) for e in evs])
    n = len(cps)

    res = cfog.results(job.out)
    dx, dy, st = (res[k].cpu().numpy() for k in ("dx", "dy", "status"))
    recovered = float(np.mean(np.hypot(dx - shift[0], dy - shift[1]) <= 1.5))

    P = cfog.fft_size(N, r)
    bytes_launch = n * algorithmic_bytes_per_cp(N, r, m)
    flops_launch = n * fft_flops_per_cp(N, r, P, m)
    t_match = float(np.mean(match_ms)) * 1e-3
    gbs = bytes_launch / t_match / 1e9
    tfs = flops_launch / t_match / 1e12
    alu_peak = 157.3
    hbm_peak = 8000.0
    t_hbm = bytes_launch / (hbm_peak * 1e9)
    t_alu = flops_launch / (alu_peak * 1e12)
    if t_alu > t_hbm:
        roof = dict(bound="alu", achieved=round(tfs, 3), peak=alu_peak, unit="TFLOP/s", frac=round(tfs / alu_peak, 4))
    else:
        roof = dict(bound="hbm", achieved=round(gbs, 1), peak=hbm_peak, unit="GB/s", frac=round(gbs / hbm_peak, 4))
    roof.update(kernel=f"match_fft_plain_kernel<P={P}>", traffic=None,
                bytes_per_launch=bytes_launch, flops_per_launch=flops_launch,
                hbm=dict(achieved=round(gbs, 1), peak=hbm_peak, unit="GB/s", frac=round(gbs / hbm_peak, 4)),
                alu=dict(achieved=round(tfs, 3), peak=alu_peak, unit="TFLOP/s", frac=round(tfs / alu_peak, 4),
                         nonpacked_peak=78.6))
    out = {
        "metric": "CP matches/sec (CFOG+3DFFT SSD) on 1 MI355X; p50/p99 match latency",
        "value": round(n / (ms * 1e-3), 1),
        "unit": "CP matches/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP64 energies)",
        "data": "synthetic",
        "config": {"workload": "plain_2048: 2048^2 pair, 400 CPs (20x20 grid), template 100, radius 20, m=9, sigma=0.8",
                   "path": args.path, "fft_size": P},
        "latency_ms": {"step_p50": round(float(np.percentile(step_ms, 50)), 4),
                       "step_p99": round(float(np.percentile(step_ms, 99)), 4),
                       "match_p50": round(float(np.percentile(match_ms, 50)), 4),
                       "match_p99": round(float(np.percentile(match_ms, 99)), 4),
                       "extract_p50": round(float(np.percentile(ext_ms, 50)), 4)},
        "match_only_cp_per_s": round(n / t_match, 1),
        "extract_gbs": round(2 * H * W * extract_bytes_per_px(m) / (np.mean(ext_ms) * 1e-3) / 1e9, 1),
        "roofline": roof,
        "recovered_1p5px": round(recovered, 4),
        "cp_status_ok": int(np.sum(st == 0)),
    }
    if args.calib_copy_mib:
        # source written first, then 1 GiB of other writes so that the copy's
        # reads come from HBM rather than the last-level cache
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        junk = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        junk.fill_(2.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = nb
        del junk
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, B, cps, N, r, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
