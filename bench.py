#!/usr/bin/env python3
"""Benchmark of the real-spherical-harmonics hot path on one MI355X.

Headline (`value`): all real Y_lm for lmax = 9 in FP64 over 2^26 isotropic
points (radius uniform in [0.01, 10]) already resident in HBM, SoA output
[100][2^26].  One step = one sh_eval call over the whole batch (normalise,
evaluate the explicit formulas, store every (l, m) row).  `value` is points/s.

The same JSON line also carries the HBM roofline of the forward kernel, the
FP32 twin and the lmax sweep {2, 4, 6, 9} x {FP64, FP32}, a plain write probe
(achievable store bandwidth) and the CPU oracle timed on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def _parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 26, help="points of the headline workload")
    ap.add_argument("--cpu-sample", type=int, default=1 << 23,
                    help="points of the oracle's CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline only")
    return ap.parse_args()


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_launches(fn, steps: int, warmup: int):
    """Run fn() warmup times, then time `steps` calls; returns (total_s, per-call
    kernel seconds from events recorded on the launch stream around each call)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    per = [a.elapsed_time(b) / 1e3 for a, b in evs]
    return total, per


def fwd_bytes_per_point(lmax: int, elem: int) -> int:
    """Algorithmic HBM bytes per point of the forward pass: 3 coordinates in,
    (lmax+1)^2 values out."""
    return 3 * elem + (lmax + 1) ** 2 * elem


def bench_forward(sh, xyz, out, lmax, steps, warmup):
    import torch
    fn = sh.sh_eval if xyz.dtype == torch.float64 else sh.sh_eval_f32
    F = (lmax + 1) ** 2
    n = xyz.shape[0]
    o = out.view(-1).view(xyz.dtype)[: F * n].view(F, n)  # reuse the buffer's bytes
    total, per = time_launches(lambda: fn(lmax, xyz, out=o), steps, warmup)
    elem = xyz.element_size()
    avg = sum(per) / len(per)
    gbs = n * fwd_bytes_per_point(lmax, elem) / avg / 1e9
    return {"points_per_s": n * steps / total, "kernel_ms": avg * 1e3, "gbs": gbs,
            "frac": gbs / HBM_PEAK_GBS, "bytes_per_point": fwd_bytes_per_point(lmax, elem)}


def write_probe(buf, steps):
    """Achievable store bandwidth: torch's fill over the same output buffer."""
    total, per = time_launches(lambda: buf.fill_(1.0), steps, 2)
    avg = sum(per) / len(per)
    return {"bytes": buf.numel() * buf.element_size(), "gbs": buf.numel() * buf.element_size() / avg / 1e9}


def cpu_baseline(pts, lmax, sample):
    import oracle
    chunk = 1 << 18
    n = min(sample, pts.shape[0])
    t0 = time.perf_counter()
    for c in range(0, n, chunk):
        oracle.eval_xyz(lmax, pts[c:min(n, c + chunk)])
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "points/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"first {n} points of the same 2^26-point workload, lmax {lmax}, long double, "
                      f"{dt:.1f} s"}


def main():
    args = _parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the method needs no communication: a multi-GPU run shards the points)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2510_05282_amd as sh
    from paper_2510_05282_amd import workloads

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.n
    _log(f"generating {n} points")
    pts = workloads.points_roofline(n=n, seed=0)
    xyz = torch.from_numpy(pts).to(dev)
    out = torch.empty((100, n), dtype=torch.float64, device=dev)

    _log("headline: lmax 9 fp64")
    head = bench_forward(sh, xyz, out, 9, args.steps, args.warmup)
    _log("  ", json.dumps(head))
    result = {
        "metric": "Y_lm points/s (lmax=9, FP64, SoA output) + % HBM peak",
        "value": head["points_per_s"],
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": n / head["points_per_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded isotropic points, radius U[0.01, 10]",
        "config": {"workload": "real Y_lm, lmax=9, FP64, 2^26 points, SoA [100][N] output",
                   "n_points": n, "lmax": 9},
        "roofline": {"bound": "hbm", "achieved": head["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": head["frac"], "traffic": None,
                     "kernel": "fwd_kernel<9,double>", "kernel_ms": head["kernel_ms"],
                     "bytes_per_point": head["bytes_per_point"]},
    }

    if not args.no_extras:
        sweep = {}
        xyz32 = xyz.float()
        for lmax in (2, 4, 6, 9):
            _log(f"sweep lmax {lmax}")
            sweep[f"f64_l{lmax}"] = bench_forward(sh, xyz, out, lmax, max(5, args.steps // 2), 2)
            sweep[f"f32_l{lmax}"] = bench_forward(sh, xyz32, out, lmax, max(5, args.steps // 2), 2)
            _log("  ", json.dumps({k: sweep[k] for k in (f"f64_l{lmax}", f"f32_l{lmax}")}))
        result["fp32"] = sweep["f32_l9"]
        result["lmax_sweep"] = sweep
        _log("write probe")
        result["write_probe"] = write_probe(out, 5)
        result["roofline"]["frac_of_write_probe"] = head["gbs"] / result["write_probe"]["gbs"]
        del xyz32

    del out
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        _log("cpu baseline")
        result["cpu_baseline"] = cpu_baseline(pts, 9, args.cpu_sample)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
