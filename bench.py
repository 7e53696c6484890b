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
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector, published
ROOT = os.path.dirname(os.path.abspath(__file__))
FWD_SOURCES = ("sh_fwd.h", "sh_core.h", "sh_eval.hip", "sh_constants.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fwd_traffic.json")


def fwd_source_hash() -> str:
    """sha256 over the compile flags and the code of the forward kernel's sources,
    comments and whitespace removed (for matching counter data to the kernel they
    were taken on)."""
    import hashlib
    import re
    from paper_2510_05282_amd import build as shbuild
    h = hashlib.sha256()
    h.update(" ".join(shbuild.compile_flags()).encode())  # the code also depends on how it is compiled
    for f in FWD_SOURCES:
        with open(os.path.join(ROOT, "paper_2510_05282_amd", "csrc", f)) as fh:
            code = re.sub(r"/\*.*?\*/", " ", fh.read(), flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()


def counter_record():
    """The committed rocprofv3 counter record of the headline kernel, or {} when it
    was taken on other kernel code."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return {}
    return t if t.get("source_sha256") == fwd_source_hash() else {}


def measured_traffic():
    """HBM bytes per launch of the headline kernel (counters), or None."""
    return counter_record().get("traffic_bytes_per_launch")


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
    ap.add_argument("--only", default="",
                    help="comma-separated extra sections to run (sweep, store_probes, interfaces, projectors, "
                         "gradient, serving); default: all")
    ap.add_argument("--serve-requests", type=int, default=10_000)
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the headline, copy 4 GiB once (calibrates HBM traffic counters)")
    ap.add_argument("--store-sweep", action="store_true",
                    help="no benchmark: time the store-pattern probe variants (rows split over XCDs, tile "
                         "orders, cache-policy bits, the forward kernel with split rows) on the headline "
                         "workload and print one JSON line per variant")
    ap.add_argument("--traffic-from", nargs="+", metavar="CSV",
                    help="no GPU work: turn the counter_collection.csv files of a --pmc FETCH_SIZE and a "
                         "--pmc WRITE_SIZE run of `--copy-probe` (and optionally a --pmc "
                         "SQ_INSTS_VALU_FLOPS_FP64 run) into the committed counter record")
    ap.add_argument("--serving-trace-summary", metavar="CSV",
                    help="no GPU work: split the serving kernels of a rocprofv3 kernel trace of "
                         "`--only serving` into its passes (at idle gaps over 2 ms) and print, per pass, "
                         "the span, how many serving kernels ran at a time, and the kernels' time")
    ap.add_argument("--counter-summary", nargs="+", metavar="CSV",
                    help="no GPU work: mean of each counter per dispatch over each run of consecutive "
                         "dispatches of one kernel and grid size, from the counter_collection.csv files of "
                         "rocprofv3 --pmc passes over the same command (one markdown row per run)")
    ap.add_argument("--counter-chunk", type=int, default=0,
                    help="with --counter-summary: cut each run into chunks of this many dispatches")
    ap.add_argument("--counter-kernels", default="",
                    help="with --counter-summary: comma-separated substrings; only kernels that contain one")
    return ap.parse_args()


HEADLINE_KERNEL = "shk::fwd_kernel<9, double, 2, (shk::In)0>"
COPY_BYTES = 8 << 29  # the copy probe's 4 GiB


def flops_from_counters(flops_csv: str) -> float:
    """FP64 flops per launch of the headline kernel: SQ_INSTS_VALU_FLOPS_FP64 counts
    the flops of each wave instruction once per wave, so it is scaled by the 64
    lanes (averaged over the launches in the file)."""
    import csv
    acc = {}
    with open(flops_csv, newline="") as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == "SQ_INSTS_VALU_FLOPS_FP64" and HEADLINE_KERNEL in r["Kernel_Name"]:
                acc[r["Dispatch_Id"]] = acc.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    if not acc:
        raise SystemExit(f"{flops_csv}: no SQ_INSTS_VALU_FLOPS_FP64 rows for the headline kernel")
    return 64.0 * sum(acc.values()) / len(acc)


def traffic_from_counters(fetch_csv: str, write_csv: str, n_points: int) -> dict:
    """HBM bytes per launch of the headline kernel from two rocprofv3 counter runs
    (KiB per dispatch), each scaled so that the copy probe's reading equals the 4 GiB
    it reads (FETCH_SIZE) and writes (WRITE_SIZE)."""
    import csv

    def per_dispatch(path, counter):
        acc = {}
        with open(path, newline="") as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                k = (r["Dispatch_Id"], r["Kernel_Name"])
                acc[k] = acc.get(k, 0.0) + float(r["Counter_Value"])
        head = [v for (d, name), v in acc.items() if HEADLINE_KERNEL in name]
        copy = [v for (d, name), v in acc.items() if "copyBuffer" in name and v * 1024 > COPY_BYTES / 4]
        if not head or len(copy) != 1:
            raise SystemExit(f"{path}: expected headline dispatches and one copy-probe dispatch")
        return head, copy[0]

    fh_, fc = per_dispatch(fetch_csv, "FETCH_SIZE")
    wh, wc = per_dispatch(write_csv, "WRITE_SIZE")
    fs, ws = COPY_BYTES / (fc * 1024), COPY_BYTES / (wc * 1024)
    fetch = fs * 1024 * sum(fh_) / len(fh_)
    write = ws * 1024 * sum(wh) / len(wh)
    return {"kernel": HEADLINE_KERNEL, "n_points": n_points, "source_sha256": fwd_source_hash(),
            "fetch_scale": fs, "write_scale": ws, "fetch_bytes_per_launch": fetch,
            "write_bytes_per_launch": write, "traffic_bytes_per_launch": fetch + write,
            "algorithmic_bytes_per_launch": n_points * (24 + 800),
            "dispatches": {"fetch": len(fh_), "write": len(wh)}}


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


def store_probe_lib():
    """libshprobe.so (store-pattern probe kernels, built with the library)."""
    import ctypes
    path = os.path.join(ROOT, "paper_2510_05282_amd", "libshprobe.so")
    if not os.path.exists(path):
        raise SystemExit(f"{path} is not built; run `python -m paper_2510_05282_amd.build`")
    P = ctypes.CDLL(path)
    i32, i64, vp = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
    P.shp_fill.argtypes = [vp, i64, i32, vp]
    P.shp_rows.argtypes = [vp, vp, i64, i64, i32, i32, i32, i32, i32, vp]
    P.shp_fwd_split.argtypes = [vp, vp, i64, i64, i32, i32, i32, vp]
    return P


def bench_store_probes(xyz, out, head, steps):
    """The headline kernel's store pattern without its arithmetic, and plain fills,
    over the same buffers: `rows100` loads each lane's two points and writes 100
    rows of 16 bytes in the headline kernel's launch shape (256 lanes, XCD-ordered
    tiles, one resident workgroup per CU); `rows100_2wg` the same with at most 2
    workgroups per CU (the shape of the kernels below lmax 8); `rows10` 10 rows, 2
    workgroups per CU; `fill` one 16-byte store per lane over the whole output
    (plain, and with the sc1 cache policy bit).  `frac_of_store_pattern` is the
    headline kernel's rate over rows100's."""
    import torch
    P = store_probe_lib()
    n = xyz.shape[0]
    st = torch.cuda.current_stream().cuda_stream

    def chk(rc):
        if rc != 0:
            raise RuntimeError(f"store probe rejected its arguments ({rc})")

    res = {}
    cases = (("rows100", n * (24 + 800), lambda: chk(P.shp_rows(xyz.data_ptr(), out.data_ptr(), n, n, 100, 1, 0, 2, 0, st))),
             ("rows100_2wg", n * (24 + 800),
              lambda: chk(P.shp_rows(xyz.data_ptr(), out.data_ptr(), n, n, 100, 1, 0, 1, 0, st))),
             ("rows10", n * (24 + 80), lambda: chk(P.shp_rows(xyz.data_ptr(), out.data_ptr(), n, n, 10, 1, 0, 1, 0, st))),
             ("fill", n * 800, lambda: chk(P.shp_fill(out.data_ptr(), n * 800, 0, st))),
             ("fill_sc1", n * 800, lambda: chk(P.shp_fill(out.data_ptr(), n * 800, 4, st))))
    for name, nbytes, fn in cases:
        _, per = time_launches(fn, steps, 2)
        avg = sum(per) / len(per)
        res[name] = {"ms": avg * 1e3, "bytes": nbytes, "gbs": nbytes / avg / 1e9,
                     "frac": nbytes / avg / 1e9 / HBM_PEAK_GBS}
    res["frac_of_store_pattern"] = head["gbs"] / res["rows100"]["gbs"]
    res["frac_of_fill"] = head["gbs"] / max(res["fill"]["gbs"], res["fill_sc1"]["gbs"])
    return res


def store_sweep(sh, xyz, out, steps):
    """Variants of the headline kernel's store pattern (libshprobe.so), each timed
    like the headline: the 100-row pattern with its rows split over 1, 2, 4 or 8
    workgroups per tile (order 0: each split on its own XCDs, XCD-contiguous tiles;
    order 1: hardware order, every XCD on the same tiles), with 16 to 128 tile
    ranges (orders 2-5), with each cache-policy variant of the store (modes 1-8),
    and the lmax 9 FP64 forward kernel itself with the same splits and orders."""
    P = store_probe_lib()
    import torch
    n = xyz.shape[0]
    st = torch.cuda.current_stream().cuda_stream
    B = n * 824

    def one(name, fn, nbytes=B):
        _, per = time_launches(fn, steps, 2)
        avg = sum(per) / len(per)
        print(json.dumps({"case": name, "ms": avg * 1e3, "gbs": nbytes / avg / 1e9,
                          "frac": nbytes / avg / 1e9 / HBM_PEAK_GBS}), flush=True)

    def chk(rc):
        if rc != 0:
            raise RuntimeError(f"store probe rejected its arguments ({rc})")

    x, o = xyz.data_ptr(), out.data_ptr()
    one("sh_eval lmax 9 fp64", lambda: sh.sh_eval(9, xyz, out=out.view(-1)[: 100 * n].view(100, n)))
    for split in (1, 2, 4, 8):
        for order in (0, 1):
            for cap in (0, 1):
                one(f"rows100 split {split} order {order} cap {cap}",
                    lambda: chk(P.shp_rows(x, o, n, n, 100, split, order, cap, 0, st)))
                one(f"fwd lmax 9 split {split} order {order} cap {cap}",
                    lambda: chk(P.shp_fwd_split(x, o, n, n, split, order, cap, st)))
    for order in (2, 3, 4, 5):
        one(f"rows100 ranges {8 << (order - 1)} cap 1", lambda: chk(P.shp_rows(x, o, n, n, 100, 1, order, 1, 0, st)))
        one(f"fwd lmax 9 ranges {8 << (order - 1)} cap 1", lambda: chk(P.shp_fwd_split(x, o, n, n, 1, order, 1, st)))
    for mode in range(1, 9):
        one(f"rows100 store mode {mode}", lambda: chk(P.shp_rows(x, o, n, n, 100, 1, 0, 1, mode, st)))
        one(f"fill store mode {mode}", lambda: chk(P.shp_fill(o, n * 800, mode, st)), n * 800)


def bench_interfaces(sh, xyz, out, steps):
    """lmax 9 through the other interfaces on the same points: unit vectors (no
    normalisation), angles (theta, phi), complex output (2^25 points, 16 B
    per value), spinor output (2^23 points, 400 complex values each); the
    recurrence at lmax 16 (2^24 points), and its complex (2^22 points) and spinor
    (2^20 points, 1156 complex values each) harmonics."""
    import torch
    n = xyz.shape[0]
    r = xyz.norm(dim=1, keepdim=True)
    unit = (xyz / r).contiguous()
    theta = torch.acos((xyz[:, 2:3] / r).clamp(-1, 1)).reshape(-1).contiguous()
    phi = torch.atan2(xyz[:, 1], xyz[:, 0]).contiguous()
    res = {}
    o = out.view(-1)[: 100 * n].view(100, n)
    for name, fn, inb in (("unit", lambda: sh.sh_eval_unit(9, unit, out=o), 24),
                          ("angles", lambda: sh.sh_eval_angles(9, theta, phi, out=o), 16)):
        _, per = time_launches(fn, steps, 2)
        avg = sum(per) / len(per)
        b = n * (inb + 800)
        res[name] = {"points_per_s": n / avg, "kernel_ms": avg * 1e3, "gbs": b / avg / 1e9,
                     "frac": b / avg / 1e9 / HBM_PEAK_GBS, "bytes_per_point": inb + 800}
    nc = n // 2
    oc = out.view(-1)[: 200 * nc].view(torch.complex128).view(100, nc)
    xc = xyz[:nc].contiguous()
    _, per = time_launches(lambda: sh.sh_eval_complex(9, xc, out=oc), steps, 2)
    avg = sum(per) / len(per)
    b = nc * (24 + 1600)
    res["complex"] = {"n_points": nc, "points_per_s": nc / avg, "kernel_ms": avg * 1e3, "gbs": b / avg / 1e9,
                      "frac": b / avg / 1e9 / HBM_PEAK_GBS, "bytes_per_point": 1624}
    oc32 = out.view(-1)[: 100 * nc].view(torch.float32).view(torch.complex64).view(100, nc)
    xc32 = xc.to(torch.float32)
    _, per = time_launches(lambda: sh.sh_eval_complex_f32(9, xc32, out=oc32), steps, 2)
    avg = sum(per) / len(per)
    b = nc * (12 + 800)
    res["complex_f32"] = {"n_points": nc, "points_per_s": nc / avg, "kernel_ms": avg * 1e3, "gbs": b / avg / 1e9,
                          "frac": b / avg / 1e9 / HBM_PEAK_GBS, "bytes_per_point": 812}
    del xc32
    # spinors: 200 (l, j, m_j) x 2 components x 16 B per point
    ns = n // 8
    os_ = out.view(-1)[: 800 * ns].view(torch.complex128).view(200, 2, ns)
    xs = xyz[:ns].contiguous()
    _, per = time_launches(lambda: sh.sh_eval_spinor(9, xs, out=os_), steps, 2)
    avg = sum(per) / len(per)
    b = ns * (24 + 6400)
    res["spinor"] = {"n_points": ns, "points_per_s": ns / avg, "kernel_ms": avg * 1e3, "gbs": b / avg / 1e9,
                     "frac": b / avg / 1e9 / HBM_PEAK_GBS, "bytes_per_point": 6424}
    # l > 9 by recurrence: lmax 16 (289 rows) on 2^24 points
    nr = n // 4
    orr = out.view(-1)[: 289 * nr].view(289, nr)
    xr = xyz[:nr].contiguous()
    _, per = time_launches(lambda: sh.sh_eval_rec(16, xr, out=orr), steps, 2)
    avg = sum(per) / len(per)
    b = nr * (24 + 289 * 8)
    res["rec_l16"] = {"n_points": nr, "points_per_s": nr / avg, "kernel_ms": avg * 1e3, "gbs": b / avg / 1e9,
                      "frac": b / avg / 1e9 / HBM_PEAK_GBS, "bytes_per_point": 24 + 289 * 8}
    orr32 = out.view(-1)[: 289 * nr // 2].view(torch.float32).view(289, nr)
    xr32 = xr.to(torch.float32)
    _, per = time_launches(lambda: sh.sh_eval_rec_f32(16, xr32, out=orr32), steps, 2)
    avg = sum(per) / len(per)
    b = nr * (12 + 289 * 4)
    res["rec_l16_f32"] = {"n_points": nr, "points_per_s": nr / avg, "kernel_ms": avg * 1e3, "gbs": b / avg / 1e9,
                          "frac": b / avg / 1e9 / HBM_PEAK_GBS, "bytes_per_point": 12 + 289 * 4}
    del xr32
    # complex and spinor harmonics by recurrence at lmax 16: 2^22 and 2^20 points
    F16 = 289
    nc16 = n // 16
    occ = out.view(-1)[: 2 * F16 * nc16].view(torch.complex128).view(F16, nc16)
    xcc = xyz[:nc16].contiguous()
    _, per = time_launches(lambda: sh.sh_eval_complex_rec(16, xcc, out=occ), steps, 2)
    avg = sum(per) / len(per)
    b = nc16 * (24 + 16 * F16)
    res["complex_rec_l16"] = {"n_points": nc16, "points_per_s": nc16 / avg, "kernel_ms": avg * 1e3,
                              "gbs": b / avg / 1e9, "frac": b / avg / 1e9 / HBM_PEAK_GBS,
                              "bytes_per_point": 24 + 16 * F16}
    ns16 = n // 64
    osp = out.view(-1)[: 8 * F16 * ns16].view(torch.complex128).view(2 * F16, 2, ns16)
    xsp = xyz[:ns16].contiguous()
    _, per = time_launches(lambda: sh.sh_eval_spinor_rec(16, xsp, out=osp), steps, 2)
    avg = sum(per) / len(per)
    b = ns16 * (24 + 64 * F16)
    res["spinor_rec_l16"] = {"n_points": ns16, "points_per_s": ns16 / avg, "kernel_ms": avg * 1e3,
                             "gbs": b / avg / 1e9, "frac": b / avg / 1e9 / HBM_PEAK_GBS,
                             "bytes_per_point": 24 + 64 * F16}
    return res


def bench_projectors(sh, workloads, dev, steps):
    """64 atoms, spheres of radius 3 on a 0.2 grid, lmax 3, 2000-knot tables."""
    import torch
    A = workloads.atom_spheres(seed=0)
    rad = sh.Radial(A.tables, A.r_max)
    c = torch.from_numpy(A.centers).to(dev)
    off = torch.from_numpy(A.offsets).to(dev)
    p = torch.from_numpy(A.points).to(dev)
    n = int(A.offsets[-1])
    out = torch.empty(16 * n, dtype=torch.float64, device=dev)
    total, per = time_launches(lambda: sh.sh_projectors(3, c, off, p, rad, out=out), steps, 3)
    avg = sum(per) / len(per)
    bpp = 16 * 8 + 24
    rad.close()
    res = {"workload": "64 atoms, r=3 spheres on a 0.2 grid, lmax 3, FP64", "n_points": n,
           "ms_per_build": avg * 1e3, "points_per_s": n / avg, "gbs": n * bpp / avg / 1e9,
           "frac": n * bpp / avg / 1e9 / HBM_PEAK_GBS, "bytes_per_point": bpp}
    del out, p
    # a large build (several adjacent points per lane): 64 atoms x 150k points uniform
    # in balls of radius 3, one 10-channel table per atom
    import numpy as np
    na, per = 64, 150_000
    gen = torch.Generator(device=dev)
    gen.manual_seed(1)
    cen = 20.0 * torch.rand((na, 3), generator=gen, dtype=torch.float64, device=dev)
    d = torch.randn((na * per, 3), generator=gen, dtype=torch.float64, device=dev)
    d = d / d.norm(dim=1, keepdim=True) * (3.0 * torch.rand((na * per, 1), generator=gen, dtype=torch.float64,
                                                            device=dev) ** (1 / 3))
    pts = (cen.repeat_interleave(per, 0) + d).contiguous()
    del d
    offl = torch.arange(0, na + 1, dtype=torch.int64, device=dev) * per
    rng = np.random.default_rng(0)
    radl = sh.Radial(np.stack([workloads.radial_table(rng, 9, 2000, 3.0) for _ in range(na)]), 3.0)
    nl = na * per
    large = {"workload": "64 atoms x 150k points, balls of radius 3", "n_points": nl}
    for name, lmax, dt in (("lmax0_f64", 0, torch.float64), ("lmax1_f64", 1, torch.float64),
                           ("lmax3_f64", 3, torch.float64), ("lmax6_f64", 6, torch.float64),
                           ("lmax9_f64", 9, torch.float64), ("lmax0_f32", 0, torch.float32),
                           ("lmax1_f32", 1, torch.float32), ("lmax3_f32", 3, torch.float32),
                           ("lmax6_f32", 6, torch.float32), ("lmax9_f32", 9, torch.float32)):
        F, sz = (lmax + 1) ** 2, (8 if dt == torch.float64 else 4)
        pl, cl = pts.to(dt), cen.to(dt)
        o = torch.empty(F * nl, dtype=dt, device=dev)
        fn = sh.sh_projectors if dt == torch.float64 else sh.sh_projectors_f32
        _, per_l = time_launches(lambda: fn(lmax, cl, offl, pl, radl, out=o), steps, 2)
        t = sum(per_l) / len(per_l)
        b = nl * (F + 3) * sz
        large[name] = {"ms": t * 1e3, "gbs": b / t / 1e9, "frac": b / t / 1e9 / HBM_PEAK_GBS,
                       "bytes_per_point": (F + 3) * sz}
        del o, pl, cl
    radl.close()
    res["large_build"] = large
    return res


def bench_gradient(sh, workloads, dev, steps):
    """2^24 points (radius in [0.5, 5]), lmax 6: forward, then backward with an
    N(0,1) upstream gradient."""
    import torch
    n, lmax = 1 << 24, 6
    x = torch.from_numpy(workloads.points_gradient(n=n, seed=0)).to(dev)
    y = torch.empty((49, n), dtype=torch.float64, device=dev)
    G = workloads.upstream_gradient_device(49, n, seed=1, device=dev)
    g = torch.empty((n, 3), dtype=torch.float64, device=dev)
    _, per_f = time_launches(lambda: sh.sh_eval(lmax, x, out=y), steps, 2)
    _, per_b = time_launches(lambda: sh.sh_eval_grad(lmax, x, G, grad_xyz=g), steps, 2)
    f, b = sum(per_f) / len(per_f), sum(per_b) / len(per_b)
    bf, bb = 24 + 49 * 8, 24 + 49 * 8 + 24
    res = {"workload": "2^24 points, lmax 6, FP64, forward + backward", "n_points": n,
           "forward_ms": f * 1e3, "backward_ms": b * 1e3,
           "forward_points_per_s": n / f, "backward_points_per_s": n / b,
           "forward_gbs": n * bf / f / 1e9, "backward_gbs": n * bb / b / 1e9,
           "backward_frac": n * bb / b / 1e9 / HBM_PEAK_GBS, "backward_bytes_per_point": bb}
    # FP32 backward on the same points and upstream gradient, rounded
    x32, G32, g32 = x.float(), G.float(), g.float()
    _, per = time_launches(lambda: sh.sh_eval_grad_f32(lmax, x32, G32, grad_xyz=g32), steps, 2)
    b32 = sum(per) / len(per)
    res["backward_f32_ms"] = b32 * 1e3
    res["backward_f32_points_per_s"] = n / b32
    res["backward_f32_frac"] = n * 220 / b32 / 1e9 / HBM_PEAK_GBS
    del x32, G32, g32, G
    # fused values + Jacobian: 24 B in, 4 F 8 B out
    jac = torch.empty((3, 49, n), dtype=torch.float64, device=dev)
    _, per = time_launches(lambda: sh.sh_eval_jac(lmax, x, out=y, jac=jac), steps, 2)
    j = sum(per) / len(per)
    bj = 24 + 4 * 49 * 8
    res["jacobian_ms"] = j * 1e3
    res["jacobian_points_per_s"] = n / j
    res["jacobian_frac"] = n * bj / j / 1e9 / HBM_PEAK_GBS
    del jac, y
    # backward beyond l = 9 (recurrence on dual numbers): lmax 16 on 2^22 points
    nr, lr = n // 4, 16
    Fr = (lr + 1) ** 2
    xr = x[:nr].contiguous()
    Gr = workloads.upstream_gradient_device(Fr, nr, seed=2, device=dev)
    gr = torch.empty((nr, 3), dtype=torch.float64, device=dev)
    _, per = time_launches(lambda: sh.sh_eval_grad_rec(lr, xr, Gr, grad_xyz=gr), steps, 2)
    br = sum(per) / len(per)
    bbr = 24 + Fr * 8 + 24
    res["backward_rec_l16"] = {"n_points": nr, "ms": br * 1e3, "points_per_s": nr / br,
                               "gbs": nr * bbr / br / 1e9, "frac": nr * bbr / br / 1e9 / HBM_PEAK_GBS,
                               "bytes_per_point": bbr}
    xr32, Gr32, gr32 = xr.float(), Gr.float(), gr.float()
    _, per = time_launches(lambda: sh.sh_eval_grad_rec_f32(lr, xr32, Gr32, grad_xyz=gr32), steps, 2)
    br32 = sum(per) / len(per)
    bb32 = bbr // 2
    res["backward_rec_l16_f32"] = {"n_points": nr, "ms": br32 * 1e3, "points_per_s": nr / br32,
                                   "gbs": nr * bb32 / br32 / 1e9, "frac": nr * bb32 / br32 / 1e9 / HBM_PEAK_GBS,
                                   "bytes_per_point": bb32}
    return res


def counter_summary(paths, chunk: int = 0, kernels: str = "") -> None:
    """Counters of several rocprofv3 --pmc passes over one command, side by side.
    Each file's dispatches (in order) are cut into runs of consecutive dispatches
    with the same kernel and grid size (and into chunks of `chunk` dispatches when
    given); the passes ran the same program, so run k of every file is the same
    work, and each row gives the mean per dispatch of every counter of every pass."""
    import csv
    import re
    keep = [k for k in kernels.split(",") if k]
    table, names, order = {}, [], []
    for path in paths:
        disp = {}
        with open(path, newline="") as fh:
            for r in csv.DictReader(fh):
                d = disp.setdefault(int(r["Dispatch_Id"]), {"kernel": r["Kernel_Name"], "grid": int(r["Grid_Size"]),
                                                            "vgpr": r.get("VGPR_Count", ""), "c": {}})
                d["c"][r["Counter_Name"]] = d["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        runs = []
        for i in sorted(disp):
            d = disp[i]
            if keep and not any(k in d["kernel"] for k in keep):
                continue
            key = (d["kernel"], d["grid"])
            if not runs or runs[-1]["key"] != key or (chunk and len(runs[-1]["ids"]) == chunk):
                runs.append({"key": key, "ids": [], "vgpr": d["vgpr"], "c": {}})
            runs[-1]["ids"].append(i)
            for n, v in d["c"].items():
                runs[-1]["c"].setdefault(n, []).append(v)
        for k, run in enumerate(runs):
            row = table.setdefault(k, {"key": run["key"], "n": len(run["ids"]), "vgpr": run["vgpr"], "c": {}})
            if row["key"] != run["key"]:
                raise SystemExit(f"{path}: run {k} is {run['key']}, other passes have {row['key']}")
            for n, v in run["c"].items():
                row["c"][n] = sum(v) / len(v)
                if n not in names:
                    names.append(n)
        order = sorted(table)
    short = lambda name: re.sub(r"\((?!anon)[^()]*\)$", "", name.replace("void ", "")
                                .replace("(anonymous namespace)::", "")).strip()
    print("| run | kernel | grid | dispatches | VGPRs | " + " | ".join(names) + " |")
    print("|" + "---|" * (5 + len(names)))
    for k in order:
        row = table[k]
        print(f"| {k} | {short(row['key'][0])} | {row['key'][1]} | {row['n']} | {row['vgpr']} | "
              + " | ".join(f"{row['c'][n]:.6g}" if n in row["c"] else "" for n in names) + " |")


def serving_trace_summary(path: str, gap_ns: int = 2_000_000) -> None:
    """Per-pass view of a rocprofv3 kernel trace (`*_kernel_trace.csv`) of the
    serving section: its serve_kernel and serve_mixed_kernel dispatches (warm-up
    launches of one tile left out) split where no serving kernel runs for more than gap_ns; for each
    pass the dispatch count, span, the share of the span with 0, 1, 2 or 3 serving
    kernels running, their summed duration, and the kernels with the most time."""
    import collections
    import csv
    import re
    with open(path, newline="") as fh:
        rows = list(csv.DictReader(fh))

    def grid(r):
        return int(r.get("Grid_Size") or r.get("Grid_Size_X") or 0)

    ds = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]) for r in rows
                if ("serve_kernel" in r["Kernel_Name"] or "serve_mixed_kernel" in r["Kernel_Name"]) and grid(r) > 256)
    passes, cur, end = [], [], 0
    for d in ds:
        if cur and d[0] - end > gap_ns:
            passes.append(cur)
            cur = []
        end = d[1] if not cur else max(end, d[1])
        cur.append(d)
    if cur:
        passes.append(cur)
    for k, p in enumerate(passes):
        t0, t1 = p[0][0], max(e for _, e, _ in p)
        span = t1 - t0
        ev = sorted([(s, 1) for s, _, _ in p] + [(e, -1) for _, e, _ in p])
        at = collections.Counter()
        c, last = 0, t0
        for t, dlt in ev:
            at[c] += t - last
            c, last = c + dlt, t
        per = collections.defaultdict(lambda: [0, 0.0])
        for s, e, name in p:
            m = re.search(r"serve_kernel<[^>]*>|serve_mixed_kernel", name)
            per[m.group(0) if m else name][0] += 1
            per[m.group(0) if m else name][1] += (e - s) / 1e6
        busy = sum(v[1] for v in per.values())
        one = sum(v[1] for kk, v in per.items() if kk.endswith(", 1>") or kk == "serve_mixed_kernel")
        print(f"pass {k}: {len(p)} dispatches over {span / 1e6:.2f} ms; share of the span with "
              + ", ".join(f"{n} running {at[n] / span:.3f}" for n in sorted(at))
              + f"; kernel time {busy:.1f} ms ({one:.1f} ms in one-point-per-lane launches)")
        for kk, v in sorted(per.items(), key=lambda kv: -kv[1][1])[:6]:
            print(f"    {kk:30s} calls {v[0]:5d} total {v[1]:8.3f} ms avg {v[1] / v[0] * 1e3:9.1f} us")


def bench_serving(sh, workloads, dev, n_req):
    """n_req projector requests (lmax ~ U{0..9}, n log-uniform in [1e3, 1e6], 80%
    FP64), per-atom points and radial tables (lmax + 1 channels) resident on the
    device, 64 GB budget.
    One server for all passes.  After an untimed closed-loop pass, three closed
    loops (everything submitted at once; the median is reported) give the
    saturation rate; then Poisson arrivals
    at 0.7x and 0.3x that rate, and at fixed 54k and 23k requests/s, give the
    latencies (rates over each pass's wall time, from its first submission to the
    end of its drain)."""
    import numpy as np
    import torch
    from paper_2510_05282_amd.serve import SH_REQ_AUTORELEASE, Server
    reqs = workloads.request_stream(n_req=n_req, rate=1.0, seed=0)
    # each request's own table of lmax + 1 channels: one radial handle per lmax
    # holding the tables of that lmax's requests
    slot = {}
    by_l = {}
    for k, r in enumerate(reqs):
        slot[k] = (r.lmax, len(by_l.setdefault(r.lmax, [])))
        by_l[r.lmax].append(workloads.radial_table(np.random.default_rng(r.seed), r.lmax, 2000, 3.0))
    radials = {l: sh.Radial(np.stack(t), 3.0) for l, t in by_l.items()}
    del by_l
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    pts = []
    for k, r in enumerate(reqs):
        dt = torch.float64 if r.dtype == "f64" else torch.float32
        d = torch.randn((r.n, 3), generator=gen, dtype=torch.float64, device=dev)
        d = d / d.norm(dim=1, keepdim=True)
        rr = 3.0 * torch.rand((r.n, 1), generator=gen, dtype=torch.float64, device=dev) ** (1 / 3)
        pts.append((torch.from_numpy(r.center).to(dev) + d * rr).to(dt).contiguous())
    total_points = sum(r.n for r in reqs)
    total_bytes = sum((r.lmax + 1) ** 2 * r.n * (8 if r.dtype == "f64" else 4) for r in reqs)
    out = {"workload": f"{n_req} projector requests, lmax U{{0..9}}, n log-U[1e3,1e6], 80% FP64, "
                       "64 GB budget, 3 streams",
           "total_points": total_points, "output_bytes": total_bytes}

    # one long-lived server, as a service would run it; an untimed closed-loop pass first
    # (the first pass through a fresh arena runs 10-15% slower)
    srv = Server(64 << 30, max_pending=n_req + 1, n_slots=3)
    atoms = [srv.add_atom(p, r.center, radials[slot[k][0]], table=slot[k][1])
             for k, (p, r) in enumerate(zip(pts, reqs))]

    def run(arrivals):
        torch.cuda.synchronize()
        st0 = srv.stats()
        n_lat0 = len(srv.latencies_ms())
        lag = np.empty(n_req)  # how far each submission fell behind its scheduled arrival
        t0 = time.perf_counter()
        for k, (a, r, ta) in enumerate(zip(atoms, reqs, arrivals)):
            now = time.perf_counter() - t0
            while now < ta:
                now = time.perf_counter() - t0
            lag[k] = now - ta
            srv.submit(a, r.lmax, SH_REQ_AUTORELEASE)
        srv.drain(600)
        wall = time.perf_counter() - t0
        st1 = srv.stats()
        st = {k: st1[k] - st0[k] for k in ("completed", "failed", "deferred", "batches")}
        st["peak_bytes"] = st1["peak_bytes"]
        st["scheduler_cpu_frac"] = (st1["scheduler_cpu_s"] - st0["scheduler_cpu_s"]) / wall
        st["lag_ms_max"], st["lag_ms_p99"] = float(lag.max() * 1e3), float(np.percentile(lag, 99) * 1e3)
        lat = srv.latencies_ms()[n_lat0:]
        return wall, st, lat

    run([0.0] * n_req)  # warm-up
    # three closed-loop passes (each under 0.1 s): the median one is reported
    cl = sorted((run([0.0] * n_req) for _ in range(3)), key=lambda x: x[0])
    wall, st, lat = cl[1]
    rate = n_req / wall
    out["closed_loop"] = {"wall_s": wall, "req_per_s": rate, "points_per_s": total_points / wall,
                          "gbs": total_bytes / wall / 1e9, "batches": st["batches"],
                          "deferred": st["deferred"], "peak_bytes": st["peak_bytes"],
                          "scheduler_cpu_frac": st["scheduler_cpu_frac"],
                          "passes_req_per_s": [n_req / x[0] for x in cl]}
    # Poisson arrivals at 0.7x and 0.3x the saturation rate, and at two fixed rates
    # (comparable between builds whose saturation rates differ)
    for key, lam in (("poisson", 0.7 * rate), ("poisson_0.3", 0.3 * rate), ("poisson_54k", 54000.0),
                     ("poisson_23k", 23000.0)):
        arr = workloads.request_stream(n_req=n_req, rate=lam, seed=0)
        wall, st, lat = run([r.arrival for r in arr])
        out[key] = {"rate_req_per_s": lam, "p50_ms": float(np.percentile(lat, 50)),
                    "p90_ms": float(np.percentile(lat, 90)), "p99_ms": float(np.percentile(lat, 99)),
                    "mean_ms": float(lat.mean()), "points_per_s": total_points / wall,
                    "gbs": total_bytes / wall / 1e9, "batches": st["batches"], "deferred": st["deferred"],
                    "peak_bytes": st["peak_bytes"], "completed": st["completed"], "failed": st["failed"],
                    "scheduler_cpu_frac": st["scheduler_cpu_frac"],
                    "submit_lag_ms_max": st["lag_ms_max"], "submit_lag_ms_p99": st["lag_ms_p99"]}
    srv.close()
    for rad in radials.values():
        rad.close()
    return out


# The paper's own timings (Section 4, Table 1), in millions of individual
# harmonics (point, l, m) per second, l <= 9, evaluated and accumulated rather than
# stored, on one NVIDIA V100 and one core of an AMD Ryzen 5950X.
PAPER_MHARM_PER_S = {
    "real_cartesian": {"V100": 9939, "Ryzen 5950X, 1 core": 228},
    "real_normalised": {"V100": 12540, "Ryzen 5950X, 1 core": 553},
    "real_angular": {"V100": 9307, "Ryzen 5950X, 1 core": 159},
    "complex_cartesian": {"V100": 5187, "Ryzen 5950X, 1 core": 85},
}


def paper_context(result: dict) -> dict:
    """This run's rates in the paper's unit next to the paper's figures (context
    only: other hardware, and the paper does not store its results)."""
    mine = {"real_cartesian": result["value"] * 100 / 1e6}
    itf = result.get("interfaces", {})
    for key, name, per in (("unit", "real_normalised", 100), ("angles", "real_angular", 100),
                           ("complex", "complex_cartesian", 100)):
        if key in itf:
            mine[name] = itf[key]["points_per_s"] * per / 1e6
    out = {"unit": "M harmonics/s (lmax 9, FP64)", "paper": PAPER_MHARM_PER_S, "this_run_mi355x": mine,
           "note": "paper: evaluated and accumulated in registers; this run: every value stored to HBM"}
    if "cpu_baseline" in result:
        cb = result["cpu_baseline"]
        out["this_run_oracle_cpu"] = {"all_threads": cb["value"] * 100 / 1e6,
                                      "one_thread": cb["one_thread_value"] * 100 / 1e6,
                                      "note": "long-double test oracle, not an optimised CPU code"}
    return out


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _timed(fn, threads=None):
    """Seconds one call of fn takes, with `threads` OpenMP threads in the oracle
    (None: all of them)."""
    import oracle
    cores = oracle.num_threads()
    if threads:
        oracle.set_num_threads(threads)
    try:
        t0 = time.perf_counter()
        fn()
        return time.perf_counter() - t0
    finally:
        oracle.set_num_threads(cores)


def cpu_baseline(pts, lmax, sample, sh=None, dev=None):
    """The oracle on the host.  Headline: all its OpenMP threads on `sample` points
    of the headline workload, then one thread on a 32x smaller sample (comparable
    with a single-core figure).  Then the other workloads, all threads and one
    thread: the plain evaluation of 100,064 points (lmax 9), the 64-atom projector
    build (lmax 3), the backward pass on 10,000 points (lmax 6).  Last, the FP32
    error per l of the headline kernel against the oracle at the float inputs, on
    2^18 points of the headline workload (re-evaluated on the GPU: a point's values
    do not depend on its batch)."""
    import numpy as np

    import oracle
    from paper_2510_05282_amd import workloads
    chunk = 1 << 18
    n = min(sample, pts.shape[0])
    cores = oracle.num_threads()

    def head(m):
        for c in range(0, m, chunk):
            oracle.eval_xyz(lmax, pts[c:min(m, c + chunk)])

    dt = _timed(lambda: head(n))
    n1 = max(1, n // 32)
    dt1 = _timed(lambda: head(n1), threads=1)
    res = {"value": n / dt, "unit": "points/s", "cores": cores, "kind": "oracle",
           "sample": f"first {n} points of the same 2^26-point workload, lmax {lmax}, long double, "
                     f"{dt:.1f} s",
           "cpu_model": _cpu_model(), "one_thread_value": n1 / dt1,
           "one_thread_sample": f"first {n1} points, 1 thread, {dt1:.1f} s"}
    cfg = {}
    p1 = workloads.points_plain_eval(seed=0)
    cfg["plain_eval"] = {"workload": "100,064 points (100,000 isotropic + 64 special), lmax 9, FP64",
                         "n_points": p1.shape[0]}
    A = workloads.atom_spheres(seed=0)
    cfg["projectors"] = {"workload": "64 atoms, r=3 spheres on a 0.2 grid, lmax 3, FP64",
                         "n_points": int(A.offsets[-1])}
    pg = workloads.points_gradient(n=10_000, seed=0)
    G = np.random.default_rng(1).standard_normal((49, pg.shape[0]))
    cfg["gradient"] = {"workload": "backward pass, 10,000 points, lmax 6, FP64", "n_points": pg.shape[0]}
    calls = {"plain_eval": lambda: oracle.eval_xyz(9, p1),
             "projectors": lambda: oracle.projectors(3, A.centers, A.offsets, A.points, A.tables, A.r_max),
             "gradient": lambda: oracle.grad_xyz(6, pg, G)}
    for key, fn in calls.items():
        ta, t1 = _timed(fn), _timed(fn, threads=1)
        cfg[key].update({"points_per_s": cfg[key]["n_points"] / ta, "one_thread_points_per_s": cfg[key]["n_points"] / t1,
                         "seconds": ta, "one_thread_seconds": t1})
    res["configs"] = cfg
    if sh is not None:
        import torch
        idx = np.sort(np.random.default_rng(11).choice(pts.shape[0], 1 << 18, replace=False))
        p32 = np.ascontiguousarray(pts[idx].astype(np.float32))
        got = sh.sh_eval_f32(lmax, torch.from_numpy(p32).to(dev)).cpu().numpy()
        ref = oracle.eval_xyz(lmax, p32)
        err = np.abs(got.astype(np.longdouble) - ref).max(axis=1).astype(np.float64)
        res["fp32_error_per_l"] = {"max_abs_err": [float(err[l * l:(l + 1) ** 2].max()) for l in range(lmax + 1)],
                                   "bound": 5e-6,
                                   "sample": "2^18 random points of the headline workload rounded to float; "
                                             "oracle at the float inputs"}
    return res


def main():
    args = _parse()
    if args.traffic_from:
        if len(args.traffic_from) not in (2, 3):
            raise SystemExit("--traffic-from takes FETCH_CSV WRITE_CSV [FLOPS_CSV]")
        t = traffic_from_counters(*args.traffic_from[:2], n_points=args.n)
        if len(args.traffic_from) == 3:
            t["fp64_flops_per_launch"] = flops_from_counters(args.traffic_from[2])
        with open(TRAFFIC_FILE, "w") as fh:
            json.dump(t, fh, indent=1)
            fh.write("\n")
        print(json.dumps(t))
        return
    if args.counter_summary:
        counter_summary(args.counter_summary, args.counter_chunk, args.counter_kernels)
        return
    if args.serving_trace_summary:
        serving_trace_summary(args.serving_trace_summary)
        return
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

    if args.store_sweep:
        if n % 4096:
            raise SystemExit("--store-sweep needs --n a multiple of 4096")
        store_sweep(sh, xyz, out, max(5, args.steps // 2))
        return
    _log("headline: lmax 9 fp64")
    head = bench_forward(sh, xyz, out, 9, args.steps, args.warmup)
    _log("  ", json.dumps(head))
    if args.copy_probe:
        src = torch.ones(1 << 29, dtype=torch.float64, device=dev)  # 4 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        _log("copy probe: 4 GiB read + 4 GiB written by one copy kernel")
        del src, dst
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
                     "frac": head["frac"], "traffic": measured_traffic(),
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated)",
                     "kernel": HEADLINE_KERNEL, "kernel_ms": head["kernel_ms"],
                     "bytes_per_point": head["bytes_per_point"]},
    }
    rec = counter_record()
    if "fp64_flops_per_launch" in rec:
        # FP64 VALU use: the counted flops of one launch over this run's launch time
        tflops = rec["fp64_flops_per_launch"] / (head["kernel_ms"] * 1e-3) / 1e12
        result["roofline"]["fp64_valu"] = {
            "flops_per_point": rec["fp64_flops_per_launch"] / n, "tflops": tflops,
            "peak_tflops": FP64_VECTOR_PEAK_TFLOPS, "frac": tflops / FP64_VECTOR_PEAK_TFLOPS,
            "source": "SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes (rocprofv3, committed counter record)"}

    want = (lambda name: not args.no_extras and (not args.only or name in args.only.split(",")))
    if want("sweep"):
        sweep = {}
        xyz32 = xyz.float()
        for lmax in (2, 4, 6, 9):
            _log(f"sweep lmax {lmax}")
            sweep[f"f64_l{lmax}"] = bench_forward(sh, xyz, out, lmax, max(5, args.steps // 2), 2)
            sweep[f"f32_l{lmax}"] = bench_forward(sh, xyz32, out, lmax, max(5, args.steps // 2), 2)
            _log("  ", json.dumps({k: sweep[k] for k in (f"f64_l{lmax}", f"f32_l{lmax}")}))
        result["fp32"] = sweep["f32_l9"]
        result["lmax_sweep"] = sweep
        # the plain-evaluation workload: 100,064 points (a parity configuration, far too
        # small to fill the GPU: launch-bound)
        p1 = torch.from_numpy(workloads.points_plain_eval(seed=0)).to(dev)
        o1 = torch.empty((100, p1.shape[0]), dtype=torch.float64, device=dev)
        _, per = time_launches(lambda: sh.sh_eval(9, p1, out=o1), 20, 3)
        t1 = sum(per) / len(per)
        result["plain_eval"] = {"workload": "100,064 points, lmax 9, FP64", "n_points": p1.shape[0],
                                "kernel_ms": t1 * 1e3, "points_per_s": p1.shape[0] / t1}
        del p1, o1
        _log("write probe")
        result["write_probe"] = write_probe(out, 5)
        result["roofline"]["frac_of_write_probe"] = head["gbs"] / result["write_probe"]["gbs"]
        del xyz32
    if want("store_probes") and n % 4096 == 0:  # the probes take whole groups of 8 tiles
        _log("store-pattern probes")
        result["store_probes"] = bench_store_probes(xyz, out, head, max(5, args.steps // 2))
        result["roofline"]["frac_of_store_pattern"] = result["store_probes"]["frac_of_store_pattern"]
        _log("  ", json.dumps(result["store_probes"]))
    if want("interfaces"):
        _log("interfaces")
        result["interfaces"] = bench_interfaces(sh, xyz, out, max(5, args.steps // 2))
        _log("  ", json.dumps(result["interfaces"]))

    del out
    torch.cuda.empty_cache()
    if want("projectors"):
        _log("projectors")
        result["projectors"] = bench_projectors(sh, workloads, dev, 20)
        _log("  ", json.dumps(result["projectors"]))
    if want("gradient"):
        _log("gradient")
        result["gradient"] = bench_gradient(sh, workloads, dev, max(5, args.steps // 2))
        _log("  ", json.dumps(result["gradient"]))
        torch.cuda.empty_cache()
    if want("serving"):
        _log("serving")
        result["serving"] = bench_serving(sh, workloads, dev, args.serve_requests)
        _log("  ", json.dumps(result["serving"]))
        torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        _log("cpu baseline")
        cb = cpu_baseline(pts, 9, args.cpu_sample, sh, dev)
        # the GPU's rate on the same workloads, where this run measured it
        gpu = {"plain_eval": result.get("plain_eval", {}).get("points_per_s"),
               "projectors": result.get("projectors", {}).get("points_per_s"),
               "gradient": result.get("gradient", {}).get("backward_points_per_s")}
        for k, v in gpu.items():
            cb["configs"][k]["gpu_points_per_s"] = v
        if "fp32_error_per_l" in cb:
            result.setdefault("fp32", {})["max_abs_err_per_l"] = cb.pop("fp32_error_per_l")
        result["cpu_baseline"] = cb
    result["paper_context"] = paper_context(result)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
