"""Benchmark: magnification-map throughput on one MI355X.

A step is one whole map of the plain FP64 workload (1e5 Kroupa stars,
kappa_* = 0.45, kappa_s = 0, gamma = 0.45, 2000 x 2000 px of half-width 25,
1 ray per pixel, FMM order 20): tree build, P2M/M2M/M2L/P2L/L2L, leaf tables,
ray shooting and IPM, with the stars already resident in device memory and
the map left in device memory.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-variants]

Beside the headline, `variants` reports the same map in mixed precision, the
256-map batched workload (one fused call against 256 single calls), and the
paper's Table 1 map (context: the paper's time is for other hardware).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
IPM_SRC = os.path.join(ROOT, "paper_2506_02114_amd", "csrc", "ipm.hip")
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rays/sec and maps/hour on 1 MI355X at ≤1e-4 pixel error; plain vs mixed/batched"
FP64_VECTOR_PEAK_TFLOPS = 78.6          # MI355X FP64 vector, dense

# HBM traffic of one launch of each IPM kernel on this workload, from two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE, KiB per dispatch), scaled by
# the same counters' reading of a plain 1 GiB device copy (--copy-check):
# FETCH_SIZE x 2.0, WRITE_SIZE x 1.0.  Valid only for the IPM source they were
# taken with, identified by its SHA-256 prefix.
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
IPM_TRAFFIC = {"ipm_sha256": "a8e4288d3ca909d0",                     # (fetch KiB, write KiB)
               "k_ipm": (719914.5, 4175274.65625), "k_band": (1486720.8125, 31250.0)}


def file_sha(path: str) -> str:
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def shoot_flops(stats: dict) -> float:
    """Algorithmic FP64 flops of the ray-shooting kernel for one map:
    10 per ray-star pair (2 sub, |dz|^2 3, divide 1, 2 x fused accumulate 4),
    8 per Horner step of the degree p-1 derivative polynomial (p-1 steps),
    26 per ray for the vertex position, zeta, macro model, sheet and pixel
    coordinates."""
    p = stats["order"]
    return 10.0 * stats["near_pairs"] + (8.0 * (p - 1) + 26.0) * stats["n_rays"]


def band_flops(stats: dict) -> float:
    """Algorithmic FP64 flops of the per-band IPM kernel for one map:
    30 per (large triangle, pixel row) item (3 edges clipped to the row, 2
    crossings x 3 each; for the ~2 edges present: extent, first and last
    column and deposit factor, 6 each) and 6 per column difference deposited
    (the squared distance 2 and its factor 1, the difference of two terms 1,
    the change from the previous column 1, the column boundary 1)."""
    return 30.0 * stats["n_band_rows"] + 6.0 * stats["n_band_pieces"]


def cells_flops(stats: dict) -> float:
    """Algorithmic FP64 flops of the per-cell IPM kernel for one map: 18 per
    cell (twice the signed area of both triangles, 9 each), 55 per triangle
    inside a 2 x 2 pixel box (local coordinates 6, area 9, weight 1, the part
    below v = 1 7, the corner cut by u = 1 and the part left of it 8, the
    corner's vertices and its part below v = 1 16, four pieces 8), 21 per
    (triangle, pixel column) item (3 edges clipped to the column, 7 each) and
    29 per pixel piece (the area below the next row line from 3 clipped
    edges, 26; the piece and its deposit, 3)."""
    return (18.0 * stats["n_cells"] + 55.0 * stats["n_small"] + 21.0 * stats["n_col_items"]
            + 29.0 * stats["n_col_pieces"])


def mixed_variant(lens, spec, out, ref) -> dict:
    """The same map in the mixed-precision mode: time per map and its
    per-pixel difference from the FP64 map just made (`ref`)."""
    import torch
    lens.map(out=out, precision="mixed", **spec)
    torch.cuda.synchronize()
    ts = []
    for _ in range(3):
        _, s = lens.map(out=out, precision="mixed", timing=1, **spec)
        ts.append(s["t_total_ms"])
    d = ((out - ref).abs() / ref.clamp_min(1e-300))
    return {"ms_per_map": sum(ts) / len(ts), "rays_per_s": s["n_rays"] / (sum(ts) / len(ts) * 1e-3),
            "max_rel_vs_fp64": float(d.max()), "median_rel_vs_fp64": float(d.median())}


def batched_variant() -> dict:
    """The 256-map batched workload (seed 4; kappa, gamma, s and star counts
    drawn; 1000^2 px, mixed precision): one fused batch call (leaf sizes from
    the autotuner, cached after a first call) against 256 single-map calls."""
    import torch
    import paper_2506_02114_amd as mlm
    import workloads as W
    dev = torch.device("cuda:0")
    lenses, reqs, outs = [], [], []
    for wl in W.batch_draws(256, seed=4):
        sf = wl.stars()
        L = wl.lens
        lenses.append(mlm.Lens(L.kappa_star, L.kappa_smooth, L.gamma, torch.from_numpy(sf.x).to(dev),
                               torch.from_numpy(sf.y).to(dev), torch.from_numpy(sf.m).to(dev)))
        reqs.append(dict(wl.map.asdict(), precision="mixed"))
        outs.append(torch.empty((wl.map.n2, wl.map.n1), dtype=torch.float64, device=dev))
    print("[bench] batched: 256 lenses ready", file=sys.stderr, flush=True)
    mlm.map_batch(lenses, reqs, outs, autotune=True)          # tunes and warms
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, b = mlm.map_batch(lenses, reqs, outs, autotune=True)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    for lens, r, o in zip(lenses, reqs, outs):
        lens.map(out=o, **r)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    print("[bench] batched: done", file=sys.stderr, flush=True)
    return {"maps": 256, "rays": b["n_rays"], "s_per_batch": t_batch, "rays_per_s": b["n_rays"] / t_batch,
            "maps_per_hour": 256 * 3600.0 / t_batch, "s_256_single_calls": t_seq, "chunks": b["n_chunks"],
            "stage_ms": {"prep": b["t_prep_ms"], "shoot": b["t_shoot_ms"], "ipm": b["t_ipm_ms"]}}


def paper_table1_variant() -> dict:
    """The paper's Table 1 map (IPM + FMM, circular star region), as far as
    the paper fixes it: kappa = kappa_* = gamma = 0.6 (its sec. 4.1
    comparison lens), equal masses, a 20 x 20 theta_* map of 2000 x 2000 px,
    1 ray per pixel, flux fraction 1/1000 (its default).  The star disc
    covers the shooting region with a 1.2 margin, about 26 700 stars (the
    paper says ~27 000).  The paper's 0.763 s was measured on an NVIDIA A100
    80 GB: context for the same map on other hardware, not a target."""
    import math
    import torch
    import paper_2506_02114_amd as mlm
    import workloads as W
    kappa = gamma = 0.6
    f = 1e-3
    r = math.sqrt(kappa / f)                      # equal masses: <m^2>/<m> = 1
    dx1, dx2 = (10.0 + r) / abs(1 - kappa + gamma), (10.0 + r) / abs(1 - kappa - gamma)
    n = int(round(kappa * (1.2 * math.hypot(dx1, dx2)) ** 2))
    sf = W.star_field(n, kappa, "equal", seed=1)
    dev = torch.device("cuda:0")
    lens = mlm.Lens(kappa, 0.0, gamma, torch.from_numpy(sf.x).to(dev), torch.from_numpy(sf.y).to(dev),
                    torch.from_numpy(sf.m).to(dev))
    spec = dict(hw1=10.0, hw2=10.0, n1=2000, n2=2000, rays_per_pixel=1.0, flux_fraction=f)
    out = torch.empty((2000, 2000), dtype=torch.float64, device=dev)
    lens.map(out=out, **spec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        _, st = lens.map(out=out, **spec)
    torch.cuda.synchronize()
    s_map = (time.perf_counter() - t0) / 3
    return {"stars": n, "rays": st["n_rays"], "order": st["order"], "s_per_map": s_map,
            "rays_per_s": st["n_rays"] / s_map, "paper_s_per_map": 0.763, "paper_hardware": "NVIDIA A100 80 GB",
            "paper_over_this": 0.763 / s_map, "precision": "fp64"}


def copy_check() -> None:
    """A plain device copy of 1 GiB (2^27 doubles), three times: the reference
    reading for the HBM byte counters."""
    import torch
    n = 1 << 27
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}), flush=True)


def cpu_baseline(wl, spec, region, nthreads: int) -> dict:
    """The oracle (plain FP64 C, FMM + per-pixel IPM) on a bounded sample of the
    same map: its full FMM build plus a strip of ray rows through the middle
    of the grid, extrapolated to all rows."""
    import numpy as np
    import oracle

    sf = wl.stars()
    L = wl.lens
    ol = oracle.Lens(L.kappa_star, L.kappa_smooth, L.gamma, sf.x, sf.y, sf.m)
    R = oracle.region(ol, **spec)
    t0 = time.perf_counter()
    F = oracle.FMM(ol, R.L0, spec["order"], nthreads=nthreads)
    t_build = time.perf_counter() - t0
    rows = 64
    r0 = R.nr2 // 2 - rows // 2
    dep = np.zeros(R.n1 * R.n2)
    st = np.zeros(5)
    t0 = time.perf_counter()
    done = 0
    while done < rows or time.perf_counter() - t0 < 8.0:
        b = r0 + done
        if b + 16 >= R.nr2:
            break
        wx, wy = oracle.shoot_rows(R, ol, b, b + 17, F, nthreads)
        oracle.ipm_rows(R, b, b + 16, wx, wy, dep, st)
        done += 16
        if time.perf_counter() - t0 > 20.0:
            break
    t_rows = time.perf_counter() - t0
    t_full = t_build + t_rows * (R.nr2 - 1) / done
    rays = R.nr1 * R.nr2
    return {"value": rays / t_full, "unit": "rays/s", "cores": nthreads, "kind": "oracle",
            "sample": f"oracle FMM build ({t_build:.1f} s, p={spec['order']}) + {done} of {R.nr2 - 1} cell rows "
                      f"shot and apportioned ({t_rows:.1f} s), extrapolated to the full map "
                      f"({t_full:.0f} s for {rays} rays)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-check", action="store_true", help="only run the plain copy used to scale HBM counters")
    ap.add_argument("--no-variants", action="store_true", help="skip the mixed-precision and batched measurements")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the map path has no multi-GPU mode); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_check:
        copy_check()
        return

    import torch

    import paper_2506_02114_amd as mlm
    import workloads as W

    wl = W.config("plain_large")
    spec = wl.map.asdict()
    sf = wl.stars()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    L = wl.lens
    lens = mlm.Lens(L.kappa_star, L.kappa_smooth, L.gamma, torch.from_numpy(sf.x).to(dev),
                    torch.from_numpy(sf.y).to(dev), torch.from_numpy(sf.m).to(dev))
    region = lens.region(**spec)
    out = torch.empty((spec["n2"], spec["n1"]), dtype=torch.float64, device=dev)
    for k in range(args.warmup):
        lens.map(out=out, **spec)
        print(f"[bench] warmup {k + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        _, s = lens.map(out=out, timing=1, **spec)
        stats.append(s)
        print(f"[bench] step {k + 1}/{args.steps}: {s['t_total_ms']:.2f} ms device", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    # one more map, untimed, for the IPM kernels' work counts (timing 2)
    _, counts = lens.map(out=out, timing=2, **spec)
    torch.cuda.synchronize()
    rays = stats[0]["n_rays"]
    value = rays / (ms * 1e-3)

    def avg(k):
        return sum(s[k] for s in stats) / len(stats)

    t_shoot, t_ipm, t_band = avg("t_shoot_ms"), avg("t_ipm_ms"), avg("t_band_ms")
    flops = shoot_flops(stats[0])
    shoot_roof = {"bound": "alu", "achieved": flops / (t_shoot * 1e-3) / 1e12, "peak": FP64_VECTOR_PEAK_TFLOPS,
                  "unit": "TFLOP/s", "kernel": "k_shoot", "launch_ms": t_shoot}
    shoot_roof["frac"] = shoot_roof["achieved"] / shoot_roof["peak"]
    # the two IPM kernels (one launch each per map on this workload); the
    # headline roofline is the one that takes longer
    fresh = IPM_TRAFFIC["ipm_sha256"] == file_sha(IPM_SRC)

    def traffic(kernel):
        t = IPM_TRAFFIC.get(kernel) if fresh else None
        return None if t is None else (t[0] * FETCH_SCALE + t[1] * WRITE_SCALE) * 1024.0

    t_cells = avg("t_cells_ms")
    cells_roof = {"bound": "alu", "achieved": cells_flops(counts) / (t_cells * 1e-3) / 1e12,
                  "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "traffic": traffic("k_ipm"), "kernel": "k_ipm",
                  "launch_ms": t_cells, "launches_per_step": stats[0]["n_ipm_launches"],
                  "cells": counts["n_cells"], "small_triangles": counts["n_small"],
                  "column_items": counts["n_col_items"], "pieces": counts["n_col_pieces"]}
    cells_roof["frac"] = cells_roof["achieved"] / cells_roof["peak"]
    band_roof = {"bound": "alu", "achieved": band_flops(counts) / (t_band * 1e-3) / 1e12,
                 "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "traffic": traffic("k_band"), "kernel": "k_band",
                 "launch_ms": t_band, "launches_per_step": stats[0]["n_ipm_launches"],
                 "row_items": counts["n_band_rows"], "pieces": counts["n_band_pieces"]}
    band_roof["frac"] = band_roof["achieved"] / band_roof["peak"]
    roof, other = (cells_roof, band_roof) if t_cells >= t_band else (band_roof, cells_roof)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded star field of the workload's shape)",
        "config": {"workload": "plain_large: 1e5 Kroupa (0.08-1.5) stars, kappa*=0.45, kappa_s=0, gamma=0.45, "
                               "2000x2000 px, half-width 25, 1 ray/px, FMM order 20, leaf <= 32 block stars",
                   "rays_per_map": rays, "grid": [region["nr1"], region["nr2"]], "precision": "fp64"},
        "maps_per_hour": 3600.0 / (ms * 1e-3),
        "stages_ms": {"tree": avg("t_tree_ms"), "fmm": avg("t_fmm_ms"), "shoot": t_shoot, "ipm": t_ipm,
                      "ipm_cells": avg("t_cells_ms"), "ipm_band": t_band, "total_device": avg("t_total_ms")},
        "roofline": roof,
        "roofline_" + other["kernel"]: other,
        "roofline_shoot": shoot_roof,
        "tree": {"nodes": stats[0]["n_nodes"], "leaves": stats[0]["n_leaves"], "levels": stats[0]["n_levels"],
                 "near_pairs_per_ray": stats[0]["near_pairs"] / rays},
        "ipm": {"triangles": 2 * stats[0]["n_cells"], "row_path_triangles": stats[0]["n_big"],
                "row_path_rows": counts["n_big_rows"]},
    }
    if not args.no_variants:
        variants = {}
        ref = out.clone()
        try:
            variants["mixed_plain_large"] = mixed_variant(lens, spec, torch.empty_like(out), ref)
        except Exception as e:   # a variant must not cost the headline line
            variants["mixed_plain_large"] = {"error": str(e)}
        try:
            variants["batched_256"] = batched_variant()
        except Exception as e:
            variants["batched_256"] = {"error": str(e)}
        try:
            variants["paper_table1"] = paper_table1_variant()
        except Exception as e:
            variants["paper_table1"] = {"error": str(e)}
        line["variants"] = variants
    if not args.no_cpu_baseline:
        nthreads = min(16, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), os.cpu_count() or 1)
        line["cpu_baseline"] = cpu_baseline(wl, spec, region, nthreads)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
