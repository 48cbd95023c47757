"""Benchmark: magnification-map throughput on one MI355X.

A step is one whole map of the plain FP64 workload (1e5 Kroupa stars,
kappa_* = 0.45, kappa_s = 0, gamma = 0.45, 2000 x 2000 px of half-width 25,
1 ray per pixel, FMM order 20): tree build, P2M/M2M/M2L/P2L/L2L, leaf tables,
ray shooting and IPM, with the stars already resident in device memory and
the map left in device memory.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-variants]

Beside the headline, `variants` reports the same map in mixed precision
(with its per-pixel error against FP64), the 256-map batched workload (one
fused call against 256 single calls, and their differences), the paper's
Table 1 maps (IPM and IRS, circular and rectangular star regions; context:
the paper's times are for other hardware) and the high-magnification
workload in FP64 and mixed precision.  `cpu_baseline` times the oracle on the
host and states the FMM's method-level error on a strip of the map against
the exact direct sum.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
IPM_SRCS = [os.path.join(ROOT, "paper_2506_02114_amd", "csrc", f) for f in ("ipm.hip", "colarea.hpp")]
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rays/sec and maps/hour on 1 MI355X at ≤1e-4 pixel error; plain vs mixed/batched"
FP64_VECTOR_PEAK_TFLOPS = 78.6          # MI355X FP64 vector, dense

# HBM traffic of one launch of each IPM kernel on this workload, from two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE, KiB per dispatch), scaled by
# the same counters' reading of a plain 1 GiB device copy (--copy-check):
# FETCH_SIZE x 2.0, WRITE_SIZE x 1.0.  Valid only for the IPM sources they were
# taken with (ipm.hip and colarea.hpp), identified by the SHA-256 prefix of
# the two files' bytes in that order.
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
IPM_TRAFFIC = {"ipm_sha256": "a530c3ebbb5bdec1",                     # (fetch KiB, write KiB)
               "k_ipm": (719906.85, 2278836.5375), "k_band_queue1": (5470672.9125, 280193.3625)}
# Wavefront vector instructions per launch of the same kernels (SQ_INSTS_VALU,
# same runs and source).  A wave64 vector instruction holds its SIMD four
# cycles, so 1024 SIMDs at 2.4 GHz issue at most 6.144e11 of them per second:
# the kernels' issue time, set against their launch time, says how close they
# run to the vector-issue limit that bounds them.
IPM_VALU = {"k_ipm": 2.057e+09, "k_band_queue1": 1.173e+09}
VALU_ISSUE_PER_S = 1024 * 2.4e9 / 4
# The IPM scatter per launch (same runs and source): FP64 deposits summed in
# LDS (SQ_INSTS_LDS_ATOMIC_BANDWIDTH x 64 B / 8 B) and atomic requests to L2
# (TCC_ATOMIC: window flushes, deposits outside the window, shared band rows)
IPM_SCATTER = {"k_ipm": {"lds_atomic_lanes": 3.239e8, "l2_atomic_requests": 5.790e7},
               "k_band_queue1": {"lds_atomic_lanes": 1.053e9, "l2_atomic_requests": 4.340e6}}
LDS_BYTES_PER_S = 256 * 2.4e9 * 128      # 128 bytes per clock per CU


def file_sha(paths) -> str:
    import hashlib
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


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


def rel_errors(a, b) -> dict:
    """max, p99.9 and median of |a - b| / b over the pixels with b > 0 (torch
    tensors on the device), and whether the rest agree exactly."""
    import torch
    pos = b > 0
    d = ((a[pos] - b[pos]).abs() / b[pos]).double()
    q = torch.quantile(d[torch.randperm(d.numel(), device=d.device)[:1 << 24]], 0.999) if d.numel() else d.sum()
    return {"max": float(d.max()), "p999": float(q), "median": float(d.median()),
            "zero_pixels_agree": bool((a[~pos] == b[~pos]).all())}


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
    ms = sum(ts) / len(ts)
    return {"ms_per_map": ms, "rays_per_s": s["n_rays"] / (ms * 1e-3), "maps_per_hour": 3600.0 / (ms * 1e-3),
            "vs_fp64": rel_errors(out, ref)}


def highmag_variant() -> dict:
    """The high-magnification workload (1e6 Salpeter stars, kappa_* = 0.01,
    kappa_s = 0.82, gamma = 0.1725, 4000^2 px of half-width 10, 1 ray per
    pixel: 2.1e10 rays) in FP64 and mixed precision, with the mixed map's
    per-pixel error against the FP64 map."""
    import torch
    import paper_2506_02114_amd as mlm
    import workloads as W
    wl = W.config("mixed_highmag")
    sf = wl.stars()
    L = wl.lens
    dev = torch.device("cuda:0")
    lens = mlm.Lens(L.kappa_star, L.kappa_smooth, L.gamma, torch.from_numpy(sf.x).to(dev),
                    torch.from_numpy(sf.y).to(dev), torch.from_numpy(sf.m).to(dev))
    spec = wl.map.asdict()
    m64 = torch.empty((spec["n2"], spec["n1"]), dtype=torch.float64, device=dev)
    m32 = torch.empty_like(m64)
    out = {}
    for prec, m in (("fp64", m64), ("mixed", m32)):
        _, s = lens.map(out=m, precision=prec, timing=1, **spec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, s = lens.map(out=m, precision=prec, timing=1, **spec)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        out[prec] = {"s_per_map": sec, "rays_per_s": s["n_rays"] / sec, "maps_per_hour": 3600.0 / sec,
                     "stages_ms": {"tree": s["t_tree_ms"], "fmm": s["t_fmm_ms"], "shoot": s["t_shoot_ms"],
                                   "ipm": s["t_ipm_ms"]}}
        print(f"[bench] high magnification {prec}: {sec:.3f} s", file=sys.stderr, flush=True)
    out["rays"] = s["n_rays"]
    out["order"] = s["order"]
    out["mixed_vs_fp64"] = rel_errors(m32, m64)
    return out


def batched_variant() -> dict:
    """The 256-map batched workload (seed 4; kappa, gamma, s and star counts
    drawn; 1000^2 px, mixed precision): one fused batch call with leaf sizes
    from the autotuner (cached after a first call), timed; the same batch at
    the default leaf size against 256 single-map calls (the fusion changes
    nothing but the order of sums); and every autotuned mixed map against an
    FP64 single-map call of the same lens (the mode's error over the whole
    batch)."""
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
    per_map, b = mlm.map_batch(lenses, reqs, outs, autotune=True)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    tuned = [o.clone() for o in outs]
    from collections import Counter
    schedules = Counter((s["leaf_max"], s["order"], s["big_pixels"]) for s in per_map)
    # fusion: the batch at the default leaf size against single calls
    mlm.map_batch(lenses, reqs, outs, autotune=False)
    fused = [o.clone() for o in outs]
    t0 = time.perf_counter()
    for lens, r, o in zip(lenses, reqs, outs):
        lens.map(out=o, **r)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    worst = 0.0
    for f, o in zip(fused, outs):
        pos = o > 0
        worst = max(worst, float(((f[pos] - o[pos]).abs() / o[pos]).max()) if bool(pos.any()) else 0.0)
        assert bool((f[~pos] == 0).all())
    del fused
    # accuracy: every autotuned mixed map against its FP64 single-map call
    errs = []
    for lens, r, f, o in zip(lenses, reqs, tuned, outs):
        lens.map(out=o, **dict(r, precision="fp64"))
        pos = o > 0
        if bool(pos.any()):
            errs.append(((f[pos] - o[pos]).abs() / o[pos]).float())
    e = torch.cat(errs)
    q = torch.quantile(e[torch.randperm(e.numel(), device=e.device)[:1 << 24]].double(), 0.999)
    torch.cuda.synchronize()
    print("[bench] batched: done", file=sys.stderr, flush=True)
    return {"maps": 256, "rays": b["n_rays"], "s_per_batch": t_batch, "rays_per_s": b["n_rays"] / t_batch,
            "maps_per_hour": 256 * 3600.0 / t_batch, "s_256_single_calls": t_seq, "chunks": b["n_chunks"],
            "stage_ms": {"prep": b["t_prep_ms"], "shoot": b["t_shoot_ms"], "ipm": b["t_ipm_ms"]},
            "fused_vs_single_max_rel_default_leaf": worst,
            "tuned_schedules": [{"leaf_max": k[0], "order": k[1], "big_pixels": k[2], "maps": v}
                                for k, v in sorted(schedules.items())],
            "autotuned_mixed_vs_fp64_single": {"max": float(e.max()), "p999": float(q),
                                               "median": float(e.median()), "pixels": int(e.numel())}}


def paper_table1_variant() -> dict:
    """The paper's Table 1 map with the FMM, as far as the paper fixes it:
    kappa = kappa_* = gamma = 0.6 (its sec. 4.1 comparison lens), equal
    masses, a 20 x 20 theta_* map of 2000 x 2000 px, flux fraction 1/1000
    (its default), IPM at 1 ray per pixel and IRS at 100, stars in a disc or
    a rectangle covering the shooting region with a 1.2 margin.  The paper's
    times were measured on an NVIDIA A100 80 GB: context for the same maps on
    other hardware, not a target."""
    import torch
    import paper_2506_02114_amd as mlm
    import workloads as W
    paper = {("ipm", "circle"): 0.763, ("ipm", "rect"): 0.839, ("irs", "circle"): 0.748, ("irs", "rect"): 2.141}
    dev = torch.device("cuda:0")
    out = torch.empty((2000, 2000), dtype=torch.float64, device=dev)
    res = {}
    for shape in ("circle", "rect"):
        L, mspec, aspect = W.paper_table1(shape)
        if shape == "circle":
            sf = W.star_field(L.n_stars, L.kappa_star, "equal", seed=L.seed)
            lens = mlm.Lens(L.kappa_star, 0.0, L.gamma, sf.x, sf.y, sf.m)
        else:
            sf = W.rect_field(L.n_stars, L.kappa_star, aspect, "equal", seed=L.seed)
            lens = mlm.Lens(L.kappa_star, 0.0, L.gamma, sf.x, sf.y, sf.m, sheet="rect", rect_aspect=aspect)
        for mapping, rho in (("ipm", 1.0), ("irs", 100.0)):
            spec = dict(mspec.asdict(), rays_per_pixel=rho, mapping=mapping)
            lens.map(out=out, **spec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(2):
                _, st = lens.map(out=out, **spec)
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) / 2
            res[f"{mapping}_{shape}"] = {"stars": L.n_stars, "rays": st["n_rays"], "order": st["order"],
                                         "s_per_map": sec, "rays_per_s": st["n_rays"] / sec,
                                         "paper_s_per_map": paper[(mapping, shape)],
                                         "paper_over_this": paper[(mapping, shape)] / sec}
            print(f"[bench] table 1 {mapping} {shape}: {sec:.4f} s", file=sys.stderr, flush=True)
    res["paper_hardware"] = "NVIDIA A100 80 GB"
    res["precision"] = "fp64"
    return res


def macrocaustic_variant() -> dict:
    """A map across a macro fold caustic (the macro potential to third order,
    app. D; workloads.macrocaustic): the library finds the macroimages of the
    map inside the star disc and maps them in FP64."""
    import torch
    import paper_2506_02114_amd as mlm
    import workloads as W
    L, mspec, psi3 = W.macrocaustic()
    sf = W.star_field(L.n_stars, L.kappa_star, "equal", seed=L.seed)
    dev = torch.device("cuda:0")
    lens = mlm.Lens(L.kappa_star, L.kappa_smooth, L.gamma, torch.from_numpy(sf.x).to(dev),
                    torch.from_numpy(sf.y).to(dev), torch.from_numpy(sf.m).to(dev), psi3=psi3)
    spec = mspec.asdict()
    R = lens.region(**spec)
    out = torch.empty((spec["n2"], spec["n1"]), dtype=torch.float64, device=dev)
    lens.map(out=out, **spec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        _, st = lens.map(out=out, timing=1, **spec)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / 3
    mu = out.cpu().numpy()
    half = spec["n2"] // 2
    print(f"[bench] macrocaustic: {sec * 1e3:.1f} ms", file=sys.stderr, flush=True)
    return {"stars": L.n_stars, "psi3": list(psi3), "rays": st["n_rays"], "order": st["order"],
            "region": {k: R[k] for k in ("X1", "X2", "dX1", "dX2", "nr1", "nr2")}, "ms_per_map": sec * 1e3,
            "rays_per_s": st["n_rays"] / sec, "stages_ms": {"tree": st["t_tree_ms"], "fmm": st["t_fmm_ms"],
                                                            "shoot": st["t_shoot_ms"], "ipm": st["t_ipm_ms"]},
            "mean_mu_below_caustic": float(mu[:half].mean()), "mean_mu_above_caustic": float(mu[half:].mean())}


def learned_variant() -> dict:
    """The learned refinement (a small network flags the cells worth the
    refinement test): cells of two fields of the 1e5-star lens type and two
    of the high-magnification type (8e3 and 2e4 stars, 1e5 sampled cells
    each) labelled by the plain refinement test on the device, the network
    trained on them by the library's kernels, then a fresh
    high-magnification field (2e4 stars, seed 3999, 400^2 px of half-width
    1) mapped with no refinement, with every cell tested, and with the
    flagged cells only: times, flags and map differences."""
    import numpy as np
    import torch
    import paper_2506_02114_amd as mlm
    import workloads as W
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(2001)
    feats, labels, domain = [], [], []
    t0 = time.perf_counter()
    for ks, kss, g, mf, lo, hi, seed, n, hw in ((0.45, 0.0, 0.45, "kroupa", 0.08, 1.5, 2001, 8000, 4.0),
                                                 (0.45, 0.0, 0.45, "kroupa", 0.08, 1.5, 2002, 8000, 4.0),
                                                 (0.01, 0.82, 0.1725, "salpeter", 0.1, 1.0, 3001, 20000, 1.0),
                                                 (0.01, 0.82, 0.1725, "salpeter", 0.1, 1.0, 3002, 20000, 1.0)):
        sf = W.star_field(n, ks, mf, seed=seed, m_lo=lo, m_hi=hi)
        gl = mlm.Lens(ks, kss, g, sf.x, sf.y, sf.m)
        spec = dict(hw1=hw, hw2=hw, n1=400, n2=400, order=16)
        R = gl.region(**spec)
        cells = np.stack([rng.integers(0, R["nr1"] - 1, 100000), rng.integers(0, R["nr2"] - 1, 100000)], 1)
        f, y = gl.cell_samples(cells, **spec)
        feats.append(f)
        labels.append(y)
        domain.append(np.full(len(y), 0 if ks > 0.1 else 1))
        gl.close()
    t_label = time.perf_counter() - t0
    X, y, dom = np.concatenate(feats), np.concatenate(labels), np.concatenate(domain)
    perm = rng.permutation(len(y))
    X, y, dom = X[perm], y[perm], dom[perm]
    ntr = int(0.8 * len(y))
    pw = float(min((1 - y.mean()) / max(y.mean(), 1e-6), 20.0))
    net = mlm.Refiner(seed=7)
    t0 = time.perf_counter()
    net.train(X[:ntr], y[:ntr], epochs=20, batch=4096, lr=2e-3, pos_weight=pw, seed=2)
    t_train = time.perf_counter() - t0
    zv, yv, dv = net.predict(X[ntr:]), y[ntr:], dom[ntr:]
    folded = np.array([len(set(r)) > 1 for r in X[ntr:, 8:]])
    thr = min(float(np.quantile(zv[(yv == 1) & ~folded & (dv == d)], 0.02)) for d in (0, 1))
    flag = (zv > thr) | folded
    sf = W.star_field(20000, 0.01, "salpeter", seed=3999, m_lo=0.1, m_hi=1.0)
    gl = mlm.Lens(0.01, 0.82, 0.1725, torch.from_numpy(sf.x).to(dev), torch.from_numpy(sf.y).to(dev),
                  torch.from_numpy(sf.m).to(dev))
    spec = dict(hw1=1.0, hw2=1.0, n1=400, n2=400, order=16)
    out = {k: torch.empty((400, 400), dtype=torch.float64, device=dev) for k in ("none", "plain", "learned")}
    st = {}
    for mode in ("none", "plain", "learned"):
        kw = dict(refine=mode, refiner=net, refine_threshold=thr) if mode == "learned" else dict(refine=mode)
        gl.map(out=out[mode], **spec, **kw)
        _, st[mode] = gl.map(out=out[mode], timing=1, **spec, **kw)
        print(f"[bench] learned refinement: refine={mode} {st[mode]['t_total_ms']:.1f} ms", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    full = out["plain"]
    norm = float(full.abs().sum())
    return {"cells_per_map": st["none"]["n_cells"], "label_s": t_label, "train_s": t_train, "train_cells": ntr,
            "heldout_recall": float(flag[yv == 1].mean()), "heldout_precision": float(yv[flag].mean()),
            "ms_per_map": {k: v["t_total_ms"] for k, v in st.items()},
            "refine_ms": {k: st[k]["t_refine_ms"] for k in ("plain", "learned")},
            "cells_tested": {k: st[k]["n_refine_candidates"] for k in ("plain", "learned")},
            "cells_refined": {k: st[k]["n_refined"] for k in ("plain", "learned")},
            "l1_vs_full_refinement": {k: float((out[k] - full).abs().sum()) / norm for k in ("none", "learned")}}


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


def host_cpu() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, spec, nthreads: int, gpu_strip=None) -> dict:
    """The oracle (plain FP64 C, FMM + per-pixel IPM), rebuilt -O3
    -march=native for this host, on a bounded sample of the same map: its
    full FMM build, then strips of cell rows through the middle of the grid,
    shot and apportioned by `nthreads` workers (each strip on one thread, its
    own deposit array), extrapolated to all rows.  With gpu_strip = (rows,
    map of those rows from the GPU), also the method-level error: the same
    rows mapped with the exact direct sum against the GPU's FMM strip."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import oracle

    tmp = tempfile.mkdtemp(prefix="oracle_native_")
    oracle.use_native_build(tmp)
    sf = wl.stars()
    L = wl.lens
    ol = oracle.Lens(L.kappa_star, L.kappa_smooth, L.gamma, sf.x, sf.y, sf.m)
    R = oracle.region(ol, **spec)
    t0 = time.perf_counter()
    F = oracle.FMM(ol, R.L0, spec["order"], nthreads=nthreads)
    t_build = time.perf_counter() - t0
    strip = 16
    times = {"shoot": 0.0, "ipm": 0.0}

    def work(b):
        dep = np.zeros(R.n1 * R.n2)
        st = np.zeros(5)
        a = time.perf_counter()
        wx, wy = oracle.shoot_rows(R, ol, b, b + strip + 1, F, 1)
        m = time.perf_counter()
        oracle.ipm_rows(R, b, b + strip, wx, wy, dep, st)
        e = time.perf_counter()
        return m - a, e - m

    r0 = R.nr2 // 2 - 8 * strip * nthreads // 2
    done = 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(nthreads) as ex:
        while time.perf_counter() - t0 < 12.0 and r0 + done + strip * nthreads < R.nr2 - 1:
            starts = [r0 + done + k * strip for k in range(nthreads)]
            for ts, ti in ex.map(work, starts):
                times["shoot"] += ts
                times["ipm"] += ti
            done += strip * nthreads
    t_rows = time.perf_counter() - t0
    t_full = t_build + t_rows * (R.nr2 - 1) / done
    rays = R.nr1 * R.nr2
    out = {"value": rays / t_full, "unit": "rays/s", "cores": nthreads, "kind": "oracle",
           "sample": f"oracle rebuilt -O3 -march=native on this host ({host_cpu()}, nproc {os.cpu_count()}, "
                     f"{nthreads} threads used: the box's CPU share for one GPU): FMM build {t_build:.1f} s (p="
                     f"{spec['order']}) + {done} of {R.nr2 - 1} cell rows shot and apportioned in {t_rows:.1f} s, "
                     f"extrapolated to the full map ({t_full:.0f} s for {rays} rays)",
           "shoot_us_per_ray_thread": times["shoot"] / (done * R.nr1) * 1e6,
           "ipm_us_per_triangle_thread": times["ipm"] / (done * 2 * (R.nr1 - 1)) * 1e6}
    if gpu_strip is not None:
        (a, b), gmu = gpu_strip
        t0 = time.perf_counter()
        ref = oracle.magnification_map(ol, spec, method="direct", rows=(a, b), nthreads=nthreads)
        big = ref.mu >= 1e-6
        rel = np.abs(gmu[big] - ref.mu[big]) / ref.mu[big]
        out["fmm_p20_vs_direct_strip"] = {"rows": [a, b], "pixels": int(big.sum()), "max_rel": float(rel.max()),
                                          "median_rel": float(np.median(rel)),
                                          "max_abs_below_1e-6": float(np.abs(gmu[~big] - ref.mu[~big]).max()),
                                          "s_direct": time.perf_counter() - t0}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-check", action="store_true", help="only run the plain copy used to scale HBM counters")
    ap.add_argument("--no-variants", action="store_true", help="skip the mixed-precision and batched measurements")
    ap.add_argument("--only", choices=["mixed", "batched", "table1", "highmag", "learned", "macrocaustic"],
                    help="run one variant alone (for profiling) and print it as the JSON line")
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

    if args.only:
        torch.cuda.set_device(0)
        fn = {"batched": batched_variant, "table1": paper_table1_variant, "highmag": highmag_variant,
              "learned": learned_variant, "macrocaustic": macrocaustic_variant}.get(args.only)
        if fn is None:
            print("--only mixed runs with the headline map: use the default run", file=sys.stderr)
            sys.exit(2)
        print(json.dumps({"variant": args.only, **fn()}), flush=True)
        return

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
    # the same map with every kernel on one stream (the large-triangle passes
    # after the cell pass instead of beside it), for comparison
    one = []
    for _ in range(3):
        _, s1 = lens.map(out=out, timing=1, one_stream=1, **spec)
        one.append(s1)
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
    fresh = IPM_TRAFFIC["ipm_sha256"] == file_sha(IPM_SRCS)

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
    # in the timed maps the cell pass shares the device with the large-triangle
    # chain; the one-stream maps time each IPM kernel alone
    t_cells1 = sum(t["t_cells_ms"] for t in one) / len(one)
    t_band1 = sum(t["t_band_ms"] for t in one) / len(one)
    cells_roof["alone"] = {"launch_ms": t_cells1, "achieved": cells_flops(counts) / (t_cells1 * 1e-3) / 1e12}
    cells_roof["alone"]["frac"] = cells_roof["alone"]["achieved"] / cells_roof["peak"]

    def valu_issue(kernel, t_alone_ms):
        if not fresh:
            return None
        issue_ms = IPM_VALU[kernel] / VALU_ISSUE_PER_S * 1e3
        return {"instructions": IPM_VALU[kernel], "issue_ms": issue_ms, "frac_of_launch_alone": issue_ms / t_alone_ms}

    cells_roof["valu_issue"] = valu_issue("k_ipm", t_cells1)

    def scatter(kernel, t_alone_ms):
        if not fresh:
            return None
        c = IPM_SCATTER[kernel]
        t = t_alone_ms * 1e-3
        return {"lds_atomic_lanes": c["lds_atomic_lanes"], "lds_atomics_per_s": c["lds_atomic_lanes"] / t,
                "lds_atomic_frac_of_lds_bytes": c["lds_atomic_lanes"] * 8 / t / LDS_BYTES_PER_S,
                "l2_atomic_requests": c["l2_atomic_requests"], "l2_atomic_requests_per_s": c["l2_atomic_requests"] / t}

    cells_roof["scatter"] = scatter("k_ipm", t_cells1)
    band_roof = {"bound": "alu", "achieved": band_flops(counts) / (t_band * 1e-3) / 1e12,
                 "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "traffic": traffic("k_band_queue1"),
                 "kernel": "k_band_queue1",
                 "launch_ms": t_band, "launches_per_step": stats[0]["n_ipm_launches"],
                 "row_items": counts["n_band_rows"], "pieces": counts["n_band_pieces"]}
    band_roof["frac"] = band_roof["achieved"] / band_roof["peak"]
    band_roof["alone"] = {"launch_ms": t_band1, "achieved": band_flops(counts) / (t_band1 * 1e-3) / 1e12}
    band_roof["alone"]["frac"] = band_roof["alone"]["achieved"] / band_roof["peak"]
    band_roof["valu_issue"] = valu_issue("k_band_queue1", t_band1)
    band_roof["scatter"] = scatter("k_band_queue1", t_band1)
    roof, other = (cells_roof, band_roof) if t_cells >= t_band else (band_roof, cells_roof)
    # the IPM stage priced per piece: 25 flops per (triangle, pixel) piece
    # and 30 per triangle, over the whole stage's time
    piece_flops = 25.0 * counts["n_pieces"] + 30.0 * 2.0 * counts["n_cells"]
    ipm_pieces = {"bound": "alu", "model": "25 flops per (triangle, pixel) piece + 30 per triangle",
                  "achieved": piece_flops / (t_ipm * 1e-3) / 1e12, "peak": FP64_VECTOR_PEAK_TFLOPS,
                  "unit": "TFLOP/s", "stage_ms": t_ipm, "pieces": counts["n_pieces"],
                  "triangles": 2 * counts["n_cells"]}
    ipm_pieces["frac"] = ipm_pieces["achieved"] / ipm_pieces["peak"]
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
        "one_stream": {"ms_per_map_device": sum(t["t_total_ms"] for t in one) / len(one),
                       "ipm_ms": sum(t["t_ipm_ms"] for t in one) / len(one),
                       "ipm_cells_ms": sum(t["t_cells_ms"] for t in one) / len(one),
                       "ipm_band_ms": sum(t["t_band_ms"] for t in one) / len(one)},
        "stages_ms": {"tree": avg("t_tree_ms"), "fmm": avg("t_fmm_ms"), "shoot": t_shoot, "ipm": t_ipm,
                      "ipm_cells": avg("t_cells_ms"), "ipm_band": t_band, "total_device": avg("t_total_ms")},
        "roofline": roof,
        "roofline_" + other["kernel"]: other,
        "roofline_shoot": shoot_roof,
        "roofline_ipm_stage_piece_model": ipm_pieces,
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
        try:
            variants["high_magnification"] = highmag_variant()
        except Exception as e:
            variants["high_magnification"] = {"error": str(e)}
        try:
            variants["learned_refinement"] = learned_variant()
        except Exception as e:
            variants["learned_refinement"] = {"error": str(e)}
        try:
            variants["macrocaustic"] = macrocaustic_variant()
        except Exception as e:
            variants["macrocaustic"] = {"error": str(e)}
        line["variants"] = variants
    if not args.no_cpu_baseline:
        # the machine's CPU share for one GPU is 16 threads
        nthreads = min(16, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), os.cpu_count() or 1)
        mid = region["nr2"] // 2
        rows = (mid - 4, mid + 4)
        gstrip, _ = lens.map(rows=rows, **spec)
        line["cpu_baseline"] = cpu_baseline(wl, spec, nthreads, gpu_strip=(rows, gstrip))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
