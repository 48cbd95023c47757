"""Batched maps (mlm_map_batch): fused persistent launches over many maps
must give each map exactly what mlm_map gives it (up to the order of FP64
additions), in FP64 and mixed precision, across chunk boundaries, with the
autotuner, and on draws of the 256-map batched workload (needs an MI355X)."""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

REPORT = {}


def _report(key, **vals):
    REPORT[key] = vals
    print(f"[batch] {key}: " + ", ".join(f"{k}={v}" for k, v in vals.items()), flush=True)


@pytest.fixture(scope="module")
def mlm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2506_02114_amd as m
    m.load()
    yield m
    out = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")
    if os.path.isdir(out):
        with open(os.path.join(out, "parity_report_batch.json"), "w") as f:
            json.dump(REPORT, f, indent=1, default=float)


def _small_batch(mlm, n_maps=6):
    """Maps of uneven size: 1e3 - 2e4 stars, several macro models, 96^2 to
    256^2 pixels, FP64 and mixed."""
    rng = np.random.default_rng(404)
    lenses, reqs = [], []
    for b in range(n_maps):
        kappa = rng.uniform(0.2, 0.8)
        gamma = rng.uniform(0.0, 0.6)
        while min(abs(1 - kappa + gamma), abs(1 - kappa - gamma)) < 0.1:
            gamma = rng.uniform(0.0, 0.6)
        s = rng.uniform(0.0, 0.7)
        ks = (1 - s) * kappa
        n = int(10 ** rng.uniform(3, 4.3))
        sf = W.star_field(n, ks, "salpeter", seed=500 + b, m_lo=0.1, m_hi=1.0)
        lenses.append((mlm.Lens(ks, kappa - ks, gamma, sf.x, sf.y, sf.m), (ks, kappa - ks, gamma, sf)))
        npx = int(rng.choice([96, 160, 256]))
        reqs.append(dict(hw1=float(rng.uniform(2, 5)), hw2=float(rng.uniform(2, 5)), n1=npx, n2=npx,
                         order=16, precision="mixed" if b % 2 else "fp64"))
    return lenses, reqs


def _single(lens, req):
    mu, st = lens.map(**req)
    return mu, st


def test_batch_equals_single_maps(mlm, orc):
    lenses, reqs = _small_batch(mlm)
    outs = [np.empty((r["n2"], r["n1"])) for r in reqs]
    stats, b = mlm.map_batch([l for l, _ in lenses], reqs, outs)
    assert b["n_maps"] == len(reqs) and b["n_chunks"] == 1
    worst = 0.0
    for (lens, _), r, mu, st in zip(lenses, reqs, outs, stats):
        ref, s1 = _single(lens, r)
        assert st["n_rays"] == s1["n_rays"] and st["order"] == s1["order"] and st["n_nodes"] == s1["n_nodes"]
        pos = ref > 0
        assert np.all(np.abs(mu[~pos]) < 1e-12)
        rel = np.abs(mu[pos] - ref[pos]) / ref[pos]
        worst = max(worst, float(rel.max()))
    _report("batch_vs_single", max_rel=worst, maps=len(reqs), rays=b["n_rays"])
    assert worst < 1e-11
    # one FP64 map of the batch against the oracle directly
    (lens, (ks, kss, g, sf)), r, mu = lenses[0], reqs[0], outs[0]
    ol = orc.Lens(ks, kss, g, sf.x, sf.y, sf.m)
    ref = orc.magnification_map(ol, {k: v for k, v in r.items() if k != "precision"}, method="fmm", p=16)
    pos = ref.mu > 0
    rel = np.abs(mu[pos] - ref.mu[pos]) / ref.mu[pos]
    _report("batch_map0_vs_oracle", max_rel=float(rel.max()))
    assert rel.max() < 1e-9


def test_batch_tall_map_many_bands(mlm):
    """A 5000 x 6000 px map (6000 one-row bands, more than 64 KiB of LDS can
    bin) batched with two small maps: the fused binning passes run with the
    larger LDS the device gives a workgroup, and every map equals its single
    call (the tall map's single call is pinned to the oracle in the parity
    tests)."""
    lenses, reqs = _small_batch(mlm, n_maps=2)
    sf = W.config("plain_small").stars()
    tall = mlm.Lens(0.3, 0.0, 0.3, sf.x, sf.y, sf.m)
    pix = 0.001
    treq = dict(hw1=0.5 * 5000 * pix, hw2=0.5 * 6000 * pix, n1=5000, n2=6000, nray1=100, nray2=120, order=16)
    ls = [lenses[0][0], tall, lenses[1][0]]
    rs = [reqs[0], treq, reqs[1]]
    outs = [np.empty((r["n2"], r["n1"])) for r in rs]
    stats, b = mlm.map_batch(ls, rs, outs)
    assert b["n_maps"] == 3 and b["n_big"] > 0
    worst = 0.0
    for lens, r, mu in zip(ls, rs, outs):
        ref, _ = _single(lens, r)
        pos = ref > 0
        assert np.all(np.abs(mu[~pos]) < 1e-12)
        worst = max(worst, float((np.abs(mu[pos] - ref[pos]) / ref[pos]).max()))
    _report("batch_tall_map_vs_single", max_rel=worst, bands=6000)
    assert worst < 1e-11


def test_batch_chunks_and_device_outputs(mlm):
    import torch
    lenses, reqs = _small_batch(mlm)
    outs = [torch.empty((r["n2"], r["n1"]), dtype=torch.float64, device="cuda") for r in reqs]
    # the smallest budget (raised to the largest map's grid) splits the batch
    # into greedy chunks of consecutive maps
    stats, b = mlm.map_batch([l for l, _ in lenses], reqs, outs, vertex_budget=1)
    torch.cuda.synchronize()
    sizes = [s["n_rays"] for s in stats]
    expect, run = 1, 0
    for n in sizes:
        if run and run + n > max(sizes):
            expect, run = expect + 1, 0
        run += n
    assert b["n_chunks"] == expect > 1
    for (lens, _), r, mu in zip(lenses, reqs, outs):
        ref, _ = _single(lens, r)
        got = mu.cpu().numpy()
        pos = ref > 0
        assert np.all(np.abs(got[~pos]) < 1e-12)
        assert (np.abs(got[pos] - ref[pos]) / ref[pos]).max() < 1e-11


def test_batch_autotune(mlm, orc):
    lenses, reqs = _small_batch(mlm, 4)
    reqs = [dict(r, precision="fp64", order=24) for r in reqs]
    outs = [np.empty((r["n2"], r["n1"])) for r in reqs]
    stats, b = mlm.map_batch([l for l, _ in lenses], reqs, outs, autotune=True)
    worst = 0.0
    for (lens, (ks, kss, g, sf)), r, mu, st in zip(lenses, reqs, outs, stats):
        ol = orc.Lens(ks, kss, g, sf.x, sf.y, sf.m)
        ref = orc.magnification_map(ol, {k: v for k, v in r.items() if k != "precision"}, method="fmm", p=24)
        pos = ref.mu > 0
        worst = max(worst, float((np.abs(mu[pos] - ref.mu[pos]) / ref.mu[pos]).max()))
    _report("batch_autotuned_vs_oracle", max_rel=worst, leaves=[s["n_leaves"] for s in stats])
    assert worst < 1e-4


def test_batch_errors(mlm):
    lenses, reqs = _small_batch(mlm, 2)
    outs = [np.empty((r["n2"], r["n1"])) for r in reqs]
    with pytest.raises(mlm.MLMError) as e:
        mlm.map_batch([lenses[0][0], lenses[0][0]], reqs, outs)
    assert e.value.status == mlm.MLM_EINVAL
    with pytest.raises(mlm.MLMError) as e:
        mlm.map_batch([l for l, _ in lenses], [dict(reqs[0], rows=(0, 3)), reqs[1]], outs)
    assert e.value.status == mlm.MLM_EINVAL
    with pytest.raises(mlm.MLMError) as e:
        mlm.map_batch([l for l, _ in lenses], [dict(reqs[0], method="direct"), reqs[1]], outs)
    assert e.value.status == mlm.MLM_EINVAL
    # a map too wide for the row bands fails while the maps are prepared
    # (on a preparing thread): the error reaches the caller and the batch
    # machinery stays usable
    wide = dict(reqs[1], n1=9000, n2=4, hw1=4.5, hw2=0.002)
    with pytest.raises(mlm.MLMError) as e:
        mlm.map_batch([l for l, _ in lenses], [reqs[0], wide], [outs[0], np.empty((4, 9000))])
    assert e.value.status == mlm.MLM_ENOTSUP
    stats, b = mlm.map_batch([l for l, _ in lenses], reqs, outs)
    ref, _ = _single(lenses[1][0], reqs[1])
    pos = ref > 0
    assert (np.abs(outs[1][pos] - ref[pos]) / ref[pos]).max() < 1e-11


def test_batched_workload_draws(mlm, orc):
    """All 256 draws of the batched workload (1000^2 px, 1 ray/px, mixed
    precision), fused, against single-map calls (compared on the device);
    sampled rays of two maps against the exact direct sum."""
    import torch
    draws = W.batch_draws(256, seed=4)
    lenses, reqs, fields = [], [], []
    dev = torch.device("cuda")
    for wl in draws:
        sf = wl.stars()
        L = wl.lens
        lenses.append(mlm.Lens(L.kappa_star, L.kappa_smooth, L.gamma, torch.from_numpy(sf.x).to(dev),
                               torch.from_numpy(sf.y).to(dev), torch.from_numpy(sf.m).to(dev)))
        reqs.append(dict(wl.map.asdict(), precision="mixed"))
        fields.append((L, sf) if len(fields) < 2 else None)
    outs = [torch.empty((r["n2"], r["n1"]), dtype=torch.float64, device=dev) for r in reqs]
    stats, b = mlm.map_batch(lenses, reqs, outs)
    torch.cuda.synchronize()
    worst = 0.0
    ref = torch.empty_like(outs[0])
    for lens, r, mu in zip(lenses, reqs, outs):
        if ref.shape != mu.shape:
            ref = torch.empty_like(mu)
        lens.map(out=ref, **r)
        pos = ref > 0
        assert bool((mu[~pos].abs() < 1e-12).all())
        worst = max(worst, float(((mu[pos] - ref[pos]).abs() / ref[pos]).max()))
    _report("batched_workload_256_maps", max_rel_vs_single=worst, rays=b["n_rays"], chunks=b["n_chunks"],
            ms_total=b["t_total_ms"])
    assert worst < 1e-11
    for k in (0, 1):
        L, sf = fields[k]
        ol = orc.Lens(L.kappa_star, L.kappa_smooth, L.gamma, sf.x, sf.y, sf.m)
        R = orc.region(ol, **{kk: v for kk, v in reqs[k].items() if kk != "precision"})
        rng = np.random.default_rng(90 + k)
        zx = R.x0 + rng.integers(0, R.nr1, 5000) * R.d1
        zy = R.y0 + rng.integers(0, R.nr2, 5000) * R.d2
        w = lenses[k].deflect(np.stack([zx, zy], 1), **reqs[k])
        mx, my = orc.lens_equation(ol, zx, zy, np.zeros_like(zx), np.zeros_like(zy))
        ax, ay = orc.alpha_direct(ol, zx, zy)
        e = np.abs((mx - w[:, 0] - ax) + 1j * (my - w[:, 1] - ay)) / np.maximum(np.abs(ax + 1j * ay), 1.0)
        _report(f"batched_workload_map{k}_deflection_vs_direct", max=float(e.max()), stars=int(sf.n))
        assert e.max() < 1e-4   # mixed precision: bound derived in test_gpu_mixed
