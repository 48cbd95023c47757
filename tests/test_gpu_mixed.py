"""Mixed-precision mode against the FP64 oracle and the FP64 map (needs an
MI355X).  In this mode the near field, the Taylor series' variation across a
leaf (its l >= 1 terms in the leaf's coordinate) and the column pass of
well-conditioned triangles run in FP32; the FMM coefficients, each leaf's
far field at its centre, positions, offsets, the macro model, the sheet,
thin triangles, the row bands and every pixel sum stay FP64.

The paper gives no error bound for its single-precision mode (sec. 5 reports
that it degrades near caustics).  The bounds here follow from FP32's unit
round-off u = 2^-24 and the size of what FP32 carries:
  * a vertex moves by delta <= ~10 u S / pix pixels, S = sum over its near
    stars of m / r plus sum_l |d_l| 2^(l/2) of its leaf's Taylor variation
    (a few to a few tens of theta_*): delta ~ 1e-6 px typically, up to
    ~1e-4 px for rays grazing a star;
  * a pixel away from caustics changes by at most ~4 delta relative (its
    four sides, each crossed by displaced cell edges): so the median pixel
    sits near 1e-6 and the p99.9 below the benchmark spec's 1e-4, which is
    asserted; the median is held to 1e-5;
  * caustic pixels amplify delta by their magnification gradient (the
    paper's sec. 5 observation), so the maximum is stated and only bounded
    loosely: 1e-3 on the two plain maps, 1e-2 on the high-magnification one
    (mu_macro ~ -1168).
A regression that puts the field's magnitude back into FP32 (about
kappa_* |z| ~ 100, i.e. ~1e-5 theta_* of absolute error) fails all three.
The coefficients are FP64 in both modes, so they match the oracle's like the
FP64 mode's (1e-11).  Measured values go to the report file
parity_report_mixed.json.
"""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

REPORT = {}
GOLDEN_PIXELS = os.path.join(os.path.dirname(__file__), "golden", "plain_large_pixels.npz")


def _report(key, **vals):
    REPORT[key] = vals
    print(f"[mixed] {key}: " + ", ".join(f"{k}={v}" for k, v in vals.items()), flush=True)


@pytest.fixture(scope="module")
def mlm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2506_02114_amd as m
    m.load()
    yield m
    out = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")
    if os.path.isdir(out):
        with open(os.path.join(out, "parity_report_mixed.json"), "w") as f:
            json.dump(REPORT, f, indent=1, default=float)


def _pair(mlm, orc, ks, kss, g, sf):
    return (mlm.Lens(ks, kss, g, sf.x, sf.y, sf.m), orc.Lens(ks, kss, g, sf.x, sf.y, sf.m))


def _alpha_from_w(ol, orc, zx, zy, wx, wy):
    mx, my = orc.lens_equation(ol, zx, zy, np.zeros_like(zx), np.zeros_like(zy))
    return mx - wx, my - wy


P999_BOUND = 1e-4      # the per-pixel target, at the 99.9th percentile
MEDIAN_BOUND = 1e-5
MAX_BOUND_PLAIN = 1e-3
MAX_BOUND_HIGHMAG = 1e-2


def _assert_map(rel, max_bound, what):
    assert np.quantile(rel, 0.999) < P999_BOUND, what
    assert np.median(rel) < MEDIAN_BOUND, what
    assert rel.max() < max_bound, what


def test_mixed_coefficients(mlm, orc):
    wl = W.config("plain_small")
    sf = wl.stars()
    gl, ol = _pair(mlm, orc, 0.3, 0.0, 0.3, sf)
    spec = wl.map.asdict()
    R = orc.region(ol, **spec)
    p = 20
    ex = gl.fmm_export(**dict(spec, order=p, precision="mixed"))
    ex64 = gl.fmm_export(**dict(spec, order=p))
    # same tree in both modes (integer work and FP64 geometry)
    for k in ("level", "i", "j", "leaf", "nstars", "block"):
        assert np.array_equal(ex[k], ex64[k])
    F = orc.FMM(ol, R.L0, p)
    nd = F.nodes()
    okey = {(int(l), int(i), int(j)): q for q, (l, i, j) in enumerate(zip(nd["level"], nd["i"], nd["j"]))}
    gq = np.array([okey[(int(l), int(i), int(j))] for l, i, j in zip(ex["level"], ex["i"], ex["j"])])
    oa, oc = F.coeffs()
    oa, oc = oa[gq], oc[gq]
    sa = np.maximum(np.abs(oa).max(axis=1, keepdims=True), 1e-300)
    sc = np.maximum(np.abs(oc[:, 1:]).max(axis=1, keepdims=True), 1e-300)
    ea = np.abs(ex["mult"] - oa) / sa
    ec = np.abs(ex["local"][:, 1:] - oc[:, 1:]) / sc
    _report("coeffs_plain_small", max_mult=float(ea.max()), max_local=float(ec.max()))
    assert ea.max() < 1e-11 and ec.max() < 1e-11


def test_mixed_deflection(mlm, orc):
    wl = W.config("plain_small")
    sf = wl.stars()
    gl, ol = _pair(mlm, orc, 0.3, 0.0, 0.3, sf)
    spec = wl.map.asdict()
    R = orc.region(ol, **spec)
    rng = np.random.default_rng(51)
    n = 20000
    zx = rng.uniform(R.x0, -R.x0, n)
    zy = rng.uniform(R.y0, -R.y0, n)
    k = rng.integers(0, sf.n, 2000)
    zx[:2000] = sf.x[k] + rng.normal(scale=1e-3, size=2000)
    zy[:2000] = sf.y[k] + rng.normal(scale=1e-3, size=2000)
    w = gl.deflect(np.stack([zx, zy], 1), **dict(spec, order=20, precision="mixed"))
    gx, gy = _alpha_from_w(ol, orc, zx, zy, w[:, 0], w[:, 1])
    ax, ay = orc.alpha_direct(ol, zx, zy)
    e = np.abs((gx - ax) + 1j * (gy - ay)) / np.maximum(np.abs(ax + 1j * ay), 1.0)
    _report("deflect_plain_small_p20", vs_direct_max=float(e.max()), p999=float(np.quantile(e, 0.999)),
            median=float(np.median(e)))
    # the FP32 parts carry at most a few tens of theta_* (relative error
    # ~10 u of that), and the order-20 truncation adds ~1e-8
    assert e.max() < 1e-5


def test_mixed_map_small(mlm, orc):
    wl = W.config("plain_small")
    sf = wl.stars()
    gl, ol = _pair(mlm, orc, 0.3, 0.0, 0.3, sf)
    spec = dict(wl.map.asdict(), order=20)
    mu, st = gl.map(**spec, precision="mixed")
    ref = orc.magnification_map(ol, spec, method="fmm", p=20)
    pos = ref.mu > 0
    rel = np.abs(mu[pos] - ref.mu[pos]) / ref.mu[pos]
    _report("map_plain_small", max=float(rel.max()), p999=float(np.quantile(rel, 0.999)),
            median=float(np.median(rel)))
    assert np.all(np.abs(mu[~pos]) < 1e-12)
    _assert_map(rel, MAX_BOUND_PLAIN, "plain_small vs oracle")


def test_mixed_map_full_size(mlm, orc):
    """The 1e5-star workload's whole map in mixed precision against the
    oracle's whole FP64 map (stored pixels), and its speed beside FP64."""
    import torch
    wl = W.config("plain_large")
    sf = wl.stars()
    dev = torch.device("cuda")
    gl = mlm.Lens(0.45, 0.0, 0.45, torch.from_numpy(sf.x).to(dev), torch.from_numpy(sf.y).to(dev),
                  torch.from_numpy(sf.m).to(dev))
    spec = wl.map.asdict()
    out = torch.empty((2000, 2000), dtype=torch.float64, device=dev)
    ref64 = torch.empty_like(out)
    gl.map(out=ref64, **spec)
    t = {}
    for prec, o in (("fp64", ref64), ("mixed", out)):
        gl.map(out=o, precision=prec, **spec)     # warm
        _, s = gl.map(out=o, precision=prec, timing=1, **spec)
        t[prec] = s["t_total_ms"]
    torch.cuda.synchronize()
    mu = out.cpu().numpy()
    gold = np.load(GOLDEN_PIXELS)
    ref = gold["mu"]
    got = mu.ravel()[gold["index"]]
    rel = np.abs(got - ref) / ref
    m64 = ref64.cpu().numpy()
    pos64 = m64 > 0
    assert np.all(mu[~pos64] == 0)
    rel64 = np.abs(mu[pos64] - m64[pos64]) / m64[pos64]
    _report("map_plain_large", vs_oracle_max=float(rel.max()), vs_oracle_p999=float(np.quantile(rel, 0.999)),
            vs_oracle_median=float(np.median(rel)), vs_fp64_whole_map_max=float(rel64.max()),
            vs_fp64_whole_map_p999=float(np.quantile(rel64, 0.999)),
            vs_fp64_whole_map_median=float(np.median(rel64)), ms_fp64=t["fp64"], ms_mixed=t["mixed"])
    _assert_map(rel, MAX_BOUND_PLAIN, "plain_large stored pixels vs oracle")
    _assert_map(rel64, MAX_BOUND_PLAIN, "plain_large whole map vs FP64")


def test_mixed_high_magnification_map(mlm, orc):
    """The high-magnification workload (1e6 Salpeter stars, kappa_* = 0.01,
    kappa_s = 0.82, gamma = 0.1725, 4000^2 px of half-width 10, 1 ray/px:
    2.1e10 rays): the whole map in mixed precision against the FP64 map of
    the same rays, sampled rays against the exact direct sum, and a strip of
    the FP64 map against the oracle's strip."""
    import torch
    wl = W.config("mixed_highmag")
    sf = wl.stars()
    L = wl.lens
    dev = torch.device("cuda")
    gl = mlm.Lens(L.kappa_star, L.kappa_smooth, L.gamma, torch.from_numpy(sf.x).to(dev),
                  torch.from_numpy(sf.y).to(dev), torch.from_numpy(sf.m).to(dev))
    ol = orc.Lens(L.kappa_star, L.kappa_smooth, L.gamma, sf.x, sf.y, sf.m)
    spec = wl.map.asdict()
    R = orc.region(ol, **spec)
    print(f"[mixed] high-magnification grid {R.nr1} x {R.nr2}", flush=True)
    m64 = torch.empty((spec["n2"], spec["n1"]), dtype=torch.float64, device=dev)
    m32 = torch.empty_like(m64)
    _, s64 = gl.map(out=m64, timing=1, **spec)
    print(f"[mixed] fp64 map {s64['t_total_ms']:.0f} ms, order {s64['order']}", flush=True)
    _, s32 = gl.map(out=m32, timing=1, precision="mixed", **spec)
    print(f"[mixed] mixed map {s32['t_total_ms']:.0f} ms", flush=True)
    a, b = m32.cpu().numpy(), m64.cpu().numpy()
    assert np.all(np.isfinite(a)) and np.all(np.isfinite(b))
    pos = b > 0
    rel = np.abs(a[pos] - b[pos]) / b[pos]
    _report("map_high_magnification_vs_fp64", max=float(rel.max()), p999=float(np.quantile(rel, 0.999)),
            median=float(np.median(rel)), mean_mu_fp64=float(b.mean()), mean_mu_mixed=float(a.mean()),
            ms_fp64=s64["t_total_ms"], ms_mixed=s32["t_total_ms"], rays=s64["n_rays"], order=s64["order"])
    # the paper's observation (sec. 5): single precision degrades at high
    # magnification; here the caustic pixels are the maximum
    assert abs(a.mean() - b.mean()) < 1e-6 * b.mean()
    _assert_map(rel, MAX_BOUND_HIGHMAG, "high-magnification map vs FP64")
    # the products sec. 5 compares the precisions by: light curves across the
    # map and the distribution of log10 mu
    lc = {}
    for name, (p0, p1) in {"row": ((-10.0, 0.0025), (10.0, 0.0025)), "diagonal": ((-9.99, -9.9), (9.9, 9.99)),
                           "column": ((0.0025, -10.0), (0.0025, 10.0))}.items():
        c32 = mlm.light_curve(m32, p0, p1, 8001, **spec).cpu().numpy()
        c64 = mlm.light_curve(m64, p0, p1, 8001, **spec).cpu().numpy()
        lc[name] = float(np.max(np.abs(c32 - c64) / c64))
    h32 = mlm.histogram(m32, 1.0, 5.0, 400, **spec).cpu().numpy()
    h64 = mlm.histogram(m64, 1.0, 5.0, 400, **spec).cpu().numpy()
    hist_l1 = float(np.abs(h32 - h64).sum() / h64.sum())
    _report("high_magnification_products_mixed_vs_fp64", light_curve_max_rel=lc, histogram_l1=hist_l1)
    assert max(lc.values()) < MAX_BOUND_HIGHMAG and hist_l1 < 1e-3
    # sampled rays of both modes against the exact direct sum
    rng = np.random.default_rng(33)
    ns = 4000
    zx = R.x0 + rng.integers(0, R.nr1, ns) * R.d1
    zy = R.y0 + rng.integers(0, R.nr2, ns) * R.d2
    ax, ay = orc.alpha_direct(ol, zx, zy)
    errs = {}
    for prec in ("fp64", "mixed"):
        w = gl.deflect(np.stack([zx, zy], 1), **dict(spec, precision=prec))
        gx, gy = _alpha_from_w(ol, orc, zx, zy, w[:, 0], w[:, 1])
        errs[prec] = float((np.abs((gx - ax) + 1j * (gy - ay)) / np.maximum(np.abs(ax + 1j * ay), 1.0)).max())
    _report("deflect_high_magnification_vs_direct", fp64=errs["fp64"], mixed=errs["mixed"], n=ns)
    assert errs["fp64"] < 1e-6 and errs["mixed"] < 1e-5
    # the FP64 map's middle strip against the oracle (pixels below 1e-6 of a
    # partial map held to an absolute bound, as for the 1e5-star strip)
    r0 = R.nr2 // 2 - 2
    part, _ = gl.map(**spec, rows=(r0, r0 + 4))
    ref = orc.magnification_map(ol, spec, method="fmm", p=s64["order"], rows=(r0, r0 + 4))
    big = ref.mu >= 1e-6
    relp = np.abs(part[big] - ref.mu[big]) / ref.mu[big]
    _report("high_magnification_strip_fp64_vs_oracle", max_rel=float(relp.max()) if relp.size else 0.0,
            pixels=int(relp.size), max_abs_small=float(np.abs(part[~big] - ref.mu[~big]).max()))
    assert relp.size == 0 or relp.max() < 1e-4
    assert np.abs(part[~big] - ref.mu[~big]).max() < 1e-10
