"""Parity of the HIP path with the FP64 CPU oracle (needs an MI355X).

Every comparison runs the library through its C ABI (via the ctypes
binding) and the oracle on the same seeded inputs from `workloads`.
Tolerances:
  * tree structure: bit-exact (integer work);
  * FMM coefficients and deflections against the oracle's FMM at the same
    order: 1e-11 relative (both are FP64; only rounding order differs);
  * deflection against the exact direct sum: 1e-6 relative
    (|da| / max(|a|, theta_*));
  * maps: 1e-4 relative per pixel.
"""
import json
import math
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

REPORT = {}


def _report(key, **vals):
    REPORT[key] = vals
    print(f"[parity] {key}: " + ", ".join(f"{k}={v}" for k, v in vals.items()), flush=True)


@pytest.fixture(scope="module")
def mlm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2506_02114_amd as m
    m.load()
    yield m
    out = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")
    if os.path.isdir(out):
        with open(os.path.join(out, "parity_report.json"), "w") as f:
            json.dump(REPORT, f, indent=1, default=float)


def _pair(mlm, orc, kappa_star, kappa_smooth, gamma, sf, sheet=True):
    g = mlm.Lens(kappa_star, kappa_smooth, gamma, sf.x, sf.y, sf.m, sheet=sheet)
    o = orc.Lens(kappa_star, kappa_smooth, gamma, sf.x, sf.y, sf.m, sheet=sheet)
    return g, o


def _spec(wl, **over):
    d = wl.map.asdict()
    d.update(over)
    return d


def _node_key(level, i, j):
    return (int(level), int(i), int(j))


@pytest.mark.parametrize("case", ["plain_small", "kroupa_20k"])
def test_tree_and_coefficients_match_oracle(mlm, orc, case):
    if case == "plain_small":
        wl = W.config("plain_small")
        sf, ks, kss, g = wl.stars(), 0.3, 0.0, 0.3
        spec, p = _spec(wl), 20
    else:
        sf = W.star_field(20000, 0.45, "kroupa", seed=21, m_lo=0.08, m_hi=1.5)
        ks, kss, g = 0.45, 0.0, 0.45
        spec, p = dict(hw1=8.0, hw2=8.0, n1=128, n2=128), 12
    gl, ol = _pair(mlm, orc, ks, kss, g, sf)
    R = orc.region(ol, **spec)
    ex = gl.fmm_export(**dict(spec, order=p))
    assert ex["info"]["L0"] == R.L0
    F = orc.FMM(ol, R.L0, p)
    nd = F.nodes()
    onodes = {_node_key(l, i, j): (int(lf), int(s), int(b), q)
              for q, (l, i, j, lf, s, b) in enumerate(zip(nd["level"], nd["i"], nd["j"], nd["leaf"], nd["nstars"], nd["block"]))}
    gnodes = {_node_key(l, i, j): (int(lf), int(s), int(b), q)
              for q, (l, i, j, lf, s, b) in enumerate(zip(ex["level"], ex["i"], ex["j"], ex["leaf"], ex["nstars"], ex["block"]))}
    assert set(onodes) == set(gnodes)
    for k in onodes:
        assert onodes[k][:3] == gnodes[k][:3], k
    oa, oc = F.coeffs()
    gq = np.array([gnodes[k][3] for k in onodes])
    oq = np.array([onodes[k][3] for k in onodes])
    ga, gc = ex["mult"][gq], ex["local"][gq]
    oa, oc = oa[oq], oc[oq]
    sa = np.maximum(np.abs(oa).max(axis=1, keepdims=True), 1e-300)
    sc = np.maximum(np.abs(oc[:, 1:]).max(axis=1, keepdims=True), 1e-300)
    ea = np.abs(ga - oa) / sa
    ec = np.abs(gc[:, 1:] - oc[:, 1:]) / sc
    _report(f"coeffs_{case}", nodes=len(onodes), max_mult=float(ea.max()), max_local=float(ec.max()))
    assert ea.max() < 1e-11
    assert ec.max() < 1e-11


def _alpha_from_w(lens_o, orc, zx, zy, wx, wy):
    # a_* = macro + sheet - w, using the oracle's lens equation with a_* = 0
    mx, my = orc.lens_equation(lens_o, zx, zy, np.zeros_like(zx), np.zeros_like(zy))
    return mx - wx, my - wy


def test_deflection_matches_oracle(mlm, orc):
    wl = W.config("plain_small")
    sf = wl.stars()
    gl, ol = _pair(mlm, orc, 0.3, 0.0, 0.3, sf)
    spec = _spec(wl)
    R = orc.region(ol, **spec)
    rng = np.random.default_rng(5)
    n = 20000
    zx = rng.uniform(R.x0, -R.x0, n)
    zy = rng.uniform(R.y0, -R.y0, n)
    # points close to stars too
    k = rng.integers(0, sf.n, 2000)
    zx[:2000] = sf.x[k] + rng.normal(scale=1e-3, size=2000)
    zy[:2000] = sf.y[k] + rng.normal(scale=1e-3, size=2000)
    for p in (8, 20, 30):
        w = gl.deflect(np.stack([zx, zy], 1), **dict(spec, order=p))
        F = orc.FMM(ol, R.L0, p)
        fx, fy = F.alpha(zx, zy)
        gx, gy = _alpha_from_w(ol, orc, zx, zy, w[:, 0], w[:, 1])
        e_fmm = np.abs((gx - fx) + 1j * (gy - fy)) / np.maximum(np.abs(fx + 1j * fy), 1.0)
        ax, ay = orc.alpha_direct(ol, zx, zy)
        e_dir = np.abs((gx - ax) + 1j * (gy - ay)) / np.maximum(np.abs(ax + 1j * ay), 1.0)
        _report(f"deflect_p{p}", vs_oracle_fmm=float(e_fmm.max()), vs_direct=float(e_dir.max()))
        assert e_fmm.max() < 1e-11
        if p >= 20:
            assert e_dir.max() < 1e-6
    # direct method through the library: exact sum
    w = gl.deflect(np.stack([zx, zy], 1), **dict(spec, method="direct"))
    gx, gy = _alpha_from_w(ol, orc, zx, zy, w[:, 0], w[:, 1])
    ax, ay = orc.alpha_direct(ol, zx, zy)
    e = np.abs((gx - ax) + 1j * (gy - ay)) / np.maximum(np.abs(ax + 1j * ay), 1.0)
    _report("deflect_direct", vs_direct=float(e.max()))
    assert e.max() < 1e-12


def _rel_map_err(mu, ref):
    pos = ref > 0
    rel = np.abs(mu[pos] - ref[pos]) / ref[pos]
    zero_ok = np.all(np.abs(mu[~pos]) < 1e-12)
    return rel, zero_ok


def test_map_small_matches_oracle(mlm, orc):
    wl = W.config("plain_small")
    sf = wl.stars()
    gl, ol = _pair(mlm, orc, 0.3, 0.0, 0.3, sf)
    spec = _spec(wl, order=20)
    mu, st = gl.map(**spec)
    ref = orc.magnification_map(ol, spec, method="fmm", p=20)
    rel, zok = _rel_map_err(mu, ref.mu)
    _report("map_plain_small_vs_oracle_fmm", max=float(rel.max()), p999=float(np.quantile(rel, 0.999)),
            median=float(np.median(rel)), skipped=st["n_skipped"], order=st["order"])
    assert zok and rel.max() < 1e-4
    assert st["n_skipped"] == ref.n_skip
    # against the exact direct sum (the FMM at order 30 is within 1e-11 of it)
    mu30, _ = gl.map(**_spec(wl, order=30))
    ref_d = orc.magnification_map(ol, spec, method="direct")
    rel, zok = _rel_map_err(mu30, ref_d.mu)
    _report("map_plain_small_vs_direct", max=float(rel.max()), p999=float(np.quantile(rel, 0.999)),
            median=float(np.median(rel)))
    assert zok and rel.max() < 1e-4
    # the library's own direct-sum method
    mud, _ = gl.map(**_spec(wl, method="direct"))
    rel, zok = _rel_map_err(mud, ref_d.mu)
    _report("map_plain_small_direct_method", max=float(rel.max()))
    assert zok and rel.max() < 1e-9
    # area bookkeeping: deposited area = oracle's
    assert mu.sum() * ref.region.pix1 * ref.region.pix2 == pytest.approx(ref.dep_total, rel=1e-9)


def test_map_with_few_large_triangles_matches_oracle(mlm, orc):
    """Coarse pixels over a fine ray grid (24^2 px, 1024^2 rays, one strip):
    fewer large triangles than cell tiles, the case where the gather strides
    a resident grid over the tiles and skips the empty ones, and 1800 cells
    per pixel, where the cell pass sums in its 16 x 16 pixel window; the map
    against the oracle's."""
    wl = W.config("plain_small")
    sf = wl.stars()
    gl, ol = _pair(mlm, orc, 0.3, 0.0, 0.3, sf)
    spec = _spec(wl, order=20, n1=24, n2=24, nray1=1024, nray2=1024)
    R = gl.region(**spec)
    tiles = -(-(R["nr1"] - 1) // 16) * -(-(R["nr2"] - 1) // 16)
    mu, st = gl.map(timing=2, **spec)
    ref = orc.magnification_map(ol, spec, method="fmm", p=20)
    rel, zok = _rel_map_err(mu, ref.mu)
    _report("map_few_large_triangles_vs_oracle_fmm", max=float(rel.max()), median=float(np.median(rel)),
            big=st["n_big"], tiles=int(tiles))
    assert 0 < st["n_big"] < tiles
    assert zok and rel.max() < 1e-9
    assert mu.sum() * ref.region.pix1 * ref.region.pix2 == pytest.approx(ref.dep_total, rel=1e-9)


def test_timing_levels_and_work_counts(mlm):
    """timing 0, 1 and 2 make the same map; only timing 2 fills the IPM
    kernels' work counts, which obey their definitions' bounds."""
    wl = W.config("plain_small")
    sf = wl.stars()
    gl = mlm.Lens(0.3, 0.0, 0.3, sf.x, sf.y, sf.m)
    spec = _spec(wl, order=20)
    maps, stats = [], []
    for t in (0, 1, 2):
        mu, st = gl.map(timing=t, **spec)
        maps.append(mu)
        stats.append(st)
    for mu in maps[1:]:
        pos = maps[0] > 0
        assert np.all(mu[~pos] == 0.0)
        assert np.abs(mu[pos] - maps[0][pos]).max() <= 1e-12 * maps[0][pos].max()
    s1, s2 = stats[1], stats[2]
    assert s1["t_cells_ms"] > 0 and s1["n_small"] == s1["n_col_items"] == s1["n_col_pieces"] == 0
    assert s1["n_band_rows"] == 0
    assert 0 < s2["n_small"] <= 2 * s2["n_cells"]
    assert 0 < s2["n_col_items"] <= s2["n_col_pieces"]
    assert s2["n_big_rows"] >= s2["n_big"] and s2["n_band_pieces"] >= 0
    _report("work_counts_plain_small", cells=s2["n_cells"], small=s2["n_small"], items=s2["n_col_items"],
            pieces=s2["n_col_pieces"], big=s2["n_big"], band_rows=s2["n_band_rows"])


@pytest.mark.parametrize("n1", [5000, 9000])
def test_wide_maps_match_oracle(mlm, orc, n1):
    """Maps wider than the row bands' usual shape: 5000 px gives one-row
    bands, 9000 px (more than an LDS row of doubles) takes the per-triangle
    row kernel with global column differences.  A coarse ray grid makes
    every triangle large, so these paths carry the whole map."""
    wl = W.config("plain_small")
    sf = wl.stars()
    gl, ol = _pair(mlm, orc, 0.3, 0.0, 0.3, sf)
    pix = 0.001
    spec = dict(hw1=0.5 * n1 * pix, hw2=1.5 * pix, n1=n1, n2=3, nray1=150, nray2=160, order=16)
    mu, st = gl.map(timing=2, **spec)
    ref = orc.magnification_map(ol, spec, method="fmm", p=16)
    rel, zok = _rel_map_err(mu, ref.mu)
    _report(f"map_wide_{n1}_vs_oracle_fmm", max=float(rel.max()), median=float(np.median(rel)), big=st["n_big"],
            band_rows=st["n_band_rows"])
    assert st["n_big"] > 0 and zok and rel.max() < 1e-9
    assert mu.sum() * pix * pix == pytest.approx(ref.dep_total, rel=1e-9)


GOLDEN_TALL = os.path.join(os.path.dirname(__file__), "golden", "tall_map_pixels.npz")


def test_tall_map_many_bands(mlm, orc):
    """6000 one-row bands (5000 x 6000 px): more bands than the binning
    passes can index in 64 KiB of LDS.  Where the device gives a workgroup
    more, the band path runs with it, else the per-triangle row kernel; either
    way the map matches the oracle's (every pixel row's sum and 22000 sampled
    pixels, stored by tests/golden/make_tall_map_pixels.py)."""
    gold = np.load(GOLDEN_TALL)
    n1, n2, pix = int(gold["n1"]), int(gold["n2"]), float(gold["pix"])
    sf = W.config("plain_small").stars()
    gl, _ = _pair(mlm, orc, 0.3, 0.0, 0.3, sf)
    spec = dict(hw1=0.5 * n1 * pix, hw2=0.5 * n2 * pix, n1=n1, n2=n2, nray1=int(gold["nray1"]),
                nray2=int(gold["nray2"]), order=int(gold["order"]))
    mu, st = gl.map(timing=2, **spec)
    assert mu.shape == (n2, n1) and np.all(np.isfinite(mu))
    rel, zok = _rel_map_err(mu.ravel()[gold["index"]], gold["mu"])
    rs = mu.sum(axis=1)
    ref_rs = gold["row_sum"]
    pos = ref_rs > 0
    rel_rows = np.abs(rs[pos] - ref_rs[pos]) / ref_rs[pos]
    _report("map_tall_6000_bands_vs_oracle_fmm", max=float(rel.max()), rows_max=float(rel_rows.max()),
            big=st["n_big"], band_rows=st["n_band_rows"], path="bands" if st["n_band_rows"] > 0 else "rows")
    assert st["n_big"] > 0 and zok and rel.max() < 1e-9
    assert rel_rows.max() < 1e-9 and np.all(np.abs(rs[~pos]) < 1e-9)
    assert mu.sum() * pix * pix == pytest.approx(float(gold["dep_total"]), rel=1e-9)


def test_large_triangle_chain_beside_cell_pass(mlm, orc):
    """The large-triangle passes run on a second stream beside the cell pass
    by default (band rows added atomically); with one_stream every kernel
    runs on the request's stream.  The two agree to rounding (only the order
    of the atomic sums differs), on the small workload with a caller's stream
    and on the 1e5-star workload's map, and the default matches the oracle."""
    import torch
    wl = W.config("plain_small")
    sf = wl.stars()
    gl, ol = _pair(mlm, orc, 0.3, 0.0, 0.3, sf)
    spec = _spec(wl, order=20)
    ref = orc.magnification_map(ol, spec, method="fmm", p=20)
    out = torch.empty((256, 256), dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        _, st2 = gl.map(out=out, **spec)
    s.synchronize()
    two = out.cpu().numpy()
    one, st1 = gl.map(one_stream=1, **spec)
    assert st1["n_big"] == st2["n_big"] > 0
    rel, zok = _rel_map_err(two, one)
    assert zok and rel.max() < 1e-12
    rel, zok = _rel_map_err(two, ref.mu)
    assert zok and rel.max() < 1e-9
    big = W.config("plain_large")
    sfb = big.stars()
    L = big.lens
    glb = mlm.Lens(L.kappa_star, L.kappa_smooth, L.gamma, torch.from_numpy(sfb.x).cuda(), torch.from_numpy(sfb.y).cuda(),
                   torch.from_numpy(sfb.m).cuda())
    specb = big.map.asdict()
    a = torch.empty((specb["n2"], specb["n1"]), dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    _, sa = glb.map(out=a, timing=1, **specb)
    _, sb = glb.map(out=b, timing=1, one_stream=1, **specb)
    torch.cuda.synchronize()
    pos = b > 0
    worst = float(((a[pos] - b[pos]).abs() / b[pos]).max())
    _report("two_streams_vs_one", max_rel=worst, ms_two=sa["t_total_ms"], ms_one=sb["t_total_ms"],
            ipm_ms_two=sa["t_ipm_ms"], ipm_ms_one=sb["t_ipm_ms"])
    assert bool((a[~pos].abs() < 1e-12).all()) and worst < 1e-10


def test_map_device_output_and_stream(mlm, orc):
    import torch
    wl = W.config("plain_small")
    sf = wl.stars()
    gl, ol = _pair(mlm, orc, 0.3, 0.0, 0.3, sf)
    spec = _spec(wl, order=16)
    host, _ = gl.map(**spec)
    out = torch.empty((256, 256), dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        gl.map(out=out, **spec)
    s.synchronize()
    dev = out.cpu().numpy()
    assert np.max(np.abs(dev - host) / np.maximum(host, 1e-300)) < 1e-12


def test_strip_additivity_and_w_out(mlm, orc):
    wl = W.config("plain_small")
    sf = wl.stars()
    gl, ol = _pair(mlm, orc, 0.3, 0.0, 0.3, sf)
    spec = _spec(wl, order=14)
    full, _ = gl.map(**spec)
    parts = [gl.map(**spec, rows=r)[0] for r in ((0, 100), (100, 101), (101, 511))]
    np.testing.assert_allclose(sum(parts), full, rtol=1e-12, atol=1e-13)
    # w_out of a strip matches the oracle's FMM vertex positions
    R = orc.region(ol, **spec)
    rows = (200, 230)
    w = np.empty((rows[1] - rows[0] + 1) * R.nr1 * 2)
    gl.map(**spec, rows=rows, w_out=w)
    F = orc.FMM(ol, R.L0, 14)
    wx, wy = orc.shoot_rows(R, ol, rows[0], rows[1] + 1, F)
    e = np.max(np.abs(w[0::2] - wx) + np.abs(w[1::2] - wy))
    _report("w_out_strip", max_abs=float(e))
    assert e < 1e-11


def test_special_lenses(mlm, orc):
    # no lens, cells = pixels: mu = 1 exactly
    g = mlm.Lens(0.0, 0.0, 0.0, [], [], [], sheet=False)
    mu, _ = g.map(hw1=1.0, hw2=1.0, n1=16, n2=16, nray1=17, nray2=17)
    assert np.max(np.abs(mu - 1.0)) < 1e-14
    # macro model only: |mu_macro| in every pixel, both parities
    for kss, gam in ((0.3, 0.25), (0.7, 0.6), (1.4, 0.2)):
        g = mlm.Lens(0.0, kss, gam, [], [], [], sheet=False)
        lam1, lam2 = 1 - kss + gam, 1 - kss - gam
        mu, _ = g.map(hw1=2.0, hw2=1.5, n1=24, n2=20, rays_per_pixel=3.0, dx1=2.6 / abs(lam1),
                      dx2=2.1 / abs(lam2), y1c=0.3, y2c=-0.2)
        np.testing.assert_allclose(mu, 1.0 / abs((1 - kss) ** 2 - gam ** 2), rtol=1e-12)
    # point lens and Chang-Refsdal lens against the oracle's maps
    for gam in (0.0, 0.6):
        g = mlm.Lens(0.0, 0.0, gam, [0.0], [0.0], [1.0], sheet=False)
        o = orc.Lens(0.0, 0.0, gam, [0.0], [0.0], [1.0], sheet=False)
        spec = dict(hw1=1.5, hw2=1.5, n1=48, n2=48, rays_per_pixel=16, dx1=3.5, dx2=4.0 / (1 - gam + 1e-9),
                    y1c=0.03, y2c=0.05)
        mu, _ = g.map(**dict(spec, method="direct"))
        ref = orc.magnification_map(o, spec, method="direct")
        rel, zok = _rel_map_err(mu, ref.mu)
        _report(f"point_lens_gamma{gam}", max=float(rel.max()))
        assert zok and rel.max() < 1e-9
        mu, _ = g.map(**dict(spec, order=20))
        rel, zok = _rel_map_err(mu, ref.mu)
        assert zok and rel.max() < 1e-9


def test_edge_cases(mlm, orc):
    # a single cell row, a 2 x 2 vertex grid, one-pixel maps
    sf = W.star_field(50, 0.2, "equal", seed=9)
    g, o = _pair(mlm, orc, 0.2, 0.1, 0.1, sf)
    for spec in (dict(hw1=1.0, hw2=1.0, n1=1, n2=1, nray1=2, nray2=2, order=10),
                 dict(hw1=1.0, hw2=2.0, n1=3, n2=7, nray1=33, nray2=2, order=10),
                 dict(hw1=0.5, hw2=0.5, n1=9, n2=5, rays_per_pixel=2.0, order=10, rows=(3, 4))):
        mu, _ = g.map(**spec)
        ref = orc.magnification_map(o, {k: v for k, v in spec.items() if k != "rows"}, method="fmm", p=10,
                                    rows=spec.get("rows"))
        rel, zok = _rel_map_err(mu, ref.mu)
        assert zok and (rel.size == 0 or rel.max() < 1e-9)
    # degenerate macro model
    bad = mlm.Lens(0.01, 0.82, 0.17, sf.x, sf.y, sf.m)
    with pytest.raises(mlm.MLMError) as e:
        bad.map(hw1=1.0, hw2=1.0, n1=4, n2=4)
    assert e.value.status == mlm.MLM_EDEGENERATE
    # mixed precision exists for the FMM only
    with pytest.raises(mlm.MLMError) as e:
        g.map(hw1=1.0, hw2=1.0, n1=4, n2=4, precision="mixed", method="direct")
    assert e.value.status == mlm.MLM_ENOTSUP
    # bad row range
    with pytest.raises(mlm.MLMError) as e:
        g.map(hw1=1.0, hw2=1.0, n1=4, n2=4, rows=(5, 2))
    assert e.value.status == mlm.MLM_EINVAL
    # no stars at all with a sheet-free lens
    z = mlm.Lens(0.0, 0.2, 0.1, [], [], [], sheet=False)
    mu, st = z.map(hw1=1.0, hw2=1.0, n1=8, n2=8, rays_per_pixel=2.0, dx1=1.5 / 0.9, dx2=1.5 / 0.7)
    np.testing.assert_allclose(mu, 1.0 / abs(0.8 ** 2 - 0.01), rtol=1e-12)


GOLDEN_PIXELS = os.path.join(os.path.dirname(__file__), "golden", "plain_large_pixels.npz")


def test_full_size_plain_large_sampled(mlm, orc):
    """The benchmark's workload and launch configuration (1e5 Kroupa stars,
    2000^2 px, 1 ray/px, p = 20): sampled vertices against the exact direct
    sum; sampled pixels of the whole map against the oracle's whole map
    (stored by tests/golden/make_plain_large_pixels.py); and a strip of the
    map against the oracle's map of the same rows."""
    import torch
    wl = W.config("plain_large")
    sf = wl.stars()
    gl, ol = _pair(mlm, orc, 0.45, 0.0, 0.45, sf)
    spec = _spec(wl)
    R = orc.region(ol, **spec)
    print(f"[parity] plain_large grid {R.nr1} x {R.nr2}", flush=True)
    out = torch.empty((2000, 2000), dtype=torch.float64, device="cuda")
    w = torch.empty((R.nr2, R.nr1, 2), dtype=torch.float64, device="cuda")
    _, st = gl.map(out=out, w_out=w, **spec)
    torch.cuda.synchronize()
    assert st["n_rays"] == R.nr1 * R.nr2 and st["order"] == 20
    rng = np.random.default_rng(77)
    ns = 100_000
    a = rng.integers(0, R.nr1, ns)
    b = rng.integers(0, R.nr2, ns)
    idx = torch.from_numpy(b * R.nr1 + a).cuda()
    ws = w.reshape(-1, 2)[idx].cpu().numpy()
    zx = R.x0 + a * R.d1
    zy = R.y0 + b * R.d2
    ax, ay = orc.alpha_direct(ol, zx, zy)
    gx, gy = _alpha_from_w(ol, orc, zx, zy, ws[:, 0], ws[:, 1])
    e = np.abs((gx - ax) + 1j * (gy - ay)) / np.maximum(np.abs(ax + 1j * ay), 1.0)
    _report("plain_large_sampled_deflection", max=float(e.max()), p999=float(np.quantile(e, 0.999)),
            median=float(np.median(e)), n=ns)
    assert e.max() < 1e-6
    mu = out.cpu().numpy()
    assert np.all(np.isfinite(mu)) and st["n_skipped"] == 0
    # whole map: per-pixel relative error on the stored oracle pixels
    gold = np.load(GOLDEN_PIXELS)
    assert int(gold["order"]) == 20 and float(gold["min_mu"]) > 0.0
    ref_px = gold["mu"]
    got_px = mu.ravel()[gold["index"]]
    rel_px = np.abs(got_px - ref_px) / ref_px
    _report("plain_large_whole_map_pixels_vs_oracle_fmm", max=float(rel_px.max()),
            p999=float(np.quantile(rel_px, 0.999)), median=float(np.median(rel_px)), pixels=int(rel_px.size),
            mean_mu_gpu=float(mu.mean()), mean_mu_oracle=float(gold["mean_mu"]))
    assert rel_px.max() < 1e-4
    assert abs(mu.mean() - float(gold["mean_mu"])) <= 1e-9 * float(gold["mean_mu"])
    # a strip of cell rows through the middle of the grid, against the oracle's
    # FMM map of the same rows.  A strip is a partial sum of the map: pixels fed
    # only by slivers of single triangles hold values down to 1e-15, and there a
    # prefix sum's rounding, not the method, sets the error; so pixels below
    # 1e-6 are held to an absolute bound instead
    r0 = R.nr2 // 2 - 3
    rows = (r0, r0 + 6)
    part, _ = gl.map(**spec, rows=rows)
    ref = orc.magnification_map(ol, spec, method="fmm", p=20, rows=rows)
    big = ref.mu >= 1e-6
    rel = np.abs(part[big] - ref.mu[big]) / ref.mu[big]
    small_abs = np.abs(part[~big] - ref.mu[~big])
    _report("plain_large_strip_vs_oracle_fmm", max_rel=float(rel.max()), pixels_rel=int(rel.size),
            max_abs_below_1em6=float(small_abs.max()), pixels_abs=int(small_abs.size))
    assert rel.max() < 1e-4 and small_abs.max() < 1e-10
