"""Inverse ray shooting, the rectangular star region and library-drawn star
fields on the GPU, through the C ABI, against the FP64 oracle (needs an
MI355X).

IRS parity is on integer counts.  A ray's pixel is floor((w - ylo) / pix);
the GPU's deflection (FMM, or a direct sum in another order) differs from the
oracle's by ~1e-12 of a pixel, so a ray that lands within 1e-6 pixels of a
pixel edge may be counted in either neighbour.  The oracle lists every ray's
landing point; with those rays set aside, every pixel's count must be exact,
and the set-aside rays must account for every difference."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
REPORT = {}
EDGE = 1e-6     # pixels: rays this close to a pixel edge may go either way


def _report(key, **vals):
    REPORT[key] = vals
    print(f"[irs/rect] {key}: " + ", ".join(f"{k}={v}" for k, v in vals.items()), flush=True)


@pytest.fixture(scope="module")
def mlm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2506_02114_amd as m
    m.load()
    yield m
    out = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")
    if os.path.isdir(out):
        with open(os.path.join(out, "parity_report_irs_rect.json"), "w") as f:
            json.dump(REPORT, f, indent=1, default=float)


def _gpu_counts(mu, R):
    w = R["d1"] * R["d2"] / (R["pix1"] * R["pix2"])
    c = mu / w
    k = np.rint(c)
    assert np.abs(c - k).max() < 1e-6
    return k.astype(np.int64)


def _check_counts(got, ref, what):
    """got: GPU counts; ref: oracle IRSResult with uv."""
    n1, n2 = ref.counts.shape[1], ref.counts.shape[0]
    u, v = ref.uv[:, 0], ref.uv[:, 1]
    fu, fv = np.floor(u), np.floor(v)
    edge = (np.abs(u - np.rint(u)) < EDGE) | (np.abs(v - np.rint(v)) < EDGE)
    inside = (fu >= 0) & (fv >= 0) & (fu < n1) & (fv < n2) & np.isfinite(u) & np.isfinite(v)
    sure = np.zeros(n1 * n2, np.int64)
    np.add.at(sure, (fv[inside & ~edge] * n1 + fu[inside & ~edge]).astype(np.int64), 1)
    sure = sure.reshape(n2, n1)
    diff = got - sure
    assert diff.min() >= 0, what
    assert diff.sum() <= int(edge.sum()), what
    # every pixel that gained a set-aside ray is next to where such a ray landed
    near = np.zeros((n2 + 2, n1 + 2), bool)
    eu, ev = np.clip(fu[edge], -1, n1).astype(int), np.clip(fv[edge], -1, n2).astype(int)
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            near[np.clip(ev + 1 + dj, 0, n2 + 1), np.clip(eu + 1 + di, 0, n1 + 1)] = True
    assert np.all(near[1:-1, 1:-1][diff > 0]), what
    _report(what, rays=int(ref.uv.shape[0]), edge_rays=int(edge.sum()), moved=int(diff.sum()),
            pixels_equal=float(np.mean(got == ref.counts)))


@pytest.mark.parametrize("method", ["fmm", "direct"])
def test_irs_counts_match_oracle(mlm, orc, method):
    wl = W.config("plain_small")
    sf = wl.stars()
    gl = mlm.Lens(0.3, 0.0, 0.3, sf.x, sf.y, sf.m)
    ol = orc.Lens(0.3, 0.0, 0.3, sf.x, sf.y, sf.m)
    spec = dict(hw1=5.0, hw2=5.0, n1=96, n2=96, rays_per_pixel=9.0)
    print(f"[irs/rect] IRS parity, {method}", flush=True)
    mu, st = gl.map(mapping="irs", method=method, order=24, **spec)
    R = gl.region(**spec)
    ref = orc.irs_map(ol, spec, method="direct", want_uv=True)
    assert st["n_rays"] == (R["nr1"] - 1) * (R["nr2"] - 1)
    _check_counts(_gpu_counts(mu, R), ref, f"irs_{method}_vs_oracle_direct")


def test_irs_strips_add_up_and_mixed(mlm):
    sf = W.star_field(2000, 0.4, "salpeter", seed=8)
    gl = mlm.Lens(0.4, 0.1, 0.15, sf.x, sf.y, sf.m)
    spec = dict(hw1=3.0, hw2=2.0, n1=150, n2=100, rays_per_pixel=25.0)
    R = gl.region(**spec)
    full, _ = gl.map(mapping="irs", **spec)
    n = R["nr2"] - 1
    parts = sum(gl.map(mapping="irs", rows=(a, min(n, a + 333)), **spec)[0] for a in range(0, n, 333))
    assert np.array_equal(_gpu_counts(parts, R), _gpu_counts(full, R))
    # mixed precision moves only rays within FP32's reach of a pixel edge,
    # the map's outer edge included (a ray that leaves or enters the map
    # changes the in-map total by one)
    mixed, _ = gl.map(mapping="irs", precision="mixed", **spec)
    a, b = _gpu_counts(mixed, R), _gpu_counts(full, R)
    moved = np.abs(a - b).sum() / 2
    _report("irs_mixed_vs_fp64", rays_moved=float(moved), rays=int(b.sum()), frac=float(moved / b.sum()),
            total_change=int(a.sum() - b.sum()))
    assert moved / b.sum() < 1e-4 and abs(int(a.sum()) - int(b.sum())) <= 2 * moved


def test_irs_agrees_with_ipm_on_table1_map(mlm):
    """The paper's consistency check (sec. 4.1) at its Table 1 size: IRS at
    100 rays per pixel against IPM at 1, the same lens and map."""
    import torch
    lens_spec, mspec, _ = W.paper_table1("circle")
    sf = W.star_field(lens_spec.n_stars, 0.6, "equal", seed=lens_spec.seed)
    dev = torch.device("cuda")
    gl = mlm.Lens(0.6, 0.0, 0.6, torch.from_numpy(sf.x).to(dev), torch.from_numpy(sf.y).to(dev),
                  torch.from_numpy(sf.m).to(dev))
    spec = mspec.asdict()
    ipm = torch.empty((2000, 2000), dtype=torch.float64, device=dev)
    irs = torch.empty_like(ipm)
    gl.map(out=ipm, **spec)
    _, st = gl.map(out=irs, mapping="irs", timing=1, **dict(spec, rays_per_pixel=100.0))
    torch.cuda.synchronize()
    a, b = irs.cpu().numpy(), ipm.cpu().numpy()
    pos = b > 0
    rel = np.abs(a[pos] - b[pos]) / b[pos]
    _report("table1_irs_vs_ipm", mean_irs=float(a.mean()), mean_ipm=float(b.mean()), median_rel=float(np.median(rel)),
            rays=st["n_rays"], ms_irs=st["t_total_ms"])
    assert abs(a.mean() / b.mean() - 1) < 1e-3
    # 100 rays per unit magnification: lattice sampling error ~ (100 mu)^(-2/3)
    assert np.median(rel) < 0.05


def test_sampled_lens_reads_back_its_field(mlm, orc):
    f = mlm.field_params(0.3, "kroupa", n_stars=1500, seed=42, m_lo=0.08, m_hi=1.5)
    x, y, m, e1, e2 = mlm.field_sample(f)
    gl = mlm.Lens.sampled(0.3, 0.05, 0.25, f)
    gx, gy, gm = gl.stars()
    assert np.array_equal(gx, x) and np.array_equal(gy, y) and np.array_equal(gm, m)
    info = gl.info()
    assert info["n_stars"] == 1500 and info["extent1"] == pytest.approx(e1, rel=1e-15)
    # the oracle maps the field the library holds (read back as data)
    ol = orc.Lens(0.3, 0.05, 0.25, gx, gy, gm)
    spec = dict(hw1=2.0, hw2=2.0, n1=64, n2=64, rays_per_pixel=2.0, order=20)
    mu, _ = gl.map(**spec)
    ref = orc.magnification_map(ol, spec, method="fmm", p=20)
    pos = ref.mu > 0
    rel = np.abs(mu[pos] - ref.mu[pos]) / ref.mu[pos]
    _report("sampled_lens_map_vs_oracle", max_rel=float(rel.max()))
    assert rel.max() < 1e-9


def _rect_pair(mlm, orc, n, kappa_star, kappa_smooth, gamma, aspect, seed):
    f = mlm.field_params(kappa_star, "salpeter", n_stars=n, seed=seed, shape="rect", rect_aspect=aspect)
    gl = mlm.Lens.sampled(kappa_star, kappa_smooth, gamma, f, sheet="rect")
    x, y, m = gl.stars()
    ol = orc.Lens(kappa_star, kappa_smooth, gamma, x, y, m, sheet="rect", rect_aspect=aspect)
    return gl, ol, (x, y, m)


def test_rect_sheet_deflection_matches_oracle(mlm, orc):
    gl, ol, (x, y, m) = _rect_pair(mlm, orc, 3000, 0.4, 0.1, 0.3, 0.5, 7)
    info = gl.info()
    assert info["extent1"] == pytest.approx(ol.e1, rel=1e-14) and info["extent2"] == pytest.approx(ol.e2, rel=1e-14)
    rng = np.random.default_rng(3)
    c1, c2 = ol.e1, ol.e2
    zx = np.r_[rng.uniform(-c1, c1, 3000), rng.uniform(-1.5 * c1, 1.5 * c1, 1000)]
    zy = np.r_[rng.uniform(-c2, c2, 3000), rng.uniform(-1.5 * c2, 1.5 * c2, 1000)]
    z = np.stack([zx, zy], 1)
    ax, ay = orc.alpha_direct(ol, zx, zy)
    wx, wy = orc.lens_equation(ol, zx, zy, ax, ay)
    # a request whose shooting region holds every point (the tree's root
    # square must contain them)
    req = dict(hw1=1.0, hw2=1.0, dx1=1.6 * c1, dx2=1.6 * c2)
    w_direct = gl.deflect(z, method="direct", **req)
    scale = np.maximum(np.hypot(wx, wy), 1.0)
    e_direct = np.hypot(w_direct[:, 0] - wx, w_direct[:, 1] - wy) / scale
    w_fmm = gl.deflect(z, order=24, **req)
    e_fmm = np.hypot(w_fmm[:, 0] - wx, w_fmm[:, 1] - wy) / scale
    _report("rect_sheet_deflection", direct_max=float(e_direct.max()), fmm_max=float(e_fmm.max()))
    assert e_direct.max() < 1e-12 and e_fmm.max() < 1e-8


def test_rect_map_matches_oracle(mlm, orc):
    gl, ol, _ = _rect_pair(mlm, orc, 2000, 0.3, 0.0, 0.4, 0.25, 9)
    spec = dict(hw1=2.0, hw2=2.0, n1=80, n2=80, rays_per_pixel=1.0, order=20)
    mu, _ = gl.map(**spec)
    ref = orc.magnification_map(ol, spec, method="fmm", p=20)
    pos = ref.mu > 0
    rel = np.abs(mu[pos] - ref.mu[pos]) / ref.mu[pos]
    _report("rect_map_vs_oracle", max_rel=float(rel.max()), pixels=int(pos.sum()))
    assert np.all(mu[~pos] == 0) and rel.max() < 1e-9


def test_circle_vs_rect_star_regions(mlm, orc):
    """The paper's sec. 4.1 comparison: the rectangle's stars reused inside a
    disc (filled out with further stars of the same density).  The two maps
    show the same caustic network, shifted by the extra stars' deflection,
    and their mean magnifications differ by what the extra stars' tidal field
    does to the macro magnification: the ratio of the mean magnifications is
    predicted from the Jacobian of the deflection difference (extra stars
    summed directly, plus the disc's sheet minus the rectangle's, by the
    oracle) averaged over the macro image of the map, and the magnification
    distributions agree once divided by their means."""
    import torch
    lens_spec, mspec, aspect = W.paper_table1("rect")
    rect = W.rect_field(lens_spec.n_stars, 0.6, aspect, "equal", seed=5)
    c1, c2 = rect.radius, aspect * rect.radius
    R = math.hypot(c1, c2)
    extra = W.star_field(int(round(0.6 * R * R)), 0.6, "equal", seed=6)
    out = (np.abs(extra.x) > c1) | (np.abs(extra.y) > c2)
    x, y = np.r_[rect.x, extra.x[out]], np.r_[rect.y, extra.y[out]]
    m = np.ones_like(x)
    spec = dict(mspec.asdict(), n1=1000, n2=1000)
    dev = torch.device("cuda")
    gr = mlm.Lens(0.6, 0.0, 0.6, rect.x, rect.y, rect.m, sheet="rect", rect_aspect=aspect)
    gc = mlm.Lens(0.6, 0.0, 0.6, x, y, m)
    mr = torch.empty((1000, 1000), dtype=torch.float64, device=dev)
    mc = torch.empty_like(mr)
    _, sr = gr.map(out=mr, timing=1, **spec)
    _, sc = gc.map(out=mc, timing=1, **spec)
    torch.cuda.synchronize()
    a, b = mr.cpu().numpy().ravel(), mc.cpu().numpy().ravel()
    # predicted ratio: the lens map's Jacobian diag(1 - k + g, 1 - k - g) minus
    # that of the deflection difference, over the macro image of the map
    # (|x1| <= hw / |1 - k + g|, |x2| <= hw / |1 - k - g|)
    extra_lens = orc.Lens(0.6, 0.0, 0.6, extra.x[out], extra.y[out], np.ones(int(out.sum())))
    r_disc = math.sqrt(len(x) / 0.6)

    def dalpha(zx, zy):
        ax, ay = orc.alpha_direct(extra_lens, zx, zy)
        cx, cy = orc.sheet_alpha(0.6, "circle", r_disc, 0.0, zx, zy)
        rx, ry = orc.sheet_alpha(0.6, "rect", c1, c2, zx, zy)
        return ax + cx - rx, ay + cy - ry

    l1, l2, h = 1.0, -0.2, 1e-3
    gx, gy = np.meshgrid(np.linspace(-10 / abs(l1), 10 / abs(l1), 9), np.linspace(-10 / abs(l2), 10 / abs(l2), 41))
    gx, gy = gx.ravel(), gy.ravel()
    a0 = dalpha(gx, gy)
    au = dalpha(gx + h, gy)
    av = dalpha(gx, gy + h)
    j11, j12 = l1 - (au[0] - a0[0]) / h, -(av[0] - a0[0]) / h
    j21, j22 = -(au[1] - a0[1]) / h, l2 - (av[1] - a0[1]) / h
    predicted = float(np.mean(np.abs(l1 * l2 / (j11 * j22 - j12 * j21))))
    measured = float(b.mean() / a.mean())

    def ks(p, q):
        bins = np.linspace(-2, 2, 81)
        hp, _ = np.histogram(np.log10(np.maximum(p, 1e-6)), bins)
        hq, _ = np.histogram(np.log10(np.maximum(q, 1e-6)), bins)
        return float(np.abs(np.cumsum(hp) - np.cumsum(hq)).max() / p.size)

    ks_norm = ks(a / a.mean(), b / b.mean())
    _report("circle_vs_rect", stars_rect=gr.n, stars_circle=gc.n, mean_rect=float(a.mean()),
            mean_circle=float(b.mean()), mean_ratio=measured, predicted_ratio=predicted, ks_log_mu=ks(a, b),
            ks_log_mu_over_mean=ks_norm, ms_rect=sr["t_total_ms"], ms_circle=sc["t_total_ms"])
    assert abs(measured / predicted - 1) < 0.05
    assert ks_norm < 0.1


def test_piece_count_statistics(mlm):
    """timing 2 counts the (triangle, pixel) pieces of the apportioning: with
    no lens and cells aligned to pixels (sizes exact in binary), every
    triangle lies in one pixel."""
    gl = mlm.Lens(0.0, 0.0, 0.0, np.zeros(0), np.zeros(0), np.zeros(0), sheet=False)
    for rho in (1.0, 4.0):
        mu, st = gl.map(hw1=4.0, hw2=4.0, n1=64, n2=64, rays_per_pixel=rho, timing=2)
        assert np.all(mu == 1.0)
        assert st["n_pieces"] == 2 * st["n_cells"]
