"""Pins of the oracle's lens equation and region set-up (CPU only).

Each test checks the oracle against something other than itself: closed
forms, an independent discretisation, or values the paper states.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_single_lens_deflection_closed_form(orc):
    # sec. 2.2: a_*(z) = m / conj(z - z_1); for one unit mass at the origin 1/conj(z)
    L = orc.Lens(0.0, 0.0, 0.0, [0.0], [0.0], [1.0], sheet=False)
    rng = np.random.default_rng(0)
    z = rng.normal(size=200) + 1j * rng.normal(size=200)
    ax, ay = orc.alpha_direct(L, z.real, z.imag)
    np.testing.assert_allclose(ax + 1j * ay, 1.0 / np.conj(z), rtol=1e-15, atol=0)
    # point lens: y = x - x/|x|^2 (vector form of the lens equation)
    wx, wy = orc.lens_equation(L, z.real, z.imag, ax, ay)
    r2 = np.abs(z) ** 2
    np.testing.assert_allclose(wx, z.real - z.real / r2, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(wy, z.imag - z.imag / r2, rtol=1e-14, atol=1e-15)


def test_shifted_massive_lens(orc):
    L = orc.Lens(0.0, 0.0, 0.0, [1.5], [-0.25], [0.37], sheet=False)
    z = np.array([0.3 + 0.2j, -4.0 + 1.0j])
    ax, ay = orc.alpha_direct(L, z.real, z.imag)
    np.testing.assert_allclose(ax + 1j * ay, 0.37 / np.conj(z - (1.5 - 0.25j)), rtol=1e-15)


def test_direct_sum_order_independent(orc):
    sf = W.star_field(2000, 0.3, "salpeter", seed=11)
    L = orc.Lens(0.3, 0.0, 0.3, sf.x, sf.y, sf.m)
    rng = np.random.default_rng(1)
    zx, zy = rng.uniform(-20, 20, 64), rng.uniform(-20, 20, 64)
    a1 = orc.alpha_direct(L, zx, zy)
    a2 = orc.alpha_direct(L, zx, zy, reversed_order=True)
    np.testing.assert_allclose(a1[0], a2[0], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(a1[1], a2[1], rtol=1e-13, atol=1e-13)


def test_macro_terms(orc):
    # w = (1-kappa) z + gamma conj(z): diag(1-k+g, 1-k-g) (sec. 2.1, 2.2)
    L = orc.Lens(0.0, 0.35, 0.2, [], [], [], sheet=False)
    z = np.array([1.0 + 2.0j, -3.0 + 0.5j])
    wx, wy = orc.lens_equation(L, z.real, z.imag, np.zeros(2), np.zeros(2))
    np.testing.assert_allclose(wx, (1 - 0.35 + 0.2) * z.real, rtol=1e-15)
    np.testing.assert_allclose(wy, (1 - 0.35 - 0.2) * z.imag, rtol=1e-15)


def test_sheet_cancels_a_uniform_disc_of_stars(orc):
    """The compensating sheet (sec. 3.1, both branches) must cancel the mean
    deflection of the stars: a dense regular lattice of equal masses filling
    the disc deflects like a uniform disc, k z inside and k R^2/conj(z) outside
    (Gauss's law), so a_* + a_s -> 0 away from the lattice points."""
    h = 0.05
    R = 3.0
    g = np.arange(-R, R + h / 2, h)
    X, Y = np.meshgrid(g, g)
    inside = X ** 2 + Y ** 2 <= R ** 2
    x, y = X[inside], Y[inside]
    kappa_star = 0.4
    m = np.full(x.size, kappa_star * h * h / math.pi)   # surface density kappa_*
    L = orc.Lens(kappa_star, 0.0, 0.0, x, y, m, sheet=True)
    # R_* from sum(m) = kappa_* R_*^2 must equal the lattice disc radius
    assert abs(L.r_star - R) < 0.02
    # points midway between lattice sites, inside and outside the disc
    pts = np.array([0.3 + 0.2j, -1.1 + 0.45j, 0.6 - 1.95j, 4.025 + 0.525j, -3.525 - 3.025j, 6.025 + 0.025j])
    pts = np.round(pts.real / h - 0.5) * h + h / 2 + 1j * (np.round(pts.imag / h - 0.5) * h + h / 2)
    ax, ay = orc.alpha_direct(L, pts.real, pts.imag)
    wx, wy = orc.lens_equation(L, pts.real, pts.imag, ax, ay)
    # with kappa_s = gamma = 0 (kappa = kappa_*): w = (1 - k_*) z - a_* - a_s,
    # so w - (1 - k_*) z = -(a_* + a_s), which must vanish
    resid = (wx + 1j * wy) - (1 - kappa_star) * pts
    alpha_mag = np.abs(ax + 1j * ay)
    assert np.all(np.abs(resid) < 0.03 * np.maximum(alpha_mag, 0.1)), (np.abs(resid), alpha_mag)


def test_star_radius(orc):
    # kappa_* = N <m> / R_*^2 (sec. 2.1, theta_* = 1)
    m = np.array([0.5, 1.0, 2.0, 0.25])
    assert orc.lib().orc_star_radius(4, m.ctypes.data_as(orc._dp), 0.3) == pytest.approx(
        math.sqrt(3.75 / 0.3), rel=1e-15)


def _solve_kappa_gamma(inv1, inv2):
    lam1, lam2 = 1.0 / inv1, 1.0 / inv2
    one_minus_kappa = 0.5 * (lam1 + lam2)
    gamma = 0.5 * (lam1 - lam2)
    return 1.0 - one_minus_kappa, gamma


def test_region_paper_examples(orc):
    gold = json.load(open(os.path.join(GOLDEN, "paper_region.json")))
    ex = gold["extreme_example"]
    kappa, gamma = _solve_kappa_gamma(ex["inv_lam1"], ex["inv_lam2"])
    ks = (1.0 - ex["smooth_fraction"]) * kappa
    sf = W.star_field(50, ks, "salpeter", seed=3, m_lo=0.1, m_hi=2.0)
    L = orc.Lens(ks, kappa - ks, gamma, sf.x, sf.y, sf.m)
    R = orc.region(L, y1c=3.0, y2c=-0.02, hw1=50.0, hw2=5.0, n1=100, n2=100, flux_fraction=0.001)
    assert R.mu_macro == pytest.approx(ex["mu_macro"], rel=1e-9)
    # centre (Y1/(1-k+g), Y2/(1-k-g)) and half-size (dY + r)/|1-k+-g| (sec. 2.3, app. A)
    r = math.sqrt(ks * np.mean(sf.m ** 2) / (0.001 * np.mean(sf.m)))
    assert R.border == pytest.approx(r, rel=1e-12)
    assert R.X1 == pytest.approx(3.0 * ex["inv_lam1"], rel=1e-12)
    assert R.X2 == pytest.approx(-0.02 * ex["inv_lam2"], rel=1e-9)
    assert R.dX1 == pytest.approx((50.0 + r) * abs(ex["inv_lam1"]), rel=1e-12)
    assert R.dX2 == pytest.approx((5.0 + r) * abs(ex["inv_lam2"]), rel=1e-9)

    mod = gold["moderate_example"]
    L = orc.Lens(mod["kappa"], 0.0, mod["gamma"], [], [], [], sheet=False)
    R = orc.region(L, hw1=1.0, hw2=1.0, n1=10, n2=10)
    assert R.mu_macro == pytest.approx(mod["mu_macro"], rel=1e-12)


def test_border_equal_mass_matches_ten_sqrt_kappa(orc):
    gold = json.load(open(os.path.join(GOLDEN, "paper_region.json")))["border_equal_mass"]
    for ks in gold["kappa_star"]:
        L = orc.Lens(ks, 0.0, 0.1, [0.0, 1.0], [0.0, 0.0], [1.0, 1.0])
        R = orc.region(L, hw1=1.0, hw2=1.0, n1=4, n2=4, flux_fraction=gold["f"])
        assert R.border == pytest.approx(gold["border_over_sqrt_kappa_star"] * math.sqrt(ks), rel=1e-14)


def test_degenerate_macro_rejected(orc):
    L = orc.Lens(0.01, 0.82, 0.17, [0.0], [0.0], [1.0])
    with pytest.raises(orc.DegenerateMacro):
        orc.region(L, hw1=10, hw2=10, n1=4000, n2=4000)


def test_grid_geometry(orc):
    L = orc.Lens(0.45, 0.0, 0.45, [0.0], [0.0], [1.0])
    R = orc.region(L, hw1=25.0, hw2=25.0, n1=2000, n2=2000, rays_per_pixel=1.0)
    # 1 ray per pixel in the absence of lensing: cell side = pixel side
    assert R.d1 == R.pix1 and R.d2 == R.pix2
    assert R.nr1 == math.ceil(2 * R.dX1 / R.d1) + 1
    assert (R.nr1 - 1) * R.d1 >= 2 * R.dX1
    zx, zy = orc.grid_points(R, 0, 2)
    assert zx[0] == pytest.approx(R.X1 - 0.5 * (R.nr1 - 1) * R.d1)
    assert zx[R.nr1 - 1] == pytest.approx(R.X1 + 0.5 * (R.nr1 - 1) * R.d1)
    # explicit vertex counts span exactly [-dX, dX]
    R2 = orc.region(L, hw1=5.0, hw2=5.0, n1=256, n2=256, nray1=512, nray2=512)
    zx, zy = orc.grid_points(R2, R2.nr2 - 1, R2.nr2)
    assert zx[0] == pytest.approx(-R2.dX1, rel=1e-15) and zx[-1] == pytest.approx(R2.dX1, rel=1e-14)
    assert zy[0] == pytest.approx(R2.dX2, rel=1e-14)
    # the root square holds all stars and rays, and is a power of two
    e = math.frexp(R.L0)
    assert e[0] == 0.5 and R.L0 > max(abs(R.X1) + R.dX1, abs(R.X2) + R.dX2)
