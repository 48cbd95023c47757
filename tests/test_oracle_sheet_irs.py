"""Pins of the oracle's rectangular compensating sheet (app. B) and of its
inverse ray shooting (sec. 2.3, 4), against what the mathematics fixes:
quadrature of the sheet integral, the field's divergence and curl, its
continuity across the rectangle's edges, its far-field limit; exact counts
for lattices mapped linearly, the point lens's closed form, and the IPM map
of the same lens."""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W

KS, C1, C2 = 0.4, 3.0, 1.5


def _alpha(orc, x, y, c1=C1, c2=C2):
    ax, ay = orc.sheet_alpha(KS, "rect", c1, c2, np.atleast_1d(x), np.atleast_1d(y))
    return ax + 1j * ay


def _quad_outside(z, c1=C1, c2=C2):
    """(1/pi) int kappa / (conj z - conj z') dA over the rectangle, kappa = -KS."""
    f = lambda yp, xp: (-KS / math.pi) / (np.conj(z) - complex(xp, -yp))
    re = integrate.dblquad(lambda yp, xp: f(yp, xp).real, -c1, c1, -c2, c2, epsabs=1e-12)[0]
    im = integrate.dblquad(lambda yp, xp: f(yp, xp).imag, -c1, c1, -c2, c2, epsabs=1e-12)[0]
    return complex(re, im)


def _quad_inside(z, c1=C1, c2=C2):
    """Inside the rectangle, in polar coordinates about z (z' = z + r e^{i phi}):
    the sheet integral becomes (KS / pi) int e^{i phi} r_max(phi) d phi, r_max
    the distance from z to the rectangle's edge along phi."""
    x, y = z.real, z.imag

    def rmax(phi):
        c, s = math.cos(phi), math.sin(phi)
        out = []
        if c > 0:
            out.append((c1 - x) / c)
        if c < 0:
            out.append((-c1 - x) / c)
        if s > 0:
            out.append((c2 - y) / s)
        if s < 0:
            out.append((-c2 - y) / s)
        return min(out)
    corners = sorted(math.atan2(cy - y, cx - x) % (2 * math.pi) for cx in (-c1, c1) for cy in (-c2, c2))
    re = integrate.quad(lambda p: math.cos(p) * rmax(p), 0, 2 * math.pi, points=corners, epsabs=1e-13, limit=200)[0]
    im = integrate.quad(lambda p: math.sin(p) * rmax(p), 0, 2 * math.pi, points=corners, epsabs=1e-13, limit=200)[0]
    return (KS / math.pi) * complex(re, im)


@pytest.mark.parametrize("z", [5 + 0.3j, -4 + 2.5j, 0.5 + 3.0j, 3.5 - 0.7j, -3.2 + 1.0j, 10 - 9j])
def test_rect_sheet_outside_matches_quadrature(orc, z):
    assert abs(_alpha(orc, z.real, z.imag)[0] - _quad_outside(z)) < 1e-9


@pytest.mark.parametrize("z", [0.3 + 0.2j, -2.1 + 1.1j, 2.9 - 1.4j, 0.0 + 0.0j, -2.99 - 1.49j, 1.7 + 1.45j])
def test_rect_sheet_inside_matches_quadrature(orc, z):
    assert abs(_alpha(orc, z.real, z.imag)[0] - _quad_inside(z)) < 1e-10


def test_rect_sheet_poisson_and_curl(orc):
    """div a = 2 kappa (-2 KS inside, 0 outside), curl a = 0."""
    h = 1e-5
    rng = np.random.default_rng(1)
    for _ in range(40):
        x, y = rng.uniform(-6, 6), rng.uniform(-4, 4)
        if min(abs(abs(x) - C1), abs(abs(y) - C2)) < 1e-3:
            continue
        a = lambda dx, dy: _alpha(orc, x + dx, y + dy)[0]
        div = (a(h, 0).real - a(-h, 0).real + a(0, h).imag - a(0, -h).imag) / (2 * h)
        curl = (a(h, 0).imag - a(-h, 0).imag - a(0, h).real + a(0, -h).real) / (2 * h)
        inside = abs(x) < C1 and abs(y) < C2
        assert abs(div - (-2 * KS if inside else 0.0)) < 1e-6, (x, y, div)
        assert abs(curl) < 1e-6


def test_rect_sheet_continuous_across_edges(orc):
    """A uniform sheet's field is continuous: the branch-cut terms must undo
    exactly the jumps of the logarithms at every edge."""
    e = 1e-9
    for t in np.linspace(-0.95, 0.95, 9):
        for z0, n in ((C1 + 1j * t * C2, 1), (-C1 + 1j * t * C2, -1), (t * C1 + 1j * C2, 1j), (t * C1 - 1j * C2, -1j)):
            zi, zo = z0 - e * n, z0 + e * n
            d = _alpha(orc, zi.real, zi.imag)[0] - _alpha(orc, zo.real, zo.imag)[0]
            assert abs(d) < 1e-7, (z0, d)


def test_rect_sheet_symmetry_and_far_field(orc):
    rng = np.random.default_rng(2)
    x, y = rng.uniform(-8, 8, 50), rng.uniform(-8, 8, 50)
    a = _alpha(orc, x, y)
    assert np.allclose(_alpha(orc, -x, -y), -a, atol=1e-12)            # odd
    assert np.allclose(_alpha(orc, x, -y), np.conj(a), atol=1e-12)     # mirror in the x1 axis
    assert abs(_alpha(orc, 0.0, 0.0)[0]) < 1e-12
    # far away: the point mass -KS (4 C1 C2) / pi, deflection M / conj(z)
    z = 4000.0 * np.exp(1j * np.linspace(0, 2 * np.pi, 7, endpoint=False))
    M = -KS * 4 * C1 * C2 / math.pi
    far = _alpha(orc, z.real, z.imag)
    assert np.allclose(far, M / np.conj(z), rtol=1e-5)


def test_rect_lens_uses_the_rect_sheet(orc):
    """A lens with sheet="rect": c2 = aspect c1 and 4 c1 c2 = pi sum m / k_*,
    and its lens equation subtracts that sheet's field."""
    sf = W.star_field(50, 0.3, "equal", seed=4)
    L = orc.Lens(0.3, 0.1, 0.2, sf.x, sf.y, sf.m, sheet="rect", rect_aspect=0.5)
    assert L.e2 == pytest.approx(0.5 * L.e1) and 4 * L.e1 * L.e2 == pytest.approx(math.pi * sf.m.sum() / 0.3)
    zx, zy = np.array([0.3, 7.0]), np.array([-0.2, 1.0])
    ax, ay = orc.alpha_direct(L, zx, zy)
    wx, wy = orc.lens_equation(L, zx, zy, ax, ay)
    sx, sy = orc.sheet_alpha(0.3, "rect", L.e1, L.e2, zx, zy)
    assert np.allclose(wx, (1 - 0.4 + 0.2) * zx - ax - sx, atol=1e-13)
    assert np.allclose(wy, (1 - 0.4 - 0.2) * zy - ay - sy, atol=1e-13)


# ---------------------------------------------------------------------------
# IRS
# ---------------------------------------------------------------------------

def test_irs_no_lens_is_exactly_one(orc):
    """No lens, a ray grid aligned with the pixels at 64 rays per pixel (all
    sizes exact in binary): every pixel receives exactly 64 rays, mu = 1."""
    L = orc.Lens(0.0, 0.0, 0.0, [], [], [], sheet=False)
    res = orc.irs_map(L, dict(hw1=4.0, hw2=4.0, n1=64, n2=64, rays_per_pixel=64.0))
    assert res.region.nr1 == 513 and res.n_out == 0
    assert np.all(res.counts == 64) and np.all(res.mu == 1.0)


def test_irs_macro_only_counts(orc):
    """A linear (diagonal) map takes the lattice to a lattice of spacing
    |lam_i| D_i: a pixel holds floor or ceil of pix_i / (|lam_i| D_i) columns
    and rows of rays, and the rays are conserved."""
    for kappa, gamma in ((0.3, 0.2), (0.7, 0.45)):
        L = orc.Lens(0.0, kappa, gamma, [], [], [], sheet=False)
        res = orc.irs_map(L, dict(hw1=3.0, hw2=2.0, n1=30, n2=20, rays_per_pixel=49.0))
        R = res.region
        A = R.pix1 / (abs(R.lam1) * R.d1)
        B = R.pix2 / (abs(R.lam2) * R.d2)
        # (a spacing that divides the pixel exactly may round either way)
        lo = math.floor(A - 1e-9) * math.floor(B - 1e-9)
        hi = math.ceil(A + 1e-9) * math.ceil(B + 1e-9)
        assert res.counts.min() >= lo and res.counts.max() <= hi
        assert res.counts.sum() + res.n_out == (R.nr1 - 1) * (R.nr2 - 1)
        assert abs(res.mu.mean() * abs(R.lam1 * R.lam2) - 1.0) < 1.0 / A + 1.0 / B


def test_irs_point_lens_closed_form(orc):
    """One unit mass: the IRS map approaches the pixel-averaged
    A(u) = (u^2 + 2) / (u sqrt(u^2 + 4)) as the rays per pixel grow."""
    L = orc.Lens(0.0, 0.0, 0.0, [0.0], [0.0], [1.0], sheet=False)
    A = lambda y1, y2: ((y1 ** 2 + y2 ** 2) + 2) / (np.hypot(y1, y2) * np.sqrt(y1 ** 2 + y2 ** 2 + 4))
    from test_oracle_ipm import _pixel_average
    errs = []
    for rho in (64, 400, 2500):
        spec = dict(hw1=1.5, hw2=1.5, n1=24, n2=24, rays_per_pixel=rho, dx1=3.0, dx2=3.0, y1c=0.03, y2c=0.05)
        res = orc.irs_map(L, spec)
        R = res.region
        rel = []
        for j in range(R.n2):
            for i in range(R.n1):
                cu = R.y1c - R.hw1 + (i + 0.5) * R.pix1
                cv = R.y2c - R.hw2 + (j + 0.5) * R.pix2
                if math.hypot(cu, cv) < 2 * R.pix1:
                    continue
                want = _pixel_average(A, R, i, j)
                rel.append(abs(res.mu[j, i] - want) / want)
        errs.append(np.mean(rel))
    assert errs[2] < errs[1] < errs[0]
    assert errs[2] < 1e-2


def test_irs_agrees_with_ipm(orc):
    """The paper's consistency check (sec. 4.1): IRS and IPM maps of the same
    lens agree, to the rays' sampling error."""
    sf = W.star_field(300, 0.3, "salpeter", seed=21)
    L = orc.Lens(0.3, 0.1, 0.2, sf.x, sf.y, sf.m)
    spec = dict(hw1=2.0, hw2=2.0, n1=40, n2=40)
    ipm = orc.magnification_map(L, dict(spec, rays_per_pixel=4.0), method="direct")
    irs = orc.irs_map(L, dict(spec, rays_per_pixel=900.0))
    assert abs(irs.mu.mean() / ipm.mu.mean() - 1) < 2e-3
    rel = np.abs(irs.mu - ipm.mu) / ipm.mu
    # rays per pixel image: 900 mu; lattice sampling error ~ (900 mu)^(-2/3)
    assert np.median(rel) < 2e-2
    assert irs.counts.sum() + irs.n_out == (irs.region.nr1 - 1) * (irs.region.nr2 - 1)


def test_irs_rows_are_additive(orc):
    sf = W.star_field(100, 0.3, "equal", seed=22)
    L = orc.Lens(0.3, 0.0, 0.3, sf.x, sf.y, sf.m)
    spec = dict(hw1=1.0, hw2=1.0, n1=16, n2=16, rays_per_pixel=16.0)
    full = orc.irs_map(L, spec)
    n = full.region.nr2 - 1
    parts = [orc.irs_map(L, spec, rows=(a, min(n, a + 37))) for a in range(0, n, 37)]
    assert np.array_equal(sum(p.counts for p in parts), full.counts)
