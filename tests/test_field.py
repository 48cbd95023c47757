"""The library's star-field sampler through the C ABI (host code only, no
GPU): the published generator it draws from, the mass functions' CDFs and
moments, the uniform disc and rectangle, the realised kappa_*, the star
count rule of sec. 2.1 and the covering region of sec. 2.3 / 3.1."""
import math

import numpy as np
import pytest
from scipy import integrate, stats


@pytest.fixture(scope="module")
def mlm():
    import paper_2506_02114_amd as m
    if not __import__("os").path.exists(m.LIB_PATH):
        from paper_2506_02114_amd import _build
        _build.build()
    m.load()
    return m


def test_philox_known_answers(mlm):
    """Known-answer vectors of Philox4x32-10 (Salmon et al. 2011)."""
    assert mlm.philox4x32_10((0, 0, 0, 0), (0, 0)) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    full = 0xFFFFFFFF
    assert mlm.philox4x32_10((full,) * 4, (full, full)) == (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)
    assert mlm.philox4x32_10((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0)) == \
        (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)


def _pdf(kind, lo, hi):
    """Unnormalised density of the mass function (definitions, sec. 2.1)."""
    if kind == "salpeter":
        return lambda m: m ** -2.35
    return lambda m: m ** -1.3 if m < 0.5 else 0.5 ** (2.3 - 1.3) * m ** -2.3


def _cdf(kind, lo, hi):
    f = _pdf(kind, lo, hi)
    z = integrate.quad(f, lo, hi, points=[0.5] if lo < 0.5 < hi else None)[0]

    def F(x):
        x = np.atleast_1d(x)
        return np.array([integrate.quad(f, lo, min(max(v, lo), hi), points=[0.5] if lo < 0.5 < v else None)[0]
                         for v in x]) / z
    return F


@pytest.mark.parametrize("kind,lo,hi", [("salpeter", 0.1, 1.0), ("salpeter", 0.1, 2.0), ("kroupa", 0.08, 1.5)])
def test_masses_follow_the_mass_function(mlm, kind, lo, hi):
    f = mlm.field_params(0.3, kind, n_stars=20000, seed=11, m_lo=lo, m_hi=hi)
    x, y, m, e1, e2 = mlm.field_sample(f)
    assert m.min() >= lo and m.max() <= hi
    # Kolmogorov-Smirnov against the CDF integrated here from the density
    F = _cdf(kind, lo, hi)
    grid = np.quantile(m, np.linspace(0.0, 1.0, 400))
    Fg = F(grid)
    emp = np.searchsorted(np.sort(m), grid, side="right") / m.size
    d = np.abs(emp - Fg).max()
    assert d < 1.63 / math.sqrt(m.size)          # 1 % level of the KS statistic
    # exact moments of the library against quadrature of the density
    z = integrate.quad(_pdf(kind, lo, hi), lo, hi, points=[0.5] if lo < 0.5 < hi else None)[0]
    q1 = integrate.quad(lambda v: v * _pdf(kind, lo, hi)(v), lo, hi, points=[0.5] if lo < 0.5 < hi else None)[0]
    q2 = integrate.quad(lambda v: v * v * _pdf(kind, lo, hi)(v), lo, hi, points=[0.5] if lo < 0.5 < hi else None)[0]
    mm, mm2 = mlm.field_moments(f)
    assert mm == pytest.approx(q1 / z, rel=1e-12) and mm2 == pytest.approx(q2 / z, rel=1e-12)
    # and the sample's
    assert abs(m.mean() - mm) < 5 * m.std() / math.sqrt(m.size)


def test_moment_table(mlm):
    # the first two moments of the mass functions by quadrature of their
    # definitions, to four places: Salpeter (slope 2.35) over 0.1-1 and 0.1-2,
    # Kroupa (slopes 1.3 below 0.5 and 2.3 above) over 0.08-1.5
    for kind, lo, hi, mm, mm2 in (("salpeter", 0.1, 1.0, 0.2234, 0.0754), ("salpeter", 0.1, 2.0, 0.2550, 0.1270),
                                  ("kroupa", 0.08, 1.5, 0.3251, 0.1830)):
        a, b = mlm.field_moments(mlm.field_params(0.3, kind, n_stars=1, m_lo=lo, m_hi=hi))
        assert round(a, 4) == mm and round(b, 4) == mm2


def test_disc_positions_and_kappa(mlm):
    f = mlm.field_params(0.45, "kroupa", n_stars=30000, seed=3, m_lo=0.08, m_hi=1.5)
    x, y, m, e1, e2 = mlm.field_sample(f)
    assert e1 == e2
    # the disc realises kappa_* exactly: kappa_* = sum m / R^2 (theta_* = 1)
    assert m.sum() / e1 ** 2 == pytest.approx(0.45, rel=1e-14)
    r2 = (x * x + y * y) / e1 ** 2
    assert r2.max() <= 1.0
    assert stats.kstest(r2, "uniform").pvalue > 0.01
    assert stats.kstest((np.arctan2(y, x) / (2 * np.pi)) % 1.0, "uniform").pvalue > 0.01


def test_rectangle_positions_and_kappa(mlm):
    f = mlm.field_params(0.2, "salpeter", n_stars=20000, seed=5, shape="rect", rect_aspect=0.25)
    x, y, m, c1, c2 = mlm.field_sample(f)
    assert c2 / c1 == pytest.approx(0.25, rel=1e-15)
    assert math.pi * m.sum() / (4 * c1 * c2) == pytest.approx(0.2, rel=1e-14)
    assert np.abs(x).max() <= c1 and np.abs(y).max() <= c2
    assert stats.kstest((x / c1 + 1) / 2, "uniform").pvalue > 0.01
    assert stats.kstest((y / c2 + 1) / 2, "uniform").pvalue > 0.01


def test_counter_based_and_seeded(mlm):
    a = mlm.field_sample(mlm.field_params(0.3, "salpeter", n_stars=500, seed=9))
    b = mlm.field_sample(mlm.field_params(0.3, "salpeter", n_stars=500, seed=9))
    c = mlm.field_sample(mlm.field_params(0.3, "salpeter", n_stars=800, seed=9))
    d = mlm.field_sample(mlm.field_params(0.3, "salpeter", n_stars=500, seed=10))
    for u, v in zip(a[:3], b[:3]):
        assert np.array_equal(u, v)
    # star i's draws depend on (seed, i) only: the masses of a larger field
    # start with the smaller one's
    assert np.array_equal(a[2], c[2][:500])
    assert not np.array_equal(a[2], d[2])
    # equal masses
    e = mlm.field_sample(mlm.field_params(0.3, "equal", n_stars=100, seed=1, m_equal=0.7))
    assert np.all(e[2] == 0.7)


def test_count_from_region(mlm):
    # n_stars = 0: kappa_* = pi N <m> / A (sec. 2.1, theta_* = 1)
    f = mlm.field_params(0.3, "salpeter", n_stars=0, extent=(40.0, 0.0), m_lo=0.1, m_hi=1.0)
    mm, _ = mlm.field_moments(f)
    assert mlm.field_count(f) == round(0.3 * 40.0 ** 2 / mm)
    g = mlm.field_params(0.3, "salpeter", n_stars=0, shape="rect", extent=(30.0, 10.0))
    assert mlm.field_count(g) == round(0.3 * 4 * 30.0 * 10.0 / (math.pi * mm))
    x, y, m, c1, c2 = mlm.field_sample(g)
    assert c2 / c1 == pytest.approx(10.0 / 30.0)   # aspect from the extents


def test_cover_contains_the_shooting_region(mlm):
    f = mlm.field_params(0.45, "kroupa", n_stars=0, m_lo=0.08, m_hi=1.5)
    mm, mm2 = mlm.field_moments(f)
    req = dict(hw1=25.0, hw2=25.0, n1=200, n2=200, flux_fraction=0.01, y1c=2.0, y2c=-1.0)
    r1, r2 = mlm.field_cover(0.45, 0.0, 0.45, f, margin=1.0, **req)
    # the region of sec. 2.3 with the border of app. A
    border = math.sqrt(0.45 * mm2 / (0.01 * mm))
    lam1, lam2 = 1 - 0.45 + 0.45, 1 - 0.45 - 0.45
    X1, X2 = 2.0 / lam1, -1.0 / lam2
    dX1, dX2 = (25 + border) / abs(lam1), (25 + border) / abs(lam2)
    assert r1 == r2 == pytest.approx(math.hypot(abs(X1) + dX1, abs(X2) + dX2), rel=1e-14)
    g = mlm.field_params(0.45, "kroupa", n_stars=0, shape="rect", m_lo=0.08, m_hi=1.5)
    c1, c2 = mlm.field_cover(0.45, 0.0, 0.45, g, margin=1.2, **req)
    assert c1 == pytest.approx(1.2 * (abs(X1) + dX1)) and c2 == pytest.approx(1.2 * (abs(X2) + dX2))


def test_field_errors(mlm):
    import ctypes as C
    lib = mlm.load()
    bad = mlm.field_params(0.3, "kroupa", n_stars=10, m_lo=0.6, m_hi=1.5)   # break not inside
    n = C.c_int64()
    assert lib.mlm_field_count(C.byref(bad), C.byref(n)) == mlm.MLM_EINVAL
    bad = mlm.field_params(-0.3, "equal", n_stars=10)
    assert lib.mlm_field_count(C.byref(bad), C.byref(n)) == mlm.MLM_EINVAL
    bad = mlm.field_params(0.3, "equal", n_stars=0)                          # no extent to count from
    assert lib.mlm_field_count(C.byref(bad), C.byref(n)) == mlm.MLM_EINVAL
    f = mlm.field_params(0.3, "equal", n_stars=10)
    x = np.empty(5)
    st = lib.mlm_field_sample(C.byref(f), x.ctypes.data_as(C.c_void_p), x.ctypes.data_as(C.c_void_p),
                              x.ctypes.data_as(C.c_void_p), 5, C.byref(n), None, None)
    assert st == mlm.MLM_ERANGE and n.value == 10
