"""The seeded input generators: mass-function samples follow their analytic
CDFs, positions fill the disc uniformly, and kappa_* is realised exactly."""
import math

import numpy as np
import pytest
from scipy import stats

import workloads as W


def _powerlaw_cdf(m, lo, hi, a):
    e = 1 - a
    return (m ** e - lo ** e) / (hi ** e - lo ** e)


def test_salpeter_ks():
    rng = np.random.default_rng(0)
    m = W.sample_masses(rng, 200_000, "salpeter", 0.1, 1.0)
    assert m.min() >= 0.1 and m.max() <= 1.0
    d, p = stats.kstest(m, lambda t: _powerlaw_cdf(t, 0.1, 1.0, 2.35))
    assert p > 1e-3
    # moments of dN/dm ~ m^-2.35 on [0.1, 1] by quadrature
    from scipy.integrate import quad
    Z = quad(lambda t: t ** -2.35, 0.1, 1.0)[0]
    m1 = quad(lambda t: t ** -1.35, 0.1, 1.0)[0] / Z
    assert m.mean() == pytest.approx(m1, rel=5e-3)
    assert m1 == pytest.approx(0.2234, abs=1e-4)


def test_kroupa_ks():
    rng = np.random.default_rng(1)
    m = W.sample_masses(rng, 200_000, "kroupa", 0.08, 1.5)
    from scipy.integrate import quad

    def f(t):
        return t ** -1.3 if t < 0.5 else 0.5 ** (2.3 - 1.3) * t ** -2.3

    Z = quad(f, 0.08, 1.5, points=[0.5])[0]
    cdf = np.vectorize(lambda t: quad(f, 0.08, min(max(t, 0.08), 1.5), points=[0.5] if t > 0.5 else None)[0] / Z)
    d, p = stats.kstest(m[:20000], cdf)
    assert p > 1e-3
    m1 = quad(lambda t: t * f(t), 0.08, 1.5, points=[0.5])[0] / Z
    m2 = quad(lambda t: t * t * f(t), 0.08, 1.5, points=[0.5])[0] / Z
    assert m1 == pytest.approx(0.3251, abs=2e-4)
    assert m2 == pytest.approx(0.1830, abs=2e-4)
    assert m.mean() == pytest.approx(m1, rel=5e-3)


def test_disc_uniform_and_kappa_realised():
    sf = W.star_field(100_000, 0.45, "kroupa", seed=2, m_lo=0.08, m_hi=1.5)
    r = np.hypot(sf.x, sf.y)
    assert r.max() <= sf.radius
    d, p = stats.kstest((r / sf.radius) ** 2, "uniform")
    assert p > 1e-3
    # kappa_* = N <m> / R_*^2
    assert sf.m.sum() / sf.radius ** 2 == pytest.approx(0.45, rel=1e-14)


def test_seeded_and_deterministic():
    a = W.config("plain_small").stars()
    b = W.config("plain_small").stars()
    assert np.array_equal(a.x, b.x) and np.array_equal(a.m, b.m)
    assert a.n == 1000 and np.all(a.m == 1.0)


def test_batch_draws_avoid_degenerate_macro():
    draws = W.batch_draws(256)
    assert len(draws) == 256
    for d in draws:
        k = d.lens.kappa_star + d.lens.kappa_smooth
        g = d.lens.gamma
        assert min(abs(1 - k + g), abs(1 - k - g)) >= 0.05
        assert 1000 <= d.lens.n_stars <= 1_000_000
