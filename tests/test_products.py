"""Light curves and magnification histograms (the products of sec. 4.1 and
5): the oracle's definitions pinned on maps whose answers are known, and the
library's (host pointers, no GPU needed for the argument checks)."""
import math

import numpy as np
import pytest


def test_light_curve_reproduces_linear_maps(orc):
    """Bilinear interpolation is exact for a map linear in the pixel
    centres' coordinates, and returns pixel values at pixel centres."""
    n1, n2, hw1, hw2, y1c, y2c = 40, 30, 2.0, 1.5, 0.3, -0.2
    pix1, pix2 = 2 * hw1 / n1, 2 * hw2 / n2
    cu = y1c - hw1 + (np.arange(n1) + 0.5) * pix1
    cv = y2c - hw2 + (np.arange(n2) + 0.5) * pix2
    f = lambda a, b: 3.0 + 0.7 * a - 1.3 * b
    mu = f(cu[None, :], cv[:, None])
    spec = dict(hw1=hw1, hw2=hw2, y1c=y1c, y2c=y2c)
    # a track inside the centres' hull
    a, b = (cu[0] + 0.01, cv[1]), (cu[-1] - 0.02, cv[-2] + 0.003)
    lc = orc.light_curve(mu, spec, a, b, 57)
    t = np.linspace(0, 1, 57)
    want = f(a[0] + t * (b[0] - a[0]), a[1] + t * (b[1] - a[1]))
    assert np.allclose(lc, want, rtol=0, atol=1e-13)
    # pixel centres give pixel values
    lc = orc.light_curve(mu, spec, (cu[3], cv[7]), (cu[3], cv[7]), 1)
    assert lc[0] == pytest.approx(mu[7, 3], abs=1e-14)
    # outside the map: NaN; in the outer half-pixel: the edge row repeated
    lc = orc.light_curve(mu, spec, (y1c - hw1 - 0.01, cv[5]), (y1c - hw1 + 0.25 * pix1, cv[5]), 2)
    assert math.isnan(lc[0]) and lc[1] == pytest.approx(mu[5, 0], abs=1e-14)


def test_histogram_counts(orc):
    lo, hi, nb = -1.0, 3.0, 8                    # bins of width 0.5 in log10
    centres = 10.0 ** (lo + (np.arange(nb) + 0.5) * 0.5)
    mu = np.r_[np.repeat(centres, np.arange(1, nb + 1)), 0.0, -1.0, 1e-5, 1e3, 5e4, np.nan]
    h = orc.histogram(mu, lo, hi, nb)
    assert h.sum() == mu.size
    assert list(h[1:-1]) == list(range(1, nb + 1))
    assert h[0] == 3 and h[-1] == 3              # {0, -1, 1e-5} and {1e3 = 10^hi, 5e4, nan}


def test_library_products_match_oracle_on_host_maps(mlm_host, orc):
    rng = np.random.default_rng(4)
    n1, n2 = 64, 48
    mu = np.exp(rng.normal(size=(n2, n1)))
    mu[0, 0] = 0.0
    spec = dict(hw1=1.5, hw2=1.0, n1=n1, n2=n2, y1c=0.1, y2c=0.0)
    with pytest.raises(mlm_host.MLMError):
        mlm_host.histogram(mu, 1.0, 1.0, 4, **spec)          # hi <= lo


@pytest.fixture(scope="module")
def mlm_host():
    import os
    import paper_2506_02114_amd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_2506_02114_amd import _build
        _build.build()
    m.load()
    return m
