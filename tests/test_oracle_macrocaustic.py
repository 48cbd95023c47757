"""Pins of the oracle's third-order macro model (app. D: the macro potential
expanded past second order near a macro critical curve).

* The added deflection is the gradient of the cubic potential
  (1/6) sum_ijk psi_ijk x_i x_j x_k, by central differences of that potential.
* A fold: 1 - kappa - gamma = 0 with only psi_222 = d set maps x2 to
  y2 = -(d/2) x2^2, so a source at y2 < 0 has two images with |det J| =
  |1 - kappa + gamma| sqrt(2 d |y2|) each and none above the caustic y2 = 0;
  the pixel average of 2 / (|lam1| sqrt(2 d |y2|)) over a pixel row
  [a, b] is 4 (sqrt|a| - sqrt|b|) / (|lam1| sqrt(2 d) (b - a)).  The IPM map
  (no stars) converges to it at second order in the cell size, and is zero
  above the caustic.
* A lens with third-order terms needs its shooting region stated.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore")


def _psi3_potential(psi, x, y):
    a, b, c, d = psi
    return (a * x ** 3 + 3 * b * x * x * y + 3 * c * x * y * y + d * y ** 3) / 6.0


def test_cubic_deflection_is_the_potential_gradient(orc):
    rng = np.random.default_rng(11)
    psi = rng.normal(size=4)
    zx, zy = rng.uniform(-3, 3, 200), rng.uniform(-3, 3, 200)
    zero = np.zeros_like(zx)
    base = orc.Lens(0.2, 0.1, 0.3, np.zeros(0), np.zeros(0), np.zeros(0), sheet=False)
    cub = orc.Lens(0.2, 0.1, 0.3, np.zeros(0), np.zeros(0), np.zeros(0), sheet=False, psi3=psi)
    w0 = orc.lens_equation(base, zx, zy, zero, zero)
    w3 = orc.lens_equation(cub, zx, zy, zero, zero)
    ax, ay = w0[0] - w3[0], w0[1] - w3[1]      # the added deflection
    h = 1e-5
    gx = (_psi3_potential(psi, zx + h, zy) - _psi3_potential(psi, zx - h, zy)) / (2 * h)
    gy = (_psi3_potential(psi, zx, zy + h) - _psi3_potential(psi, zx, zy - h)) / (2 * h)
    scale = np.abs(psi).sum() * 9.0
    assert np.abs(ax - gx).max() < 1e-8 * scale
    assert np.abs(ay - gy).max() < 1e-8 * scale
    # the macro terms of second order are unchanged
    w0b = orc.lens_equation(base, zx, zy, zero, zero)
    assert np.array_equal(w0[0], w0b[0]) and np.array_equal(w0[1], w0b[1])


def _fold_errors(orc, rho):
    d, lam1 = 0.5, 1.0
    lens = orc.Lens(0.0, 0.5, 0.5, np.zeros(0), np.zeros(0), np.zeros(0), sheet=False, psi3=[0, 0, 0, d])
    spec = dict(y1c=0.0, y2c=-0.5, hw1=1.0, hw2=1.0, n1=64, n2=64, rays_per_pixel=rho, x1c=0.0, x2c=0.0,
                dx1=1.05, dx2=2.6)
    mu = orc.magnification_map(lens, spec, method="direct").mu
    pix = 2.0 / 64
    edges = -1.5 + pix * np.arange(65)
    a, b = edges[:-1], edges[1:]
    rows = np.flatnonzero(b <= -2 * pix)          # rows at least two pixels below the caustic
    exact = 4.0 * (np.sqrt(-a[rows]) - np.sqrt(-b[rows])) / (lam1 * math.sqrt(2 * d) * (b[rows] - a[rows]))
    rel = np.abs(mu[rows, :] - exact[:, None]) / exact[:, None]
    above = mu[np.flatnonzero(a >= pix), :]
    return rel.max(), np.abs(above).max()


def test_fold_map_converges_to_closed_form(orc):
    e4, z4 = _fold_errors(orc, 4.0)
    e16, z16 = _fold_errors(orc, 16.0)
    assert z4 == 0.0 and z16 == 0.0
    assert e16 < 2e-4
    assert e4 / e16 > 3.0      # second order in the cell size: 4x per 4x rays per pixel


def test_cubic_lens_needs_its_region(orc):
    lens = orc.Lens(0.0, 0.5, 0.5, np.zeros(0), np.zeros(0), np.zeros(0), sheet=False, psi3=[0, 0, 0, 0.5])
    with pytest.raises(ValueError):
        orc.region(lens, hw1=1.0, hw2=1.0, n1=16, n2=16)
    R = orc.region(lens, hw1=1.0, hw2=1.0, n1=16, n2=16, x1c=0.0, x2c=0.5, dx1=1.0, dx2=2.0)
    assert R.X2 == 0.5 and R.dX2 == 2.0
