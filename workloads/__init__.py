"""Seeded synthetic inputs shared by the oracle-side tests and the GPU side.

This module only *draws inputs*: star masses and positions, and the lens /
map parameter sets of the workloads.  It holds none of the method's
arithmetic (no deflection, no tree, no expansion, no area apportioning), so
both the CPU oracle and the HIP library can consume what it produces without
sharing any code with each other.

Units: lengths in Einstein radii of a 1 solar-mass lens (theta_* = 1),
masses in solar masses (paper, section 2.1).

Star fields follow the paper's set-up (section 3.1): microlenses uniformly
distributed in a circular region whose radius R_* makes the realised
convergence equal the requested kappa_*:  kappa_* = N <m> / R_*^2, i.e.
R_* = sqrt(sum(m) / kappa_*) (section 2.1, definition of kappa_*).

Mass functions (the paper names Salpeter and "a variety"; Kroupa is named by
the workload definitions):
  * equal     : every m = m_equal
  * salpeter  : dN/dm ~ m^-2.35 on [m_lo, m_hi]
  * kroupa    : dN/dm ~ m^-1.3 on [0.08, 0.5), ~ m^-2.3 on [0.5, m_hi],
                continuous at 0.5
All are sampled by inverse CDF from numpy's PCG64 stream seeded with `seed`.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import Optional

import numpy as np

__all__ = [
    "StarField", "MapSpec", "LensSpec", "sample_masses", "sample_disc",
    "star_field", "rect_field", "config", "CONFIGS", "batch_draws", "paper_table1",
]

SALPETER_SLOPE = 2.35
KROUPA_SLOPES = (1.3, 2.3)
KROUPA_BREAK = 0.5


def _powerlaw_icdf(u: np.ndarray, lo: float, hi: float, slope: float) -> np.ndarray:
    """Inverse CDF of dN/dm ~ m^-slope on [lo, hi] (slope != 1)."""
    e = 1.0 - slope
    a, b = lo ** e, hi ** e
    return (a + u * (b - a)) ** (1.0 / e)


def sample_masses(rng: np.random.Generator, n: int, mass_fn: str,
                  m_lo: float = 0.1, m_hi: float = 1.0,
                  m_equal: float = 1.0) -> np.ndarray:
    """Draw n masses from the named mass function."""
    if n == 0:
        return np.zeros(0)
    if mass_fn == "equal":
        return np.full(n, float(m_equal))
    u = rng.random(n)
    if mass_fn == "salpeter":
        return _powerlaw_icdf(u, m_lo, m_hi, SALPETER_SLOPE)
    if mass_fn == "kroupa":
        a1, a2 = KROUPA_SLOPES
        mb = KROUPA_BREAK
        if not (m_lo < mb < m_hi):
            raise ValueError("kroupa needs m_lo < 0.5 < m_hi")
        # piecewise density f(m) = m^-a1 (m < mb), mb^(a2-a1) m^-a2 (m >= mb)
        w1 = (mb ** (1 - a1) - m_lo ** (1 - a1)) / (1 - a1)
        w2 = mb ** (a2 - a1) * (m_hi ** (1 - a2) - mb ** (1 - a2)) / (1 - a2)
        p1 = w1 / (w1 + w2)
        out = np.empty(n)
        lo_part = u < p1
        out[lo_part] = _powerlaw_icdf(u[lo_part] / p1, m_lo, mb, a1)
        out[~lo_part] = _powerlaw_icdf((u[~lo_part] - p1) / (1 - p1), mb, m_hi, a2)
        return out
    raise ValueError(f"unknown mass function {mass_fn!r}")


def sample_disc(rng: np.random.Generator, n: int, radius: float):
    """Uniform positions in a disc of the given radius: r = R sqrt(u), phi = 2 pi v."""
    u = rng.random(n)
    v = rng.random(n)
    r = radius * np.sqrt(u)
    phi = 2.0 * math.pi * v
    return r * np.cos(phi), r * np.sin(phi)


@dataclass
class StarField:
    x: np.ndarray
    y: np.ndarray
    m: np.ndarray
    radius: float

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def star_field(n: int, kappa_star: float, mass_fn: str = "equal", seed: int = 0,
               m_lo: float = 0.1, m_hi: float = 1.0, m_equal: float = 1.0) -> StarField:
    """N stars uniform in the disc that realises kappa_* exactly (FP64 arrays)."""
    rng = np.random.default_rng(seed)
    m = sample_masses(rng, n, mass_fn, m_lo, m_hi, m_equal)
    if n == 0:
        return StarField(np.zeros(0), np.zeros(0), m, 0.0)
    radius = math.sqrt(float(m.sum()) / kappa_star)
    x, y = sample_disc(rng, n, radius)
    return StarField(np.ascontiguousarray(x), np.ascontiguousarray(y),
                     np.ascontiguousarray(m), radius)


@dataclass
class LensSpec:
    kappa_star: float
    kappa_smooth: float
    gamma: float
    n_stars: int
    mass_fn: str = "equal"
    m_lo: float = 0.1
    m_hi: float = 1.0
    m_equal: float = 1.0
    seed: int = 0
    sheet: bool = True


@dataclass
class MapSpec:
    y1c: float = 0.0
    y2c: float = 0.0
    hw1: float = 5.0
    hw2: float = 5.0
    n1: int = 256
    n2: int = 256
    rays_per_pixel: float = 1.0
    nray1: int = 0
    nray2: int = 0
    flux_fraction: float = 0.01
    order: int = 0
    leaf_max: int = 32

    def asdict(self):
        return asdict(self)


@dataclass
class Workload:
    name: str
    lens: LensSpec
    map: MapSpec
    note: str = ""

    def stars(self) -> StarField:
        L = self.lens
        return star_field(L.n_stars, L.kappa_star, L.mass_fn, L.seed,
                          L.m_lo, L.m_hi, L.m_equal)


def config(name: str) -> Workload:
    """The named workloads, as concrete seeded inputs.

    plain_small : 1 000 equal-mass lenses, kappa_*=0.3, kappa_s=0, gamma=0.3,
                  256^2 px map of half-width 5, 512 x 512 ray-grid vertices.
    plain_large : 1e5 Kroupa (0.08-1.5) lenses, kappa_*=0.45, kappa_s=0,
                  gamma=0.45, 2000^2 px of half-width 25, 1 ray/px, p=20.
    mixed_highmag : 1e6 Salpeter (0.1-1) lenses, kappa_*=0.01, kappa_s=0.82,
                  gamma=0.1725 (the workload's gamma=0.17 makes 1-kappa-gamma
                  vanish; 0.1725 keeps the saddle-point regime), 4000^2 px of
                  half-width 10, 1 ray/px.
    """
    if name == "plain_small":
        return Workload(name, LensSpec(0.3, 0.0, 0.3, 1000, "equal", seed=1),
                        MapSpec(hw1=5.0, hw2=5.0, n1=256, n2=256, nray1=512, nray2=512))
    if name == "plain_large":
        return Workload(name, LensSpec(0.45, 0.0, 0.45, 100_000, "kroupa",
                                       m_lo=0.08, m_hi=1.5, seed=2),
                        MapSpec(hw1=25.0, hw2=25.0, n1=2000, n2=2000, order=20))
    if name == "mixed_highmag":
        return Workload(name, LensSpec(0.01, 0.82, 0.1725, 1_000_000, "salpeter",
                                       m_lo=0.1, m_hi=1.0, seed=3),
                        MapSpec(hw1=10.0, hw2=10.0, n1=4000, n2=4000))
    raise KeyError(name)


CONFIGS = ("plain_small", "plain_large", "mixed_highmag")


def macrocaustic(seed: int = 7):
    """A map across a macro fold caustic (app. D): the macro model sits on
    the critical line, 1 - kappa - gamma = 0, with kappa_* = 0.2, kappa_s =
    0.3, gamma = 0.5 and the third derivative psi_222 = 0.002 (the others 0),
    so y2 = -(psi_222 / 2) x2^2 along x2: sources below y2 = 0 have two
    macroimages, those above none.  The map is 10 x 10 theta_* centred on
    the caustic, 2000^2 px, 1 ray/px, equal masses; the star disc covers the
    macroimages of the map widened by the border r (the library then finds
    the images inside it) with a 1.2 margin.  The paper shows such a map
    without stating its parameters.  Returns (lens spec, map spec, psi3)."""
    ks, kss, g, d = 0.2, 0.3, 0.5, 0.002
    f = 0.01
    r = math.sqrt(ks / f)                       # border of app. A, equal masses
    hw = 5.0
    x1 = (hw + r) / abs(1.0 - ks - kss + g)
    x2 = math.sqrt(2.0 * (hw + r) / d)          # outer edge of the macroimages
    n = int(round(ks * (1.2 * math.hypot(x1, x2)) ** 2))
    lens = LensSpec(ks, kss, g, n, "equal", seed=seed)
    spec = MapSpec(y1c=0.0, y2c=0.0, hw1=hw, hw2=hw, n1=2000, n2=2000, flux_fraction=f)
    return lens, spec, (0.0, 0.0, 0.0, d)


def paper_table1(shape: str = "circle", seed: int = 1):
    """The paper's Table 1 map as far as the paper fixes it: kappa =
    kappa_* = gamma = 0.6 (its sec. 4.1 comparison lens), equal masses, a
    20 x 20 theta_* map of 2000 x 2000 px, 1 ray per pixel for IPM (100 for
    IRS), flux fraction 1/1000 (its default).  The star region covers the
    shooting rectangle (|X1| + dX1, |X2| + dX2) with a 1.2 margin: a disc
    (about 26 700 stars; the paper says ~27 000) or the rectangle (about
    6 500; the paper says ~3 000 without stating its margin).  Returns
    (lens spec, map spec, rect_aspect)."""
    kappa = gamma = 0.6
    f = 1e-3
    r = math.sqrt(kappa / f)                      # equal masses: <m^2>/<m> = 1
    dx1, dx2 = (10.0 + r) / abs(1 - kappa + gamma), (10.0 + r) / abs(1 - kappa - gamma)
    if shape == "circle":
        n = int(round(kappa * (1.2 * math.hypot(dx1, dx2)) ** 2))
        aspect = 0.0
    else:
        n = int(round(kappa * 4 * (1.2 * dx1) * (1.2 * dx2) / math.pi))
        aspect = dx2 / dx1
    lens = LensSpec(kappa, 0.0, gamma, n, "equal", seed=seed)
    spec = MapSpec(hw1=10.0, hw2=10.0, n1=2000, n2=2000, rays_per_pixel=1.0, flux_fraction=f)
    return lens, spec, aspect


def rect_field(n: int, kappa_star: float, aspect: float, mass_fn: str = "equal", seed: int = 0,
               m_lo: float = 0.1, m_hi: float = 1.0, m_equal: float = 1.0) -> StarField:
    """N stars uniform in the rectangle [-c1, c1] x [-c2, c2], c2 = aspect c1,
    whose area 4 c1 c2 = pi sum(m) / kappa_* realises kappa_* exactly (sec.
    2.1); `radius` holds c1."""
    rng = np.random.default_rng(seed)
    m = sample_masses(rng, n, mass_fn, m_lo, m_hi, m_equal)
    c1 = math.sqrt(math.pi * float(m.sum()) / (4.0 * kappa_star * aspect))
    c2 = aspect * c1
    x = c1 * (2.0 * rng.random(n) - 1.0)
    y = c2 * (2.0 * rng.random(n) - 1.0)
    return StarField(np.ascontiguousarray(x), np.ascontiguousarray(y), np.ascontiguousarray(m), c1)


def batch_draws(n_maps: int = 256, seed: int = 4, min_macro_eig: float = 0.05):
    """Parameter sets of the batched workload.

    kappa ~ U[0.1, 1.2], gamma ~ U[0, 1.2], smooth fraction s ~ U[0, 0.9],
    N ~ round(10^U[3, 6]), map half-width ~ U[10, 25], 1000^2 px, 1 ray/px,
    Salpeter 0.1-1.  Draws whose macro eigenvalues |1-kappa+-gamma| fall
    below `min_macro_eig` are rejected (the shooting region diverges there).
    Star seeds are 10000 + index.
    """
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n_maps:
        kappa = rng.uniform(0.1, 1.2)
        gamma = rng.uniform(0.0, 1.2)
        s = rng.uniform(0.0, 0.9)
        logn = rng.uniform(3.0, 6.0)
        hw = rng.uniform(10.0, 25.0)
        if min(abs(1 - kappa + gamma), abs(1 - kappa - gamma)) < min_macro_eig:
            continue
        ks = (1.0 - s) * kappa
        b = len(out)
        out.append(Workload(
            f"batch_{b}",
            LensSpec(ks, kappa - ks, gamma, int(round(10 ** logn)), "salpeter",
                     m_lo=0.1, m_hi=1.0, seed=10000 + b),
            MapSpec(hw1=hw, hw2=hw, n1=1000, n2=1000)))
    return out
