"""Pins of the oracle's FMM (appendix C) against the direct sum, exact
re-expansion identities and a brute-force tree built independently here."""
import math
from collections import Counter

import numpy as np
import pytest

import workloads as W


def _cell(t, L0, level):
    side = 2 ** level
    k = np.floor((np.asarray(t) + L0) * (side / (2.0 * L0))).astype(np.int64)
    return np.clip(k, 0, side - 1)


def brute_tree(x, y, L0, nmax, lmax):
    """Tree of appendix C.1 from its definition, with dictionaries: a node is
    split when the stars of the 3x3 block of same-level squares around it
    exceed nmax (and it is above lmax); its 4 children are nodes."""
    out = {}
    frontier = [(0, 0)]
    level = 0
    while frontier:
        cnt = Counter(zip(_cell(x, L0, level).tolist(), _cell(y, L0, level).tolist()))
        nxt = []
        for a, b in frontier:
            blk = sum(cnt.get((a + da, b + db), 0) for da in (-1, 0, 1) for db in (-1, 0, 1))
            leaf = not (blk > nmax and level < lmax)
            out[(level, a, b)] = (int(leaf), cnt.get((a, b), 0), blk)
            if not leaf:
                nxt += [(2 * a + qi, 2 * b + qj) for qi in (0, 1) for qj in (0, 1)]
        frontier = nxt
        level += 1
    return out


@pytest.mark.parametrize("n,nmax,seed", [(300, 8, 0), (700, 32, 1), (60, 4, 2)])
def test_tree_matches_brute_force(orc, n, nmax, seed):
    sf = W.star_field(n, 0.3, "salpeter", seed=seed)
    lens = orc.Lens(0.3, 0.0, 0.3, sf.x, sf.y, sf.m)
    L0 = 2.0 ** math.ceil(math.log2(np.abs(np.r_[sf.x, sf.y]).max() * 1.0001))
    F = orc.FMM(lens, L0, 4, nmax=nmax)
    nd = F.nodes()
    got = {(int(l), int(i), int(j)): (int(lf), int(s), int(b))
           for l, i, j, lf, s, b in zip(nd["level"], nd["i"], nd["j"], nd["leaf"], nd["nstars"], nd["block"])}
    want = brute_tree(sf.x, sf.y, L0, nmax, 24)
    assert got == want


def test_tree_invariants(orc):
    wl = W.config("plain_small")
    sf = wl.stars()
    lens = orc.Lens(0.3, 0.0, 0.3, sf.x, sf.y, sf.m)
    R = orc.region(lens, **wl.map.asdict())
    F = orc.FMM(lens, R.L0, 4)
    nd = F.nodes()
    leaf = nd["leaf"] == 1
    # leaves tile the root square and hold every star exactly once
    area = np.sum((2.0 * R.L0 / 2.0 ** nd["level"][leaf]) ** 2)
    assert area == (2 * R.L0) ** 2
    assert nd["nstars"][leaf].sum() == sf.n
    # the near field of every leaf (its 3x3 block) is within nmax
    assert nd["block"][leaf].max() <= 32
    assert np.all(nd["block"][~leaf] > 32)


def _multipole(zs, ms, centre, L, p):
    """Multipole coefficients of appendix C.2 (P2M): a_0 = sum m,
    a_k = -(1/k) sum m zeta^k, zeta in half-length units about the centre."""
    zeta = (zs - centre) / L
    a = np.zeros(p + 1, complex)
    a[0] = ms.sum()
    for k in range(1, p + 1):
        a[k] = -(ms * zeta ** k).sum() / k
    return a


def _local_grad(c, centre, L, z):
    zeta = (z - centre) / L
    d = np.zeros_like(zeta)
    for l in range(len(c) - 1, 0, -1):
        d = d * zeta + l * c[l]
    return d / L


def _rand_square(rng, n, centre, L):
    return centre + L * (rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n))


def _square_members(x, y, L0, level, i, j, halo=0):
    """Stars in the square (level, i, j) of the root [-L0, L0)^2, or in its
    (2 halo + 1)^2 block of same-level squares."""
    ci, cj = _cell(x, L0, level), _cell(y, L0, level)
    return (np.abs(ci - i) <= halo) & (np.abs(cj - j) <= halo)


def test_p2m_converges_to_direct_sum(orc):
    """The oracle's multipole expansion of a leaf (P2M, appendix C.2),
    evaluated far outside the leaf, converges to the direct sum over the
    leaf's own stars, with error shrinking like (sqrt2 / dist)^p."""
    sf = W.star_field(400, 0.3, "salpeter", seed=31)
    lens = orc.Lens(0.3, 0.0, 0.3, sf.x, sf.y, sf.m)
    L0 = 2.0 ** math.ceil(math.log2(np.abs(np.r_[sf.x, sf.y]).max() * 1.0001))
    errs = []
    for p in (5, 10, 20, 30):
        F = orc.FMM(lens, L0, p, nmax=8)
        nd = F.nodes()
        cand = np.flatnonzero((nd["leaf"] == 1) & (nd["nstars"] >= 3) & (nd["level"] >= 2))
        q = int(cand[0])
        lev, i, j = int(nd["level"][q]), int(nd["i"][q]), int(nd["j"][q])
        L = L0 / 2 ** lev
        cen = complex(-L0 + (2 * i + 1) * L, -L0 + (2 * j + 1) * L)
        inside = _square_members(sf.x, sf.y, L0, lev, i, j)
        assert inside.sum() == nd["nstars"][q]
        zs = sf.x[inside] + 1j * sf.y[inside]
        z = cen + 4.0 * L * np.exp(1j * np.linspace(0, 2 * np.pi, 50, endpoint=False))
        exact = (sf.m[inside][None, :] / (z[:, None] - zs[None, :])).sum(1)
        got = F.eval_multipole(q, z.real, z.imag)
        errs.append(np.abs(got - exact).max() / sf.m[inside].sum() * L)
    for e, p in zip(errs, (5, 10, 20, 30)):
        assert e < 4 * (math.sqrt(2) / 4) ** p
    assert errs[-1] < 1e-12


def test_local_expansion_is_far_field(orc):
    """A leaf's Taylor series (appendix C.2, from M2L, P2L and L2L) evaluated
    inside the leaf converges to the direct sum over every star outside the
    leaf's 3x3 block of same-level squares (the far stars)."""
    sf = W.star_field(3000, 0.3, "salpeter", seed=32)
    lens = orc.Lens(0.3, 0.0, 0.3, sf.x, sf.y, sf.m)
    L0 = 2.0 ** math.ceil(math.log2(np.abs(np.r_[sf.x, sf.y]).max() * 1.0001))
    rng = np.random.default_rng(33)
    prev = None
    for p in (8, 16, 30):
        F = orc.FMM(lens, L0, p)
        nd = F.nodes()
        leaves = np.flatnonzero((nd["leaf"] == 1) & (nd["level"] >= 3))
        worst = 0.0
        for q in leaves[:: max(1, leaves.size // 12)]:
            lev, i, j = int(nd["level"][q]), int(nd["i"][q]), int(nd["j"][q])
            L = L0 / 2 ** lev
            cen = complex(-L0 + (2 * i + 1) * L, -L0 + (2 * j + 1) * L)
            far = ~_square_members(sf.x, sf.y, L0, lev, i, j, halo=1)
            z = cen + L * (rng.uniform(-1, 1, 20) + 1j * rng.uniform(-1, 1, 20))
            exact = (sf.m[far][None, :] / (z[:, None] - (sf.x[far] + 1j * sf.y[far])[None, :])).sum(1)
            got = F.eval_local(q, z.real, z.imag)
            worst = max(worst, np.abs(got - exact).max() / max(np.abs(exact).max(), 1.0))
        if prev is not None:
            assert worst < prev / 10
        prev = worst
    assert prev < 1e-9


@pytest.mark.parametrize("qi,qj", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_m2m_is_exact_reexpansion(orc, qi, qj):
    """M2M of a child's expansion equals the multipole taken directly about the
    parent (every l <= p), in parent half-length units (appendix C.2)."""
    rng = np.random.default_rng(4 + qi + 2 * qj)
    p = 25
    Lp, cp = 1.0, 0.2 - 0.7j
    Lc = Lp / 2
    cc = cp + Lc * complex(2 * qi - 1, 2 * qj - 1)
    zs = _rand_square(rng, 15, cc, Lc)
    ms = rng.uniform(0.1, 1.5, 15)
    a_child = _multipole(zs, ms, cc, Lc, p)
    b = orc.op_m2m(p, a_child, complex(2 * qi - 1, 2 * qj - 1))
    a_parent = _multipole(zs, ms, cp, Lp, p)
    np.testing.assert_allclose(b, a_parent, rtol=1e-12, atol=1e-13 * np.abs(a_parent).max())


@pytest.mark.parametrize("qi,qj", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_l2l_is_exact_reexpansion(orc, qi, qj):
    """The shifted Taylor series is the same polynomial: at points in the
    child both give the same value (appendix C.2, z0 = parent centre relative
    to the child, in parent half-lengths)."""
    rng = np.random.default_rng(10 + qi)
    p = 20
    c = (rng.normal(size=p + 1) + 1j * rng.normal(size=p + 1)) / (1.0 + np.arange(p + 1)) ** 2
    delta = 0.5 * complex(2 * qi - 1, 2 * qj - 1)        # child centre - parent centre
    d = orc.op_l2l(p, c, -delta)
    zc = rng.uniform(-1, 1, 40) + 1j * rng.uniform(-1, 1, 40)   # child units
    zp = delta + zc / 2                                          # same points, parent units
    val_p = np.polyval(c[::-1], zp)
    val_c = np.polyval(d[::-1], zc)
    np.testing.assert_allclose(val_c, val_p, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("off", [(2, 0), (3, -2), (-2, 2), (3, 3), (-3, 1)])
def test_m2l_converges_to_direct_sum(orc, off):
    rng = np.random.default_rng(20)
    L = 0.7
    ct = 1.0 + 2.0j
    cs = ct + 2 * L * complex(*off)
    zs = _rand_square(rng, 30, cs, L)
    ms = rng.uniform(0.1, 1.0, 30)
    z = _rand_square(rng, 100, ct, L)
    exact = (ms[None, :] / (z[:, None] - zs[None, :])).sum(1)
    prev = None
    for p in (8, 16, 31):
        b = _multipole(zs, ms, cs, L, p)
        c = orc.op_m2l(p, b, complex(2 * off[0], 2 * off[1]))
        err = np.abs(_local_grad(c, ct, L, z) - exact).max() / np.abs(exact).max()
        if prev is not None:
            assert err < prev
        prev = err
    assert prev < 1e-7


def test_fmm_converges_to_direct_sum(orc):
    wl = W.config("plain_small")
    sf = wl.stars()
    lens = orc.Lens(0.3, 0.0, 0.3, sf.x, sf.y, sf.m)
    R = orc.region(lens, **wl.map.asdict())
    zx, zy = orc.grid_points(R, 200, 204)
    ax, ay = orc.alpha_direct(lens, zx, zy)
    prev = None
    for p in (6, 12, 20, 30):
        F = orc.FMM(lens, R.L0, p)
        fx, fy = F.alpha(zx, zy)
        err = np.max(np.abs((fx - ax) + 1j * (fy - ay)) / np.maximum(np.abs(ax + 1j * ay), 1.0))
        if prev is not None:
            assert err < prev / 10
        prev = err
    assert prev < 1e-10


def test_fmm_random_points_and_mass_spectrum(orc):
    sf = W.star_field(5000, 0.45, "kroupa", seed=7, m_lo=0.08, m_hi=1.5)
    lens = orc.Lens(0.45, 0.0, 0.45, sf.x, sf.y, sf.m)
    L0 = 2.0 ** math.ceil(math.log2(sf.radius * 1.01))
    rng = np.random.default_rng(8)
    zx, zy = rng.uniform(-L0, L0, 4000) * 0.999, rng.uniform(-L0, L0, 4000) * 0.999
    F = orc.FMM(lens, L0, 28)
    fx, fy, leaf = F.alpha(zx, zy, want_leaf=True)
    assert np.all(leaf >= 0)
    ax, ay = orc.alpha_direct(lens, zx, zy)
    err = np.abs((fx - ax) + 1j * (fy - ay)) / np.maximum(np.abs(ax + 1j * ay), 1.0)
    assert err.max() < 1e-8


def test_local_expansions_vanish_near_root(orc):
    # levels 0 and 1: every star is in the node's 3x3 block (no far field)
    sf = W.star_field(500, 0.3, "equal", seed=9)
    lens = orc.Lens(0.3, 0.0, 0.3, sf.x, sf.y, sf.m)
    F = orc.FMM(lens, 64.0, 6)
    nd = F.nodes()
    a, c = F.coeffs()
    assert np.all(c[nd["level"] <= 1] == 0)
    # the root's monopole is the total mass
    assert a[0, 0].real == pytest.approx(sf.m.sum(), rel=1e-14)


def test_auto_order_rule(orc):
    # appendix C.3: p > log2((<m^2>/<m>) / (L eps))
    p = orc.auto_order(1.0, 1.0, 1.0, 1e-6)
    assert p == math.floor(math.log2(1e6)) + 1
    assert orc.auto_order(0.2234, 0.0754, 0.5, 1e-12) == 31   # capped at 31
