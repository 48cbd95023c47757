"""Pins of the oracle's cell refinement, cell features and refinement
network (test infrastructure for the learned variant; the paper itself
apportions every cell as two triangles, sec. 3.2)."""
import math

import numpy as np
import pytest

import workloads as W


def test_mlp_gradients_match_finite_differences(orc):
    """Every parameter's analytic gradient against central differences of the
    loss in FP64 (P10)."""
    rng = np.random.default_rng(3)
    P = orc.mlp_init(seed=5)
    for k in ("b1", "b2", "b3"):
        P[k] = rng.normal(0, 0.1, P[k].shape)
    X = rng.normal(0, 1.0, (40, 12))
    y = (rng.random(40) < 0.3).astype(np.uint8)
    loss, G = orc.mlp_loss_grad(P, X, y, pos_weight=3.0)
    h = 1e-6
    for name, arr in P.items():
        flat = arr.reshape(-1)
        idx = rng.choice(flat.size, size=min(flat.size, 25), replace=False)
        for k in idx:
            old = flat[k]
            flat[k] = old + h
            lp, _ = orc.mlp_loss_grad(P, X, y, pos_weight=3.0)
            flat[k] = old - h
            lm, _ = orc.mlp_loss_grad(P, X, y, pos_weight=3.0)
            flat[k] = old
            fd = (lp - lm) / (2 * h)
            g = G[name].reshape(-1)[k]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(fd)), (name, k, fd, g)


def test_mlp_closed_forms(orc):
    """Zero weights give the bias as logit and loss softplus terms; a ReLU
    network is positively homogeneous in its input when biases vanish."""
    P = {k: np.zeros_like(v) for k, v in orc.mlp_init().items()}
    P["b3"][:] = 0.7
    X = np.random.default_rng(1).normal(size=(8, 12))
    y = np.array([1, 0, 1, 1, 0, 0, 0, 1], np.uint8)
    z, _ = orc.mlp_forward(P, X)
    assert np.all(z == 0.7)
    loss, G = orc.mlp_loss_grad(P, X, y, pos_weight=2.0)
    sp = lambda t: math.log1p(math.exp(t))
    want = np.mean([2.0 * sp(-0.7) if t else sp(0.7) for t in y])
    assert abs(loss - want) < 1e-15
    s = 1 / (1 + math.exp(-0.7))
    assert abs(G["b3"][0] - np.mean([2.0 * (s - 1) if t else s for t in y])) < 1e-15
    Q = orc.mlp_init(seed=2)
    z1, _ = orc.mlp_forward(Q, X)
    z3, _ = orc.mlp_forward(Q, 3.0 * X)
    np.testing.assert_allclose(z3, 3.0 * z1, rtol=1e-12, atol=1e-12)


def test_cell_features(orc):
    rng = np.random.default_rng(8)
    u = rng.normal(size=4) * 3
    v = rng.normal(size=4) * 3
    f = orc.cell_features(u, v)
    # offsets from the pixel corner: unchanged by a whole-pixel translation
    np.testing.assert_allclose(orc.cell_features(u + 5.0, v - 7.0)[:8], f[:8], rtol=0, atol=1e-14)
    # ... but not by a fraction of a pixel (the grid phase shows)
    assert np.abs(orc.cell_features(u + 0.5, v)[:8:2] - f[:8:2]).max() > 0.1
    # a unit square with positive orientation: ears all +1; mirrored: all -1
    su, sv = np.array([0, 1, 1, 0.0]) + 0.25, np.array([0, 0, 1, 1.0]) + 0.25
    assert list(orc.cell_features(su, sv)[8:]) == [1, 1, 1, 1]
    assert list(orc.cell_features(su, -sv)[8:]) == [-1, -1, -1, -1]
    # offsets are log-compressed: the mean (0.75, 0.75) lies in pixel (0, 0),
    # so corner 11 sits at (1.25, 1.25)
    ff = orc.cell_features(su, sv)
    assert abs(ff[4] - math.log1p(1.25)) < 1e-15 and abs(ff[0] - math.log1p(0.25)) < 1e-15
    # a folded cell (corner 11 pulled across the diagonal): ears disagree
    fu, fv = np.array([0, 1, 0.2, 0.0]), np.array([0, 0, 0.2, 1.0])
    e = orc.cell_features(fu, fv)[8:]
    assert len(set(e)) > 1


def test_linear_mapping_is_never_refined(orc):
    """Macro model only: the mapping is linear, so the 2 x 2 split tiles the
    cell's image exactly; no cell is refined and the map does not change."""
    L = orc.Lens(0.0, 0.35, 0.2, [], [], [], sheet=False)
    spec = dict(hw1=2.0, hw2=2.0, n1=16, n2=16, rays_per_pixel=1.0, y1c=0.1, y2c=-0.05)
    R = orc.region(L, **spec)
    a, b = np.meshgrid(np.arange(R.nr1 - 1), np.arange(R.nr2 - 1))
    labels, dmu, st = orc.refine_cells(R, L, a.ravel(), b.ravel())
    assert labels.sum() == 0 and st[1] == 0
    assert np.abs(dmu).max() < 1e-12


def test_point_lens_refinement(orc):
    """Point lens: refined cells are the folded ones across the Einstein ring
    plus those where the map is curved; full refinement moves the map toward
    the pixel-averaged closed form (u^2 + 2) / (u sqrt(u^2 + 4))."""
    from test_oracle_ipm import _pixel_average
    L = orc.Lens(0.0, 0.0, 0.0, [0.0], [0.0], [1.0], sheet=False)
    A = lambda y1, y2: ((y1 ** 2 + y2 ** 2) + 2) / (np.hypot(y1, y2) * np.sqrt(y1 ** 2 + y2 ** 2 + 4))
    spec = dict(hw1=1.5, hw2=1.5, n1=24, n2=24, rays_per_pixel=1.0, dx1=3.0, dx2=3.0, y1c=0.03, y2c=0.05)
    res = orc.magnification_map(L, spec, method="direct")
    R = res.region
    a, b = np.meshgrid(np.arange(R.nr1 - 1), np.arange(R.nr2 - 1))
    a, b = a.ravel(), b.ravel()
    labels, dmu, st = orc.refine_cells(R, L, a, b)
    assert st[1] > 0 and labels.sum() > 0
    # folded cells straddle the critical curve |z| = 1
    zc = np.hypot(R.x0 + (a + 0.5) * R.d1, R.y0 + (b + 0.5) * R.d2)
    ring = np.abs(zc - 1.0) < 2 * max(R.d1, R.d2)
    assert labels[ring].mean() > 0.9
    refined = res.mu + dmu
    e_plain, e_ref = [], []
    for j in range(R.n2):
        for i in range(R.n1):
            cu = R.y1c - R.hw1 + (i + 0.5) * R.pix1
            cv = R.y2c - R.hw2 + (j + 0.5) * R.pix2
            if math.hypot(cu, cv) < 2 * R.pix1:
                continue
            want = _pixel_average(A, R, i, j)
            e_plain.append(abs(res.mu[j, i] - want) / want)
            e_ref.append(abs(refined[j, i] - want) / want)
    assert np.mean(e_ref) < 0.5 * np.mean(e_plain)


def test_refinement_depth_and_threshold_monotone(orc):
    """More depth refines more subcells; a looser threshold refines fewer
    cells; with depth 0 nothing is tested."""
    sf = W.star_field(30, 0.4, "equal", seed=9)
    L = orc.Lens(0.4, 0.0, 0.3, sf.x, sf.y, sf.m)
    spec = dict(hw1=2.0, hw2=2.0, n1=20, n2=20, rays_per_pixel=1.0)
    R = orc.region(L, **spec)
    a, b = np.meshgrid(np.arange(R.nr1 - 1), np.arange(R.nr2 - 1))
    a, b = a.ravel()[::3], b.ravel()[::3]
    l1, _, s1 = orc.refine_cells(R, L, a, b, max_depth=1)
    l3, _, s3 = orc.refine_cells(R, L, a, b, max_depth=3)
    np.testing.assert_array_equal(l1, l3)          # the label is decided at the first level
    assert s3[1] >= s1[1] and s3[0] >= s1[0]
    lt, _, _ = orc.refine_cells(R, L, a, b, tau=1e-1)
    assert lt.sum() <= l3.sum()
    l0, d0, s0 = orc.refine_cells(R, L, a, b, max_depth=0)
    assert l0.sum() == 0 and s0[0] == 0 and np.abs(d0).max() == 0.0
