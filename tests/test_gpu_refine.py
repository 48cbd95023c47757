"""Cell refinement and the refinement network on the GPU against the FP64
oracle (needs an MI355X): the BF16 network's forward pass and gradients
(P10: within a BF16-scaled bound of the FP64 values computed from the same
rounded weights and inputs), training, the features and labels of sampled
cells, the plainly refined map, and what the trained network gains over
refining every cell."""
import json
import os
import time

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

REPORT = {}


def _report(key, **vals):
    REPORT[key] = vals
    print(f"[refine] {key}: " + ", ".join(f"{k}={v}" for k, v in vals.items()), flush=True)


@pytest.fixture(scope="module")
def mlm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2506_02114_amd as m
    m.load()
    yield m
    out = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")
    if os.path.isdir(out):
        with open(os.path.join(out, "parity_report_refine.json"), "w") as f:
            json.dump(REPORT, f, indent=1, default=float)


def _bf16(a):
    """Round to bfloat16 (nearest even), returned as float64."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _random_case(orc, n=300, seed=0):
    rng = np.random.default_rng(seed)
    P = orc.mlp_init(seed=seed + 1)
    for k in ("b1", "b2", "b3"):
        P[k] = rng.normal(0, 0.1, P[k].shape)
    flat = np.concatenate([P["W1"].ravel(), P["b1"], P["W2"].ravel(), P["b2"], P["W3"], P["b3"]]).astype(np.float32)
    X = rng.normal(0, 1.0, (n, 12)).astype(np.float32)
    X[:, 8:] = np.sign(X[:, 8:])
    y = (rng.random(n) < 0.3).astype(np.uint8)
    return flat, X, y


def _rounded(mlm, flat, X):
    """The oracle's parameters and inputs as the GPU kernels see them."""
    Q = mlm.params_to_dict(flat)
    for k in ("W1", "W2", "W3"):
        Q[k] = _bf16(Q[k])
    return Q, _bf16(X)


def test_network_forward_and_gradients_match_oracle(mlm, orc):
    flat, X, y = _random_case(orc)
    net = mlm.Refiner(flat)
    assert np.array_equal(net.params, flat)
    Q, Xr = _rounded(mlm, flat, X)
    z_ref, _ = orc.mlp_forward(Q, Xr)
    z = net.predict(X)
    # bf16 weights are in the oracle too; what remains is the rounding of the
    # inputs of each product to bf16 (2^-9 relative, the first hidden layer
    # carried to 16 bits) and FP32 accumulation
    scale = np.abs(z_ref).max() + 1.0
    ez = np.abs(z - z_ref).max() / scale
    loss_ref, G = orc.mlp_loss_grad(Q, Xr, y, pos_weight=2.0)
    loss, g = net.grads(X, y, pos_weight=2.0)
    gd = mlm.params_to_dict(g)
    errs = {k: float(np.linalg.norm(gd[k] - G[k]) / max(np.linalg.norm(G[k]), 1e-30)) for k in G}
    _report("network_vs_oracle", logit_err=float(ez), loss=loss, loss_ref=float(loss_ref), grad_rel=errs)
    assert ez < 2.0 ** -8
    assert abs(loss - loss_ref) < 2.0 ** -9 * abs(loss_ref)
    for k, e in errs.items():
        assert e < 2.0 ** -7, (k, e)


def test_network_training_learns(mlm, orc):
    """A separable rule (label = folded, or the first corner far from the
    mean) is learnt by the GPU training kernels; the loss falls."""
    rng = np.random.default_rng(12)
    n = 40000
    X = rng.normal(0, 1.5, (n, 12)).astype(np.float32)
    ears = np.sign(rng.normal(size=(n, 4)))
    ears[rng.random(n) < 0.7] = 1.0
    X[:, 8:] = ears
    y = ((np.abs(X[:, 0]) > 2.0) | (ears.min(1) != ears.max(1))).astype(np.uint8)
    net = mlm.Refiner(seed=3)
    losses = net.train(X, y, epochs=6, batch=2048, lr=3e-3, pos_weight=1.0, seed=1)
    acc = np.mean((net.predict(X) > 0) == (y == 1))
    _report("network_training", losses=[float(v) for v in losses], accuracy=float(acc), positives=float(y.mean()))
    assert losses[-1] < 0.5 * losses[0] and acc > 0.97


def test_training_graph_replays_match_eager(mlm):
    """Training with each epoch's steps captured once in a HIP graph and
    replayed per epoch (with the permutation upload, a reset and a
    synchronisation between replays) against the same steps launched one by
    one.  A batch's gradient is summed in a fixed order (per-wavefront rows,
    then one ordered sum), so two eager runs and the graph run agree bit for
    bit: every epoch's loss, the parameters and the predictions; a second call
    continues from the device step count."""
    import time
    rng = np.random.default_rng(31)
    n = 12000
    X = rng.normal(0, 1.5, (n, 12)).astype(np.float32)
    ears = np.sign(rng.normal(size=(n, 4)))
    ears[rng.random(n) < 0.7] = 1.0
    X[:, 8:] = ears
    y = ((np.abs(X[:, 0]) > 2.0) | (ears.min(1) != ears.max(1))).astype(np.uint8)
    kw = dict(epochs=4, batch=512, lr=3e-3, pos_weight=1.0, seed=2)
    runs = []
    for graph in (False, False, True):
        net = mlm.Refiner(seed=5)
        t0 = time.perf_counter()
        losses = net.train(X, y, graph=graph, **kw)
        dt = time.perf_counter() - t0
        more = net.train(X, y, graph=graph, **dict(kw, epochs=2, seed=3))
        runs.append((np.asarray(losses), np.asarray(more), net.params, net.predict(X), dt))
    (le, me, pe, ze, te), (le2, me2, pe2, ze2, _), (lg, mg, pg, zg, tg) = runs
    _report("training_graph_vs_eager", loss_eager=[float(v) for v in le], loss_graph=[float(v) for v in lg],
            loss_more_eager=[float(v) for v in me], loss_more_graph=[float(v) for v in mg],
            param_diff=float(np.abs(pe - pg).max()), param_diff_eager_runs=float(np.abs(pe2 - pe).max()),
            logit_diff=float(np.abs(ze - zg).max()), s_eager=te, s_graph=tg)
    for a, b in ((le2, le), (me2, me), (pe2, pe), (ze2, ze), (lg, le), (mg, me), (pg, pe), (zg, ze)):
        assert np.array_equal(a, b)
    assert lg[-1] < lg[0] and mg[-1] < lg[0]


def _lens_pair(mlm, orc, ks, kss, g, sf):
    return mlm.Lens(ks, kss, g, sf.x, sf.y, sf.m), orc.Lens(ks, kss, g, sf.x, sf.y, sf.m)


def test_cell_samples_match_oracle(mlm, orc):
    wl = W.config("plain_small")
    sf = wl.stars()
    gl, ol = _lens_pair(mlm, orc, 0.3, 0.0, 0.3, sf)
    spec = dict(wl.map.asdict(), order=20)
    R = orc.region(ol, **spec)
    rng = np.random.default_rng(21)
    cells = np.stack([rng.integers(0, R.nr1 - 1, 3000), rng.integers(0, R.nr2 - 1, 3000)], 1)
    feats, labels = gl.cell_samples(cells, **spec)
    F = orc.FMM(ol, R.L0, 20)
    lab_ref, _, _ = orc.refine_cells(R, ol, cells[:, 0], cells[:, 1], fmm=F, max_depth=1)
    # features against the oracle's from the same corners
    w = gl.deflect(np.concatenate([np.stack([R.x0 + (cells[:, 0] + da) * R.d1, R.y0 + (cells[:, 1] + db) * R.d2], 1)
                                   for da, db in ((0, 0), (1, 0), (1, 1), (0, 1))]), **spec)
    n = cells.shape[0]
    u = (w[:, 0] - (spec.get("y1c", 0.0) - spec["hw1"])) / R.pix1
    v = (w[:, 1] - (spec.get("y2c", 0.0) - spec["hw2"])) / R.pix2
    fe = 0.0
    for k in range(0, n, 7):
        f = orc.cell_features(u[k::n][:4], v[k::n][:4])
        fe = max(fe, float(np.abs(feats[k] - f).max()))
    mism = int((labels != lab_ref).sum())
    _report("cell_samples", feature_err=fe, label_mismatches=mism, positives=int(lab_ref.sum()), cells=n)
    assert fe < 1e-5
    assert mism <= max(1, n // 1000)


def test_plain_refined_map_matches_oracle(mlm, orc):
    sf = W.star_field(200, 0.35, "salpeter", seed=31, m_lo=0.1, m_hi=1.0)
    gl, ol = _lens_pair(mlm, orc, 0.35, 0.1, 0.25, sf)
    spec = dict(hw1=2.0, hw2=2.0, n1=48, n2=48, order=20)
    plain, s0 = gl.map(**spec)
    mu, st = gl.map(**spec, refine="plain")
    ref = orc.magnification_map(ol, spec, method="fmm", p=20)
    R = ref.region
    a, b = np.meshgrid(np.arange(R.nr1 - 1), np.arange(R.nr2 - 1))
    labels, dmu, ost = orc.refine_cells(R, ol, a.ravel(), b.ravel(), fmm=orc.FMM(ol, R.L0, 20))
    want = ref.mu + dmu
    pos = want > 0
    rel = np.abs(mu[pos] - want[pos]) / want[pos]
    change = np.abs(want - ref.mu).max()
    _report("plain_refined_map", max_rel=float(rel.max()), refined_cells=st["n_refined"],
            oracle_refined_cells=int(labels.sum()), tests=st["n_refine_tests"], oracle_tests=int(ost[0]),
            largest_change=float(change))
    assert change > 1e-3            # refinement matters on this map
    assert abs(st["n_refined"] - int(labels.sum())) <= 2
    assert rel.max() < 1e-6


def test_learned_refinement_gain(mlm, orc):
    """Train on cells of two draws of the 1e5-star plain workload's lens
    type and two of the high-magnification type (smaller fields of the same
    parameters), then map a fresh high-magnification field: the learned
    refinement against refining every cell (the method without the
    network): flag recall and precision, its map error relative to full
    refinement, and its time."""
    import torch
    dev = torch.device("cuda")
    feats, labels, domain = [], [], []
    rng = np.random.default_rng(2001)
    draws = [(0.45, 0.0, 0.45, "kroupa", 0.08, 1.5, 2001, 8000, 4.0),
             (0.45, 0.0, 0.45, "kroupa", 0.08, 1.5, 2002, 8000, 4.0),
             (0.01, 0.82, 0.1725, "salpeter", 0.1, 1.0, 3001, 20000, 1.0),
             (0.01, 0.82, 0.1725, "salpeter", 0.1, 1.0, 3002, 20000, 1.0)]
    for ks, kss, g, mf, lo, hi, seed, n, hw in draws:
        sf = W.star_field(n, ks, mf, seed=seed, m_lo=lo, m_hi=hi)
        gl = mlm.Lens(ks, kss, g, sf.x, sf.y, sf.m)
        spec = dict(hw1=hw, hw2=hw, n1=400, n2=400, order=16)
        R = gl.region(**spec)
        cells = np.stack([rng.integers(0, R["nr1"] - 1, 100000), rng.integers(0, R["nr2"] - 1, 100000)], 1)
        f, y = gl.cell_samples(cells, **spec)
        feats.append(f)
        labels.append(y)
        domain.append(np.full(len(y), 0 if ks > 0.1 else 1))
    X, y, dom = np.concatenate(feats), np.concatenate(labels), np.concatenate(domain)
    perm = rng.permutation(len(y))
    X, y, dom = X[perm], y[perm], dom[perm]
    ntr = int(0.8 * len(y))
    pw = float(min((1 - y.mean()) / max(y.mean(), 1e-6), 20.0))
    net = mlm.Refiner(seed=7)
    t0 = time.time()
    losses = net.train(X[:ntr], y[:ntr], epochs=20, batch=4096, lr=2e-3, pos_weight=pw, seed=2)
    t_train = time.time() - t0
    # threshold for 98% recall of the held-out positives of each lens type
    zv, yv, dv = net.predict(X[ntr:]), y[ntr:], dom[ntr:]
    folded = np.array([len(set(r)) > 1 for r in X[ntr:, 8:]])
    thr = min(float(np.quantile(zv[(yv == 1) & ~folded & (dv == d)], 0.02)) for d in (0, 1))
    flag = (zv > thr) | folded                  # folded cells are candidates anyway
    recall = float(flag[yv == 1].mean())
    precision = float(yv[flag].mean())
    # a fresh field of the high-magnification type
    sf = W.star_field(20000, 0.01, "salpeter", seed=3999, m_lo=0.1, m_hi=1.0)
    gl = mlm.Lens(0.01, 0.82, 0.1725, torch.from_numpy(sf.x).to(dev), torch.from_numpy(sf.y).to(dev),
                  torch.from_numpy(sf.m).to(dev))
    spec = dict(hw1=1.0, hw2=1.0, n1=400, n2=400, order=16)
    out = {k: torch.empty((400, 400), dtype=torch.float64, device=dev) for k in ("none", "plain", "learned")}
    stats = {}
    for mode in ("none", "plain", "learned"):
        kw = dict(refine=mode, refiner=net, refine_threshold=thr) if mode == "learned" else dict(refine=mode)
        gl.map(out=out[mode], **spec, **kw)                     # warm
        _, stats[mode] = gl.map(out=out[mode], timing=1, **spec, **kw)
    torch.cuda.synchronize()
    plain, full, learned = (out[k].cpu().numpy() for k in ("none", "plain", "learned"))
    e_plain = float(np.abs(plain - full).sum() / np.abs(full).sum())
    e_learned = float(np.abs(learned - full).sum() / np.abs(full).sum())
    t_full, t_learned = stats["plain"]["t_refine_ms"], stats["learned"]["t_refine_ms"]
    _report("learned_gain", train_losses=[float(v) for v in losses[::4]], train_s=t_train, positives=float(y.mean()),
            threshold=thr, heldout_recall=recall, heldout_precision=precision,
            l1_plain_vs_full=e_plain, l1_learned_vs_full=e_learned, t_refine_full_ms=t_full,
            t_refine_learned_ms=t_learned, candidates=stats["learned"]["n_refine_candidates"],
            cells=stats["learned"]["n_cells"], refined_full=stats["plain"]["n_refined"],
            refined_learned=stats["learned"]["n_refined"], t_map_ms={k: v["t_total_ms"] for k, v in stats.items()})
    assert recall > 0.95
    assert e_learned < 0.2 * e_plain      # most of the refinement's correction is kept
    assert t_learned < t_full             # for less work than testing every cell


def test_learned_refinement_at_workload_size(mlm):
    """The learned workload at its stated size: 1e7 labelled cells, half from
    ten draws of the 1e5-star plain lens type (seeds 2001-2010, its 2000^2 px
    map) and half from ten draws of the 1e6-star high-magnification type
    (seeds 3001-3010, its 4000^2 px map), sampled uniformly from each ray
    grid; the network trained on them by the library's kernels; then a fresh
    high-magnification field (seed 3999) mapped over 16 384 cell rows through
    the middle of its grid (2.0e8 cells) with no refinement, with full
    refinement (every cell tested) and with the learned one."""
    import torch
    dev = torch.device("cuda")
    rng = np.random.default_rng(5)
    feats, labels, domain = [], [], []
    t0 = time.time()
    for kind, seeds in (("plain_large", range(2001, 2011)), ("mixed_highmag", range(3001, 3011))):
        wl = W.config(kind)
        L = wl.lens
        spec = dict(wl.map.asdict(), order=16)
        for seed in seeds:
            sf = W.star_field(L.n_stars, L.kappa_star, L.mass_fn, seed=seed, m_lo=L.m_lo, m_hi=L.m_hi)
            gl = mlm.Lens(L.kappa_star, L.kappa_smooth, L.gamma, torch.from_numpy(sf.x).to(dev),
                          torch.from_numpy(sf.y).to(dev), torch.from_numpy(sf.m).to(dev))
            R = gl.region(**spec)
            cells = np.stack([rng.integers(0, R["nr1"] - 1, 500_000), rng.integers(0, R["nr2"] - 1, 500_000)], 1)
            f, y = gl.cell_samples(cells, **spec)
            feats.append(f)
            labels.append(y)
            domain.append(np.full(len(y), 0 if kind == "plain_large" else 1, np.int8))
            gl.close()
        print(f"[refine] {kind}: 5e6 cells labelled, {time.time() - t0:.0f} s", flush=True)
    X, y, dom = np.concatenate(feats), np.concatenate(labels), np.concatenate(domain)
    del feats, labels
    perm = rng.permutation(len(y))
    X, y, dom = X[perm], y[perm], dom[perm]
    ntr = len(y) - 500_000
    pw = float(min((1 - y.mean()) / max(y.mean(), 1e-6), 20.0))
    net = mlm.Refiner(seed=7)
    t1 = time.time()
    losses = net.train(X[:ntr], y[:ntr], epochs=6, batch=8192, lr=2e-3, pos_weight=pw, seed=2)
    t_train = time.time() - t1
    print(f"[refine] trained on {ntr} cells in {t_train:.1f} s", flush=True)
    zv, yv, dv = net.predict(X[ntr:]), y[ntr:], dom[ntr:]
    folded = np.array([len(set(r)) > 1 for r in X[ntr:, 8:]])
    thr = min(float(np.quantile(zv[(yv == 1) & ~folded & (dv == d)], 0.02)) for d in (0, 1))
    flag = (zv > thr) | folded
    recall = float(flag[yv == 1].mean())
    precision = float(yv[flag].mean())
    # the fresh high-magnification field, a 16 384-row strip of its map
    wl = W.config("mixed_highmag")
    L = wl.lens
    sf = W.star_field(L.n_stars, L.kappa_star, L.mass_fn, seed=3999, m_lo=L.m_lo, m_hi=L.m_hi)
    gl = mlm.Lens(L.kappa_star, L.kappa_smooth, L.gamma, torch.from_numpy(sf.x).to(dev),
                  torch.from_numpy(sf.y).to(dev), torch.from_numpy(sf.m).to(dev))
    spec = dict(wl.map.asdict(), order=16)
    R = gl.region(**spec)
    mid = R["nr2"] // 2
    rows = (mid - 8192, mid + 8192)
    out = {k: torch.empty((spec["n2"], spec["n1"]), dtype=torch.float64, device=dev)
           for k in ("none", "plain", "learned")}
    stats = {}
    for mode in ("none", "plain", "learned"):
        kw = dict(refine=mode, refiner=net, refine_threshold=thr) if mode == "learned" else dict(refine=mode)
        _, stats[mode] = gl.map(out=out[mode], rows=rows, timing=1, **spec, **kw)
        print(f"[refine] strip, refine={mode}: {stats[mode]['t_total_ms']:.0f} ms", flush=True)
    torch.cuda.synchronize()
    plain, full, learned = (out[k] for k in ("none", "plain", "learned"))
    norm = float(full.abs().sum())
    e_plain = float((plain - full).abs().sum()) / norm
    e_learned = float((learned - full).abs().sum()) / norm
    t_full, t_learned = stats["plain"]["t_refine_ms"], stats["learned"]["t_refine_ms"]
    _report("learned_gain_at_size", cells_trained=ntr, train_s=t_train, label_s=t1 - t0,
            train_losses=[float(v) for v in losses], positives=float(y.mean()), threshold=thr,
            heldout_recall=recall, heldout_precision=precision, eval_cells=stats["learned"]["n_cells"],
            l1_plain_vs_full=e_plain, l1_learned_vs_full=e_learned, t_refine_full_ms=t_full,
            t_refine_learned_ms=t_learned, candidates=stats["learned"]["n_refine_candidates"],
            refined_full=stats["plain"]["n_refined"], refined_learned=stats["learned"]["n_refined"],
            t_map_ms={k: v["t_total_ms"] for k, v in stats.items()})
    assert recall > 0.95
    assert e_learned < 0.2 * e_plain
    assert t_learned < t_full
