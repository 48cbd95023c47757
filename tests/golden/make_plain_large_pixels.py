"""Writes plain_large_pixels.npz: sampled pixels of the oracle's whole FP64 map
of the plain 1e5-star workload (Kroupa 0.08-1.5, kappa_* = 0.45, kappa_s = 0,
gamma = 0.45, 2000 x 2000 px of half-width 25, 1 ray per pixel, FMM order 20).

Only the oracle is called.  The map is made strip by strip (strips of cell
rows are independent and their deposits add, as the tests of the oracle
check) on a pool of threads; each oracle call runs single-threaded and
releases the interpreter lock.  The sample: every pixel of five whole pixel
rows, the 2000 pixels of highest magnification and 8000 further pixels drawn
with seed 7.

    python tests/golden/make_plain_large_pixels.py [--threads 8]
"""
from __future__ import annotations

import argparse
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "plain_large_pixels.npz")
ORDER = 20
WHOLE_ROWS = (0, 500, 1000, 1500, 1999)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--strip", type=int, default=64, help="cell rows per oracle call")
    args = ap.parse_args()
    wl = W.config("plain_large")
    sf = wl.stars()
    L = wl.lens
    lens = oracle.Lens(L.kappa_star, L.kappa_smooth, L.gamma, sf.x, sf.y, sf.m)
    spec = wl.map.asdict()
    R = oracle.region(lens, **spec)
    t0 = time.time()
    fmm = oracle.FMM(lens, R.L0, ORDER, nthreads=args.threads)
    print(f"FMM built in {time.time() - t0:.1f} s; grid {R.nr1} x {R.nr2}", flush=True)
    strips = [(b, min(R.nr2 - 1, b + args.strip)) for b in range(0, R.nr2 - 1, args.strip)]

    def run(chunk):
        dep = np.zeros(R.n1 * R.n2)
        st = np.zeros(5)
        for b, e in chunk:
            wx, wy = oracle.shoot_rows(R, lens, b, e + 1, fmm, 1)
            oracle.ipm_rows(R, b, e, wx, wy, dep, st)
        return dep, st

    # interleave the strips over the workers so each gets a similar mix
    chunks = [strips[k::args.threads * 4] for k in range(args.threads * 4)]
    dep = np.zeros(R.n1 * R.n2)
    stats = np.zeros(5)
    done = 0
    with ThreadPoolExecutor(args.threads) as ex:
        for d, s in ex.map(run, chunks):
            dep += d
            stats += s
            done += 1
            print(f"{done}/{len(chunks)} chunks, {time.time() - t0:.0f} s", flush=True)
    mu = np.empty_like(dep)
    oracle.lib().orc_normalise(oracle.C.byref(R), oracle._d(dep), oracle._d(mu))
    mu = mu.reshape(R.n2, R.n1)
    rng = np.random.default_rng(7)
    idx = set()
    for j in WHOLE_ROWS:
        idx.update(range(j * R.n1, (j + 1) * R.n1))
    idx.update(np.argsort(mu.ravel())[-2000:].tolist())
    target = len(idx) + 8000
    while len(idx) < target:
        idx.add(int(rng.integers(0, mu.size)))
    idx = np.array(sorted(idx), dtype=np.int64)
    np.savez_compressed(OUT, index=idx, mu=mu.ravel()[idx], order=np.int64(ORDER),
                        dep_total=stats[0], a_out=stats[1], a_skip=stats[2], n_skip=stats[3],
                        mean_mu=mu.mean(), min_mu=mu.min(), max_mu=mu.max())
    print(f"wrote {OUT}: {idx.size} pixels; mean mu {mu.mean():.6f}, min {mu.min():.3e}, max {mu.max():.3e}; "
          f"{time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
