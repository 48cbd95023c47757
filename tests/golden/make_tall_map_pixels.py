"""Writes tall_map_pixels.npz: the oracle's FP64 map of a tall map with many
row bands, sampled.  The lens is the small test workload's star field
(kappa_* = 0.3, kappa_s = 0, gamma = 0.3); the map is 5000 x 6000 px of
0.001 (6000 pixel rows), shot on a coarse 100 x 120 ray grid, FMM order 16.

Only the oracle is called.  Stored: every pixel row's sum, the total
deposited, the 2000 pixels of highest magnification and 20000 further pixels
drawn with seed 11.

    python tests/golden/make_tall_map_pixels.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "tall_map_pixels.npz")
PIX = 0.001
N1, N2 = 5000, 6000
SPEC = dict(hw1=0.5 * N1 * PIX, hw2=0.5 * N2 * PIX, n1=N1, n2=N2, nray1=100, nray2=120, order=16)


def main():
    sf = W.config("plain_small").stars()
    lens = oracle.Lens(0.3, 0.0, 0.3, sf.x, sf.y, sf.m, sheet=True)
    t0 = time.time()
    ref = oracle.magnification_map(lens, SPEC, method="fmm", p=16)
    mu = ref.mu
    print(f"oracle map in {time.time() - t0:.1f} s", flush=True)
    assert mu.shape == (N2, N1)
    flat = mu.ravel()
    top = np.argsort(flat)[-2000:]
    rng = np.random.default_rng(11)
    rest = rng.choice(flat.size, 20000, replace=False)
    index = np.unique(np.concatenate([top, rest])).astype(np.int64)
    np.savez_compressed(OUT, index=index, mu=flat[index], row_sum=mu.sum(axis=1), dep_total=ref.dep_total,
                        n1=N1, n2=N2, pix=PIX, nray1=SPEC["nray1"], nray2=SPEC["nray2"], order=16)
    print(f"wrote {OUT}: {index.size} pixels, total {ref.dep_total:.12g}")


if __name__ == "__main__":
    main()
