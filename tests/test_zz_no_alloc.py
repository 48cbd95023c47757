"""mlm_map_noalloc (scratch carved from the library's static device array,
no device allocation) against mlm_map on the same inputs (needs an MI355X).

Two calls in a row, the second with a smaller input, then a map too large
for the array, which must be refused before any device work.  The maps are
FP64 and go through the same kernels; only the order of the atomic pixel
additions differs, so they agree to rounding (bound 1e-12 relative, pixels
of zero magnification exactly zero in both)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mlm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2506_02114_amd as m
    m.load()
    return m


def _compare(a, b, what):
    assert np.all(np.isfinite(a)) and np.all(np.isfinite(b)), what
    pos = b > 0
    assert np.array_equal(a > 0, pos), what
    rel = np.abs(a[pos] - b[pos]) / b[pos]
    print(f"[noalloc] {what}: max rel {rel.max():.2e} over {pos.sum()} pixels", flush=True)
    assert rel.max() < 1e-12, what


def test_noalloc_matches_mlm_map_twice(mlm):
    import torch
    dev = torch.device("cuda")
    # first call: the 1000-star workload's map on the device
    wl = W.config("plain_small")
    sf = wl.stars()
    print("[noalloc] call 1: plain_small, 256^2 px, 512^2 rays, device output", flush=True)
    lens = mlm.Lens(0.3, 0.0, 0.3, sf.x, sf.y, sf.m)
    spec = wl.map.asdict()
    ref = torch.empty((256, 256), dtype=torch.float64, device=dev)
    got = torch.full_like(ref, -1.0)
    _, s_ref = lens.map(out=ref, **spec)
    _, s_got = lens.map(out=got, noalloc=True, **spec)
    torch.cuda.synchronize()
    assert s_got["n_rays"] == s_ref["n_rays"] and s_got["n_leaves"] == s_ref["n_leaves"]
    assert s_got["order"] == s_ref["order"] and s_got["n_big"] == s_ref["n_big"]
    _compare(got.cpu().numpy(), ref.cpu().numpy(), "call 1")
    # second call, smaller: another lens, a 96 x 80 map to the host, mixed
    # precision and the FMM order rule
    sf2 = W.star_field(300, 0.2, "salpeter", seed=77)
    print("[noalloc] call 2: 300 stars, 96 x 80 px, host output, mixed precision", flush=True)
    lens2 = mlm.Lens(0.2, 0.1, -0.15, sf2.x, sf2.y, sf2.m)
    spec2 = dict(hw1=3.0, hw2=2.5, n1=96, n2=80, rays_per_pixel=2.0, precision="mixed")
    ref2, s2r = lens2.map(**spec2)
    got2, s2g = lens2.map(noalloc=True, **spec2)
    assert s2g["n_rays"] == s2r["n_rays"]
    _compare(got2, ref2, "call 2")
    # the first lens again through mlm_map: its own buffers were put back
    again = torch.empty_like(ref)
    lens.map(out=again, **spec)
    torch.cuda.synchronize()
    _compare(again.cpu().numpy(), ref.cpu().numpy(), "mlm_map after the scratch calls")


def test_noalloc_refuses_what_does_not_fit(mlm):
    # 1.6e6 stars need 77 MiB for their sorted copies alone: refused on the
    # host, before any device work
    n = 1_600_000
    rng = np.random.default_rng(5)
    x = rng.uniform(-2000, 2000, n)
    y = rng.uniform(-2000, 2000, n)
    m = np.full(n, 0.3)
    print("[noalloc] 1.6e6 stars: expect MLM_ERANGE", flush=True)
    lens = mlm.Lens(0.01, 0.0, 0.1, x, y, m)
    with pytest.raises(mlm.MLMError) as e:
        lens.map(noalloc=True, hw1=1.0, hw2=1.0, n1=16, n2=16)
    assert e.value.status == mlm.MLM_ERANGE
    # refinement is not offered
    sf = W.star_field(50, 0.3, "equal", seed=3)
    small = mlm.Lens(0.3, 0.0, 0.3, sf.x, sf.y, sf.m)
    with pytest.raises(mlm.MLMError) as e:
        small.map(noalloc=True, hw1=1.0, hw2=1.0, n1=16, n2=16, refine="plain")
    assert e.value.status == mlm.MLM_ENOTSUP
