"""GPU parity of the CDF 9/7 path (dwt2_fwd_cdf97 / dwt2_inv_cdf97, through the
C ABI) against the float64 9/7 oracle.

Bar: float32 within TOL97 absolute on 8-bit-range data.  The bound is the
unit roundoff 2^-24, times 2^13 (every intermediate value of a fused level
on 8-bit input stays below 2^13), times 2^3 (roundings that can reach an
output at full weight), which is 2^-8 < 4e-3."""
import numpy as np
import pytest
import torch

from oracle import dwt97
from paper_1708_07853_amd import synth

pytestmark = pytest.mark.gpu
TOL97 = 4e-3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def D():
    import paper_1708_07853_amd as d
    return d


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def max_levels(w, h, cap=6):
    lv = 1
    while lv < cap and -(-w // (1 << lv)) >= 2 and -(-h // (1 << lv)) >= 2:
        lv += 1
    return lv


def maxdiff(a, b):
    return float(np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)).max())


# tiles are 128 x 32 pixels: these span several tiles per axis, ragged
# edges, odd sizes, and inputs narrower than the halo
SHAPES = [(2, 2), (3, 5), (17, 2), (2, 300), (5, 7), (64, 64), (65, 33), (33, 129), (300, 517), (129, 1030),
          (97, 258), (260, 131)]


def _img(h, w, seed):
    return np.random.default_rng(seed).integers(0, 256, size=(h, w)).astype(np.float64)


def test_cdf97_forward_matches_oracle():
    d = D()
    worst = 0.0
    for idx, (h, w) in enumerate(SHAPES):
        x = _img(h, w, 9700 + idx)
        for levels in sorted({1, 2, max_levels(w, h)}):
            if levels > max_levels(w, h):
                continue
            got = d.fwd_cdf97(to_gpu(x), levels).cpu().numpy()
            err = maxdiff(got, dwt97.fwd(x, levels))
            worst = max(worst, err)
            assert err <= TOL97, (h, w, levels, err)
    print(f"worst forward error {worst:.3g}")


# the forward's strip kernel (level inputs of at least 16 x 16): widths
# around multiples of its 224-pixel strip pitch and of the 256-pixel wave,
# heights across segment boundaries
STRIP_SHAPES = [(16, 16), (17, 23), (16, 221), (33, 224), (40, 225), (19, 226), (64, 446), (65, 448), (31, 449),
                (100, 479), (130, 672), (129, 673), (37, 1030), (300, 517), (260, 131), (16, 256), (23, 257)]


@pytest.mark.parametrize("stores", ["auto", "direct", "staged"])
def test_cdf97_strip_kernel_equals_tiled(monkeypatch, stores):
    """The register-resident forward and inverse (default from 16 x 16) are
    bit-identical to the LDS-tiled kernels at every size, level count and
    work-item shape, and match the oracle; the forward's stores either go
    out directly or are staged through LDS (forced here both ways)."""
    d = D()
    if stores != "auto":
        monkeypatch.setenv("DWT2_PAIR_STAGE", "1" if stores == "staged" else "0")
    for idx, (h, w) in enumerate(STRIP_SHAPES):
        xn = _img(h, w, 9900 + idx)
        x = to_gpu(xn)
        for levels in sorted({1, 2, max_levels(w, h)}):
            print(f"cdf97 strip ({stores}): {h}x{w} levels {levels}", flush=True)
            monkeypatch.setenv("DWT2_CDF97_TILED", "1")
            ref = d.fwd_cdf97(x, levels)
            ref_i = d.inv_cdf97(ref, levels)
            monkeypatch.setenv("DWT2_CDF97_TILED", "0")  # strip kernels at every level
            got = d.fwd_cdf97(x, levels)
            assert torch.equal(got, ref), (h, w, levels, float((got - ref).abs().max()))
            assert maxdiff(got.cpu().numpy(), dwt97.fwd(xn, levels)) <= TOL97, (h, w, levels)
            got_i = d.inv_cdf97(ref, levels)
            assert torch.equal(got_i, ref_i), (h, w, levels, float((got_i - ref_i).abs().max()))
            assert float((got_i - x).abs().max()) <= TOL97, (h, w, levels)
    x = to_gpu(_img(300, 517, 9999))
    monkeypatch.setenv("DWT2_CDF97_TILED", "1")
    ref = d.fwd_cdf97(x, 3)
    ref_i = d.inv_cdf97(ref, 3)
    monkeypatch.setenv("DWT2_CDF97_TILED", "0")
    try:
        for seg, ch in [(1, 1), (2, 2), (3, 1), (5, 2), (64, 2), (1000, 1)]:
            print(f"cdf97 strip tiling: seg {seg} chunk {ch}", flush=True)
            d.set_tiling(seg, ch)
            assert torch.equal(d.fwd_cdf97(x, 3), ref), (seg, ch)
            assert torch.equal(d.inv_cdf97(ref, 3), ref_i), (seg, ch)
    finally:
        d.set_tiling(0, 0)


def test_cdf97_inverse_matches_oracle_and_round_trips():
    d = D()
    for idx, (h, w) in enumerate(SHAPES):
        x = _img(h, w, 9750 + idx)
        for levels in sorted({1, max_levels(w, h)}):
            c32 = dwt97.fwd(x, levels).astype(np.float32)
            got = d.inv_cdf97(to_gpu(c32), levels).cpu().numpy()
            assert maxdiff(got, dwt97.inv(c32.astype(np.float64), levels)) <= TOL97, (h, w, levels)
            xg = to_gpu(x)
            rt = d.inv_cdf97(d.fwd_cdf97(xg, levels), levels)
            assert float((rt - xg).abs().max()) <= TOL97, (h, w, levels)


def test_cdf97_separable_comparison_kernel():
    """The separable comparison kernel (eight barrier-separated steps per
    level) computes the same transform: within the bound of the oracle and of
    the non-separable kernels, on the size sweep, a batch and 8192^2."""
    d = D()
    for idx, (h, w) in enumerate(SHAPES):
        x = _img(h, w, 9900 + idx)
        for levels in sorted({1, max_levels(w, h)}):
            xg = to_gpu(x)
            got = d.fwd_cdf97_separable(xg, levels)
            assert maxdiff(got.cpu().numpy(), dwt97.fwd(x, levels)) <= TOL97, (h, w, levels)
            assert float((got - d.fwd_cdf97(xg, levels)).abs().max()) <= TOL97, (h, w, levels)
    xs = torch.stack([to_gpu(_img(250, 333, 9950 + b)) for b in range(2)])
    assert float((d.fwd_cdf97_separable(xs, 3) - d.fwd_cdf97(xs, 3)).abs().max()) <= TOL97
    x = synth.image_device(8192, 8192, 2)
    assert float((d.fwd_cdf97_separable(x, 6) - d.fwd_cdf97(x, 6)).abs().max()) <= TOL97


def test_cdf97_batch_strides():
    d = D()
    xs = torch.stack([to_gpu(_img(250, 333, 9800 + b)) for b in range(3)])
    base = torch.zeros((3, 250, 340), device="cuda")
    xv = base[:, :, 2:335]
    xv.copy_(xs)
    got = d.fwd_cdf97(xv, 3)
    for b in range(3):
        ref = dwt97.fwd(xs[b].cpu().numpy().astype(np.float64), 3)
        assert maxdiff(got[b].cpu().numpy(), ref) <= TOL97
    assert float((d.inv_cdf97(got, 3) - xs).abs().max()) <= TOL97
    # a single image into a strided 2-D view: nothing outside the view is written
    obase = torch.full((252, 341), -5.0, device="cuda")
    ov = obase[1:251, 1:334]
    d.inv_cdf97(got[1].contiguous(), 3, out=ov)
    assert float((ov - xs[1]).abs().max()) <= TOL97
    assert torch.all(obase[0] == -5) and torch.all(obase[251] == -5)
    assert torch.all(obase[:, 0] == -5) and torch.all(obase[:, 334:] == -5)


# the forward's fused tail (DWT2_CDF97_TAIL=1: its last 2-3 levels of at most
# 1024^2 pixels over the batch, each at least 8 x 8, in one launch on 64 x 64
# pixel tiles): ragged and odd sizes, tiles past the edge, two or three
# levels in the tail, whole transforms in it, batches; bit-identical to the
# per-level kernels
TAIL_CASES = [((64, 64), 3), ((300, 517), 4), ((97, 131), 3), ((1000, 1000), 2), ((33, 70), 2), ((256, 256), 5),
              ((130, 65), 3), ((9, 200), 1)]


def test_cdf97_tail_equals_per_level(monkeypatch):
    d = D()
    for idx, ((h, w), levels) in enumerate(TAIL_CASES):
        for batch in (1, 3):
            xn = np.stack([_img(h, w, 9600 + 10 * idx + b) for b in range(batch)])
            x = to_gpu(xn if batch > 1 else xn[0])
            print(f"cdf97 tail: {batch} x {h}x{w} levels {levels}", flush=True)
            monkeypatch.delenv("DWT2_CDF97_TAIL", raising=False)
            ref = d.fwd_cdf97(x, levels)
            monkeypatch.setenv("DWT2_CDF97_TAIL", "1")
            got = d.fwd_cdf97(x, levels)
            assert torch.equal(got, ref), (batch, h, w, levels, float((got - ref).abs().max()))
            g0 = got[0] if batch > 1 else got
            assert maxdiff(g0.cpu().numpy(), dwt97.fwd(xn[0], levels)) <= TOL97, (batch, h, w, levels)


def test_cdf97_full_size():
    """The 8192^2 6-level workload: the forward against the oracle element
    by element, the inverse through the round trip."""
    d = D()
    x = synth.image_device(8192, 8192, 2)
    c = d.fwd_cdf97(x, 6)
    ref = dwt97.fwd(x.cpu().numpy().astype(np.float64), 6)
    assert maxdiff(c.cpu().numpy(), ref) <= TOL97
    r = d.inv_cdf97(c, 6)
    assert float((r - x).abs().max()) <= TOL97
