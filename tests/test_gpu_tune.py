"""dwt2_tune: per-shape tuning of the work-item heights changes no result
(the tuning call's own output and every later call's are bit-identical to
untuned calls), restores a user's timing probe, records nothing under a
forced tiling, and dwt2_tune_clear forgets every height."""
import numpy as np
import pytest
import torch

from paper_1708_07853_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1708_07853_amd as d
    d.tune_clear()
    yield
    d.tune_clear()
    d.set_tiling(0, 0)


def D():
    import paper_1708_07853_amd as d
    return d


CASES = [(4096, 4096, 1, 4, torch.float32), (1500, 900, 3, 5, torch.float32), (2048, 2048, 2, 3, torch.int32),
         (8192, 8192, 1, 6, torch.float32)]


@pytest.mark.parametrize("w,h,b,L,dt", CASES)
def test_tuned_results_are_unchanged(w, h, b, L, dt):
    d = D()
    print(f"tune case {w}x{h} batch {b} levels {L} {dt}", flush=True)
    x = torch.stack([synth.image_device(w, h, 11 + i, dtype=dt) for i in range(b)])
    g = torch.stack([synth.image_device(w, h, 41 + i) for i in range(b)]) - 128.0
    d.tune_clear()
    ref_f = d.fwd(x, L)
    ref_i = d.inv(ref_f, L)
    ref_b = d.bwd(g, L) if dt == torch.float32 else None
    assert torch.equal(d.tune("fwd", x, L), ref_f)
    assert torch.equal(d.tune("inv", ref_f, L), ref_i)
    if ref_b is not None:
        assert torch.equal(d.tune("bwd", g, L), ref_b)
    print(f"tuned launch shapes: {d.tune_entries()}", flush=True)
    for _ in range(2):
        assert torch.equal(d.fwd(x, L), ref_f)
        assert torch.equal(d.inv(ref_f, L), ref_i)
        if ref_b is not None:
            assert torch.equal(d.bwd(g, L), ref_b)
    if dt == torch.int32:
        assert torch.equal(ref_i, x)


@pytest.mark.parametrize("w,h,b,L", [(4096, 4096, 1, 6), (1500, 900, 3, 5), (600, 2000, 2, 4)])
def test_tuned_cdf97_results_are_unchanged(w, h, b, L):
    """The CDF 9/7 strip levels (dwt2_tune directions 3 and 4): the tuning
    calls and later calls give the untuned bits."""
    d = D()
    print(f"tune cdf97 case {w}x{h} batch {b} levels {L}", flush=True)
    x = torch.stack([synth.image_device(w, h, 61 + i) for i in range(b)])
    d.tune_clear()
    ref_f = d.fwd_cdf97(x, L)
    ref_i = d.inv_cdf97(ref_f, L)
    assert torch.equal(d.tune("fwd_cdf97", x, L), ref_f)
    assert torch.equal(d.tune("inv_cdf97", ref_f, L), ref_i)
    print(f"tuned launch shapes: {d.tune_entries()}", flush=True)
    for _ in range(2):
        assert torch.equal(d.fwd_cdf97(x, L), ref_f)
        assert torch.equal(d.inv_cdf97(ref_f, L), ref_i)


def test_tune_restores_probe_and_respects_forced_tiling():
    d = D()
    x = synth.image_device(2048, 2048, 3)
    b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.record()
    for _ in range(50):  # a long gap between the events' first records
        z = (x * 2.0).cumsum(0)
    e.record()
    torch.cuda.synchronize()
    gap = b.elapsed_time(e)
    d.set_probe("fwd", 1, b, e)
    d.tune("fwd", x, 3)
    y = d.fwd(x, 3)
    torch.cuda.synchronize()
    d.set_probe(None)
    # the probe (restored after tuning) re-recorded the events around the
    # plain call's first launch
    assert 0.0 < b.elapsed_time(e) < 0.5 * gap, (b.elapsed_time(e), gap)
    del z
    d.tune_clear()
    d.set_tiling(8, 2)
    assert torch.equal(d.tune("fwd", x, 3), y)
    assert d.tune_entries() == 0
    d.set_tiling(0, 0)
    d.tune("fwd", x, 3)
    d.tune_clear()
    assert d.tune_entries() == 0
