"""GPU checks of the boundary's failure reporting and resource bounds:
a persistent launch whose dependency waits give up (forced from the host
with a tiny poll budget and an unreachable target, so every kernel still
exits normally) is reported by dwt2_synchronize and by the next call, and the
batched plan cache stays bounded however many calls are made."""
import os

import numpy as np
import pytest
import torch

from paper_1708_07853_amd import _lib, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def D():
    import paper_1708_07853_amd as d
    return d


def test_persistent_give_up_is_reported_and_recovers():
    d = D()
    x = torch.from_numpy(synth.image(1024, 768, 31)).cuda()
    ref = d.fwd(x, 3)
    torch.cuda.synchronize()
    try:
        d.set_path("persistent")
        d.set_job_wait(8, True)
        d.fwd(x, 3)                       # launches; every level-2/3 wait gives up
        with pytest.raises(_lib.Dwt2Error) as e:
            d.synchronize()
        assert e.value.status == -6 and "gave up" in str(e.value)
        d.synchronize()                   # reported once
        # the next transform call reports a give-up that nobody collected
        d.fwd(x, 3)
        torch.cuda.synchronize()
        with pytest.raises(_lib.Dwt2Error):
            d.inv(ref, 3)
        d.set_job_wait(0, False)
        d.synchronize()
        assert torch.equal(d.fwd(x, 3), ref)
        d.synchronize()
    finally:
        d.set_job_wait(0, False)
        d.set_path("levels")
        torch.cuda.synchronize()
        _lib.load().dwt2_synchronize(None)


def test_batched_persistent_give_up_is_reported():
    d = D()
    saved = os.environ.get("DWT2_BATCH_SCHEDULE")
    imgs = [torch.from_numpy(synth.image(w, h, 50 + i)).cuda() for i, (w, h) in enumerate([(300, 200), (97, 515)])]
    refs = [d.fwd(im, 3) for im in imgs]
    try:
        os.environ["DWT2_BATCH_SCHEDULE"] = "0"
        d.clear_plan_cache()
        d.set_job_wait(8, True)           # plans built now keep this budget
        d.fwd_batched(imgs, 3)
        with pytest.raises(_lib.Dwt2Error):
            d.synchronize()
        d.set_job_wait(0, False)
        d.clear_plan_cache()              # rebuild with the default budget
        for o, r in zip(d.fwd_batched(imgs, 3), refs):
            assert torch.equal(o, r)
        d.synchronize()
    finally:
        d.set_job_wait(0, False)
        if saved is None:
            os.environ.pop("DWT2_BATCH_SCHEDULE", None)
        else:
            os.environ["DWT2_BATCH_SCHEDULE"] = saved
        d.clear_plan_cache()
        _lib.load().dwt2_synchronize(None)


def test_batched_plan_cache_stays_bounded():
    d = D()
    d.clear_plan_cache()
    sizes = [(130, 70), (64, 99), (257, 33)]
    imgs = [torch.from_numpy(synth.image(w, h, 90 + i)).cuda() for i, (w, h) in enumerate(sizes)]
    refs = [d.fwd(im, 2) for im in imgs]
    # without a workspace: the binding keeps one per shape set, so 20 calls
    # share one plan
    for _ in range(20):
        for o, r in zip(d.fwd_batched(imgs, 2), refs):
            assert torch.equal(o, r)
    assert d.plan_cache_size() == 1
    # a new workspace on every call: the library evicts down to its bound
    nbytes = d.batched_workspace_size(imgs, 2)
    for _ in range(20):
        ws = torch.empty(nbytes + 4096, dtype=torch.uint8, device="cuda")
        for o, r in zip(d.fwd_batched(imgs, 2, workspace=ws), refs):
            assert torch.equal(o, r)
        assert d.plan_cache_size() <= 16
    d.clear_plan_cache()
    assert d.plan_cache_size() == 0
