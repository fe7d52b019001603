"""The launch planner of the per-level path (host logic, no GPU): which
levels each launch of a plain call covers, per chaining path."""
import os

import pytest

from paper_1708_07853_amd import _lib, api


@pytest.fixture(scope="module", autouse=True)
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1708_07853_amd import build
        build.build()
    yield _lib.load()
    api.set_path("levels")


def _levels(w, h, L):
    out = []
    for _ in range(L):
        out.append((w, h))
        w, h = (w + 1) // 2, (h + 1) // 2
    return out  # level-k inputs, k = 1..L


SHAPES = [(8192, 8192, 1, 6), (16384, 16384, 1, 6), (1024, 1024, 96, 4), (512, 512, 96, 4), (512, 512, 1, 6),
          (2048, 2048, 1, 6), (600, 333, 1, 5), (9, 9, 1, 3), (37, 250, 2, 6), (5, 7, 1, 2), (2, 2, 1, 1)]


@pytest.mark.parametrize("path", ["levels", "levels-only", "pairs", "pairs-only", "no-pairs"])
@pytest.mark.parametrize("w,h,b,L", SHAPES)
@pytest.mark.parametrize("d", ["fwd", "inv", "bwd"])
def test_launches_cover_every_level_once(path, w, h, b, L, d):
    api.set_path(path)
    plan = api.launch_levels(w, h, L, d, batch=b)
    order = plan if d == "fwd" else plan[::-1]  # the inverses run coarsest first
    k = 1
    ins = _levels(w, h, L)
    for first, last in order:
        assert first == k and last >= first
        n = last - first + 1
        if n == 2 and last < L:
            # a pair (a two-level fused tail ends at level L): level-k input of at least 8 x 8
            assert min(ins[first - 1]) >= 8
        if path in ("levels-only",):
            assert n == 1
        if path == "no-pairs" and last < L:
            assert n == 1
        k = last + 1
    assert k == L + 1


def test_default_forward_pairs_follow_strip_fill():
    """A forward pair needs its strips (112 quadruple columns each) at least
    60 % filled, or a small level (at most 2 x 1024^2 input pixels over the
    batch); the inverse and adjoint pair wherever a pair applies.  The fused
    tail stays only where it saves a launch."""
    api.set_path("levels")
    assert api.launch_levels(8192, 8192, 6, "fwd") == [(1, 2), (3, 4), (5, 6)]
    assert api.launch_levels(8192, 8192, 6, "inv") == [(5, 6), (3, 4), (1, 2)]
    assert api.launch_levels(8192, 8192, 6, "bwd") == [(5, 6), (3, 4), (1, 2)]
    assert api.launch_levels(16384, 16384, 6, "fwd") == [(1, 2), (3, 4), (5, 6)]
    # 256^2 at five levels: the tail of levels 3-5 replaces two launches
    assert api.launch_levels(256, 256, 5, "fwd") == [(1, 2), (3, 5)]
    # 8 x 2048^2: level 3 (512 wide, 2 Mpx, 76 %) pairs too, and the tail would
    # save no launch
    assert api.launch_levels(2048, 2048, 6, "fwd", batch=8) == [(1, 2), (3, 4), (5, 6)]
    # 512 wide: 256 quadruple columns in 3 strips (336, 76 %) -> pair; level 3
    # (128 wide): 64 columns in one strip (57 %), but 1.6 Mpx -> pair
    assert api.launch_levels(512, 512, 4, "fwd", batch=96) == [(1, 2), (3, 4)]
    # 300 wide: 150 columns in 2 strips (67 %) -> pair
    assert api.launch_levels(300, 300, 3, "fwd", batch=96) == [(1, 2), (3, 3)]
    # 256 wide: 128 columns in 2 strips (57 %, 6.3 Mpx) -> single; level 2
    # (1.6 Mpx) -> pair
    assert api.launch_levels(256, 256, 3, "fwd", batch=96) == [(1, 1), (2, 3)]
    assert api.launch_levels(512, 512, 4, "inv", batch=96) == [(3, 4), (1, 2)]
    # 1024 wide: 512 in 5 strips (560) -> pair; level 3 (256 wide): 128 in 2 strips (224) -> single
    assert api.launch_levels(1024, 1024, 4, "fwd", batch=96) == [(1, 2), (3, 3), (4, 4)]
    api.set_path("pairs")
    assert api.launch_levels(512, 512, 4, "fwd", batch=96) == [(1, 2), (3, 4)]
    api.set_path("levels")


def test_persistent_is_one_launch():
    api.set_path("persistent")
    assert api.launch_levels(8192, 8192, 6, "fwd") == [(1, 6)]
    api.set_path("levels")
