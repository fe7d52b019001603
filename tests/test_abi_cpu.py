"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, sizes workspaces, and rejects every invalid argument before
any HIP call (all pointers below are never dereferenced)."""
import ctypes
import os
import re

import pytest

from paper_1708_07853_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE_A, FAKE_B, FAKE_WS = 0x10000, 0x20000, 0x30000


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1708_07853_amd import build
        build.build()
    return _lib.load()


def header_functions():
    text = open(os.path.join(ROOT, "include", "dwt2.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dwt2_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 9
    assert sorted(names) == sorted(_lib.EXPORTS)
    for n in names:
        assert getattr(lib, n) is not None


def test_missing_library_fails_loudly(tmp_path):
    saved = _lib._lib
    try:
        _lib._lib = None
        with pytest.raises(RuntimeError, match="not built"):
            _lib.load(str(tmp_path / "nope.so"))
    finally:
        _lib._lib = saved


def _sync_bytes(h, levels, batch):
    rows, hh = 0, h
    for _ in range(levels):
        hh = (hh + 1) // 2
        rows += hh
    return ((16 + 16 * batch * rows) * 4 + 255) // 256 * 256


def test_workspace_sizes(lib):
    # sync area: 16 words + one counter (on its own 64-byte line) per level
    # row, rounded up to 256 bytes; then one LL buffer per intermediate level
    # with the row pitch padded to 64 elements
    assert lib.dwt2_workspace_size(512, 512, 1, 1, 0) == _sync_bytes(512, 1, 1)
    assert lib.dwt2_workspace_size(512, 512, 1, 2, 0) == _sync_bytes(512, 2, 1) + 256 * 256 * 4
    assert lib.dwt2_workspace_size(512, 512, 1, 3, 0) == _sync_bytes(512, 3, 1) + (256 * 256 + 128 * 128) * 4
    assert lib.dwt2_workspace_size(512, 512, 3, 3, 1) == _sync_bytes(512, 3, 3) + 3 * (256 * 256 + 128 * 128) * 4
    assert lib.dwt2_workspace_size(101, 40, 1, 2, 0) == _sync_bytes(40, 2, 1) + 64 * 20 * 4   # 51 -> pitch 64
    assert _sync_bytes(512, 1, 1) == 16640
    assert lib.dwt2_workspace_size(4, 4, 1, 3, 0) == 0               # invalid: level 3 input 1 x 1
    assert lib.dwt2_workspace_size(4, 4, 1, 2, 5) == 0               # invalid mode


def test_separable_workspace_adds_one_work_array_per_image(lib):
    for (w, h, b, L, m) in [(512, 512, 1, 3, 0), (101, 40, 2, 2, 1), (4096, 64, 3, 1, 0)]:
        work = ((w + 63) // 64 * 64 * h * 4 + 255) // 256 * 256
        assert lib.dwt2_separable_workspace_size(w, h, b, L, m) == lib.dwt2_workspace_size(w, h, b, L, m) + b * work
    assert lib.dwt2_separable_workspace_size(4, 4, 1, 3, 0) == 0
    # the plain transform's workspace is too small for the separable baseline
    need = lib.dwt2_separable_workspace_size(64, 64, 1, 2, 0)
    assert call(lib, "dwt2_fwd_separable", wsb=need - 1) == -4


def call(lib, fn, **kw):
    a = dict(src=FAKE_A, ss=64, sb=0, dst=FAKE_B, ds=64, db=0, w=64, h=64, batch=1, levels=2,
             mode=0, boundary=0, ws=FAKE_WS, wsb=1 << 30, stream=None)
    a.update(kw)
    return getattr(lib, fn)(a["src"], a["ss"], a["sb"], a["dst"], a["ds"], a["db"], a["w"], a["h"],
                            a["batch"], a["levels"], a["mode"], a["boundary"], a["ws"], a["wsb"], a["stream"])


BAD = [
    (dict(src=None), -1), (dict(dst=None), -1), (dict(w=1), -1), (dict(h=1), -1),
    (dict(ss=63), -1), (dict(ds=10), -1), (dict(batch=0), -1), (dict(batch=2, sb=64 * 63), -1),
    (dict(boundary=1), -1), (dict(levels=0), -2), (dict(levels=7), -2), (dict(levels=99), -2),
    (dict(w=1 << 29, ss=1 << 29, ds=1 << 29), -2), (dict(mode=2), -3), (dict(dst=FAKE_A), -5),
    (dict(ws=None), -4), (dict(wsb=100), -4),
    (dict(src=FAKE_A + 2), -1), (dict(dst=FAKE_B + 6), -1), (dict(ws=FAKE_WS + 1), -1),
]


@pytest.mark.parametrize("fn", ["dwt2_fwd", "dwt2_inv", "dwt2_bwd", "dwt2_fwd_separable", "dwt2_fwd_cdf97",
                                "dwt2_inv_cdf97", "dwt2_fwd_cdf97_separable"])
@pytest.mark.parametrize("kw,code", BAD, ids=[str(b[0]) for b in BAD])
def test_validation_errors(lib, fn, kw, code):
    assert call(lib, fn, **kw) == code
    assert lib.dwt2_last_error().decode() != ""


def call_lds(lib, scheme=0, **kw):
    a = dict(src=FAKE_A, ss=64, sb=0, dst=FAKE_B, ds=64, db=0, w=64, h=64, batch=1, levels=2,
             mode=0, boundary=0, ws=FAKE_WS, wsb=1 << 30, stream=None)
    a.update(kw)
    return lib.dwt2_fwd_lds(a["src"], a["ss"], a["sb"], a["dst"], a["ds"], a["db"], a["w"], a["h"], a["batch"],
                            a["levels"], a["mode"], a["boundary"], scheme, a["ws"], a["wsb"], a["stream"])


@pytest.mark.parametrize("scheme", [0, 1, 2])
@pytest.mark.parametrize("kw,code", BAD, ids=[str(b[0]) for b in BAD])
def test_lds_validation_errors(lib, scheme, kw, code):
    assert call_lds(lib, scheme, **kw) == code
    assert lib.dwt2_last_error().decode() != ""


def test_lds_rejects_unknown_scheme(lib):
    for scheme in (-1, 3, 7):
        assert call_lds(lib, scheme) == -1
        assert "scheme" in lib.dwt2_last_error().decode()
    # the adapted scheme splits the filters, which floor rounding does not allow
    assert call_lds(lib, 2, mode=1) == -3
    assert "adapted" in lib.dwt2_last_error().decode()
    # the LDS kernels use the plain workspace
    need = lib.dwt2_workspace_size(64, 64, 1, 2, 0)
    assert call_lds(lib, 1, wsb=need - 1) == -4


@pytest.mark.parametrize("fn", ["dwt2_fwd_cdf97", "dwt2_inv_cdf97", "dwt2_fwd_cdf97_separable"])
def test_cdf97_rejects_integer_mode(lib, fn):
    assert call(lib, fn, mode=1) == -3
    assert "9/7" in lib.dwt2_last_error().decode()


def test_adjoint_rejects_integer_mode(lib):
    assert call(lib, "dwt2_bwd", mode=1) == -3
    assert "F32" in lib.dwt2_last_error().decode()


def test_status_strings(lib):
    for code in range(-7, 1):
        assert lib.dwt2_status_string(code)
    assert lib.dwt2_status_string(-100) == b"unknown status"


def _images(specs):
    arr = (_lib.Dwt2Image * len(specs))()
    for i, (w, h, s) in enumerate(specs):
        arr[i].src, arr[i].dst = FAKE_A + i * 0x1000000, FAKE_B + i * 0x1000000
        arr[i].src_stride = arr[i].dst_stride = s
        arr[i].width, arr[i].height = w, h
    return arr


@pytest.mark.parametrize("fn", ["dwt2_fwd_batched", "dwt2_inv_batched", "dwt2_bwd_batched"])
def test_batched_validation(lib, fn):
    call_b = getattr(lib, fn)
    ok = _images([(64, 64, 64), (33, 17, 40)])
    assert lib.dwt2_batched_workspace_size(ok, 2, 2, 0) > 0
    geo_only = _images([(64, 64, 64), (33, 17, 40)])       # the size query reads only the geometry
    for i in range(2):
        geo_only[i].src = geo_only[i].dst = None
    assert lib.dwt2_batched_workspace_size(geo_only, 2, 2, 0) == lib.dwt2_batched_workspace_size(ok, 2, 2, 0)
    assert lib.dwt2_batched_workspace_size(_images([(64, 64, 64), (3, 3, 3)]), 2, 3, 0) == 0
    misaligned = _images([(64, 64, 64), (33, 17, 40)])
    misaligned[1].dst += 2                                 # image 1: dst not 4-byte aligned
    assert call_b(misaligned, 2, 2, 0, 0, FAKE_WS, 1 << 30, None) == -1
    assert "image 1" in lib.dwt2_last_error().decode()
    bad = _images([(64, 64, 64), (33, 17, 20)])           # image 1: stride < width
    assert call_b(bad, 2, 2, 0, 0, FAKE_WS, 1 << 30, None) == -1
    assert "image 1" in lib.dwt2_last_error().decode()
    tiny = _images([(64, 64, 64), (3, 3, 3)])             # image 1: level 2 input 2 x 2 ok, level 3 not
    assert call_b(tiny, 2, 3, 0, 0, FAKE_WS, 1 << 30, None) == -2
    assert call_b(ok, 2, 2, 0, 0, FAKE_WS, 10, None) == -4
    assert call_b(ok, 0, 2, 0, 0, FAKE_WS, 1 << 30, None) == -1
    assert call_b(ok, 2, 2, 9, 0, FAKE_WS, 1 << 30, None) == -3
    assert call_b(ok, 2, 2, 0, 3, FAKE_WS, 1 << 30, None) == -1
    if fn == "dwt2_bwd_batched":
        assert call_b(ok, 2, 2, 1, 0, FAKE_WS, 1 << 30, None) == -3   # the adjoint is float only
        assert "F32" in lib.dwt2_last_error().decode()


def test_set_path_validation(lib):
    assert lib.dwt2_set_path(6) == -1
    assert lib.dwt2_set_path(-1) == -1
    for path in (1, 2, 3, 4, 5, 0):
        assert lib.dwt2_set_path(path) == 0


def test_set_probe_validation(lib):
    ev = 0x1000
    assert lib.dwt2_set_probe(3, 1, ev, ev) == -1
    assert lib.dwt2_set_probe(0, 0, ev, ev) == -1
    assert lib.dwt2_set_probe(0, 25, ev, ev) == -1
    assert lib.dwt2_set_probe(0, 1, None, ev) == -1
    assert lib.dwt2_set_probe(-1, 0, None, None) == 0


def test_set_tiling_validation(lib):
    assert lib.dwt2_set_tiling(-1, 0) == -1
    assert lib.dwt2_set_tiling(8, 3) == -1
    assert lib.dwt2_set_tiling(0, 0) == 0


# Byte ranges from the first to one past the last element: a 64 x 64 float
# image with stride 64 spans 16 KiB.
SPAN = 64 * 64 * 4
ALIAS = [
    dict(dst=FAKE_A + 4 * 64 * 10),                 # dst starts inside src
    dict(src=FAKE_B + SPAN - 4),                    # src's first element is dst's last
    dict(dst=FAKE_A - SPAN + 4),                    # dst's last element is src's first
    dict(ws=FAKE_A + 64),                           # workspace inside src
    dict(ws=FAKE_B - 256),                          # workspace runs into dst
    dict(batch=2, sb=64 * 64, db=64 * 64, dst=FAKE_A + 2 * SPAN - 4),  # second image of src meets dst
]


@pytest.mark.parametrize("fn", ["dwt2_fwd", "dwt2_inv", "dwt2_bwd", "dwt2_fwd_separable", "dwt2_fwd_cdf97"])
@pytest.mark.parametrize("kw", ALIAS, ids=[str(k) for k in ALIAS])
def test_overlapping_ranges_are_rejected(lib, fn, kw):
    assert call(lib, fn, **kw) == -5
    assert "overlap" in lib.dwt2_last_error().decode()


def test_adjacent_ranges_pass_validation(lib):
    # touching but not overlapping ranges pass every check; with no GPU the
    # call then fails at the first HIP call, not in validation
    st = call(lib, "dwt2_fwd", dst=FAKE_A + SPAN)
    assert st in (0, -6)
    assert "overlap" not in lib.dwt2_last_error().decode()


@pytest.mark.parametrize("fn", ["dwt2_fwd_batched", "dwt2_inv_batched", "dwt2_bwd_batched"])
def test_batched_overlapping_ranges_are_rejected(lib, fn):
    call_b = getattr(lib, fn)
    imgs = _images([(64, 64, 64), (64, 64, 64)])
    imgs[1].dst = imgs[0].dst + 4 * 64 * 63            # two outputs overlap
    assert call_b(imgs, 2, 2, 0, 0, FAKE_WS, 1 << 30, None) == -5
    assert "overlaps" in lib.dwt2_last_error().decode()
    imgs = _images([(64, 64, 64), (64, 64, 64)])
    imgs[1].src = imgs[0].dst + 4                      # an input overlaps another image's output
    assert call_b(imgs, 2, 2, 0, 0, FAKE_WS, 1 << 30, None) == -5
    assert "image 1's src" in lib.dwt2_last_error().decode()
    imgs = _images([(64, 64, 64), (64, 64, 64)])
    ws = imgs[1].dst - 64                              # the workspace runs into an output
    assert call_b(imgs, 2, 2, 0, 0, ws, 1 << 30, None) == -5
    assert "workspace" in lib.dwt2_last_error().decode()
    imgs = _images([(64, 64, 64), (64, 64, 64)])
    imgs[0].src = imgs[0].dst                          # an image's own input and output
    assert call_b(imgs, 2, 2, 0, 0, FAKE_WS, 1 << 30, None) == -5
    # inputs may overlap each other: they are only read
    imgs = _images([(64, 64, 64), (64, 64, 64)])
    imgs[1].src = imgs[0].src
    assert call_b(imgs, 2, 2, 0, 0, FAKE_WS, 1 << 30, None) in (0, -6)
    assert "overlap" not in lib.dwt2_last_error().decode()


def test_set_job_wait_validation(lib):
    assert lib.dwt2_set_job_wait(-1, 0) == -1
    assert lib.dwt2_set_job_wait(8, 2) == -1
    assert lib.dwt2_set_job_wait(8, 1) == 0
    assert lib.dwt2_set_job_wait(0, 0) == 0


def test_plan_cache_starts_empty_and_clears(lib):
    lib.dwt2_clear_plan_cache()
    assert lib.dwt2_plan_cache_size() == 0


def test_noalloc_validation(lib):
    # sizes beyond the 96 MiB scratch array are rejected before any HIP call
    st = lib.dwt2_fwd_noalloc(FAKE_A, 16384, 0, FAKE_B, 16384, 0, 16384, 16384, 1, 6, 0, 0, None)
    assert st == -4 and b"scratch" in lib.dwt2_last_error()
    assert lib.dwt2_fwd_noalloc(FAKE_A, 64, 0, FAKE_B, 64, 0, 1, 64, 1, 1, 0, 0, None) == -1
    assert lib.dwt2_fwd_noalloc(FAKE_A, 64, 0, FAKE_B, 64, 0, 64, 64, 1, 9, 0, 0, None) == -2
    assert lib.dwt2_fwd_noalloc(FAKE_A, 64, 0, FAKE_B, 64, 0, 64, 64, 1, 2, 7, 0, None) == -3


def call_tune(lib, d=0, **kw):
    a = dict(src=FAKE_A, ss=64, sb=0, dst=FAKE_B, ds=64, db=0, w=64, h=64, batch=1, levels=2,
             mode=0, boundary=0, ws=FAKE_WS, wsb=1 << 30, stream=None)
    a.update(kw)
    return lib.dwt2_tune(d, a["src"], a["ss"], a["sb"], a["dst"], a["ds"], a["db"], a["w"], a["h"], a["batch"],
                         a["levels"], a["mode"], a["boundary"], a["ws"], a["wsb"], a["stream"])


@pytest.mark.parametrize("d", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("kw,code", BAD, ids=[str(b[0]) for b in BAD])
def test_tune_validation_errors(lib, d, kw, code):
    """dwt2_tune validates as the call it tunes, before any HIP call."""
    assert call_tune(lib, d, **kw) == code
    assert lib.dwt2_last_error().decode() != ""


def test_tune_direction_and_table(lib):
    assert call_tune(lib, 5) == -1
    assert call_tune(lib, -1) == -1
    assert call_tune(lib, 2, mode=1) == -3      # the adjoint is float only
    assert call_tune(lib, 3, mode=1) == -3      # so is the CDF 9/7
    assert call_tune(lib, 4, mode=1) == -3
    assert lib.dwt2_tune_clear() == 0
    assert lib.dwt2_tune_entries() == 0
