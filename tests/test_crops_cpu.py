"""The windowed (crop) comparison used at full sizes, validated on the CPU
against the full oracle, and shown to catch a planted error."""
import numpy as np

import oracle
from oracle import FLOAT, INT
import crops


def _fwd_f(x, levels):
    return oracle.fwd(x, levels, FLOAT)


def _fwd_i(x, levels):
    return oracle.fwd(x, levels, INT)


def test_crops_reproduce_full_forward():
    rng = np.random.default_rng(21)
    for h, w, levels, s in [(700, 611, 3, 256), (517, 900, 4, 320)]:
        img = rng.integers(0, 256, size=(h, w))
        full_f = oracle.fwd(img.astype(float), levels)
        full_i = oracle.fwd(img, levels, INT)
        for (y0, x0, sz) in crops.standard_crops(h, w, s, levels):
            worst, n = crops.compare_fwd_crop(full_f, img.astype(float), y0, x0, sz, levels, _fwd_f)
            assert n > 0 and worst < 1e-9, (y0, x0, sz, worst)
            worst, n = crops.compare_fwd_crop(full_i, img, y0, x0, sz, levels, _fwd_i)
            assert n > 0 and worst == 0, (y0, x0, sz)


def test_crops_reproduce_full_inverse_and_adjoint():
    rng = np.random.default_rng(22)
    h, w, levels, s = 640, 577, 3, 300
    c = rng.normal(size=(h, w)) * 30
    inv_full = oracle.inv(c, levels)
    adj_full = oracle.adj(c, levels)
    for (y0, x0, sz) in crops.standard_crops(h, w, s, levels):
        worst, n = crops.compare_pixels_crop(inv_full, c, y0, x0, sz, levels, lambda p, L: oracle.inv(p, L))
        assert n > 0 and worst < 1e-9
        worst, n = crops.compare_pixels_crop(adj_full, c, y0, x0, sz, levels, lambda p, L: oracle.adj(p, L))
        assert n > 0 and worst < 1e-9


def test_crops_catch_a_planted_error():
    rng = np.random.default_rng(23)
    img = rng.integers(0, 256, size=(512, 512)).astype(float)
    full = oracle.fwd(img, 3)
    bad = full.copy()
    bad[5, 300] += 1e-3          # a level-1 HL coefficient inside the top-right crop
    hit = 0
    for (y0, x0, sz) in crops.standard_crops(512, 512, 256, 3):
        worst, _ = crops.compare_fwd_crop(bad, img, y0, x0, sz, 3, _fwd_f)
        hit += worst > 1e-4
    assert hit >= 1
