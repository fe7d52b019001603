"""Pins of the CDF 9/7 oracle to facts outside it: the published analysis
filter taps (tests/golden/cdf97_analysis_taps.txt), the wavelet's vanishing
moments, convolution with those taps on an explicitly mirrored signal (which
fixes the boundary handling), perfect reconstruction, the tensor-product
structure of the 2-D level (§2), and constant images.  A last test plants
mistakes in the oracle's constants and checks that the pins catch them."""
import os

import numpy as np
import pytest

from oracle import dwt97

HERE = os.path.dirname(os.path.abspath(__file__))


def _taps():
    vals = {}
    with open(os.path.join(HERE, "golden", "cdf97_analysis_taps.txt")) as f:
        for line in f:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            vals[k.strip()] = np.array([float(t) for t in v.split(",")])
    low, high = vals["low"], vals["high"]
    return np.concatenate([low[:0:-1], low]), np.concatenate([high[:0:-1], high])


LOW, HIGH = _taps()   # full symmetric filters, lengths 9 and 7


def _conv_reference(x):
    """s and d by direct convolution with the published taps on the
    whole-sample symmetric extension built by numpy's reflect padding."""
    n = len(x)
    pad = 8
    xt = np.pad(np.asarray(x, dtype=np.float64), pad, mode="reflect")
    s = [sum(LOW[k + 4] * xt[pad + 2 * i + k] for k in range(-4, 5)) for i in range((n + 1) // 2)]
    d = [sum(HIGH[k + 3] * xt[pad + 2 * i + 1 + k] for k in range(-3, 4)) for i in range(n // 2)]
    return np.array(s + d)


def _impulse_rows(n=64):
    """Rows: responses of s[16] and d[16] to unit impulses at x[0..n)."""
    eye = np.eye(n)
    out = np.array([dwt97.fwd_1d(eye[k]) for k in range(n)])   # out[k] = transform of impulse k
    ns = (n + 1) // 2
    return out[:, 16], out[:, ns + 16]


def test_impulse_responses_are_the_published_analysis_filters():
    s16, d16 = _impulse_rows()
    assert np.allclose(s16[32 - 4:32 + 5], LOW, atol=1e-9, rtol=0)
    assert np.allclose(d16[33 - 3:33 + 4], HIGH, atol=1e-9, rtol=0)
    # and nothing outside the supports
    assert np.abs(np.delete(s16, range(28, 37))).max() < 1e-12
    assert np.abs(np.delete(d16, range(30, 37))).max() < 1e-12


def test_filter_gains():
    assert abs(LOW.sum() - 1) < 1e-9                                    # DC gain 1
    assert abs(HIGH.sum()) < 1e-9                                       # highpass rejects DC
    assert abs(sum(h * (-1) ** (k - 3) for k, h in enumerate(HIGH)) - 2) < 1e-9   # gain 2 at Nyquist


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
def test_highpass_has_four_vanishing_moments(degree):
    n = 101
    t = np.arange(n, dtype=np.float64) / n
    x = (3 * t - 1) ** degree * 50
    c = dwt97.fwd_1d(x)
    d = c[(n + 1) // 2:]
    assert np.abs(d[3:-3]).max() < 1e-9                                # interior, away from the edges
    if degree == 0:
        assert np.allclose(c[:(n + 1) // 2], 50.0, atol=1e-9)        # lowpass keeps constants


def test_fifth_moment_does_not_vanish():
    n = 101
    t = np.arange(n, dtype=np.float64) / n
    d = dwt97.fwd_1d((3 * t - 1) ** 4 * 50)[(n + 1) // 2:]
    assert np.abs(d[3:-3]).max() > 1e-6


@pytest.mark.parametrize("n", list(range(2, 41)))
def test_boundaries_equal_convolution_on_the_mirrored_signal(n):
    x = np.random.default_rng(970 + n).uniform(0, 255, n)
    assert np.allclose(dwt97.fwd_1d(x), _conv_reference(x), atol=1e-9, rtol=0)


@pytest.mark.parametrize("h,w,levels", [(2, 2, 1), (3, 5, 1), (17, 2, 1), (64, 64, 5), (65, 33, 4),
                                        (130, 257, 6), (9, 300, 3)])
def test_perfect_reconstruction(h, w, levels):
    x = np.random.default_rng(h * 1000 + w).uniform(0, 255, (h, w))
    c = dwt97.fwd(x, levels)
    assert np.abs(dwt97.inv(c, levels) - x).max() < 1e-9


def _dense97(n):
    """n x n analysis matrix, rows [s; d], from the published taps applied to
    the reflect-padded unit impulses (no lifting involved)."""
    eye = np.eye(n)
    return np.array([_conv_reference(eye[j]) for j in range(n)]).T


def _dense97_multilevel(x, levels):
    """Dyadic recursion on the LL corner (Mallat), each level the tensor
    product A_h X A_w^T of the dense matrices: the rows [s; d] of A put the
    quadrants in Mallat order."""
    out = np.array(x, dtype=np.float64)
    h, w = out.shape
    for _ in range(levels):
        out[:h, :w] = _dense97(h) @ out[:h, :w] @ _dense97(w).T
        h, w = (h + 1) // 2, (w + 1) // 2
    return out


@pytest.mark.parametrize("h,w,levels", [(16, 16, 3), (37, 29, 3), (64, 65, 5), (9, 130, 3), (2, 2, 1),
                                        (5, 3, 2), (130, 40, 6)])
def test_multilevel_equals_recursive_dense(h, w, levels):
    """The oracle's multi-level forward equals the recursive dense form built
    from the published taps, at every level; its inverse undoes it."""
    x = np.random.default_rng(h * 31 + w).uniform(0, 255, (h, w))
    want = _dense97_multilevel(x, levels)
    assert np.allclose(dwt97.fwd(x, levels), want, atol=1e-8, rtol=0)
    assert np.allclose(dwt97.inv(want, levels), x, atol=1e-8, rtol=0)


@pytest.mark.parametrize("h,w", [(2, 2), (7, 12), (33, 65), (64, 31)])
def test_2d_level_is_the_tensor_product(h, w):
    rng = np.random.default_rng(h + 7 * w)
    u, v = rng.uniform(-1, 1, h), rng.uniform(-1, 1, w)
    got = dwt97.fwd_level(np.outer(u, v))
    assert np.allclose(got, np.outer(_conv_reference(u), _conv_reference(v)), atol=1e-9, rtol=0)


@pytest.mark.parametrize("h,w,levels", [(64, 64, 6), (37, 90, 4), (5, 3, 2)])
def test_constant_image(h, w, levels):
    c = dwt97.fwd(np.full((h, w), 77.0), levels)
    lw, lh = w, h
    for _ in range(levels):
        lw, lh = (lw + 1) // 2, (lh + 1) // 2
    assert np.allclose(c[:lh, :lw], 77.0, atol=1e-9)
    mask = np.ones_like(c, dtype=bool)
    mask[:lh, :lw] = False
    assert np.abs(c[mask]).max() < 1e-9


@pytest.mark.parametrize("mistake", ["swap_gamma_delta", "alpha_sign", "scale_inverted", "drop_delta"])
def test_planted_mistakes_are_caught(monkeypatch, mistake):
    a, b, g, d = dwt97.ALPHA, dwt97.BETA, dwt97.GAMMA, dwt97.DELTA
    steps = {"swap_gamma_delta": ((a, 1), (b, 0), (d, 1), (g, 0)),
             "alpha_sign": ((-a, 1), (b, 0), (g, 1), (d, 0)),
             "scale_inverted": ((a, 1), (b, 0), (g, 1), (d, 0)),
             "drop_delta": ((a, 1), (b, 0), (g, 1))}[mistake]
    monkeypatch.setattr(dwt97, "_STEPS", steps)
    if mistake == "scale_inverted":
        monkeypatch.setattr(dwt97, "K", 1 / dwt97.K)
    s16, d16 = _impulse_rows()
    ok = (np.allclose(s16[28:37], LOW, atol=1e-9, rtol=0) and np.allclose(d16[30:37], HIGH, atol=1e-9, rtol=0))
    assert not ok
