"""CPU statement of the non-separable CDF 9/7 formulas that the HIP kernels
evaluate, checked in float64 against the separable oracle.

Per §2 each lifting pair is treated in turn; per §3, eq. (5), a pair with
predict P = p (1 + z) and update U = u (1 + z^-1) becomes one spatial predict
and one spatial update on the quadruple (a, b, c, d):
    b' = b + p (a + aR)            c' = c + p (a + aD)
    d' = d + p (c + cR) + p (b + bD) + p^2 (a + aR + aD + aDR)
    HL = b' + u (d'U + d')         LH = c' + u (d'L + d')
    LL = a + u (b'L + b') + u (c'U + c') + u^2 (d'UL + d'U + d'L + d')
(R / D: next quadruple column / row, L / U: previous).  After both pairs
the quadrants are scaled: LL / K^2, HL and LH by 1, HH * K^2.  The inverse
undoes the update first; solved for the unknowns, each inverse step needs
only the step's inputs:
    b' = HL - u (d'U + d')         c' = LH - u (d'L + d')
    a  = LL - u (HL_L + HL + LH_U + LH) + u^2 (d'UL + d'U + d'L + d')
    b  = b' - p (a + aR)           c  = c' - p (a + aD)
    d  = d' - p (c' + c'R) - p (b' + b'D) + p^2 (a + aR + aD + aDR)
Both directions run on the whole-sample symmetric extension of their input
(of the pixels, or of the interleaved coefficients), which commutes with
lifting because it keeps every index's parity."""
import numpy as np
import pytest

from oracle import dwt97

M = 4  # quadruples of extension on each side


def _ext(x):
    h, w = x.shape
    return np.pad(x, ((2 * M, 2 * M + h % 2), (2 * M, 2 * M + w % 2)), mode="reflect")


def _sh(c, dj, di):
    """value at (i, j) becomes c[i + di, j + dj]"""
    return np.roll(np.roll(c, -di, axis=0), -dj, axis=1)


def sp_pred(p, a, b, c, d):
    aR, aD, aDR = _sh(a, 1, 0), _sh(a, 0, 1), _sh(a, 1, 1)
    return (b + p * (a + aR), c + p * (a + aD),
            d + p * (c + _sh(c, 1, 0)) + p * (b + _sh(b, 0, 1)) + p * p * (a + aR + aD + aDR))


def sp_upd(u, a, b, c, d):
    dU, dL, dUL = _sh(d, 0, -1), _sh(d, -1, 0), _sh(d, -1, -1)
    return (a + u * (_sh(b, -1, 0) + b) + u * (_sh(c, 0, -1) + c) + u * u * (dUL + dU + dL + d),
            b + u * (dU + d), c + u * (dL + d))


def sp_inv_upd(u, ll, hl, lh, d):
    dU, dL, dUL = _sh(d, 0, -1), _sh(d, -1, 0), _sh(d, -1, -1)
    return (ll - u * (_sh(hl, -1, 0) + hl + _sh(lh, 0, -1) + lh) + u * u * (dUL + dU + dL + d),
            hl - u * (dU + d), lh - u * (dL + d))


def sp_inv_pred(p, a, b1, c1, d1):
    aR, aD, aDR = _sh(a, 1, 0), _sh(a, 0, 1), _sh(a, 1, 1)
    return (b1 - p * (a + aR), c1 - p * (a + aD),
            d1 - p * (c1 + _sh(c1, 1, 0)) - p * (b1 + _sh(b1, 0, 1)) + p * p * (a + aR + aD + aDR))


def fwd_level_regrouped(x):
    h, w = x.shape
    X = _ext(x)
    a, b, c, d = X[0::2, 0::2], X[0::2, 1::2], X[1::2, 0::2], X[1::2, 1::2]
    for p, u in ((dwt97.ALPHA, dwt97.BETA), (dwt97.GAMMA, dwt97.DELTA)):
        b, c, d = sp_pred(p, a, b, c, d)
        a, b, c = sp_upd(u, a, b, c, d)
    K2 = dwt97.K * dwt97.K
    a, d = a / K2, d * K2
    ns_h, nd_h, ns_w, nd_w = (h + 1) // 2, h // 2, (w + 1) // 2, w // 2
    return np.block([[a[M:M + ns_h, M:M + ns_w], b[M:M + ns_h, M:M + nd_w]],
                     [c[M:M + nd_h, M:M + ns_w], d[M:M + nd_h, M:M + nd_w]]])


def inv_level_regrouped(cf):
    h, w = cf.shape
    ns_h, ns_w = (h + 1) // 2, (w + 1) // 2
    inter = np.empty_like(cf)
    inter[0::2, 0::2] = cf[:ns_h, :ns_w]
    inter[0::2, 1::2] = cf[:ns_h, ns_w:]
    inter[1::2, 0::2] = cf[ns_h:, :ns_w]
    inter[1::2, 1::2] = cf[ns_h:, ns_w:]
    X = _ext(inter)
    K2 = dwt97.K * dwt97.K
    a, b, c, d = X[0::2, 0::2] * K2, X[0::2, 1::2], X[1::2, 0::2], X[1::2, 1::2] / K2
    for p, u in ((dwt97.GAMMA, dwt97.DELTA), (dwt97.ALPHA, dwt97.BETA)):
        a, b, c = sp_inv_upd(u, a, b, c, d)
        b, c, d = sp_inv_pred(p, a, b, c, d)
    out = np.empty((2 * a.shape[0], 2 * a.shape[1]))
    out[0::2, 0::2], out[0::2, 1::2], out[1::2, 0::2], out[1::2, 1::2] = a, b, c, d
    return out[2 * M:2 * M + h, 2 * M:2 * M + w]


SHAPES = [(2, 2), (2, 3), (3, 2), (3, 3), (4, 5), (7, 6), (16, 16), (17, 31), (40, 9)]


@pytest.mark.parametrize("h,w", SHAPES)
def test_spatial_steps_equal_separable(h, w):
    x = np.random.default_rng(h * 100 + w).uniform(0, 255, (h, w))
    assert np.abs(fwd_level_regrouped(x) - dwt97.fwd_level(x)).max() < 1e-9


@pytest.mark.parametrize("h,w", SHAPES)
def test_inverse_spatial_steps(h, w):
    x = np.random.default_rng(h * 100 + w + 1).uniform(0, 255, (h, w))
    assert np.abs(inv_level_regrouped(dwt97.fwd_level(x)) - x).max() < 1e-9
