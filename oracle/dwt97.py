"""CPU oracle for the multi-level 2-D CDF 9/7 discrete wavelet transform.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The product path (the
HIP library and its Python binding) never calls it and shares no code with it.

What it computes
----------------
Barina et al., §2, eq. (2): the polyphase matrix of a wavelet factors into
pairs of lifting steps, a predict followed by an update, and for several
pairs the 2-D scheme treats each pair in turn.  The CDF 9/7 wavelet
(Cohen-Daubechies-Feauveau, cited in §2) has two pairs and a scaling.  The
paper prints no 9/7 coefficients.  This module uses the lifting factorisation
by Daubechies and Sweldens (also cited in §2), normalised as JPEG 2000's
irreversible transform is: the lowpass has gain 1 at DC and the highpass has
gain 2 at Nyquist.  With s[n] = x[2n] and d[n] = x[2n+1] (even samples
are L, as for the 5/3):

    predict 1   d[n] += ALPHA * (s[n] + s[n+1])
    update 1    s[n] += BETA  * (d[n-1] + d[n])
    predict 2   d[n] += GAMMA * (s[n] + s[n+1])
    update 2    s[n] += DELTA * (d[n-1] + d[n])
    scaling     s[n] /= K,  d[n] *= K

* Boundaries: whole-sample symmetric extension, with every lifting neighbour
  index folded.
* Level recursion and packing: dyadic recursion on LL, Mallat packing.
* 2-D: the tensor product of 1-D transforms (§2), so one level is the full
  1-D transform along rows, then along columns.  In exact arithmetic the
  horizontal and vertical steps may be interleaved in any order (§2), so this
  is also the result of the per-pair spatial steps of eq. (5).

Float64 only: the paper evaluates single precision, and the 9/7 has no
reversible integer form here.
"""
from __future__ import annotations

import numpy as np

__all__ = ["ALPHA", "BETA", "GAMMA", "DELTA", "K", "fold", "fwd_1d", "inv_1d",
           "fwd_level", "inv_level", "fwd", "inv", "level_sizes"]

ALPHA = -1.586134342059924
BETA = -0.052980118572961
GAMMA = 0.882911075530934
DELTA = 0.443506852043971
K = 1.230174104914001

# (coefficient, parity of the samples it changes), in forward order
_STEPS = ((ALPHA, 1), (BETA, 0), (GAMMA, 1), (DELTA, 0))


def fold(i, n):
    """Whole-sample symmetric extension of index i onto [0, n), n >= 2."""
    i = np.asarray(i)
    m = 2 * (n - 1)
    i = np.mod(i, m)
    return np.where(i >= n, m - i, i)


def _targets(n, parity):
    t = np.arange(parity, n, 2)
    return t, fold(t - 1, n), fold(t + 1, n)


def fwd_1d(x, axis=0):
    """One 1-D level along `axis`: the four lifting steps and the scaling;
    returns [s; d] (ceil(N/2) lowpass then floor(N/2) highpass) along axis."""
    y = np.moveaxis(np.array(x, dtype=np.float64, copy=True), axis, 0)
    n = y.shape[0]
    if n < 2:
        raise ValueError("length must be >= 2")
    for coef, parity in _STEPS:
        t, l, r = _targets(n, parity)
        # the neighbours have the other parity, so this step reads only
        # values it does not change
        y[t] += coef * (y[l] + y[r])
    s = y[0::2] / K
    d = y[1::2] * K
    return np.moveaxis(np.concatenate([s, d], axis=0), 0, axis)


def inv_1d(c, axis=0):
    """Inverse of fwd_1d: undo the scaling, then the steps in reverse order."""
    c = np.moveaxis(np.array(c, dtype=np.float64, copy=True), axis, 0)
    n = c.shape[0]
    ns = (n + 1) // 2
    y = np.empty_like(c)
    y[0::2] = c[:ns] * K
    y[1::2] = c[ns:] / K
    for coef, parity in reversed(_STEPS):
        t, l, r = _targets(n, parity)
        y[t] -= coef * (y[l] + y[r])
    return np.moveaxis(y, 0, axis)


def fwd_level(x):
    """One 2-D level: rows, then columns.  [s | d] along rows followed by
    [s; d] along columns is the Mallat quadrant layout (LL, HL / LH, HH)."""
    return fwd_1d(fwd_1d(x, axis=1), axis=0)


def inv_level(c):
    return inv_1d(inv_1d(c, axis=0), axis=1)


def level_sizes(w, h, levels):
    """Level input sizes (w_{k-1}, h_{k-1}) for k = 1..levels."""
    out = []
    for _ in range(levels):
        out.append((w, h))
        w, h = (w + 1) // 2, (h + 1) // 2
    return out


def _check(w, h, levels):
    if levels < 1:
        raise ValueError("levels must be >= 1")
    for (lw, lh) in level_sizes(w, h, levels):
        if lw < 2 or lh < 2:
            raise ValueError("every level input must be at least 2 x 2")


def fwd(x, levels):
    """Multi-level forward transform of a 2-D array; Mallat-packed result."""
    out = np.array(x, dtype=np.float64, copy=True)
    h, w = out.shape
    _check(w, h, levels)
    for (lw, lh) in level_sizes(w, h, levels):
        out[:lh, :lw] = fwd_level(out[:lh, :lw])
    return out


def inv(c, levels):
    """Inverse of fwd: levels coarsest first."""
    out = np.array(c, dtype=np.float64, copy=True)
    h, w = out.shape
    _check(w, h, levels)
    for (lw, lh) in reversed(level_sizes(w, h, levels)):
        out[:lh, :lw] = inv_level(out[:lh, :lw])
    return out
