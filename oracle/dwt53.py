"""CPU oracle for the multi-level 2-D CDF 5/3 discrete wavelet transform.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The product path (the
HIP library and its Python binding) never calls it and shares no code with it.

What it computes
----------------
Barina et al., "The Parallel Algorithm for the 2-D Discrete Wavelet
Transform", §2: a 2-D DWT is the tensor product of 1-D transforms; one level
splits the image into the quadruple (LL, HL, LH, HH).  The separable lifting
scheme of §2, eq. (3), applies the horizontal predict, vertical predict,
horizontal update and vertical update in that order (the right-most matrix of
eq. (3) acts first).  The non-separable scheme of §3, eq. (5), regroups those
four matrices pairwise and therefore reaches exactly the same result in exact
arithmetic; this oracle is the plain separable definition, in float64 (or in
exact Python-int-sized int64 for the reversible integer mode), so that it can
serve as the yardstick for any regrouping.

Readings of the paper (it prints neither filter taps nor boundary rules):

* CDF 5/3 lifting filters (§2, eq. (2) with K = 1; the wavelet is named in §1
  and §2): predict P(z) = -1/2 (1 + z), update U(z) = 1/4 (1 + z^-1).  No
  scaling step.
* The L/H split is by sample parity (§2): even 0-based indices are L, odd are
  H; a length-N axis has ceil(N/2) L and floor(N/2) H coefficients.
* Boundaries use whole-sample symmetric extension (x[-i] = x[i],
  x[N-1+i] = x[N-1-i]); every lifting neighbour index is folded with that rule.
* Reversible integer mode (JPEG 2000 style, not in the paper, which evaluates
  single precision only): predict d -= floor((l + r) / 2), update
  s += floor((l + r + 2) / 4), applied in the eq. (3) order.
* Multi-level: dyadic recursion on LL (Mallat's construction cited in §2);
  coefficients are stored Mallat-packed: LL_L in the top-left corner, and for
  level k, HL_k right of LL_k, LH_k below it, HH_k diagonal.
* The adjoint is the exact transpose of the forward linear map (float only).

Every 1-D lifting step is described by one table: for each target index t,
the two (folded) source indices l(t), r(t).  The forward, the inverse and the
transpose are all read off the same table, so a boundary mistake cannot hide
in only one of them.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "fold", "predict_table", "update_table", "level_sizes",
    "fwd_1d", "inv_1d",
    "fwd_level", "inv_level", "adj_level",
    "fwd", "inv", "adj", "subbands",
    "FLOAT", "INT",
]

FLOAT = "f64"
INT = "int"


# --------------------------------------------------------------------------
# Index tables (symmetric extension, parity split)
# --------------------------------------------------------------------------

def fold(p, n: int):
    """Whole-sample symmetric extension of index p onto [0, n) (n >= 2).

    The extended signal is even about 0 and about n-1, hence periodic with
    period 2(n-1); p is reduced modulo that period and reflected.
    """
    if n < 2:
        raise ValueError("axis length must be >= 2")
    period = 2 * (n - 1)
    q = np.mod(np.asarray(p, dtype=np.int64), period)
    return np.where(q >= n, period - q, q)


def predict_table(n: int):
    """Predict step of §2, eq. (2): every odd sample 2k+1 (k < floor(n/2)) is
    corrected from its even neighbours 2k and 2k+2 (folded)."""
    k = np.arange(n // 2, dtype=np.int64)
    return 2 * k + 1, fold(2 * k, n), fold(2 * k + 2, n)


def update_table(n: int):
    """Update step of §2, eq. (2): every even sample 2k (k < ceil(n/2)) is
    corrected from its odd neighbours 2k-1 and 2k+1 (folded)."""
    k = np.arange((n + 1) // 2, dtype=np.int64)
    return 2 * k, fold(2 * k - 1, n), fold(2 * k + 1, n)


def level_sizes(w: int, h: int, levels: int):
    """[(w_0, h_0), (w_1, h_1), ...]: each level keeps ceil(n/2) L samples."""
    sizes = [(w, h)]
    for _ in range(levels):
        w, h = (w + 1) // 2, (h + 1) // 2
        sizes.append((w, h))
    return sizes


# --------------------------------------------------------------------------
# One lifting step along one axis (in place on the interleaved array)
# --------------------------------------------------------------------------

def _take(x, idx, axis):
    return np.take(x, idx, axis=axis)


def _assign(x, idx, val, axis):
    sl = [slice(None)] * x.ndim
    sl[axis] = idx
    x[tuple(sl)] = val


def _predict(x, axis, mode, sign=+1):
    """d += P s (sign=+1) or d -= P s (sign=-1).

    Float: P s = -1/2 (l + r).  Integer: P s = -floor((l + r) / 2)."""
    t, l, r = predict_table(x.shape[axis])
    if len(t) == 0:
        return
    s = _take(x, l, axis) + _take(x, r, axis)
    if mode == INT:
        corr = -np.floor_divide(s, 2)
    else:
        corr = -0.5 * s
    _assign(x, t, _take(x, t, axis) + sign * corr, axis)


def _update(x, axis, mode, sign=+1):
    """s += U d (sign=+1) or s -= U d (sign=-1).

    Float: U d = 1/4 (l + r).  Integer: U d = floor((l + r + 2) / 4)."""
    t, l, r = update_table(x.shape[axis])
    s = _take(x, l, axis) + _take(x, r, axis)
    if mode == INT:
        corr = np.floor_divide(s + 2, 4)
    else:
        corr = 0.25 * s
    _assign(x, t, _take(x, t, axis) + sign * corr, axis)


def _predict_T(x, axis):
    """Transpose of the float predict step: every source gets -1/2 of the
    target's value (np.add.at accumulates folded duplicates)."""
    t, l, r = predict_table(x.shape[axis])
    if len(t) == 0:
        return
    xm = np.moveaxis(x, axis, 0)
    g = -0.5 * xm[t]
    np.add.at(xm, l, g)
    np.add.at(xm, r, g)


def _update_T(x, axis):
    """Transpose of the float update step (+1/4 to each source)."""
    t, l, r = update_table(x.shape[axis])
    xm = np.moveaxis(x, axis, 0)
    g = 0.25 * xm[t]
    np.add.at(xm, l, g)
    np.add.at(xm, r, g)


def _as_work(x, mode):
    if mode == INT:
        a = np.asarray(x)
        if not np.issubdtype(a.dtype, np.integer):
            raise TypeError("integer mode needs an integer array")
        return a.astype(np.int64, copy=True)
    if mode == FLOAT:
        return np.asarray(x, dtype=np.float64).copy()
    raise ValueError(f"unknown mode {mode!r}")


# --------------------------------------------------------------------------
# 1-D transform (used by the dense and hand-derived pins)
# --------------------------------------------------------------------------

def fwd_1d(x, mode=FLOAT):
    """One level of the 1-D lifting transform; returns (s, d)."""
    y = _as_work(x, mode)
    _predict(y, 0, mode)
    _update(y, 0, mode)
    return y[0::2].copy(), y[1::2].copy()


def inv_1d(s, d, mode=FLOAT):
    """Inverse of fwd_1d: undo the update, then undo the predict."""
    n = len(s) + len(d)
    y = np.empty(n, dtype=np.int64 if mode == INT else np.float64)
    y[0::2], y[1::2] = s, d
    _update(y, 0, mode, sign=-1)
    _predict(y, 0, mode, sign=-1)
    return y


# --------------------------------------------------------------------------
# One 2-D level (separable lifting, §2 eq. (3)), rows = axis 0, cols = axis 1
# --------------------------------------------------------------------------

def _deinterleave(r):
    return r[0::2, 0::2], r[0::2, 1::2], r[1::2, 0::2], r[1::2, 1::2]


def _pack(ll, hl, lh, hh):
    hk, wk = ll.shape
    h, w = hk + lh.shape[0], wk + hl.shape[1]
    out = np.empty((h, w), dtype=ll.dtype)
    out[:hk, :wk], out[:hk, wk:] = ll, hl
    out[hk:, :wk], out[hk:, wk:] = lh, hh
    return out


def _interleave(p, wk, hk):
    h, w = p.shape
    r = np.empty_like(p)
    r[0::2, 0::2], r[0::2, 1::2] = p[:hk, :wk], p[:hk, wk:]
    r[1::2, 0::2], r[1::2, 1::2] = p[hk:, :wk], p[hk:, wk:]
    return r


def fwd_level(x, mode=FLOAT):
    """One level: horizontal predict | vertical predict | horizontal update |
    vertical update (§2 eq. (3), right-most matrix first), then the
    quadruple (LL, HL, LH, HH) is stored Mallat-packed."""
    r = _as_work(x, mode)
    _predict(r, 1, mode)   # HP: HL += P LL, HH += P LH
    _predict(r, 0, mode)   # VP: LH += P* LL, HH += P* HL
    _update(r, 1, mode)    # HU: LL += U HL, LH += U HH
    _update(r, 0, mode)    # VU: LL += U* LH, HL += U* HH
    return _pack(*_deinterleave(r))


def inv_level(p, mode=FLOAT):
    """Exact inverse of fwd_level: the four steps undone in reverse order."""
    h, w = p.shape
    r = _interleave(_as_work(p, mode), (w + 1) // 2, (h + 1) // 2)
    _update(r, 0, mode, sign=-1)
    _update(r, 1, mode, sign=-1)
    _predict(r, 0, mode, sign=-1)
    _predict(r, 1, mode, sign=-1)
    return r


def adj_level(g):
    """Transpose of fwd_level (float): the transposed steps in reverse order,
    applied to the interleaved coefficient gradient."""
    h, w = g.shape
    r = _interleave(np.asarray(g, dtype=np.float64).copy(), (w + 1) // 2, (h + 1) // 2)
    _update_T(r, 0)
    _update_T(r, 1)
    _predict_T(r, 0)
    _predict_T(r, 1)
    return r


# --------------------------------------------------------------------------
# Multi-level (dyadic recursion on LL, Mallat packing)
# --------------------------------------------------------------------------

def _check(shape, levels):
    h, w = shape
    if levels < 1:
        raise ValueError("levels must be >= 1")
    for (wk, hk) in level_sizes(w, h, levels)[:-1]:
        if wk < 2 or hk < 2:
            raise ValueError("every level input must be at least 2x2")


def fwd(x, levels, mode=FLOAT):
    """Multi-level forward transform; returns the Mallat-packed array."""
    out = _as_work(x, mode)
    _check(out.shape, levels)
    h, w = out.shape
    for (wk, hk) in level_sizes(w, h, levels)[:-1]:
        out[:hk, :wk] = fwd_level(out[:hk, :wk], mode)
    return out


def inv(c, levels, mode=FLOAT):
    """Multi-level inverse: coarsest level first."""
    out = _as_work(c, mode)
    _check(out.shape, levels)
    h, w = out.shape
    for (wk, hk) in reversed(level_sizes(w, h, levels)[:-1]):
        out[:hk, :wk] = inv_level(out[:hk, :wk], mode)
    return out


def adj(g, levels):
    """Multi-level adjoint W^T (float): coarsest level first, the mirror of
    the forward's composition order."""
    out = _as_work(g, FLOAT)
    _check(out.shape, levels)
    h, w = out.shape
    for (wk, hk) in reversed(level_sizes(w, h, levels)[:-1]):
        out[:hk, :wk] = adj_level(out[:hk, :wk])
    return out


def subbands(c, levels):
    """Views of the packed result: {"LL": LL_L, (k, "HL"|"LH"|"HH"): band}."""
    h, w = c.shape
    sizes = level_sizes(w, h, levels)
    out = {}
    for k in range(1, levels + 1):
        (wp, hp), (wk, hk) = sizes[k - 1], sizes[k]
        out[(k, "HL")] = c[:hk, wk:wp]
        out[(k, "LH")] = c[hk:hp, :wk]
        out[(k, "HH")] = c[hk:hp, wk:wp]
    wL, hL = sizes[levels]
    out["LL"] = c[:hL, :wL]
    return out
