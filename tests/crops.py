"""Windowed oracle checks for images too large for the full CPU oracle.

A coefficient of level k depends only on pixels within R_k = 2^(k+1) - 2 of
its footprint (each level's 5-tap support doubles), so the transform of a
crop whose origin and size are multiples of 2^levels reproduces every
coefficient whose footprint stays `margin` pixels away from the crop's
artificial edges.  Edges of the crop that coincide with image edges are real
and need no margin.  The same holds for the inverse and the adjoint, whose
outputs (pixels) depend on coefficients within the same radius.
"""
from __future__ import annotations

import numpy as np


def level_sizes(w, h, levels):
    out = [(w, h)]
    for _ in range(levels):
        w, h = (w + 1) // 2, (h + 1) // 2
        out.append((w, h))
    return out


def radius(levels):
    return (1 << (levels + 1)) - 2 + (1 << levels)


def band_slices(w, h, levels):
    """{(k, band): (row slice, col slice)} of the packed array, plus "LL"."""
    sz = level_sizes(w, h, levels)
    out = {}
    for k in range(1, levels + 1):
        (wp, hp), (wk, hk) = sz[k - 1], sz[k]
        out[(k, "HL")] = (slice(0, hk), slice(wk, wp))
        out[(k, "LH")] = (slice(hk, hp), slice(0, wk))
        out[(k, "HH")] = (slice(hk, hp), slice(wk, wp))
    wl, hl = sz[levels]
    out[(levels, "LL")] = (slice(0, hl), slice(0, wl))
    return out


def crop_packed(c, y0, x0, s, levels):
    """The packed coefficients of the crop [y0, y0+sh) x [x0, x0+sw) (s is
    (sh, sw)), taken from the packed coefficients c of the full image.  The
    origin must be a multiple of 2^levels; then every level's parity split of
    the crop matches the image's, including at the image's far edges."""
    h, w = c.shape
    sh, sw = s
    assert y0 % (1 << levels) == 0 and x0 % (1 << levels) == 0
    full = band_slices(w, h, levels)
    part = band_slices(sw, sh, levels)
    out = np.empty((sh, sw), dtype=c.dtype)
    for key, (rs, cs) in part.items():
        k = key[0]
        oy, ox = y0 >> k, x0 >> k
        frs, fcs = full[key]
        out[rs, cs] = c[frs.start + oy: frs.start + oy + (rs.stop - rs.start),
                        fcs.start + ox: fcs.start + ox + (cs.stop - cs.start)]
    return out


def valid_coeff_masks(h, w, y0, x0, s, levels, margin):
    """Per band of the crop: boolean mask of coefficients unaffected by the
    crop's artificial edges."""
    sh, sw = s
    part = band_slices(sw, sh, levels)
    masks = {}
    for key, (rs, cs) in part.items():
        k = key[0]
        n_r, n_c = rs.stop - rs.start, cs.stop - cs.start
        py = (np.arange(n_r) << k)           # footprint start, crop coordinates
        px = (np.arange(n_c) << k)
        ok_y = np.ones(n_r, bool)
        ok_x = np.ones(n_c, bool)
        if y0 > 0:
            ok_y &= py >= margin
        if y0 + sh < h:
            ok_y &= py + (1 << k) <= sh - margin
        if x0 > 0:
            ok_x &= px >= margin
        if x0 + sw < w:
            ok_x &= px + (1 << k) <= sw - margin
        masks[key] = np.outer(ok_y, ok_x)
    return masks


def compare_fwd_crop(gpu_packed, img, y0, x0, s, levels, oracle_fwd, margin=None):
    """Max |gpu - oracle| over the valid coefficients of one crop, and the
    number of coefficients compared."""
    h, w = img.shape
    margin = radius(levels) if margin is None else margin
    sh, sw = s
    ref = oracle_fwd(img[y0:y0 + sh, x0:x0 + sw], levels)
    got = crop_packed(gpu_packed, y0, x0, s, levels)
    part = band_slices(sw, sh, levels)
    worst, n = 0.0, 0
    for key, m in valid_coeff_masks(h, w, y0, x0, s, levels, margin).items():
        rs, cs = part[key]
        d = np.abs(got[rs, cs].astype(np.float64) - ref[rs, cs].astype(np.float64))[m]
        if d.size:
            worst = max(worst, float(d.max()))
            n += d.size
    return worst, n


def compare_pixels_crop(gpu_pixels, coeffs, y0, x0, s, levels, oracle_fn, margin=None):
    """Max |gpu - oracle| over the valid pixels of one crop, for a map from
    packed coefficients to pixels (inverse or adjoint)."""
    h, w = coeffs.shape
    margin = 2 * radius(levels) if margin is None else margin
    sh, sw = s
    ref = oracle_fn(crop_packed(coeffs, y0, x0, s, levels), levels)
    got = gpu_pixels[y0:y0 + sh, x0:x0 + sw]
    ys, xs = np.arange(sh), np.arange(sw)
    ok_y = np.ones(sh, bool)
    ok_x = np.ones(sw, bool)
    if y0 > 0:
        ok_y &= ys >= margin
    if y0 + sh < h:
        ok_y &= ys < sh - margin
    if x0 > 0:
        ok_x &= xs >= margin
    if x0 + sw < w:
        ok_x &= xs < sw - margin
    m = np.outer(ok_y, ok_x)
    d = np.abs(got.astype(np.float64) - ref.astype(np.float64))[m]
    return (float(d.max()) if d.size else 0.0), int(d.size)


def standard_crops(h, w, s, levels):
    """(y0, x0, (sh, sw)) for the four corner crops (two real edges each; the
    far ones run to the image edge) and a central one."""
    a = 1 << levels

    def al(v):
        return max(0, (v // a) * a)

    out = []
    for y0 in (0, al(h - s), al((h - s) // 2)):
        for x0 in (0, al(w - s), al((w - s) // 2)):
            if (y0 in (0, al(h - s))) != (x0 in (0, al(w - s))) and not (y0 == al((h - s) // 2) and x0 == al((w - s) // 2)):
                continue
            sh = h - y0 if y0 == al(h - s) else min(s, h - y0)
            sw = w - x0 if x0 == al(w - s) else min(s, w - x0)
            out.append((y0, x0, (sh, sw)))
    return out
