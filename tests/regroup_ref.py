"""CPU statement of the regrouped (non-separable) formulas that the HIP
kernels evaluate, used only by tests to show, on the CPU, that they reach the
separable oracle's result.

* Float forward: the spatial predict and spatial update matrices of §3,
  eq. (5), applied to the whole-sample symmetric extension of the level input.
* Integer forward: the four rounded separable steps of §2, eq. (3) composed
  inside one spatial predict (horizontal then vertical) and one spatial update.
* Float inverse: the matrix inverses of the two eq. (5) steps, update undone
  first, on the symmetric extension of the interleaved coefficients.
* Integer inverse: the composed integer steps undone in reverse order.
* Adjoint: the transposes of the eq. (5) steps (update transpose first), with
  the boundary weights that fold the symmetric extension back (no mirroring).

Laurent polynomials in (z_m, z_n) are dicts {(e_m, e_n): Fraction}; z_m is a
shift by one quadruple column (horizontal), z_n by one quadruple row.
"""
from fractions import Fraction as Fr

import numpy as np

# ----------------------------------------------------------- symbolic layer

def padd(p, q):
    r = dict(p)
    for k, v in q.items():
        r[k] = r.get(k, 0) + v
    return {k: v for k, v in r.items() if v != 0}


def pmul(p, q):
    r = {}
    for (a, b), c in p.items():
        for (d, e), f in q.items():
            r[(a + d, b + e)] = r.get((a + d, b + e), 0) + c * f
    return {k: v for k, v in r.items() if v != 0}


def pneg(p):
    return {k: -v for k, v in p.items()}


ONE, ZERO = {(0, 0): Fr(1)}, {}
P = {(0, 0): Fr(-1, 2), (1, 0): Fr(-1, 2)}      # horizontal predict
PS = {(0, 0): Fr(-1, 2), (0, 1): Fr(-1, 2)}     # P*: the same filter, vertical
U = {(0, 0): Fr(1, 4), (-1, 0): Fr(1, 4)}       # horizontal update
US = {(0, 0): Fr(1, 4), (0, -1): Fr(1, 4)}      # U*


def mmul(a, b):
    return [[_sum(pmul(a[i][k], b[k][j]) for k in range(4)) for j in range(4)] for i in range(4)]


def _sum(it):
    r = {}
    for p in it:
        r = padd(r, p)
    return r


def mat(rows):
    return [[ONE if e == 1 else ZERO if e == 0 else e for e in row] for row in rows]


# eq. (3), component order (LL, HL, LH, HH)
HP = mat([[1, 0, 0, 0], [P, 1, 0, 0], [0, 0, 1, 0], [0, 0, P, 1]])
VP = mat([[1, 0, 0, 0], [0, 1, 0, 0], [PS, 0, 1, 0], [0, PS, 0, 1]])
HU = mat([[1, U, 0, 0], [0, 1, 0, 0], [0, 0, 1, U], [0, 0, 0, 1]])
VU = mat([[1, 0, US, 0], [0, 1, 0, US], [0, 0, 1, 0], [0, 0, 0, 1]])
# eq. (5)
SP = mat([[1, 0, 0, 0], [P, 1, 0, 0], [PS, 0, 1, 0], [pmul(P, PS), PS, P, 1]])
SU = mat([[1, U, US, pmul(U, US)], [0, 1, 0, US], [0, 0, 1, U], [0, 0, 0, 1]])
# their inverses
SP_INV = mat([[1, 0, 0, 0], [pneg(P), 1, 0, 0], [pneg(PS), 0, 1, 0],
              [pmul(P, PS), pneg(PS), pneg(P), 1]])
SU_INV = mat([[1, pneg(U), pneg(US), pmul(U, US)], [0, 1, 0, pneg(US)],
              [0, 0, 1, pneg(U)], [0, 0, 0, 1]])
IDENT = mat([[1 if i == j else 0 for j in range(4)] for i in range(4)])

# ------------------------------------------------------------ numeric layer

MARGIN = 2  # quadruples of symmetric extension around the level input


def _quads(x):
    return [x[0::2, 0::2], x[0::2, 1::2], x[1::2, 0::2], x[1::2, 1::2]]


def _extend(x):
    h, w = x.shape
    m = 2 * MARGIN
    return np.pad(x, ((m, m + h % 2), (m, m + w % 2)), mode="reflect")


def _shift(c, em, en):
    # value at (i, j) becomes c[i + en, j + em]
    return np.roll(np.roll(c, -en, axis=0), -em, axis=1)


def apply_poly_matrix(m, comps):
    out = []
    for row in m:
        acc = np.zeros_like(comps[0], dtype=np.float64)
        for poly, c in zip(row, comps):
            for (em, en), coef in poly.items():
                acc = acc + float(coef) * _shift(c, em, en)
        out.append(acc)
    return out


def _crop(comps, h, w):
    ns_h, nd_h, ns_w, nd_w = (h + 1) // 2, h // 2, (w + 1) // 2, w // 2
    a, b, c, d = comps
    o = MARGIN
    return (a[o:o + ns_h, o:o + ns_w], b[o:o + ns_h, o:o + nd_w],
            c[o:o + nd_h, o:o + ns_w], d[o:o + nd_h, o:o + nd_w])


def _pack(ll, hl, lh, hh):
    return np.block([[ll, hl], [lh, hh]])


def _interleave(p):
    h, w = p.shape
    hk, wk = (h + 1) // 2, (w + 1) // 2
    r = np.empty_like(p)
    r[0::2, 0::2], r[0::2, 1::2] = p[:hk, :wk], p[:hk, wk:]
    r[1::2, 0::2], r[1::2, 1::2] = p[hk:, :wk], p[hk:, wk:]
    return r


def float_fwd_level(x):
    h, w = x.shape
    q = _quads(_extend(np.asarray(x, dtype=np.float64)))
    q = apply_poly_matrix(SP, q)     # spatial predict
    q = apply_poly_matrix(SU, q)     # spatial update
    return _pack(*_crop(q, h, w))


def float_inv_level(p):
    h, w = p.shape
    q = _quads(_extend(_interleave(np.asarray(p, dtype=np.float64))))
    q = apply_poly_matrix(SU_INV, q)
    q = apply_poly_matrix(SP_INV, q)
    a, b, c, d = (t[MARGIN:-MARGIN, MARGIN:-MARGIN] for t in q)
    out = np.empty((h, w))
    out[0::2, 0::2] = a[:(h + 1) // 2, :(w + 1) // 2]
    out[0::2, 1::2] = b[:(h + 1) // 2, :w // 2]
    out[1::2, 0::2] = c[:h // 2, :(w + 1) // 2]
    out[1::2, 1::2] = d[:h // 2, :w // 2]
    return out


def _R(c):   # right neighbour (j + 1)
    return _shift(c, 1, 0)


def _D(c):   # neighbour below (i + 1)
    return _shift(c, 0, 1)


def _L(c):
    return _shift(c, -1, 0)


def _Up(c):
    return _shift(c, 0, -1)


def int_fwd_level(x):
    """Eq. (3)'s four rounded steps composed inside the two spatial steps."""
    h, w = x.shape
    a, b, c, d = _quads(_extend(np.asarray(x, dtype=np.int64)))
    # spatial predict = VP o HP
    b1 = b - ((a + _R(a)) >> 1)
    d1 = d - ((c + _R(c)) >> 1)
    c1 = c - ((a + _D(a)) >> 1)
    d2 = d1 - ((b1 + _D(b1)) >> 1)
    # spatial update = VU o HU
    a1 = a + ((_L(b1) + b1 + 2) >> 2)
    c2 = c1 + ((_L(d2) + d2 + 2) >> 2)
    a2 = a1 + ((_Up(c2) + c2 + 2) >> 2)
    b2 = b1 + ((_Up(d2) + d2 + 2) >> 2)
    return _pack(*_crop([a2, b2, c2, d2], h, w))


def int_inv_level(p):
    h, w = p.shape
    a2, b2, c2, d2 = _quads(_extend(_interleave(np.asarray(p, dtype=np.int64))))
    a1 = a2 - ((_Up(c2) + c2 + 2) >> 2)
    b1 = b2 - ((_Up(d2) + d2 + 2) >> 2)
    a = a1 - ((_L(b1) + b1 + 2) >> 2)
    c1 = c2 - ((_L(d2) + d2 + 2) >> 2)
    c = c1 + ((a + _D(a)) >> 1)
    d1 = d2 + ((b1 + _D(b1)) >> 1)
    b = b1 + ((a + _R(a)) >> 1)
    d = d1 + ((c + _R(c)) >> 1)
    o = MARGIN
    out = np.empty((h, w), dtype=np.int64)
    out[0::2, 0::2] = a[o:o + (h + 1) // 2, o:o + (w + 1) // 2]
    out[0::2, 1::2] = b[o:o + (h + 1) // 2, o:o + w // 2]
    out[1::2, 0::2] = c[o:o + h // 2, o:o + (w + 1) // 2]
    out[1::2, 1::2] = d[o:o + h // 2, o:o + w // 2]
    return out


def ut_weights(n):
    """Boundary weights of U^T (per H index m) for an axis of length n."""
    ns, nd = (n + 1) // 2, n // 2
    alpha = np.ones(ns + 1)
    beta = np.ones(ns + 1)
    alpha[0] = 2.0
    for m in range(ns + 1):
        if m + 1 >= ns and n % 2 == 0:
            beta[m] = 0.0
        elif n % 2 == 1 and m == nd - 1:
            beta[m] = 2.0
        elif m >= nd:
            beta[m] = 0.0
    return alpha, beta


def pt_weights(n):
    """Boundary weights of P^T (per L index m) for an axis of length n."""
    ns, nd = (n + 1) // 2, n // 2
    gamma = np.ones(ns + 1)
    delta = np.ones(ns + 1)
    gamma[0] = 0.0
    for m in range(ns + 1):
        if n % 2 == 1 and m == nd:
            delta[m] = 0.0
        elif n % 2 == 0 and m == nd - 1:
            delta[m] = 2.0
        elif m >= ns:
            delta[m] = 0.0
    return gamma, delta


def float_adj_level(g):
    """Transpose of the level: M_U^T then M_P^T, weights instead of mirrors."""
    h, w = g.shape
    ns_h, ns_w = (h + 1) // 2, (w + 1) // 2
    x = _interleave(np.asarray(g, dtype=np.float64))
    full = np.zeros((2 * ns_h + 2, 2 * ns_w + 2))
    full[:h, :w] = x            # out-of-range samples are zero
    ga, gb, gc, gd = _quads(full)
    ah, bh = ut_weights(w)
    av, bv = ut_weights(h)
    gh, dh = pt_weights(w)
    gv, dv = pt_weights(h)
    AH, BH, GH, DH = (v[None, :] for v in (ah, bh, gh, dh))
    AV, BV, GV, DV = (v[:, None] for v in (av, bv, gv, dv))
    # step A = M_U^T (predict-shaped)
    gb1 = gb + 0.25 * (AH * ga + BH * _R(ga))
    gc1 = gc + 0.25 * (AV * ga + BV * _D(ga))
    gd1 = (gd + 0.0625 * (AV * AH * ga + AV * BH * _R(ga) + BV * AH * _D(ga) + BV * BH * _R(_D(ga)))
           + 0.25 * (AV * gb + BV * _D(gb)) + 0.25 * (AH * gc + BH * _R(gc)))
    # step B = M_P^T (update-shaped); the wrapped-around neighbour at index 0
    # always carries weight 0
    ga2 = (ga - 0.5 * (GH * _L(gb1) + DH * gb1) - 0.5 * (GV * _Up(gc1) + DV * gc1)
           + 0.25 * (GV * GH * _Up(_L(gd1)) + GV * DH * _Up(gd1) + DV * GH * _L(gd1) + DV * DH * gd1))
    gb2 = gb1 - 0.5 * (GV * _Up(gd1) + DV * gd1)
    gc2 = gc1 - 0.5 * (GH * _L(gd1) + DH * gd1)
    out = np.empty((h, w))
    out[0::2, 0::2] = ga2[:ns_h, :ns_w]
    out[0::2, 1::2] = gb2[:ns_h, :w // 2]
    out[1::2, 0::2] = gc2[:h // 2, :ns_w]
    out[1::2, 1::2] = gd1[:h // 2, :w // 2]
    return out
