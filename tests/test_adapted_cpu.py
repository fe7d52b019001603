"""The adapted non-separable scheme (§3), written out in float64 for the CDF
5/3 and checked against the separable oracle.

§3 splits each lifting filter into its constant term and the rest, P = P0 + P1
and U = U0 + U1.  The constant terms touch only a quadruple's own samples, so
they run separably with no exchange; only P1 and U1 read neighbours.  For the
5/3, P0 = -1/2, P1 = -1/2 z, U0 = 1/4, U1 = 1/4 z^-1.  The horizontal and
vertical constant steps commute with the other parts (polynomials commute), so
one level is:
  load:     b += P0 a,  d += P0 c   (HP0);   c += P0 a,  d += P0 b   (VP0)
  step 1:   b' = b + P1 a:  b - 1/2 aR;       c' = c - 1/2 aD
            d' = d - 1/2 cR - 1/2 bD + 1/4 aDR     (neighbours after P0)
            a += 1/4 b',  c' += 1/4 d'   (HU0);   a += 1/4 c',  b' += 1/4 d'  (VU0)
  step 2:   LL = a + 1/4 bL + 1/4 cU + 1/16 dUL    (neighbours after U0)
            HL = b' + 1/4 dU,   LH = c' + 1/4 dL,   HH = d'
(R / D: next quadruple column / row; L / U: previous).  The HIP kernel for
this scheme evaluates these expressions; this test shows they reach the
oracle's transform."""
import numpy as np
import pytest

import oracle

M = 2


def _sh(c, dj, di):
    return np.roll(np.roll(c, -di, axis=0), -dj, axis=1)


def adapted_level(x):
    h, w = x.shape
    X = np.pad(x.astype(np.float64), ((2 * M, 2 * M + h % 2), (2 * M, 2 * M + w % 2)), mode="reflect")
    a, b, c, d = X[0::2, 0::2], X[0::2, 1::2], X[1::2, 0::2], X[1::2, 1::2]
    # constant predict parts, own quadruple only
    b = b - 0.5 * a
    d = d - 0.5 * c
    c = c - 0.5 * a
    d = d - 0.5 * b
    # step 1: the rest of the predict, then the constant update parts
    bp = b - 0.5 * _sh(a, 1, 0)
    cp = c - 0.5 * _sh(a, 0, 1)
    dp = d - 0.5 * _sh(c, 1, 0) - 0.5 * _sh(b, 0, 1) + 0.25 * _sh(a, 1, 1)
    a = a + 0.25 * bp
    cp = cp + 0.25 * dp
    a = a + 0.25 * cp
    bp = bp + 0.25 * dp
    # step 2: the rest of the update
    ll = a + 0.25 * _sh(bp, -1, 0) + 0.25 * _sh(cp, 0, -1) + 0.0625 * _sh(dp, -1, -1)
    hl = bp + 0.25 * _sh(dp, 0, -1)
    lh = cp + 0.25 * _sh(dp, -1, 0)
    ns_h, nd_h, ns_w, nd_w = (h + 1) // 2, h // 2, (w + 1) // 2, w // 2
    return np.block([[ll[M:M + ns_h, M:M + ns_w], hl[M:M + ns_h, M:M + nd_w]],
                     [lh[M:M + nd_h, M:M + ns_w], dp[M:M + nd_h, M:M + nd_w]]])


@pytest.mark.parametrize("h,w", [(2, 2), (2, 3), (3, 3), (4, 5), (7, 6), (16, 16), (17, 31), (40, 9)])
def test_adapted_scheme_equals_separable(h, w):
    x = np.random.default_rng(h * 31 + w).uniform(0, 255, (h, w))
    assert np.abs(adapted_level(x) - oracle.fwd(x, 1)).max() < 1e-10
