"""Pins for the CPU oracle: every check here compares the oracle with
something other than itself (dense convolution matrices built with numpy's
own symmetric padding, hand-derived values, closed-form invariants, exact
inverses, pure-Python textbook loops, the dense transpose)."""
import itertools
import os

import numpy as np
import pytest

import oracle
from oracle import FLOAT, INT

HERE = os.path.dirname(os.path.abspath(__file__))

# CDF 5/3 analysis taps (convolution form of the lifting pair of §2, eq. (2),
# with P(z) = -1/2 (1 + z) and U(z) = 1/4 (1 + z^-1)).
LOW = {-2: -1 / 8, -1: 1 / 4, 0: 3 / 4, 1: 1 / 4, 2: -1 / 8}
HIGH = {-1: -1 / 2, 0: 1.0, 1: -1 / 2}


def dense_1d(n):
    """n x n analysis matrix, rows [s; d], from the convolution taps applied to
    the whole-sample symmetric extension produced by numpy.pad('reflect')."""
    pad = 4
    a = np.zeros((n, n))
    ns = (n + 1) // 2
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        xe = np.pad(e, pad, mode="reflect")
        for k in range(ns):
            a[k, j] = sum(t * xe[pad + 2 * k + o] for o, t in LOW.items())
        for k in range(n // 2):
            a[ns + k, j] = sum(t * xe[pad + 2 * k + 1 + o] for o, t in HIGH.items())
    return a


def dense_multilevel(x, levels):
    out = np.array(x, dtype=np.float64)
    h, w = out.shape
    for _ in range(levels):
        out[:h, :w] = dense_1d(h) @ out[:h, :w] @ dense_1d(w).T
        h, w = (h + 1) // 2, (w + 1) // 2
    return out


def test_fold_matches_numpy_reflect():
    for n in range(2, 12):
        ref = np.pad(np.arange(n), 3 * n, mode="reflect")
        p = np.arange(-3 * n, 4 * n)
        assert np.array_equal(oracle.fold(p, n), ref)


@pytest.mark.parametrize("n", range(2, 34))
def test_1d_lifting_equals_dense_convolution(n):
    a = dense_1d(n)
    ns = (n + 1) // 2
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        s, d = oracle.fwd_1d(e)
        np.testing.assert_allclose(np.concatenate([s, d]), a[:, j], atol=1e-12, rtol=0)
    assert len(s) == ns and len(d) == n // 2


def test_2d_level_equals_dense_tensor_product():
    rng = np.random.default_rng(7)
    for h, w in itertools.product(range(2, 14), range(2, 14)):
        x = rng.normal(size=(h, w))
        want = dense_1d(h) @ x @ dense_1d(w).T     # [s;d] x [s;d]^T = Mallat order
        np.testing.assert_allclose(oracle.fwd(x, 1), want, atol=1e-12, rtol=0)


@pytest.mark.parametrize("h,w,levels", [(16, 16, 3), (37, 29, 3), (64, 65, 5), (9, 130, 3), (2, 2, 1), (4, 3, 2)])
def test_multilevel_equals_recursive_dense(h, w, levels):
    x = np.random.default_rng(h * 100 + w).normal(size=(h, w)) * 50
    np.testing.assert_allclose(oracle.fwd(x, levels), dense_multilevel(x, levels), atol=1e-10, rtol=0)


def _read_golden():
    cases, cur = [], None
    with open(os.path.join(HERE, "golden", "cdf53_hand.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                if not line and cur:
                    cases.append(cur)
                    cur = None
                continue
            key, val = (t.strip() for t in line.split(":", 1))
            if key == "case":
                cur = {"case": val}
            else:
                cur[key] = val
    if cur:
        cases.append(cur)
    return cases


def _parse(v):
    return np.array([[float(t) for t in row.split(",")] for row in v.split(";")])


GOLDEN = _read_golden()


@pytest.mark.parametrize("case", GOLDEN, ids=[c["case"] for c in GOLDEN])
def test_hand_derived_golden(case):
    x = _parse(case["input"])
    if case["kind"] == "1d":
        x = x[0]
        s, d = oracle.fwd_1d(x, FLOAT)
        np.testing.assert_array_equal(s, _parse(case["f64_s"])[0])
        np.testing.assert_array_equal(d, _parse(case["f64_d"])[0])
        s, d = oracle.fwd_1d(x.astype(np.int64), INT)
        np.testing.assert_array_equal(s, _parse(case["int_s"])[0])
        np.testing.assert_array_equal(d, _parse(case["int_d"])[0])
    else:
        lv = int(case["levels"])
        np.testing.assert_array_equal(oracle.fwd(x, lv, FLOAT), _parse(case["f64"]))
        np.testing.assert_array_equal(oracle.fwd(x.astype(np.int64), lv, INT), _parse(case["int"]))
    assert len(GOLDEN) >= 7


@pytest.mark.parametrize("case", [c for c in GOLDEN if c["kind"] == "1d"], ids=lambda c: c["case"])
def test_inv_1d_rebuilds_hand_derived_inputs(case):
    """inv_1d applied to the hand-derived coefficients gives back the hand
    example's input, in both modes (an inverse that undid the steps in the
    wrong order, or with a wrong sign, would not)."""
    x = _parse(case["input"])[0]
    got = oracle.inv_1d(_parse(case["f64_s"])[0], _parse(case["f64_d"])[0], FLOAT)
    np.testing.assert_array_equal(got, x)
    got = oracle.inv_1d(_parse(case["int_s"])[0].astype(np.int64), _parse(case["int_d"])[0].astype(np.int64), INT)
    np.testing.assert_array_equal(got, x.astype(np.int64))


@pytest.mark.parametrize("n", range(2, 34))
def test_inv_1d_equals_dense_inverse(n):
    """inv_1d is the inverse of the dense convolution matrix built from the
    taps (not of the oracle's own forward)."""
    c = np.random.default_rng(500 + n).normal(size=n) * 30
    ns = (n + 1) // 2
    want = np.linalg.solve(dense_1d(n), c)
    np.testing.assert_allclose(oracle.inv_1d(c[:ns], c[ns:], FLOAT), want, atol=1e-9, rtol=0)


# ---------------------------------------------------------------- integer mode

def _int_predict_rows(x):
    """Textbook reversible 5/3 predict on every row, pure Python, with the
    boundary written out (x[N] := x[N-2])."""
    out = [list(r) for r in x]
    for r in out:
        n = len(r)
        for k in range(n // 2):
            left = r[2 * k]
            right = r[2 * k + 2] if 2 * k + 2 < n else r[n - 2]
            r[2 * k + 1] -= (left + right) // 2
    return out


def _int_update_rows(x):
    """Textbook reversible 5/3 update on every row (d[-1] := d[0],
    d[nd] := d[nd-1] for odd N), pure Python."""
    out = [list(r) for r in x]
    for r in out:
        n = len(r)
        nd = n // 2
        d = [r[2 * k + 1] for k in range(nd)]
        for k in range((n + 1) // 2):
            dl = d[k - 1] if k >= 1 else d[0]
            dr = d[k] if k < nd else d[nd - 1]
            r[2 * k] += (dl + dr + 2) // 4
    return out


def _T(x):
    return [list(c) for c in zip(*x)]


def _int_2d_textbook(x):
    x = [list(map(int, r)) for r in x]
    x = _int_predict_rows(x)              # HP
    x = _T(_int_predict_rows(_T(x)))      # VP
    x = _int_update_rows(x)               # HU
    x = _T(_int_update_rows(_T(x)))       # VU
    a = np.array(x, dtype=np.int64)
    return np.block([[a[0::2, 0::2], a[0::2, 1::2]], [a[1::2, 0::2], a[1::2, 1::2]]])


def test_int_1d_equals_textbook_floor_form():
    rng = np.random.default_rng(3)
    for n in range(2, 40):
        for _ in range(5):
            x = rng.integers(-300, 300, size=n)
            s, d = oracle.fwd_1d(x, INT)
            y = _int_update_rows(_int_predict_rows([list(map(int, x))]))[0]
            assert list(s) == y[0::2] and list(d) == y[1::2]


def test_int_2d_equals_textbook_eq3_order():
    rng = np.random.default_rng(4)
    for h, w in itertools.product(range(2, 12), range(2, 12)):
        x = rng.integers(0, 256, size=(h, w))
        assert np.array_equal(oracle.fwd(x, 1, INT), _int_2d_textbook(x))


def test_int_step_order_matters():
    """H and V steps commute in exact arithmetic (§2) but not with floors, so
    the eq. (3) order is part of the integer definition."""
    rng = np.random.default_rng(5)
    x = rng.integers(0, 256, size=(16, 17))
    ref = oracle.fwd(x, 1, INT)
    xx = [list(map(int, r)) for r in x]
    y = _int_update_rows(_int_predict_rows(xx))                # rows first
    y = _T(_int_update_rows(_int_predict_rows(_T(y))))         # then columns
    y = np.array(y)
    alt = np.block([[y[0::2, 0::2], y[0::2, 1::2]], [y[1::2, 0::2], y[1::2, 1::2]]])
    assert (alt != ref).sum() > 0


# ------------------------------------------------------- reconstruction & co.

SIZES = [(2, 2), (2, 3), (3, 2), (5, 7), (16, 16), (33, 65), (64, 63), (100, 37)]


@pytest.mark.parametrize("h,w", SIZES)
def test_perfect_reconstruction(h, w):
    rng = np.random.default_rng(h * w)
    x = rng.integers(0, 256, size=(h, w))
    lv = 1
    while ((w + (1 << lv) - 1) >> lv) >= 2 and ((h + (1 << lv) - 1) >> lv) >= 2 and lv < 6:
        lv += 1
    for levels in range(1, lv + 1):
        c = oracle.fwd(x, levels, INT)
        assert np.array_equal(oracle.inv(c, levels, INT), x)
        cf = oracle.fwd(x.astype(float), levels, FLOAT)
        assert np.abs(oracle.inv(cf, levels, FLOAT) - x).max() < 1e-12


@pytest.mark.parametrize("mode", [FLOAT, INT])
def test_constant_image(mode):
    x = np.full((37, 50), 173, dtype=np.int64)
    c = oracle.fwd(x if mode == INT else x.astype(float), 4, mode)
    b = oracle.subbands(c, 4)
    assert np.all(b["LL"] == 173)
    for k in range(1, 5):
        for band in ("HL", "LH", "HH"):
            assert np.all(b[(k, band)] == 0)


@pytest.mark.parametrize("mode", [FLOAT, INT])
def test_bilinear_ramp_odd_lengths_kills_every_h(mode):
    # 65 -> 33 -> 17 -> 9 -> 5 and 33 -> 17 -> 9 -> 5 -> 3: all odd
    h, w, levels = 33, 65, 4
    y, x = np.mgrid[0:h, 0:w]
    img = 3 * x + 5 * y + 2 * x * y + 7
    c = oracle.fwd(img if mode == INT else img.astype(float), levels, mode)
    b = oracle.subbands(c, levels)
    for k in range(1, levels + 1):
        for band in ("HL", "LH", "HH"):
            assert np.all(b[(k, band)] == 0), (k, band)
    assert np.array_equal(b["LL"], img[:: 1 << levels, :: 1 << levels])


def test_linear_ramp_even_length_only_last_column():
    h, w = 9, 64
    img = np.tile(np.arange(w, dtype=float) * 2.0, (h, 1))
    b = oracle.subbands(oracle.fwd(img, 1), 1)
    hl = b[(1, "HL")]
    assert np.all(hl[:, :-1] == 0) and np.all(hl[:, -1] != 0)
    assert np.all(b[(1, "LH")] == 0) and np.all(b[(1, "HH")] == 0)


# ------------------------------------------------------------------ adjoint

@pytest.mark.parametrize("h,w,levels", [(2, 2, 1), (3, 5, 2), (6, 7, 2), (9, 8, 3), (12, 13, 3), (5, 2, 1), (2, 9, 1)])
def test_adjoint_equals_dense_transpose(h, w, levels):
    n = h * w
    dense = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        dense[:, j] = oracle.fwd(e.reshape(h, w), levels).ravel()
    rng = np.random.default_rng(n)
    g = rng.normal(size=(h, w))
    np.testing.assert_allclose(oracle.adj(g, levels).ravel(), dense.T @ g.ravel(), atol=1e-12, rtol=0)
    np.testing.assert_allclose(dense, np.vstack([dense_multilevel(np.eye(n)[:, j].reshape(h, w), levels).ravel()
                                                 for j in range(n)]).T, atol=1e-12)


@pytest.mark.parametrize("h,w,levels", [(64, 64, 4), (101, 77, 5), (1000, 3, 1)])
def test_adjoint_dot_product(h, w, levels):
    rng = np.random.default_rng(h + w)
    x, y = rng.normal(size=(h, w)), rng.normal(size=(h, w))
    lhs = np.vdot(oracle.fwd(x, levels), y)
    rhs = np.vdot(x, oracle.adj(y, levels))
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))


def test_level_checks():
    with pytest.raises(ValueError):
        oracle.fwd(np.zeros((4, 4)), 3)   # level-3 input would be 1x1
    with pytest.raises(ValueError):
        oracle.fwd(np.zeros((4, 4)), 0)
    with pytest.raises(TypeError):
        oracle.fwd(np.zeros((4, 4)), 1, INT)
