"""The regrouped formulas the GPU kernels use, checked on the CPU against the
separable oracle (and the paper's algebra checked symbolically)."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import FLOAT, INT
import regroup_ref as R


def test_eq5_is_the_pairwise_product_of_eq3():
    """§3 eq. (5): spatial predict = VP.HP, spatial update = VU.HU; so the
    product of the eq. (5) pair equals the product of the four eq. (3)
    matrices."""
    assert R.mmul(R.VP, R.HP) == R.SP
    assert R.mmul(R.VU, R.HU) == R.SU
    assert R.mmul(R.SU, R.SP) == R.mmul(R.mmul(R.VU, R.HU), R.mmul(R.VP, R.HP))
    # the predict leaves LL alone and fixes HH; the update fixes LL only
    assert R.SP[0] == R.IDENT[0] and R.SU[3] == R.IDENT[3]


def test_inverse_matrices():
    assert R.mmul(R.SP_INV, R.SP) == R.IDENT
    assert R.mmul(R.SU_INV, R.SU) == R.IDENT


SIZES = list(itertools.product(range(2, 14), range(2, 14)))


def test_float_spatial_steps_equal_separable():
    rng = np.random.default_rng(11)
    for h, w in SIZES:
        x = rng.normal(size=(h, w)) * 100
        np.testing.assert_allclose(R.float_fwd_level(x), oracle.fwd_level(x), atol=1e-11, rtol=0)


def test_int_composed_steps_equal_separable():
    rng = np.random.default_rng(12)
    for h, w in SIZES:
        x = rng.integers(0, 256, size=(h, w))
        assert np.array_equal(R.int_fwd_level(x), oracle.fwd_level(x, INT)), (h, w)


def test_float_inverse_steps():
    rng = np.random.default_rng(13)
    for h, w in SIZES:
        x = rng.normal(size=(h, w)) * 100
        c = oracle.fwd_level(x)
        np.testing.assert_allclose(R.float_inv_level(c), x, atol=1e-11, rtol=0)
        np.testing.assert_allclose(R.float_inv_level(c), oracle.inv_level(c), atol=1e-11, rtol=0)


def test_int_inverse_steps():
    rng = np.random.default_rng(14)
    for h, w in SIZES:
        x = rng.integers(0, 256, size=(h, w))
        c = oracle.fwd_level(x, INT)
        assert np.array_equal(R.int_inv_level(c), x), (h, w)


def test_adjoint_weights_equal_transpose():
    rng = np.random.default_rng(15)
    for h, w in SIZES:
        g = rng.normal(size=(h, w))
        np.testing.assert_allclose(R.float_adj_level(g), oracle.adj_level(g), atol=1e-12, rtol=0)


@pytest.mark.parametrize("h,w", [(40, 33), (17, 64), (3, 100)])
def test_regrouped_multilevel(h, w):
    """Chaining the regrouped level over the LL quadrant reproduces the
    oracle's multi-level transform."""
    x = np.random.default_rng(h * w).integers(0, 256, size=(h, w))
    levels = 2
    out_f, out_i = x.astype(float).copy(), x.copy()
    hh, ww = h, w
    for _ in range(levels):
        out_f[:hh, :ww] = R.float_fwd_level(out_f[:hh, :ww])
        out_i[:hh, :ww] = R.int_fwd_level(out_i[:hh, :ww])
        hh, ww = (hh + 1) // 2, (ww + 1) // 2
    np.testing.assert_allclose(out_f, oracle.fwd(x, levels), atol=1e-11, rtol=0)
    assert np.array_equal(out_i, oracle.fwd(x, levels, INT))
