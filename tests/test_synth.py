"""The seeded input generator: range, integrality, determinism, draw order."""
import numpy as np

from paper_1708_07853_amd import synth


def test_image_range_and_determinism():
    a = synth.image(300, 200, 1)
    b = synth.image(300, 200, 1)
    assert a.shape == (200, 300) and a.dtype == np.float32
    assert np.array_equal(a, b)
    assert a.min() >= 0 and a.max() <= 255
    assert np.array_equal(a, np.rint(a))
    assert not np.array_equal(a, synth.image(300, 200, 2))
    i = synth.image(300, 200, 1, np.int32)
    assert i.dtype == np.int32 and np.array_equal(i, a.astype(np.int32))


def test_row_blocking_does_not_change_the_image():
    old = synth.ROW_BLOCK
    try:
        a = synth.image(97, 70, 9)
        synth.ROW_BLOCK = 16
        b = synth.image(97, 70, 9)
    finally:
        synth.ROW_BLOCK = old
    assert np.array_equal(a, b)


def test_ragged_sizes():
    s = synth.ragged_sizes()
    assert len(s) == 256
    assert all(64 <= w <= 4096 and 64 <= h <= 4096 for w, h in s)
    assert any(w % 2 for w, _ in s) and any(h % 2 for _, h in s)
    assert s == synth.ragged_sizes()
