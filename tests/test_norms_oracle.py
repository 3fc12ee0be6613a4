"""The oracle's error norms against hand-computed values and exact identities."""
import math

import numpy as np

from oracle import norms


def test_hand_computed():
    got = [1.0, 2.0, 3.0, 4.0]
    ref = [1.0, 2.5, 0.0, 8.0]
    # d = 0, 0.5, 3, 4; d/|o| = 0, 0.2, (o = 0: d) 3, 0.5
    want = [4.0, 8.0, 3.0, math.sqrt((0.25 + 9 + 16) / 4), math.sqrt((1 + 6.25 + 64) / 4)]
    np.testing.assert_allclose(norms.error_norms(got, ref), want, rtol=1e-15, atol=0)
    assert norms.error_norms(got, ref)[2] == 3.0


def test_negative_values_and_order():
    got = np.array([-2.0, 5.0, -1.0])
    ref = np.array([-4.0, 4.0, 1.0])
    # d = 2, 1, 2; rel = 0.5, 0.25, 2
    r = norms.error_norms(got, ref)
    assert list(r[:3]) == [2.0, 4.0, 2.0]
    # invariant under a permutation of the cells
    p = [2, 0, 1]
    np.testing.assert_array_equal(norms.error_norms(got[p], ref[p])[:3], r[:3])


def test_power_of_two_scaling_is_exact():
    rng = np.random.default_rng(0)
    g, o = rng.random(1000), rng.random(1000)
    a, b = norms.error_norms(g, o), norms.error_norms(g * 8, o * 8)
    np.testing.assert_array_equal(b[[0, 1, 3, 4]], a[[0, 1, 3, 4]] * 8)
    assert b[2] == a[2]


def test_identical_inputs_and_empty():
    x = np.random.default_rng(1).random((7, 9))
    r = norms.error_norms(x, x)
    assert r[0] == r[2] == r[3] == 0.0 and r[1] == x.max()
    np.testing.assert_array_equal(norms.error_norms([], []), np.zeros(5))


def test_nan_propagates():
    r = norms.error_norms([1.0, float("nan"), 2.0], [1.0, 1.0, 1.0])
    assert math.isnan(r[0]) and math.isnan(r[2]) and math.isnan(r[3])
    assert r[1] == 1.0


def test_float32_promoted_exactly():
    g = np.array([0.1, 0.2], dtype=np.float32)
    o = np.array([0.1, 0.2], dtype=np.float64)
    r = norms.error_norms(g, o)
    assert r[0] == max(abs(float(np.float32(0.1)) - 0.1), abs(float(np.float32(0.2)) - 0.2)) > 0
