"""GPU float64 error/norm reductions (s5d_error_norms) against the numpy
definition in oracle.norms.

Bar: the three maxima are bit-exact (|g - o| and d/|o| are single correctly
rounded float64 operations on both sides); the two root-mean-squares agree
within 1e-13 relative (only the order of the float64 sums differs); repeated
calls give identical bits.
"""
import math

import numpy as np
import pytest

import paper_2001_01473_amd as s5d
from gpu_util import say, torch
from oracle import norms

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch().from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _gpu(g, o):
    r = s5d.error_norms(_dev(g), _dev(o))
    torch().cuda.synchronize()
    return r.cpu().numpy()


def _compare(got, want):
    np.testing.assert_array_equal(got[:3], want[:3])
    np.testing.assert_allclose(got[3:], want[3:], rtol=1e-13, atol=0)


@pytest.mark.parametrize("gd,od", [(np.float32, np.float64), (np.float64, np.float64),
                                   (np.float32, np.float32), (np.float64, np.float32)])
@pytest.mark.parametrize("n", [1, 3, 4, 5, 1023, 4099, 1 << 20, 3 * (1 << 20) + 7])
def test_norms_match_definition(gd, od, n):
    rng = np.random.default_rng(n)
    o = rng.random(n).astype(od)
    g = (o.astype(np.float64) + rng.standard_normal(n) * 1e-6).astype(gd)
    o[rng.random(n) < 0.01] = 0  # exercise the o = 0 branch
    say("norms", gd.__name__, od.__name__, n)
    _compare(_gpu(g, o), norms.error_norms(g, o))


def test_norms_grid_sized_and_deterministic():
    """A padded 4098 x 4099 float32 result against a float64 reference, as
    after a sweep; two calls agree bit for bit."""
    rng = np.random.default_rng(7)
    o = rng.random((4098, 4099))
    g = (o + rng.standard_normal(o.shape) * 1e-7).astype(np.float32)
    gt, ot = _dev(g), _dev(o)
    say("norms 4098x4099")
    a = s5d.error_norms(gt, ot).cpu().numpy()
    b = s5d.error_norms(gt, ot).cpu().numpy()
    np.testing.assert_array_equal(a, b)
    _compare(a, norms.error_norms(g, o))


def test_norms_nan_and_empty():
    g = np.array([1.0, np.nan, 2.0, 3.0, 5.0])
    o = np.array([1.0, 1.0, 1.0, 1.0, 1.0])
    r = _gpu(g, o)
    assert math.isnan(r[0]) and math.isnan(r[2]) and math.isnan(r[3]) and r[1] == 1.0
    t = torch()
    e = t.empty(0, dtype=t.float64, device="cuda:0")
    np.testing.assert_array_equal(s5d.error_norms(e, e).cpu().numpy(), np.zeros(5))


def test_norms_argument_errors():
    t = torch()
    a = t.zeros(64, dtype=t.float32, device="cuda:0")
    b = t.zeros(64, dtype=t.float64, device="cuda:0")
    with pytest.raises(s5d.Stencil5DError) as err:  # misaligned: checked before any launch
        s5d.error_norms(a[1:17], b[:16])
    assert err.value.status == 1
    with pytest.raises(s5d.Stencil5DError) as err:
        s5d.error_norms(a, b, workspace=t.empty(8, dtype=t.uint8, device="cuda:0"))
    assert err.value.status == 1
