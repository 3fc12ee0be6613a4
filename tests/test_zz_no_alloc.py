"""The allocation-free norm entry point (s5d_error_norms_noalloc) against the
entry point with a caller workspace (s5d_error_norms) and the numpy
definition in oracle.norms.

Two calls in a row on the shared per-device scratch, the second with a
smaller input, must each give the same bits as s5d_error_norms on the same
inputs: the scratch keeps the first call's partials, and the second call's
final pass must read only what it wrote itself.  The bar is that of the norm
tests: maxima bit-exact against the definition, root-mean-squares within
1e-13.
"""
import numpy as np
import pytest

import paper_2001_01473_amd as s5d
from gpu_util import say, torch
from oracle import norms

pytestmark = pytest.mark.gpu


def _pair(n, seed, gd, od):
    rng = np.random.default_rng(seed)
    o = rng.random(n).astype(od)
    g = (o.astype(np.float64) + rng.standard_normal(n) * 1e-6).astype(gd)
    o[rng.random(n) < 0.01] = 0
    return g, o


def _check(g, o, out):
    t = torch()
    gt = t.from_numpy(g).to("cuda:0")
    ot = t.from_numpy(o).to("cuda:0")
    got = s5d.error_norms_noalloc(gt, ot, out)
    want = s5d.error_norms(gt, ot)
    t.cuda.synchronize()
    a, b = got.cpu().numpy(), want.cpu().numpy()
    np.testing.assert_array_equal(a, b)
    ref = norms.error_norms(g, o)
    np.testing.assert_array_equal(a[:3], ref[:3])
    np.testing.assert_allclose(a[3:], ref[3:], rtol=1e-13, atol=0)


@pytest.mark.parametrize("gd,od", [(np.float32, np.float64), (np.float64, np.float64)])
def test_noalloc_norms_two_calls_second_smaller(gd, od):
    out = torch().empty(5, dtype=torch().float64, device="cuda:0")
    # first call: the largest first pass (2048 workgroups); second: 3 workgroups
    for n, seed in ((5 * (1 << 20) + 3, 11), (9000 + 1, 12)):
        say("noalloc norms", gd.__name__, od.__name__, n)
        g, o = _pair(n, seed, gd, od)
        _check(g, o, out)


def test_noalloc_norms_empty_and_tiny():
    out = torch().empty(5, dtype=torch().float64, device="cuda:0")
    for n in (1 << 16, 0, 1, 5):
        say("noalloc norms n =", n)
        g, o = _pair(n, 100 + n, np.float32, np.float32)
        if n == 0:
            t = torch()
            s5d.error_norms_noalloc(t.from_numpy(g).to("cuda:0"), t.from_numpy(o).to("cuda:0"), out)
            t.cuda.synchronize()
            np.testing.assert_array_equal(out.cpu().numpy(), norms.error_norms(g, o))
        else:
            _check(g, o, out)


def test_noalloc_norms_rejects_bad_arguments():
    t = torch()
    x = t.zeros(8, dtype=t.float32, device="cuda:0")
    small = t.empty(3, dtype=t.float64, device="cuda:0")
    with pytest.raises(ValueError):
        s5d.error_norms_noalloc(x, x, small)
    with pytest.raises(ValueError):
        s5d.error_norms_noalloc(x, x[:4], t.empty(5, dtype=t.float64, device="cuda:0"))
