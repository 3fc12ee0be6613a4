"""GPU parity of the 2D stream-block layout: bands of rows (one per XCD, or
fewer when a band would not hold one block), long blocks of h_SN rows first
and a tail of h_SN/2-row blocks last, ragged bands and ragged last blocks.

Bars: every stream-block length gives the same bits (the method's result does
not depend on the blocking); the compensated kernels equal the compensated
oracle bit for bit; float64 is within 1e-12 (normwise and elementwise) of the
oracle; plain float32 is within the a-priori bound T * (gamma_n + u) * max|A0|
of the float64 oracle run on the same float32-rounded inputs.
"""
import numpy as np
import pytest

import oracle
import pins
import stencil_inputs as si
from geometry import stream_blocks_2d
from gpu_util import rel_errors, run_gpu, say

pytestmark = pytest.mark.gpu

INTERIOR = (8 * 150 + 37, 300)   # bands of 155 rows, the last one 122
CHUNKS = (32, 40, 155, 7, 64, 400, 1237)  # 400: two bands; 1237: one band
STEPS = 23


def test_chunks_cover_tails():
    """The chosen h_SN values exercise long blocks followed by half-length
    blocks, bands without long blocks, and ragged last blocks."""
    shapes = {ch: stream_blocks_2d(INTERIOR[0], 1, ch) for ch in CHUNKS}
    assert any(len({b - a for a, b in bl}) >= 3 for bl in shapes.values())
    for ch, bl in shapes.items():
        rows = sorted(r for a, b in bl for r in range(a, b))
        assert rows == list(range(1, INTERIOR[0] + 1)), ch


@pytest.mark.parametrize("kind", ["f32", "f64", "f32c"])
@pytest.mark.parametrize("r,box", [(1, False), (1, True), (2, False)])
def test_band_layout(kind, r, box):
    dt = np.float64 if kind == "f64" else np.float32
    accum = "compensated" if kind == "f32c" else "plain"
    case = si.make_case(81 + r + 3 * box, 2, r, box, INTERIOR, STEPS)
    c_in, g_in = case.as_dtype(dt)
    outs = []
    for ch in CHUNKS:
        say("bands", kind, "r", r, "box", box, "chunk", ch)
        got, info = run_gpu(g_in, radius=r, box=box, coeffs=case.coeffs, steps=STEPS, accum=accum,
                            kernel="blocked", stream_chunk=ch)
        assert info["stream_chunk"] == ch
        outs.append(got)
    for ch, o in zip(CHUNKS[1:], outs[1:]):
        np.testing.assert_array_equal(o, outs[0], err_msg="h_SN %d" % ch)
    if kind == "f32c":
        want = oracle.sweep(g_in, radius=r, box=box, coeffs=c_in, steps=STEPS, accum="compensated")
        np.testing.assert_array_equal(outs[0], want)
        return
    ref = oracle.sweep(g_in.astype(np.float64), radius=r, box=box, coeffs=c_in.astype(np.float64),
                       steps=STEPS)
    norm, elem = rel_errors(outs[0], ref)
    if kind == "f64":
        assert norm <= 1e-12 and elem <= 1e-12, (norm, elem)
    else:
        n = len(c_in)
        gamma = n * pins.U32 / (1 - n * pins.U32)
        bound = STEPS * (gamma + pins.U32) * float(np.abs(g_in).max())
        assert float(np.abs(outs[0].astype(np.float64) - ref).max()) <= bound
