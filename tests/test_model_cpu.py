"""Performance model and tuning cache, on the CPU (no kernel runs).

The model's traffic and work counts are pinned by brute force: every
(wave, row, column) a launch touches is enumerated cell by cell on a tiny
grid and counted with the rules the model states (lanes outside the grid move
no data; every lane computes every level over its stream block plus the
shrinking warm-up), then turned into seconds with the stated device rates.
"""
import ctypes
import math
import os

import numpy as np
import pytest

from geometry import compute_width, overlap_left, stream_blocks_2d
from paper_2001_01473_amd import _lib

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH),
                                reason="libstencil5d.so not built")

HBM = 6.0e12
VALU = {4: 256 * 64 * 2.4e9, 8: 256 * 64 * 2.4e9}  # lane-operations/s (no packed float32)


def _plan(ndim, r, box, dtype, interior, steps, accum=0, **tuning):
    import paper_2001_01473_amd as s5d
    n = (2 * r + 1) ** ndim if box else 2 * r * ndim + 1
    return s5d.Plan(ndim=ndim, radius=r, box=box, dtype=dtype, interior=interior, steps=steps,
                    coeffs=np.full(n, 1.0 / n), accum="compensated" if accum else "plain", **tuning)


def _brute2d(I0, I1, r, bt, cpl, h, w):
    """Bytes moved and lane-cell-levels of one 2D round, cell by cell."""
    lo = overlap_left(bt, r, w)
    W, C = 64 * cpl, compute_width(64 * cpl, bt, r, w)
    P0, P1 = I0 + 2 * r, I1 + 2 * r
    ntiles = -(-I1 // C)
    blocks = stream_blocks_2d(I0, r, h)
    read = write = comp = 0
    for t in range(ntiles):
        col0 = r + t * C - lo
        cols_in = [c for c in range(col0, col0 + W) if 0 <= c < P1]
        cols_out = [c for c in range(r + t * C, r + t * C + C) if r <= c < r + I1]
        for ra, rb in blocks:
            rows_in = [x for x in range(ra - bt * r, rb + bt * r) if 0 <= x < P0]
            read += len(rows_in) * len(cols_in)
            write += (rb - ra) * len(cols_out)
            for T in range(1, bt + 1):
                comp += W * ((rb - ra) + 2 * (bt - T) * r)
    return (read + write) * w, comp, -(-(ntiles * len(blocks)) // 4)


@pytest.mark.parametrize("I,r,box,dtype,bt,cpl,h", [
    ((40, 300), 1, False, "f32", 3, 4, 16), ((37, 517), 2, False, "f64", 2, 2, 9),
    ((64, 250), 1, True, "f32", 5, 4, 64), ((5, 3), 1, False, "f64", 1, 2, 2),
    ((2000, 300), 1, False, "f32", 3, 4, 40), ((1203, 130), 2, False, "f64", 2, 2, 35)])
def test_model2d_counts_match_brute_force(I, r, box, dtype, bt, cpl, h):
    w = 4 if dtype == "f32" else 8
    p = _plan(2, r, box, dtype, I, 2 * bt, bt=bt, cells_per_lane=cpl, stream_chunk=h)
    m = p.model()
    nbytes, comp, wgs = _brute2d(I[0], I[1], r, bt, cpl, h, w)
    assert m["hbm_bytes"] == pytest.approx(2 * nbytes, rel=1e-12)  # two rounds
    assert m["workgroups"] == wgs
    n = (2 * r + 1) ** 2 if box else 4 * r + 1
    # float32 stars and 3x3 boxes fold the lane shifts into their FMAs
    folded = dtype == "f32" and (not box or r == 1)
    ops = n + (0 if folded else (2 * r + 1 if box else 1) * 2 * r * (w // 4) / cpl) + 0.5
    assert m["valu_ops"] == pytest.approx(2 * comp * ops, rel=1e-12)
    assert m["t_hbm"] == pytest.approx(2 * nbytes / HBM, rel=1e-9)
    assert m["t_alu"] == pytest.approx(2 * comp * ops / VALU[w], rel=1e-9)
    # the slot efficiency divides the larger of the two terms
    slots = 256 * 2  # occupancy is unknown without a device: two workgroups per CU
    frac = slots / wgs
    fill = 1.0 / (max(1.0, frac) + 0.75 * min(1.0, frac))
    assert m["seconds"] == pytest.approx(max(m["t_hbm"], m["t_alu"]) / fill, rel=1e-9)
    p.close()


def test_model_regimes():
    # float32 5-point star at b_T = 1 moves 8 bytes per update and does ~6
    # operations: bound by HBM
    p = _plan(2, 1, False, "f32", (16384, 16384), 10, bt=1, kernel="blocked")
    assert p.model()["bound"] == "hbm"
    p.close()
    # compensated 25-point box: ~220 operations per update, bound by the ALU
    p = _plan(2, 2, True, "f32", (16384, 16384), 8, accum=1, bt=2)
    assert p.model()["bound"] == "alu"
    p.close()
    # deeper temporal blocking moves fewer bytes per update
    a = _plan(2, 1, False, "f32", (16384, 16384), 100, bt=1, kernel="blocked").model()
    b = _plan(2, 1, False, "f32", (16384, 16384), 100, bt=10).model()
    assert b["hbm_bytes"] < a["hbm_bytes"] / 5
    assert b["seconds"] < a["seconds"]


def test_model_scales_with_steps_and_3d_has_lds():
    a = _plan(3, 1, False, "f64", (256, 256, 256), 40).model()
    b = _plan(3, 1, False, "f64", (256, 256, 256), 80).model()
    assert b["seconds"] == pytest.approx(2 * a["seconds"], rel=0.05)
    assert a["t_lds"] > 0


def test_autotune_model_only_and_cache_roundtrip(tmp_path):
    import paper_2001_01473_amd as s5d
    s5d.tune_cache_clear()
    kw = dict(ndim=2, radius=1, box=False, dtype="f32", interior=(3000, 2000), steps=100,
              coeffs=np.full(5, 0.2))
    tun, rep = s5d.autotune(top_k=0, **kw)
    assert rep["n_candidates"] > 20 and rep["n_measured"] == 0
    # a later plan without tuning, same stencil and extent bucket, takes the
    # cached depth and tile; the stream-block length is the cached one for the
    # very extents it was chosen for, and chosen again for other extents
    p = s5d.Plan(**{**kw, "interior": (2900, 1900)})
    got = p.query()
    assert (got["bt"], got["cells_per_lane"]) == (tun["bt"], tun["cells_per_lane"])
    own = s5d.Plan(**{**kw, "interior": (2900, 1900)}, bt=tun["bt"],
                   cells_per_lane=tun["cells_per_lane"])
    assert got["stream_chunk"] == own.query()["stream_chunk"]
    own.close()
    p.close()
    p = s5d.Plan(**kw)
    got = p.query()
    assert (got["bt"], got["cells_per_lane"], got["stream_chunk"]) == \
        (tun["bt"], tun["cells_per_lane"], tun["stream_chunk"])
    p.close()
    path = tmp_path / "tune.txt"
    s5d.tune_cache_save(path)
    s5d.tune_cache_clear()
    p = s5d.Plan(**kw)
    default_bt = p.query()["bt"]
    p.close()
    s5d.tune_cache_load(path)
    p = s5d.Plan(**kw)
    assert p.query()["bt"] == tun["bt"]
    p.close()
    s5d.tune_cache_clear()
    assert default_bt >= 1
    bad = tmp_path / "bad.txt"
    bad.write_text("1 2 3\n")
    with pytest.raises(s5d.Stencil5DError):
        s5d.tune_cache_load(bad)


def test_model_ranking_prefers_deep_blocking_for_low_order_star():
    import paper_2001_01473_amd as s5d
    s5d.tune_cache_clear()
    tun, rep = s5d.autotune(top_k=0, ndim=2, radius=1, box=False, dtype="f32",
                            interior=(16384, 16384), steps=1000, coeffs=np.full(5, 0.2))
    assert tun["bt"] >= 4
    s5d.tune_cache_clear()


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_DEFAULT_FILE_SNIPPET = r"""
import sys
sys.path.insert(0, %r)
import numpy as np
import paper_2001_01473_amd as s5d
p = s5d.Plan(ndim=2, radius=1, box=False, dtype="f64", interior=(16384, 16384), steps=1000,
             coeffs=np.full(5, 0.2))
print(p.query()["bt"], p.query()["cells_per_lane"])
"""


def _default_bt_with(env_value, tmp_path):
    import os
    import subprocess
    import sys
    env = dict(os.environ)
    if env_value is None:
        env.pop("S5D_TUNING_FILE", None)
    else:
        env["S5D_TUNING_FILE"] = env_value
    out = subprocess.run([sys.executable, "-c", _DEFAULT_FILE_SNIPPET % ROOT], env=env, capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    bt, cpl = out.stdout.split()
    return int(bt), int(cpl)


def test_tuning_file_is_merged_at_the_first_plan(tmp_path):
    """The first plan of a process takes the entries of S5D_TUNING_FILE; an
    empty value keeps the built-in defaults."""
    f = tmp_path / "tuning.txt"
    # star, r = 1, float64, plain, linear, buckets 14 x 14: b_T 3, 4 cells per lane
    f.write_text("# test entry\n2 0 1 1 0 0 14 14 0 : 3 0 0 0 4 0 : 0.001 : 16384 16384 1\n")
    assert _default_bt_with(str(f), tmp_path) == (3, 4)
    builtin = _default_bt_with("", tmp_path)
    assert builtin != (3, 4) and builtin[0] >= 1


def test_shipped_tuning_file_parses():
    import os
    import paper_2001_01473_amd as s5d
    path = os.path.join(ROOT, "paper_2001_01473_amd", "tuning_gfx950.txt")
    if not os.path.exists(path):
        pytest.skip("no shipped tuning file")
    s5d.tune_cache_clear()
    s5d.tune_cache_load(path)
    s5d.tune_cache_clear()
