"""Helpers for the GPU tests: run the library on numpy inputs, compare results."""
import sys

import numpy as np

import paper_2001_01473_amd as s5d


def torch():
    import torch as _t
    return _t


def say(*a):
    """Flush a line naming the case before a GPU step."""
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(grid, *, radius, box, coeffs, steps, accum="plain", **tuning):
    """Sweep a padded numpy grid on cuda:0 through the C ABI; returns (result, plan info)."""
    t = torch()
    x = t.from_numpy(np.ascontiguousarray(grid)).to("cuda:0")
    other = t.empty_like(x)
    interior = tuple(s - 2 * radius for s in grid.shape)
    plan = s5d.Plan(ndim=grid.ndim, radius=radius, box=box, dtype=grid.dtype,
                    interior=interior, steps=steps, coeffs=coeffs, accum=accum, **tuning)
    info = plan.query()
    idx = plan.run(x, other)
    t.cuda.synchronize()
    out = (x if idx == 0 else other).cpu().numpy()
    plan.close()
    assert idx == steps % 2
    return out, info


def rel_errors(got, ref):
    """(normwise max|g-o|/max|o|, elementwise max |g-o|/|o|) in float64."""
    g = np.asarray(got, dtype=np.float64)
    o = np.asarray(ref, dtype=np.float64)
    d = np.abs(g - o)
    norm = float(d.max() / max(np.abs(o).max(), 1e-300))
    nz = np.abs(o) > 0
    elem = float((d[nz] / np.abs(o[nz])).max()) if nz.any() else 0.0
    if (~nz).any():
        elem = max(elem, float(d[~nz].max()))
    return norm, elem
