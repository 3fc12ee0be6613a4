"""Error norms between a computed grid and a reference -- test infrastructure
only (the float64 reductions the GPU library offers for checking its results).

Plain numpy definition, in float64: with d = |g - o|,
  max d, max |o|, max d/|o| (d where o = 0), sqrt(mean d^2), sqrt(mean o^2).
NaN in either input propagates into the maxima of d and d/|o| and the RMS of d.
Pinned in tests/test_norms_oracle.py against hand-computed values and exact
scaling identities.
"""
from __future__ import annotations

import numpy as np

NAMES = ("max_abs_err", "max_abs_ref", "max_rel_err", "rms_err", "rms_ref")


def error_norms(got, ref) -> np.ndarray:
    g = np.asarray(got, dtype=np.float64).ravel()
    o = np.asarray(ref, dtype=np.float64).ravel()
    if g.size != o.size:
        raise ValueError("got and ref differ in size")
    n = g.size
    if n == 0:
        return np.zeros(5)
    d = np.abs(g - o)
    ao = np.abs(o)
    nz = ao != 0
    rel = d.copy()
    rel[nz] = d[nz] / ao[nz]
    return np.array([d.max(), ao.max(), rel.max(),
                     np.sqrt(np.sum(d * d) / n), np.sqrt(np.sum(ao * ao) / n)])
