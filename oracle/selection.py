"""Adaptive source/target selection as exact set operations (oracle side).

Strategy 1 (Sec. 3, eq. (18); Sec. 4.3, eq. (22)): keep source y_j when
I(y_j) >= I_pct * I_max, with I_max the maximum over every point (Sec. 4.1).
Strategy 2 (Sec. 3; Sec. 5): keep target x_i when
|E(x_i)| >= E_applied + eps * (E_max - E_applied); the streamer workloads also
use a plain absolute field floor |E| >= e_abs.

Each decision is a comparison of the stored value (FP32 inputs widened to FP64
exactly) against a threshold formed in FP64; the HIP path decides in FP64 the
same way, so the masks must agree bit for bit.
"""
from __future__ import annotations

import numpy as np


def source_mask(I, src_rel: float) -> np.ndarray:
    I = np.asarray(I, dtype=np.float64)
    if src_rel <= 0.0:
        return np.ones(I.shape, dtype=bool)
    thr = float(src_rel) * float(I.max())
    return I >= thr


def target_mask(E, e_abs: float = -1.0, e_applied: float = 0.0, e_rel: float = -1.0) -> np.ndarray:
    """All targets when no rule is on; otherwise the conjunction of the rules that are on."""
    if E is None:
        return None
    E = np.asarray(E, dtype=np.float64)
    m = np.ones(E.shape, dtype=bool)
    if e_abs >= 0.0:
        m &= E >= float(e_abs)
    if e_rel >= 0.0:
        thr = float(e_applied) + float(e_rel) * (float(E.max()) - float(e_applied))
        m &= E >= thr
    return m
