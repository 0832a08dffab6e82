"""Error measures of Sec. 4, eq. (19) (oracle side).

E_V: global relative discrete L2 error ||S_num - S_ref||_2 / ||S_ref||_2 (returned as a
fraction, not a percentage); E_delta: mean pointwise relative error over the ball
|x - x0| <= delta.  The reference is the discrete direct quadrature.
"""
from __future__ import annotations

import numpy as np


def rel_l2(S_num, S_ref) -> float:
    S_num = np.asarray(S_num, dtype=np.float64)
    S_ref = np.asarray(S_ref, dtype=np.float64)
    den = float(np.linalg.norm(S_ref))
    if den == 0.0:
        return float(np.linalg.norm(S_num))
    return float(np.linalg.norm(S_num - S_ref) / den)


def local_ball_error(S_num, S_ref, xyz, x0, delta) -> float:
    xyz = np.asarray(xyz, dtype=np.float64)
    m = np.linalg.norm(xyz - np.asarray(x0)[None, :], axis=1) <= delta
    if not m.any():
        return float("nan")
    S_ref = np.asarray(S_ref)[m]
    return float(np.mean(np.abs(np.asarray(S_num)[m] - S_ref) / S_ref))
