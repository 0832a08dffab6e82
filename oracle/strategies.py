"""The third adaptive strategy of Sec. 3 (the r_s skip), oracle side.  TEST INFRASTRUCTURE ONLY.

In the multipole sum every target box B splits the sources into the far field F(B) and the
near field N(B), which is summed directly (Sec. 2.4).  Some boxes of N(B) are not adjacent to
B (Fig. of the near-field cross section: boxes of a finer level next to B's neighbours).  The
strategy: first accumulate everything except the sources of those non-adjacent boxes (far
field, B itself, the adjacent boxes), which estimates S at each target; then drop the
remaining sources when they are small against that estimate, as measured by the ratio r_s.

The ratio as printed compares a remaining source strength with an estimated S, which have
different units.  Reading taken here: the remaining sources are compared through an upper
bound of their field anywhere in B,

    bound(B) = sum over the remaining boxes A of  Q_A * K(d_min(A, B)),
    Q_A = sum_{j in A, j selected} w_j I_j,   d_min = smallest distance between the cubes,

which bounds the field of A's sources at every point of B because K decreases with r; at
target i of B the remaining sources are dropped iff bound(B) < r_s * est_i.  A dropped set then
changes S_i by at most r_s * est_i <= r_s * S_i.

Everything is an exact FP64 direct sum (``direct_sum``); the box structure (which sources are
the remaining ones for which targets, and their d_min) is an input: it is a property of the
tree the method builds, not of the integral.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from .direct import direct_sum, direct_sum_numpy
from .physics import cube_self_coefficient, gas_constants, kernel_K


@dataclass
class ThirdStrategyResult:
    S_t: np.ndarray        # S at the targets (with the skip applied)
    est_t: np.ndarray      # the estimate: S without the remaining sources (P included)
    rest_t: np.ndarray     # the remaining sources' field at each target (P included)
    bound_t: np.ndarray    # bound(B) of each target's box (P included; 0 without remaining boxes)
    skipped: np.ndarray    # bool per target: its remaining sources were dropped


def third_strategy(xyz, I, gas: dict, targets, target_group, groups: Sequence[Sequence[tuple]],
                   r_s: float, h: float = 0.0, w=None, smask=None, c_self: Optional[float] = None,
                   use_numpy: bool = False) -> ThirdStrategyResult:
    """S at ``targets`` under the r_s skip.

    target_group[t] is the index into ``groups`` of target t's box, or -1 when that box has no
    remaining (non-adjacent near) boxes; groups[g] lists the remaining boxes of box g as pairs
    (indices of the points in the box, d_min between the box and box g).  Only selected sources
    (smask) count.
    """
    gc = gas_constants(gas)
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    I = np.asarray(I, dtype=np.float64)
    n = xyz.shape[0]
    smask = np.ones(n, dtype=bool) if smask is None else np.asarray(smask, dtype=bool)
    weights = np.asarray(w, dtype=np.float64) if w is not None else np.full(n, h ** 3)
    if c_self is None:
        c_self = cube_self_coefficient(h, gc) if h > 0 else 0.0
    tgt = np.asarray(targets, dtype=np.int64)
    grp = np.asarray(target_group, dtype=np.int64)
    ssum = direct_sum_numpy if use_numpy else direct_sum
    est = np.empty(tgt.size)
    rest = np.zeros(tgt.size)
    bound = np.zeros(tgt.size)
    tself = np.where(smask[tgt], c_self * I[tgt], 0.0)
    src_all = np.flatnonzero(smask)
    # targets whose box has no remaining boxes: the plain sum
    m0 = grp < 0
    if m0.any():
        t0 = tgt[m0]
        est[m0] = ssum(xyz[src_all], weights[src_all] * I[src_all], src_all, xyz[t0], t0, tself[m0], gc)
    for g in np.unique(grp[grp >= 0]):
        mt = grp == g
        tg = tgt[mt]
        in_rest = np.zeros(n, dtype=bool)
        bnd = 0.0
        for idx, dmin in groups[g]:
            idx = np.asarray(idx, dtype=np.int64)
            sel = idx[smask[idx]]
            in_rest[sel] = True
            q = float(np.sum(weights[sel] * I[sel]))
            if q > 0.0:
                bnd += q * float(kernel_K(np.array([dmin]), gc)[0])
        s_est = np.flatnonzero(smask & ~in_rest)
        s_rest = np.flatnonzero(in_rest)
        est[mt] = ssum(xyz[s_est], weights[s_est] * I[s_est], s_est, xyz[tg], tg, tself[mt], gc)
        if s_rest.size:
            rest[mt] = ssum(xyz[s_rest], weights[s_rest] * I[s_rest], s_rest, xyz[tg], tg, np.zeros(tg.size), gc)
        bound[mt] = gc.P * bnd
    skipped = (grp >= 0) & (bound < r_s * est)
    S = est + np.where(skipped, 0.0, rest)
    return ThirdStrategyResult(S, est, rest, bound, skipped)
