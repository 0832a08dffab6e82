"""Shared test helpers: NumPy references for integer work (keys, sort, tree) and plan construction."""
from __future__ import annotations

import numpy as np

import gen

MORTON_BITS = 21


def _spread(v):
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    v = (v | (v << np.uint64(32))) & np.uint64(0x001F00000000FFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x001F0000FF0000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
    return v


def morton_keys(xyz, lo, size):
    """63-bit Morton keys of 21-bit quantised coordinates (x most significant)."""
    q = np.floor((np.asarray(xyz, dtype=np.float64) - np.asarray(lo)[None, :]) / size * 2097152.0)
    q = np.clip(q, 0, 2097151).astype(np.uint64)
    return (_spread(q[:, 0]) << np.uint64(2)) | (_spread(q[:, 1]) << np.uint64(1)) | _spread(q[:, 2])


def reference_tree(s_keys, t_keys, leaf_cap, max_depth):
    """Adaptive octree over two sorted key lists, split while max(#s, #t) > leaf_cap.

    Returns rows (level, ax, ay, az, s_first, s_cnt, t_first, t_cnt, leaf) level by level,
    children in octant (Morton) order.
    """
    s_keys = np.asarray(s_keys, dtype=np.uint64)
    t_keys = np.asarray(t_keys, dtype=np.uint64)
    rows = []
    cur = [(0, 0, 0, 0, 0, len(s_keys), 0, len(t_keys))]
    for level in range(max_depth + 1):
        nxt = []
        for (l, ax, ay, az, sf, sn, tf, tn) in cur:
            split = max(sn, tn) > leaf_cap and level < max_depth
            rows.append((l, ax, ay, az, sf, sn, tf, tn, 0 if split else 1))
            if not split:
                continue
            shift = np.uint64(3 * (MORTON_BITS - (level + 1)))
            sd = (s_keys[sf:sf + sn] >> shift) & np.uint64(7)
            td = (t_keys[tf:tf + tn] >> shift) & np.uint64(7)
            for o in range(8):
                s0 = sf + int(np.searchsorted(sd, o, side="left"))
                s1 = sf + int(np.searchsorted(sd, o, side="right"))
                t0 = tf + int(np.searchsorted(td, o, side="left"))
                t1 = tf + int(np.searchsorted(td, o, side="right"))
                if (s1 - s0) + (t1 - t0) == 0:
                    continue
                nxt.append((level + 1, 2 * ax + ((o >> 2) & 1), 2 * ay + ((o >> 1) & 1), 2 * az + (o & 1),
                            s0, s1 - s0, t0, t1 - t0))
        if not nxt:
            break
        cur = nxt
    return np.array(rows, dtype=np.int64)


def plan_kwargs(wl: gen.Workload, **kw):
    lo, hi = wl.domain
    args = dict(h=wl.h, w=wl.w, cube_lo=(lo, lo, lo), cube_size=hi - lo)
    if wl.h <= 0:
        args["self_coeff"] = 0.0
    args.update(kw)
    return args


def _adjacent(A, B):
    """Closed cubes of two octree boxes (level, ax, ay, az) touch or overlap (A != B)."""
    la, lb = int(A[0]), int(B[0])
    L = max(la, lb)
    sa, sb = 1 << (L - la), 1 << (L - lb)
    for d in range(1, 4):
        a0, b0 = int(A[d]) * sa, int(B[d]) * sb
        if a0 > b0 + sb or b0 > a0 + sa:
            return False
    return tuple(int(v) for v in A[:4]) != tuple(int(v) for v in B[:4])


def w_lists(rows):
    """W list of every target leaf of a tree from ``reference_tree``: the boxes with sources
    that descend from a colleague of the leaf, are not adjacent to it, and whose parent is
    (kernel-independent FMM lists, Sec. 2.4).  Returns {leaf row: [rows of its W boxes]}."""
    key = {tuple(int(v) for v in r[:4]): i for i, r in enumerate(rows)}

    def children(i):
        l, ax, ay, az = (int(v) for v in rows[i][:4])
        out = []
        for o in range(8):
            k = (l + 1, 2 * ax + ((o >> 2) & 1), 2 * ay + ((o >> 1) & 1), 2 * az + (o & 1))
            if k in key:
                out.append(key[k])
        return out

    res = {}
    for b, r in enumerate(rows):
        if not (r[8] == 1 and r[7] > 0):
            continue
        l, ax, ay, az = (int(v) for v in r[:4])
        stack = []
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    k = (l, ax + dx, ay + dy, az + dz)
                    if k in key and k != (l, ax, ay, az):
                        stack.append(key[k])
        W = []
        while stack:
            c = stack.pop()
            if rows[c][8] == 1:
                continue
            for a in children(c):
                if _adjacent(rows[a], r):
                    stack.append(a)
                elif rows[a][5] > 0:
                    W.append(a)
        if W:
            res[b] = sorted(W)
    return res


def box_gap(A, B, lo, size):
    """Smallest distance between the cubes of two octree boxes (cube [lo, lo + size]^3)."""
    ha, hb = size / (1 << int(A[0])), size / (1 << int(B[0]))
    g2 = 0.0
    for d in range(1, 4):
        a0, b0 = lo + int(A[d]) * ha, lo + int(B[d]) * hb
        g = max(0.0, max(a0, b0) - min(a0 + ha, b0 + hb))
        g2 += g * g
    return float(np.sqrt(g2))
