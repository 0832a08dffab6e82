"""Direct FP64 quadrature of eq. (15) restricted to the adaptive sets (oracle side).

``direct_sum`` calls the OpenMP C routine in ``direct.c``; ``direct_sum_numpy``
is an all-pairs NumPy twin for small inputs.  ``photoionization`` applies the
selection rules of Sec. 3 / Sec. 4.3 / Sec. 5 as exact set operations and
returns S at the selected targets:

  S_i = P * ( sum_{j in S, j != i} w_j I_j K(|x_i - x_j|) + [i in S] c_self I_i ),  i in T,
  S_i = 0 for i not in T.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

from .physics import GasConstants, cube_self_coefficient, gas_constants, kernel_K
from .selection import source_mask, target_mask

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_direct.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile direct.c with gcc (OpenMP, -O2, no fast-math) into liboracle_direct.so."""
    import subprocess
    src = os.path.join(_HERE, "direct.c")
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    f = lib.oracle_direct_sum
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int64)
    f.argtypes = [ctypes.c_int64, dp, dp, ip, ctypes.c_int64, dp, ip, dp,
                  ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                  ctypes.c_int, dp]
    f.restype = ctypes.c_int
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def direct_sum(src_xyz, src_q, src_id, tgt_xyz, tgt_id, tgt_self, gc: GasConstants,
               nthreads: int = 0, return_threads: bool = False):
    """P * (sum_j q_j K(r_ij) over sources with a different id and r > 0, + tgt_self_i)."""
    lib = _load()
    sx = np.ascontiguousarray(src_xyz, dtype=np.float64)
    sq = np.ascontiguousarray(src_q, dtype=np.float64)
    si = np.ascontiguousarray(src_id, dtype=np.int64)
    tx = np.ascontiguousarray(tgt_xyz, dtype=np.float64)
    ti = np.ascontiguousarray(tgt_id, dtype=np.int64)
    ts = np.ascontiguousarray(tgt_self, dtype=np.float64)
    out = np.empty(tx.shape[0], dtype=np.float64)
    used = lib.oracle_direct_sum(sx.shape[0], _dptr(sx), _dptr(sq), _iptr(si), tx.shape[0], _dptr(tx),
                                 _iptr(ti), _dptr(ts), gc.a, gc.b, gc.L, gc.P, int(nthreads), _dptr(out))
    return (out, used) if return_threads else out


def direct_sum_numpy(src_xyz, src_q, src_id, tgt_xyz, tgt_id, tgt_self, gc: GasConstants):
    """All-pairs NumPy twin of ``direct_sum`` (plain summation), for at most a few thousand points."""
    d = tgt_xyz[:, None, :] - src_xyz[None, :, :]
    r = np.sqrt((d ** 2).sum(axis=2))
    keep = (np.asarray(tgt_id)[:, None] != np.asarray(src_id)[None, :]) & (r > 0)
    rr = np.where(keep, r, 1.0)
    Kmat = np.where(keep, kernel_K(rr, gc), 0.0)
    return gc.P * (Kmat @ np.asarray(src_q, dtype=np.float64) + np.asarray(tgt_self, dtype=np.float64))


@dataclass
class OracleResult:
    S_t: np.ndarray          # S at the evaluated targets
    tgt: np.ndarray          # evaluated target indices (caller order)
    src: np.ndarray          # selected source indices (caller order)
    smask: np.ndarray
    tmask: np.ndarray
    c_self: float
    threads: int
    gc: GasConstants

    def full(self, n: int) -> np.ndarray:
        out = np.zeros(n)
        out[self.tgt] = self.S_t
        return out


def photoionization(xyz, I, gas: dict, h: float = 0.0, w=None, src_rel: float = 0.0, E=None,
                    e_abs: float = -1.0, e_applied: float = 0.0, e_rel: float = -1.0,
                    c_self: Optional[float] = None, targets=None, smask=None,
                    nthreads: int = 0, use_numpy: bool = False) -> OracleResult:
    """S_ph at the selected targets (or at ``targets``, a subset of them) over the selected sources."""
    gc = gas_constants(gas)
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    I = np.asarray(I, dtype=np.float64)
    n = xyz.shape[0]
    if smask is None:
        smask = source_mask(I, src_rel)
    tm = target_mask(E, e_abs, e_applied, e_rel)
    if tm is None:
        tm = np.ones(n, dtype=bool)
    weights = np.asarray(w, dtype=np.float64) if w is not None else np.full(n, h ** 3)
    if c_self is None:
        c_self = cube_self_coefficient(h, gc) if h > 0 else 0.0
    tgt = np.flatnonzero(tm) if targets is None else np.asarray(targets, dtype=np.int64)
    src = np.flatnonzero(smask)
    q = weights[src] * I[src]
    tself = np.where(smask[tgt], c_self * I[tgt], 0.0)
    threads = 1
    if use_numpy:
        S_t = direct_sum_numpy(xyz[src], q, src, xyz[tgt], tgt, tself, gc)
    else:
        S_t, threads = direct_sum(xyz[src], q, src, xyz[tgt], tgt, tself, gc, nthreads=nthreads,
                                  return_threads=True)
    return OracleResult(S_t, tgt, src, smask, tm, float(c_self), threads, gc)
