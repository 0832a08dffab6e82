"""ctypes binding of libph (the C ABI declared in include/ph.h).

Argument marshalling only: every step of an evaluation runs in the library's
HIP kernels.  Device buffers are torch CUDA (HIP) tensors passed by
``data_ptr()``; the stream is torch's current stream unless one is given.
Loading fails loudly when libph.so is missing; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libph.so")

PH_OK, PH_EINVAL, PH_ENOMEM, PH_EDEVICE, PH_ENUMERIC, PH_EUNSUPPORTED, PH_EFALLBACK = range(7)
PRECISION = {"fp64": 0, "fp32": 1, "bf16split": 2}
SELECTOR = {"threshold": 0, "learned": 1}
METHOD = {"fmm": 0, "direct": 1}
NPHASES = 12
BOX_FIELDS = 10
MLP_NIN, MLP_NHID = 8, 64
MLP_NPARAM = 64 * 8 + 64 + 64 * 64 + 64 + 64 + 1
DEBUG = {"keys": 0, "perm": 1, "src": 2, "tgt": 3, "boxes": 4, "level_start": 5, "c_self": 6,
         "scale_exp": 7, "features": 8, "feature_boxes": 9, "rs_skip": 10}


class PhPoints(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("xyz", ctypes.POINTER(ctypes.c_double)),
                ("w", ctypes.POINTER(ctypes.c_double)), ("h", ctypes.c_double),
                ("self_coeff", ctypes.c_double), ("cube_lo", ctypes.c_double * 3),
                ("cube_size", ctypes.c_double)]


class PhGas(ctypes.Structure):
    _fields_ = [("p_torr", ctypes.c_double), ("o2_fraction", ctypes.c_double), ("pq_torr", ctypes.c_double),
                ("xi_omega_over_alpha", ctypes.c_double), ("chi_min", ctypes.c_double),
                ("chi_max", ctypes.c_double)]


class PhThresholds(ctypes.Structure):
    _fields_ = [("src_rel", ctypes.c_double), ("e_abs", ctypes.c_double), ("e_applied", ctypes.c_double),
                ("e_rel", ctypes.c_double), ("r_s", ctypes.c_double)]


class PhOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("selector", ctypes.c_int), ("method", ctypes.c_int),
                ("order_q", ctypes.c_int), ("leaf_capacity", ctypes.c_int), ("max_depth", ctypes.c_int),
                ("pinv_rel_cutoff", ctypes.c_double), ("selector_weights", ctypes.POINTER(ctypes.c_float)),
                ("selector_logit_threshold", ctypes.c_float), ("selector_fallback_rel", ctypes.c_double),
                ("workspace_cap_bytes", ctypes.c_size_t), ("validate", ctypes.c_int), ("tol", ctypes.c_double)]


class PhStats(ctypes.Structure):
    _fields_ = [("n_src", ctypes.c_int64), ("n_tgt", ctypes.c_int64), ("n_boxes", ctypes.c_int64),
                ("n_leaves", ctypes.c_int64), ("levels", ctypes.c_int32), ("fell_back", ctypes.c_int32),
                ("n_src_dropped", ctypes.c_int64), ("t_ms", ctypes.c_double * NPHASES),
                ("work", ctypes.c_int64 * 12), ("check_rel_l2", ctypes.c_double)]


WORK = ("p2p_pairs", "l2p_evals", "m2p_evals", "p2m_evals", "p2l_evals", "m2l_pairs", "m2m_children",
        "l2l_boxes", "grid_l2p_madds", "grid_p2m_madds", "near_targets", "p2p_table_pairs")


EXPORTED = ["ph_status_string", "ph_last_error", "ph_options_default", "ph_plan_create", "ph_plan_destroy",
            "ph_evaluate", "ph_plan_check", "ph_plan_size", "ph_debug_fetch", "ph_mlp_forward",
            "ph_mlp_backward", "ph_adam_step", "ph_selector_features", "ph_phase_times", "ph_selector_fields",
            "ph_plan_set_graph", "ph_mlp_backward_noalloc", "ph_evaluate_workspace_bytes", "ph_evaluate_ws",
            "ph_plan_set_targets", "ph_plan_set_gas", "ph_evaluate_same_sets"]

_lib = None


class PhError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{_status_name(status)}: {detail}")
        self.status = status


def _status_name(s):
    return {0: "PH_OK", 1: "PH_EINVAL", 2: "PH_ENOMEM", 3: "PH_EDEVICE", 4: "PH_ENUMERIC",
            5: "PH_EUNSUPPORTED", 6: "PH_EFALLBACK"}.get(s, f"status {s}")


def load(path: Optional[str] = None):
    """Load libph.so (built by ``build.py``); raises OSError if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise OSError(f"libph.so not found at {path}; run paper_2112_10059_amd/build.py (HIP build)")
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.ph_status_string.restype = ctypes.c_char_p
    lib.ph_status_string.argtypes = [ctypes.c_int]
    lib.ph_last_error.restype = ctypes.c_char_p
    lib.ph_last_error.argtypes = []
    lib.ph_options_default.restype = None
    lib.ph_options_default.argtypes = [ctypes.POINTER(PhOptions)]
    lib.ph_plan_create.restype = ctypes.c_int
    lib.ph_plan_create.argtypes = [ctypes.POINTER(PhPoints), ctypes.POINTER(PhGas), ctypes.POINTER(PhThresholds),
                                   ctypes.POINTER(PhOptions), ctypes.POINTER(vp)]
    lib.ph_plan_destroy.restype = None
    lib.ph_plan_destroy.argtypes = [vp]
    lib.ph_evaluate.restype = ctypes.c_int
    lib.ph_evaluate.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(PhStats)]
    lib.ph_evaluate_workspace_bytes.restype = ctypes.c_size_t
    lib.ph_evaluate_workspace_bytes.argtypes = [vp]
    lib.ph_evaluate_ws.restype = ctypes.c_int
    lib.ph_evaluate_ws.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(PhStats)]
    lib.ph_plan_set_targets.restype = ctypes.c_int
    lib.ph_plan_set_targets.argtypes = [vp, vp, ctypes.c_int64]
    lib.ph_evaluate_same_sets.restype = ctypes.c_int
    lib.ph_evaluate_same_sets.argtypes = [vp, vp, vp, vp, ctypes.POINTER(PhStats)]
    lib.ph_plan_set_gas.restype = ctypes.c_int
    lib.ph_plan_set_gas.argtypes = [vp, ctypes.POINTER(PhGas), ctypes.POINTER(ctypes.c_int)]
    lib.ph_plan_set_graph.restype = ctypes.c_int
    lib.ph_plan_set_graph.argtypes = [vp, ctypes.c_int]
    lib.ph_plan_check.restype = ctypes.c_int
    lib.ph_plan_check.argtypes = [vp, vp]
    lib.ph_plan_size.restype = ctypes.c_int64
    lib.ph_plan_size.argtypes = [vp]
    lib.ph_debug_fetch.restype = ctypes.c_int
    lib.ph_debug_fetch.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.ph_mlp_forward.restype = ctypes.c_int
    lib.ph_mlp_forward.argtypes = [vp, vp, ctypes.c_int64, vp, ctypes.c_int, vp]
    lib.ph_mlp_backward.restype = ctypes.c_int
    lib.ph_mlp_backward.argtypes = [vp, vp, vp, ctypes.c_float, ctypes.c_int64, vp, vp, vp]
    lib.ph_mlp_backward_noalloc.restype = ctypes.c_int
    lib.ph_mlp_backward_noalloc.argtypes = [vp, vp, vp, ctypes.c_float, ctypes.c_int64, vp, vp, vp]
    lib.ph_adam_step.restype = ctypes.c_int
    lib.ph_adam_step.argtypes = [vp, vp, vp, vp, ctypes.c_int64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_int64, vp]
    lib.ph_phase_times.restype = ctypes.c_int
    lib.ph_phase_times.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.ph_selector_features.restype = ctypes.c_int
    lib.ph_selector_features.argtypes = [vp, vp, vp, vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), vp]
    lib.ph_selector_fields.restype = ctypes.c_int
    lib.ph_selector_fields.argtypes = [vp, vp, vp, ctypes.c_int64, vp, ctypes.c_int64, ctypes.c_int64, vp]
    _lib = lib
    return lib


def _check(status: int):
    if status not in (PH_OK, PH_EFALLBACK):
        raise PhError(status, _lib.ph_last_error().decode())
    return status


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def make_gas(gas: dict) -> PhGas:
    return PhGas(gas["p_torr"], gas["o2_fraction"], gas["pq_torr"], gas["xi_omega_over_alpha"],
                 gas["chi_min"], gas["chi_max"])


def make_thresholds(thr: dict) -> PhThresholds:
    return PhThresholds(thr.get("src_rel", 0.0), thr.get("e_abs", -1.0), thr.get("e_applied", 0.0),
                        thr.get("e_rel", -1.0), thr.get("r_s", 0.0))


class Plan:
    """Owns a ph_plan; see ph_plan_create / ph_evaluate in include/ph.h."""

    def __init__(self, xyz, gas: dict, thresholds: dict, h: float = 0.0, w=None, self_coeff: float = math.nan,
                 cube_lo=None, cube_size: float = 0.0, precision: str = "fp32", method: str = "fmm",
                 selector: str = "threshold", order_q: int = 0, leaf_capacity: int = 0, max_depth: int = 0,
                 pinv_rel_cutoff: float = 0.0, selector_weights=None, selector_logit_threshold: float = 0.0,
                 selector_fallback_rel: float = 0.0, workspace_cap: int = 0, validate: bool = False,
                 tol: float = 0.0):
        lib = load()
        self._xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.n = int(self._xyz.shape[0])
        self._w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        pts = PhPoints()
        pts.n = self.n
        pts.xyz = self._xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        pts.w = self._w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if self._w is not None else None
        pts.h = float(h)
        pts.self_coeff = float(self_coeff)
        lo = cube_lo if cube_lo is not None else (0.0, 0.0, 0.0)
        pts.cube_lo[0], pts.cube_lo[1], pts.cube_lo[2] = (float(v) for v in lo)
        pts.cube_size = float(cube_size)
        opt = PhOptions()
        lib.ph_options_default(ctypes.byref(opt))
        opt.precision = PRECISION[precision]
        opt.selector = SELECTOR[selector]
        opt.method = METHOD[method]
        opt.order_q = int(order_q)
        opt.leaf_capacity = int(leaf_capacity)
        opt.max_depth = int(max_depth)
        opt.pinv_rel_cutoff = float(pinv_rel_cutoff)
        self._selw = None
        if selector_weights is not None:
            self._selw = np.ascontiguousarray(selector_weights, dtype=np.float32)
            opt.selector_weights = self._selw.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        opt.selector_logit_threshold = float(selector_logit_threshold)
        opt.selector_fallback_rel = float(selector_fallback_rel)
        opt.workspace_cap_bytes = int(workspace_cap)
        opt.validate = 1 if validate else 0
        opt.tol = float(tol)
        self.precision = precision
        self.thresholds = dict(thresholds)
        handle = ctypes.c_void_p()
        g = make_gas(gas)
        t = make_thresholds(thresholds)
        _check(lib.ph_plan_create(ctypes.byref(pts), ctypes.byref(g), ctypes.byref(t), ctypes.byref(opt),
                                  ctypes.byref(handle)))
        self._h = handle

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.precision == "fp64" else torch.float32

    def workspace_bytes(self) -> int:
        return int(_lib.ph_evaluate_workspace_bytes(self._h))

    def new_workspace(self, device="cuda"):
        """A zero-filled workspace for evaluate(workspace=...)."""
        import torch
        return torch.zeros(self.workspace_bytes(), dtype=torch.uint8, device=device)

    def evaluate(self, I, E=None, out=None, stream=None, stats: bool = False, workspace=None,
                 same_sets: bool = False):
        """S_ph for device tensors I (dtype of the plan) and |E| (float32 or None); with a
        workspace (from new_workspace) the call runs on it (ph_evaluate_ws); same_sets: on the
        sets, tree and lists of the previous call (ph_evaluate_same_sets, E unused)."""
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=self.dtype, device=I.device)
        st = PhStats() if stats else None
        if same_sets:
            _check(_lib.ph_evaluate_same_sets(self._h, _dptr(I), _dptr(out), _stream_ptr(stream),
                                              ctypes.byref(st) if stats else None))
        elif workspace is None:
            _check(_lib.ph_evaluate(self._h, _dptr(I), _dptr(E), _dptr(out), _stream_ptr(stream),
                                    ctypes.byref(st) if stats else None))
        else:
            _check(_lib.ph_evaluate_ws(self._h, _dptr(I), _dptr(E), _dptr(out), _dptr(workspace),
                                       _stream_ptr(stream), ctypes.byref(st) if stats else None))
        if stats:
            return out, {"n_src": st.n_src, "n_tgt": st.n_tgt, "n_boxes": st.n_boxes, "n_leaves": st.n_leaves,
                         "levels": st.levels,
                         "fell_back": st.fell_back, "n_src_dropped": st.n_src_dropped,
                         "t_ms": list(st.t_ms), "work": dict(zip(WORK, list(st.work))),
                         "check_rel_l2": st.check_rel_l2}
        return out

    def set_targets(self, mask=None):
        """Caller-supplied target set (boolean array over the points, caller order), or None for all."""
        if mask is None:
            _check(_lib.ph_plan_set_targets(self._h, None, 0))
            return
        self._tmask = np.ascontiguousarray(np.asarray(mask, dtype=bool).astype(np.uint8).ravel())
        _check(_lib.ph_plan_set_targets(self._h, self._tmask.ctypes.data_as(ctypes.c_void_p), self._tmask.size))

    def set_gas(self, gas: dict) -> int:
        """Moves the plan to another gas (same points and tree); returns the number of far-field
        levels taken from the plan's operator cache."""
        g = make_gas(gas)
        n = ctypes.c_int(0)
        _check(_lib.ph_plan_set_gas(self._h, ctypes.byref(g), ctypes.byref(n)))
        return n.value

    def set_graph(self, enable: bool = True):
        """Later evaluate() calls without stats run as one replayed HIP graph (per set of buffers)."""
        _check(_lib.ph_plan_set_graph(self._h, 1 if enable else 0))

    PHASES = ("reduce", "flags", "compact", "tree", "lists", "upward", "downward", "leaf", "near", "m2l")

    def phase_times(self, record: int = -1):
        """Summed per-phase device ms since the last query, and the number of calls."""
        sums = (ctypes.c_double * NPHASES)()
        n = ctypes.c_int64()
        _check(_lib.ph_phase_times(self._h, int(record), sums, ctypes.byref(n)))
        return {name: sums[i] for i, name in enumerate(self.PHASES)}, n.value

    def check(self, stream=None):
        return _check(_lib.ph_plan_check(self._h, _stream_ptr(stream)))

    def debug_fetch(self, what: str) -> np.ndarray:
        code = DEBUG[what]
        n = ctypes.c_int64()
        _check(_lib.ph_debug_fetch(self._h, code, None, 0, ctypes.byref(n)))
        dt = {0: np.uint64, 1: np.int32, 2: np.int32, 3: np.int32, 4: np.int32, 5: np.int32, 6: np.float64,
              7: np.int32, 8: np.float32, 9: np.int32, 10: np.uint8}[code]
        width = {4: BOX_FIELDS, 8: 8}.get(code, 1)
        buf = np.zeros(n.value * width, dtype=dt)
        _check(_lib.ph_debug_fetch(self._h, code, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes,
                                   ctypes.byref(n)))
        return buf.reshape(-1, width) if width > 1 else buf

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.ph_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_forward(params, X, logits=None, bf16: bool = False, stream=None):
    import torch
    m = X.shape[0]
    if logits is None:
        logits = torch.empty(m, dtype=torch.float32, device=X.device)
    _check(load().ph_mlp_forward(_dptr(params), _dptr(X), m, _dptr(logits), int(bf16), _stream_ptr(stream)))
    return logits


def mlp_backward(params, X, y, pos_weight: float, grad=None, loss=None, stream=None):
    import torch
    if grad is None:
        grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device=X.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
    _check(load().ph_mlp_backward(_dptr(params), _dptr(X), _dptr(y), float(pos_weight), X.shape[0], _dptr(grad),
                                  _dptr(loss), _stream_ptr(stream)))
    return grad, loss


MLP_NOALLOC_MAX_ROWS = 8192


def mlp_backward_noalloc(params, X, y, pos_weight: float, grad, loss, stream=None):
    """ph_mlp_backward without any allocation: grad (MLP_NPARAM floats) and loss (1 float) are
    caller-provided device tensors; at most MLP_NOALLOC_MAX_ROWS rows."""
    _check(load().ph_mlp_backward_noalloc(_dptr(params), _dptr(X), _dptr(y), float(pos_weight), X.shape[0],
                                          _dptr(grad), _dptr(loss), _stream_ptr(stream)))
    return grad, loss


def adam_step(params, m1, m2, grad, lr, beta1, beta2, eps, step, stream=None):
    _check(load().ph_adam_step(_dptr(params), _dptr(m1), _dptr(m2), _dptr(grad), params.numel(), float(lr),
                               float(beta1), float(beta2), float(eps), int(step), _stream_ptr(stream)))


def selector_features(plan: Plan, I, E=None, stream=None):
    """Features (rows x 8, device) of the source leaves of the plan's last evaluation."""
    import torch
    n = ctypes.c_int64()
    _check(load().ph_selector_features(plan._h, _dptr(I), _dptr(E), None, 0, ctypes.byref(n),
                                       _stream_ptr(stream)))
    feats = torch.empty((max(n.value, 1), 8), dtype=torch.float32, device=I.device)
    _check(load().ph_selector_features(plan._h, _dptr(I), _dptr(E), _dptr(feats), feats.shape[0],
                                       ctypes.byref(n), _stream_ptr(stream)))
    return feats[: n.value]


def selector_fields(plan: Plan, I, targets, rows: int, ld: int = 0, out=None, stream=None):
    """Fields (rows x n_targets, device FP32, units of S) of the first ``rows`` selector rows at the
    caller-order target indices (int32 device tensor), for the I of the last selector_features call."""
    import torch
    nt = targets.numel()
    ld = ld or nt
    if out is None:
        out = torch.empty((max(rows, 1), ld), dtype=torch.float32, device=targets.device)
    _check(load().ph_selector_fields(plan._h, _dptr(I), _dptr(targets), nt, _dptr(out), ld, rows,
                                     _stream_ptr(stream)))
    return out[:rows, :nt]
