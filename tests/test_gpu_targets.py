"""Caller-supplied target sets (the demand-oriented second strategy of Sec. 3, Sec. 4.1): S is
evaluated only at the given points, intersected with the field rules, and 0 elsewhere; parity
against the FP64 oracle on those targets, and bit-exact target masks."""
import numpy as np
import pytest

import gen
from oracle import photoionization, rel_l2, source_mask, target_mask
from tests.helpers import plan_kwargs

pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    import torch
    return torch.tensor(np.asarray(a), dtype=dtype or torch.float32, device="cuda")


def _planes_and_line(wl, n_axis):
    """Three orthogonal cell planes through the head and the axis line through it (the cross
    sections and line of interest of a streamer study)."""
    h = wl.h
    idx = np.floor((wl.xyz - wl.domain[0]) / h).astype(np.int64)
    hidx = np.floor((wl.head - wl.domain[0]) / h).astype(np.int64)
    m = (idx[:, 0] == hidx[0]) | (idx[:, 1] == hidx[1]) | (idx[:, 2] == hidx[2])
    line = (idx[:, 0] == hidx[0] + 3) & (idx[:, 1] == hidx[1] - 2)
    return m | line


@pytest.mark.parametrize("precision,tol,rule", [("fp32", 1e-3, "abs"), ("fp64", 1e-6, "abs"), ("fp32", 1e-3, "rel")])
def test_target_set_parity(gpu_lib, precision, tol, rule):
    import torch
    wl = gen.config2(seed=1041, n_axis=64)
    thr = dict(src_rel=1e-4, e_abs=3e6) if rule == "abs" else dict(src_rel=1e-4, e_applied=5e6, e_rel=0.005)
    print(f"target set {precision} {rule}", flush=True)
    dt = torch.float64 if precision == "fp64" else torch.float32
    plan = gpu_lib.Plan(wl.xyz, wl.gas, thr, precision=precision, **plan_kwargs(wl))
    mask = _planes_and_line(wl, 64)
    plan.set_targets(mask)
    Iin = wl.I if precision == "fp64" else wl.I.astype(np.float32).astype(np.float64)
    E32 = wl.E.astype(np.float32)
    S, st = plan.evaluate(_t(Iin, dt), _t(E32), stats=True)
    S = S.double().cpu().numpy()
    tm = target_mask(E32.astype(np.float64), thr.get("e_abs", -1.0), thr.get("e_applied", 0.0),
                     thr.get("e_rel", -1.0)) & mask
    assert st["n_tgt"] == int(tm.sum()) and 0 < st["n_tgt"] < wl.n
    perm = plan.debug_fetch("perm")
    assert np.array_equal(plan.debug_fetch("tgt"), np.flatnonzero(tm[perm]).astype(np.int32))
    assert np.all(S[~tm] == 0.0)
    r = photoionization(wl.xyz, Iin, wl.gas, h=wl.h, src_rel=1e-4, targets=np.flatnonzero(tm))
    err = rel_l2(S[tm], r.S_t)
    print(f"  {int(tm.sum())} targets, rel-L2 {err:.3e}", flush=True)
    assert err <= tol
    # back to every point: the same as a plan that never had a target set
    plan.set_targets(None)
    S2 = plan.evaluate(_t(Iin, dt), _t(E32)).double().cpu().numpy()
    fresh = gpu_lib.Plan(wl.xyz, wl.gas, thr, precision=precision, **plan_kwargs(wl))
    S3 = fresh.evaluate(_t(Iin, dt), _t(E32)).double().cpu().numpy()
    assert np.array_equal(S2, S3)
    plan.close()
    fresh.close()


def test_target_set_at_full_size(gpu_lib):
    """The streamer workload on the 128^3 grid with three planes and a line as the target set:
    parity on sampled targets, every other point exactly 0."""
    import torch
    wl = gen.config2(seed=1000, n_axis=128)
    print("target set 128^3", flush=True)
    plan = gpu_lib.Plan(wl.xyz, wl.gas, wl.thresholds, **plan_kwargs(wl))
    mask = _planes_and_line(wl, 128)
    plan.set_targets(mask)
    I32 = wl.I.astype(np.float32)
    S, st = plan.evaluate(_t(I32), _t(wl.E.astype(np.float32)), stats=True)
    S = S.double().cpu().numpy()
    assert st["n_tgt"] == int(mask.sum())
    assert np.all(S[~mask] == 0.0)
    tg = gen.sample_targets(np.flatnonzero(mask), wl.xyz, wl.head, k=3000, head_cap=3000)
    r = photoionization(wl.xyz, I32.astype(np.float64), wl.gas, h=wl.h, src_rel=1e-4, targets=tg)
    assert rel_l2(S[tg], r.S_t) <= 1e-3
    with pytest.raises(gpu_lib.PhError):
        plan.set_targets(mask[:-1])
    plan.close()
