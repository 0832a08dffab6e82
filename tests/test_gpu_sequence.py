"""A plan reused across calls whose inputs (and with them the selected sources, the tree, the
lists and the V/X target boxes) change from call to call gives, at every call, exactly the
output of a fresh plan on the same input: nothing of an earlier call (check values, V-list
slots, list ranges, call-tagged boxes) leaks into a later one, whichever precision's kernels
run (FP32 with the composite L2L, which reads only the check values written in the call,
split BF16, and FP64 with the per-level L2L)."""
import numpy as np
import pytest

import gen
from tests.helpers import plan_kwargs

pytestmark = pytest.mark.gpu


def _inputs(wl, k):
    """Input k: the field and the intensities moved and rescaled, so the source set changes."""
    rng = np.random.default_rng(300 + k)
    # a power of I / max I changes the ratios to the maximum, so the relative rule keeps another
    # count (the values stay within FP32 range)
    Ir = np.roll(wl.I, 7 * k, axis=0)
    I = (Ir / Ir.max()) ** (1.0 + 0.15 * k) * Ir.max() * (1.0 + 0.5 * k)
    I = I * (1.0 + 0.05 * rng.random(I.shape))
    E = np.roll(wl.E, -11 * k, axis=0)
    return I, E.astype(np.float32)


@pytest.mark.parametrize("precision", ["fp32", "bf16split", "fp64"])
def test_reused_plan_equals_fresh_plan(gpu_lib, precision):
    import torch
    wl = gen.config2(seed=1031, n_axis=64)
    thr = dict(src_rel=1e-5, e_abs=3e6)
    kw = dict(leaf_capacity=64, precision=precision, **plan_kwargs(wl))
    dt = torch.float64 if precision == "fp64" else torch.float32
    print(f"reused plan vs fresh plans, {precision}", flush=True)
    pr = gpu_lib.Plan(wl.xyz, wl.gas, thr, **kw)
    n_src = set()
    # a large source set first, then smaller and shifted ones, then the first again
    for k in (3, 0, 1, 2, 3):
        I, E = _inputs(wl, k)
        tI = torch.tensor(I, dtype=dt, device="cuda")
        tE = torch.tensor(E, dtype=torch.float32, device="cuda")
        got, st = pr.evaluate(tI, tE, stats=True)
        pf = gpu_lib.Plan(wl.xyz, wl.gas, thr, **kw)
        ref = pf.evaluate(tI, tE)
        torch.cuda.synchronize()
        n_src.add(st["n_src"])
        g = got.cpu().numpy()
        r = ref.cpu().numpy()
        print(f"  input {k}: n_src {st['n_src']}", flush=True)
        assert np.isfinite(g).all()
        assert np.array_equal(g.view(np.uint64 if precision == "fp64" else np.uint32),
                              r.view(np.uint64 if precision == "fp64" else np.uint32)), k
        pf.close()
    assert len(n_src) >= 3  # the calls saw different source sets
    pr.close()
