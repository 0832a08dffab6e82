"""Degenerate and edge inputs of the HIP path, against the FP64 oracle or exact values."""
import numpy as np
import pytest

import gen
from oracle import photoionization, rel_l2
from tests.helpers import plan_kwargs

pytestmark = pytest.mark.gpu


def _t(a, dtype):
    import torch
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_all_zero_sources_give_exact_zero(gpu_lib, precision):
    import torch
    wl = gen.config1()
    _say(f"zero I {precision}")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, dict(src_rel=1e-4), precision=precision, leaf_capacity=27, **plan_kwargs(wl))
    dt = torch.float64 if precision == "fp64" else torch.float32
    S = plan.evaluate(_t(np.zeros(wl.n), dt)).double().cpu().numpy()
    assert np.all(S == 0.0)
    plan.check()
    plan.close()


def test_no_active_targets(gpu_lib):
    import torch
    wl = gen.config2(seed=1020, n_axis=32)
    _say("no targets")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, dict(src_rel=1e-4, e_abs=1e12), **plan_kwargs(wl))
    out = torch.full((wl.n,), 7.0, dtype=torch.float32, device="cuda")
    S, st = plan.evaluate(_t(wl.I, torch.float32), _t(wl.E, torch.float32), out=out, stats=True)
    assert st["n_tgt"] == 0 and st["n_src"] > 0
    assert np.all(S.cpu().numpy() == 0.0)
    plan.close()


def test_single_source_is_the_kernel_row(gpu_lib):
    """src_rel = 1 keeps only the largest I: S is that one column of the quadrature."""
    import torch
    wl = gen.config2(seed=1021, n_axis=32)
    _say("single source")
    I = wl.I.copy()
    I[np.argmax(I)] *= 2.0  # a unique maximum
    plan = gpu_lib.Plan(wl.xyz, wl.gas, dict(src_rel=1.0), precision="fp64", **plan_kwargs(wl))
    S, st = plan.evaluate(_t(I, torch.float64), stats=True)
    assert st["n_src"] == 1
    ref = photoionization(wl.xyz, I, wl.gas, h=wl.h, src_rel=1.0)
    assert rel_l2(S.cpu().numpy(), ref.full(wl.n)) <= 1e-6
    plan.close()


@pytest.mark.parametrize("n", [1, 2, 65])
def test_tiny_clouds(gpu_lib, n):
    """A handful of points (one box; one leaf split into children for 65): the direct sum exactly."""
    import torch
    rng = np.random.default_rng(n)
    xyz = rng.uniform(0.2, 0.8, size=(n, 3))
    w = rng.uniform(1e-4, 1e-3, size=n)
    I = rng.uniform(0.5, 2.0, size=n) * 1e20
    _say(f"tiny cloud n={n}")
    plan = gpu_lib.Plan(xyz, gen.GAS_760, dict(src_rel=0.0), precision="fp64", w=w, self_coeff=0.0,
                        cube_lo=(0, 0, 0), cube_size=1.0)
    S = plan.evaluate(_t(I, torch.float64)).cpu().numpy()
    ref = photoionization(xyz, I, gen.GAS_760, w=w).full(n)
    if n == 1:
        assert S[0] == 0.0 and ref[0] == 0.0
    else:
        assert rel_l2(S, ref) <= 1e-6
    plan.close()


def test_coincident_points_are_skipped_pairs(gpu_lib):
    """Duplicated points in a cloud: pairs at distance zero contribute nothing, on both sides."""
    import torch
    wl = gen.config3(seed=2002, n=30_000, src_rel=0.0)
    xyz = wl.xyz.copy()
    xyz[100:200] = xyz[5]           # a stack of 101 coincident points
    xyz[1000:1010] = xyz[20000]
    _say("coincident points")
    plan = gpu_lib.Plan(xyz, wl.gas, dict(src_rel=0.0), precision="fp64", w=wl.w, self_coeff=0.0,
                        cube_lo=(0, 0, 0), cube_size=4.0)
    S = plan.evaluate(_t(wl.I, torch.float64)).cpu().numpy()
    tg = np.unique(np.concatenate([np.arange(95, 205), np.arange(995, 1015),
                                   np.random.default_rng(1).choice(wl.n, 300, replace=False)]))
    ref = photoionization(xyz, wl.I, wl.gas, w=wl.w, targets=tg)
    assert rel_l2(S[tg], ref.S_t) <= 1e-6
    plan.close()


def test_non_finite_source_is_reported(gpu_lib):
    import torch
    wl = gen.config1()
    _say("NaN in I")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, wl.thresholds, leaf_capacity=27, **plan_kwargs(wl))
    I = wl.I.astype(np.float32)
    I[17] = np.nan
    plan.evaluate(_t(I, torch.float32))
    with pytest.raises(gpu_lib.PhError) as e:
        plan.check()
    assert e.value.status == 4  # PH_ENUMERIC
    plan.close()


def test_error_of_an_earlier_call_stays_until_checked(gpu_lib):
    """A bad call followed by a good one: the next check still reports the bad one (the error
    word is sticky across calls), and a second check finds nothing left."""
    import torch
    wl = gen.config1()
    _say("sticky error: bad call, good call, check, check")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, wl.thresholds, leaf_capacity=27, **plan_kwargs(wl))
    good = wl.I.astype(np.float32)
    bad = good.copy()
    bad[300] = -1.0
    plan.evaluate(_t(bad, torch.float32))
    S = plan.evaluate(_t(good, torch.float32))
    with pytest.raises(gpu_lib.PhError) as e:
        plan.check()
    assert e.value.status == gpu_lib.PH_ENUMERIC
    plan.check()  # cleared by the first check
    ref = photoionization(wl.xyz, good.astype(np.float64), wl.gas, h=wl.h).full(wl.n)
    assert rel_l2(S.double().cpu().numpy(), ref) <= 1e-3
    # a call with statistics reports its own fault at once
    with pytest.raises(gpu_lib.PhError) as e:
        plan.evaluate(_t(bad, torch.float32), stats=True)
    assert e.value.status == gpu_lib.PH_ENUMERIC
    plan.close()


def test_list_overflow_is_reported_and_stays_in_bounds(gpu_lib, monkeypatch):
    """Interaction lists far too small for the tree: the ranges are cut at the capacity (no read
    past a list), the call completes, and the overflow is reported as PH_ENOMEM."""
    import torch
    wl = gen.config2(seed=1022, n_axis=32)
    monkeypatch.setenv("PH_LIST_ENTRIES_PER_BOX", "1")
    _say("list overflow: one list entry per box")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, dict(src_rel=0.0), leaf_capacity=16, **plan_kwargs(wl))
    monkeypatch.delenv("PH_LIST_ENTRIES_PER_BOX")
    I = _t(wl.I.astype(np.float32), torch.float32)
    plan.evaluate(I)
    with pytest.raises(gpu_lib.PhError) as e:
        plan.check()
    assert e.value.status == gpu_lib.PH_ENOMEM
    with pytest.raises(gpu_lib.PhError) as e:
        plan.evaluate(I, stats=True)
    assert e.value.status == gpu_lib.PH_ENOMEM
    plan.close()
