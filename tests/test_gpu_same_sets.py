"""Two evaluations per time step on one set of sources and targets (Sec. 5): a call on the
previous call's sets (ph_evaluate_same_sets) against a full call and the FP64 oracle over those
sets, its statistics, its speed, and its error paths."""
import numpy as np
import pytest

import gen
from oracle import photoionization, rel_l2, source_mask, target_mask
from tests.helpers import plan_kwargs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _t(a, dtype=None):
    import torch
    return torch.tensor(np.asarray(a), dtype=dtype or torch.float32, device="cuda")


def _ms(fn, torch, calls=30):
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(calls):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / calls


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_same_sets_equals_full_call_on_same_input(gpu_lib, precision):
    """The same I twice: the second call (previous sets) equals the first bit for bit, with the
    same counts and work."""
    import torch
    wl = gen.config2(seed=1003, n_axis=64)
    dt = torch.float64 if precision == "fp64" else torch.float32
    I = _t(wl.I, dt)
    E = _t(wl.E.astype(np.float32))
    _say(f"same sets, {precision}, identical input")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, wl.thresholds, precision=precision, **plan_kwargs(wl))
    S1, st1 = plan.evaluate(I, E, stats=True)
    S2, st2 = plan.evaluate(I, same_sets=True, stats=True)
    assert np.array_equal(S1.cpu().numpy().view(np.uint8), S2.cpu().numpy().view(np.uint8))
    for k in ("n_src", "n_tgt", "n_boxes", "levels"):
        assert st1[k] == st2[k]
    assert st1["work"] == st2["work"]
    plan.close()


def test_same_sets_new_strengths_match_oracle(gpu_lib):
    """Second call of a time step: the strengths change by a few per cent (and the maximum
    moves), the sets stay those of the first call; the result is the FP64 sum over those sets."""
    import torch
    wl = gen.config2(seed=1004, n_axis=64)
    I1 = wl.I.astype(np.float32)
    E1 = wl.E.astype(np.float32)
    x = wl.xyz
    I2 = (I1 * (1.0 + 0.05 * np.sin(7.0 * x[:, 0]) * np.cos(5.0 * x[:, 2]))).astype(np.float32)
    _say("same sets, new strengths")
    thr = dict(src_rel=1e-4, e_abs=3e6, e_applied=5e6, e_rel=0.005)  # the field rule of Sec. 5
    plan = gpu_lib.Plan(wl.xyz, wl.gas, thr, **plan_kwargs(wl))
    plan.evaluate(_t(I1), _t(E1))
    out = _t(np.full(wl.n, 7.0, dtype=np.float32))  # stale values: the call clears the non-targets
    S2, st = plan.evaluate(_t(I2), out=out, same_sets=True, stats=True)
    S2 = S2.double().cpu().numpy()
    smask = source_mask(I1.astype(np.float64), thr["src_rel"])
    tmask = target_mask(E1.astype(np.float64), thr["e_abs"], thr["e_applied"], thr["e_rel"])
    assert 0 < tmask.sum() < wl.n
    assert st["n_src"] == int(smask.sum()) and st["n_tgt"] == int(tmask.sum())
    assert np.all(S2[~tmask] == 0)
    tg = gen.sample_targets(np.flatnonzero(tmask), wl.xyz, wl.head, k=2000, seed=9, head_cap=500)
    ref = photoionization(wl.xyz, I2.astype(np.float64), wl.gas, h=wl.h, smask=smask, targets=tg)
    err = rel_l2(S2[tg], ref.S_t)
    _say(f"  rel-L2 {err:.3e} against the oracle over the first call's sets")
    assert err <= 1e-3
    plan.close()


def test_same_sets_learned_and_speed(gpu_lib):
    """On the 128^3 streamer workload with the learned selector: the call on the previous sets
    equals a full call for the same I bit for bit, and takes less time than a full call."""
    import torch
    from paper_2112_10059_amd.train_selector import load_selector
    w, meta = load_selector()
    wl = gen.config2(seed=1000, n_axis=128)
    I, E = _t(wl.I.astype(np.float32)), _t(wl.E.astype(np.float32))
    _say("same sets, learned selector, 128^3")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, dict(src_rel=meta["base_src_rel"], e_abs=3e6), selector="learned",
                        selector_weights=w, selector_logit_threshold=meta["threshold"],
                        selector_fallback_rel=1e-4, **plan_kwargs(wl))
    out1 = torch.empty(wl.n, dtype=torch.float32, device="cuda")
    out2 = torch.empty_like(out1)
    plan.evaluate(I, E, out=out1)
    plan.evaluate(I, out=out2, same_sets=True)
    assert np.array_equal(out1.cpu().numpy().view(np.uint32), out2.cpu().numpy().view(np.uint32))
    # the fastest of three runs each, in turn (a transient stall of the device says nothing)
    full, same = float("inf"), float("inf")
    for _ in range(3):
        full = min(full, _ms(lambda: plan.evaluate(I, E, out=out1), torch))
        same = min(same, _ms(lambda: plan.evaluate(I, out=out2, same_sets=True), torch))
    _say(f"  full call {full:.4f} ms, call on the previous sets {same:.4f} ms")
    assert same < full
    plan.close()


def test_same_sets_error_paths(gpu_lib):
    import torch
    wl = gen.config1()
    _say("same sets: error paths")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, wl.thresholds, leaf_capacity=27, **plan_kwargs(wl))
    I = wl.I.astype(np.float32)
    with pytest.raises(gpu_lib.PhError) as e:
        plan.evaluate(_t(I), same_sets=True)
    assert e.value.status == gpu_lib.PH_EINVAL
    plan.evaluate(_t(I))
    plan.set_targets(np.ones(wl.n, dtype=bool))
    with pytest.raises(gpu_lib.PhError) as e:
        plan.evaluate(_t(I), same_sets=True)
    assert e.value.status == gpu_lib.PH_EINVAL
    plan.evaluate(_t(I))
    bad = I.copy()
    bad[int(np.argmax(I))] = np.nan  # a selected source
    with pytest.raises(gpu_lib.PhError) as e:
        plan.evaluate(_t(bad), same_sets=True, stats=True)
    assert e.value.status == gpu_lib.PH_ENUMERIC
    plan.close()
    direct = gpu_lib.Plan(wl.xyz, wl.gas, wl.thresholds, method="direct", **plan_kwargs(wl))
    direct.evaluate(_t(I))
    with pytest.raises(gpu_lib.PhError) as e:
        direct.evaluate(_t(I), same_sets=True)
    assert e.value.status == gpu_lib.PH_EUNSUPPORTED
    direct.close()
