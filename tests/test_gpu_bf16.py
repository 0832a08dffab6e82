"""GPU parity of the split-BF16 M2L form (hi/lo operands on the BF16 matrix cores, FP32 accumulate)."""
import numpy as np
import pytest

import gen
from oracle import photoionization, rel_l2
from tests.helpers import plan_kwargs

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.tensor(np.asarray(a, dtype=np.float32), device="cuda")


def _say(msg):
    print(msg, flush=True)


def test_bf16split_matches_fp32_and_oracle(gpu_lib):
    wl = gen.config2(seed=1030, n_axis=64)
    _say("bf16 split vs fp32, c2_64")
    I32, E32 = wl.I.astype(np.float32), wl.E.astype(np.float32)
    out = {}
    for prec in ("fp32", "bf16split"):
        plan = gpu_lib.Plan(wl.xyz, wl.gas, wl.thresholds, precision=prec, **plan_kwargs(wl))
        out[prec] = plan.evaluate(_t(I32), _t(E32)).double().cpu().numpy()
        plan.close()
    d = rel_l2(out["bf16split"], out["fp32"])
    _say(f"  split vs fp32 rel-L2 {d:.3e}")
    assert 0.0 < d <= 1e-4  # a different computation, within the split's 2^-16 per product
    r = photoionization(wl.xyz, I32.astype(np.float64), wl.gas, h=wl.h, src_rel=1e-4, E=E32.astype(np.float64),
                        e_abs=3e6)
    err = rel_l2(out["bf16split"], r.full(wl.n))
    _say(f"  split vs oracle rel-L2 {err:.3e}")
    assert err <= 1e-3


def _c5_sample(wl, k, seed):
    cloud = wl.meta["cloud"]
    near_cloud = np.flatnonzero(np.abs(np.linalg.norm(wl.xyz - cloud[None, :], axis=1) - 0.2) < 0.03)
    rng = np.random.default_rng(seed)
    pick = rng.choice(near_cloud, size=min(200, near_cloud.size), replace=False)
    return np.unique(np.concatenate([gen.sample_targets(np.arange(wl.n), wl.xyz, wl.head, k=k, seed=seed,
                                                        head_radius=0.1, head_cap=200), pick]))


def test_c5_256_bf16split_threshold(gpu_lib):
    """The 256^3 head + plasma-cloud grid, sources I >= 1e-4 max I, split-BF16 M2L, sampled targets."""
    wl = gen.config5()
    _say("c5 256^3 bf16 split, threshold 1e-4")
    I32, E32 = wl.I.astype(np.float32), wl.E.astype(np.float32)
    plan = gpu_lib.Plan(wl.xyz, wl.gas, wl.thresholds, precision="bf16split", **plan_kwargs(wl))
    S, st = plan.evaluate(_t(I32), _t(E32), stats=True)
    _say(f"  n_src {st['n_src']} levels {st['levels']} boxes {st['n_boxes']}")
    tg = _c5_sample(wl, 400, 9)
    r = photoionization(wl.xyz, I32.astype(np.float64), wl.gas, h=wl.h, src_rel=1e-4, E=E32.astype(np.float64),
                        e_abs=3e6, targets=tg)
    assert int(r.smask.sum()) == st["n_src"]
    err = rel_l2(S.double().cpu().numpy()[tg], r.S_t)
    _say(f"  rel-L2 {err:.3e} on {tg.size} targets")
    assert err <= 1e-3
    plan.close()


def test_c5_256_learned_bf16split(gpu_lib):
    """The 256^3 grid with the committed learned selector (trained on the 128^3 streamer fields) and
    split-BF16 M2L: within 1e-3 of the FP64 direct sum over all sources on sampled targets, or the
    selector reports its fallback and then the threshold rule's result is checked."""
    from paper_2112_10059_amd.train_selector import load_selector
    w, meta = load_selector()
    wl = gen.config5()
    _say("c5 256^3 learned + bf16 split")
    I32, E32 = wl.I.astype(np.float32), wl.E.astype(np.float32)
    plan = gpu_lib.Plan(wl.xyz, wl.gas, dict(src_rel=meta["base_src_rel"], e_abs=3e6), precision="bf16split",
                        selector="learned", selector_weights=w, selector_logit_threshold=meta["threshold"],
                        selector_fallback_rel=1e-4, **plan_kwargs(wl))
    S, st = plan.evaluate(_t(I32), _t(E32), stats=True)
    _say(f"  kept {st['n_src']} dropped {st['n_src_dropped']} rows {st['n_leaves']} fell back {st['fell_back']}")
    tg = _c5_sample(wl, 200, 10)
    r = photoionization(wl.xyz, I32.astype(np.float64), wl.gas, h=wl.h, targets=tg)
    err = rel_l2(S.double().cpu().numpy()[tg], r.S_t)
    _say(f"  method rel-L2 vs all sources {err:.3e} on {tg.size} targets")
    assert err <= 1e-3
    plan.close()
