"""What the trained leaf selector gains over the paper's source rule (Sec. 3, eq. (18): keep
I >= 1e-4 max I) on held-out streamer fields: it keeps fewer sources on every field, its method
error against the FP64 direct sum over all sources stays within 1e-3 (the gate of the FP32
forms), and a call takes at most 15 % longer than the rule's (the decisions cost more time
than the fewer sources save on this workload: about 8 % measured).  The selector was trained on seeds 0-179 and calibrated on
180-199; these seeds come from the held-out range 200-249."""
import numpy as np
import pytest

import gen
from oracle import photoionization, rel_l2
from tests.helpers import plan_kwargs

pytestmark = pytest.mark.gpu

SEEDS = list(range(200, 250, 5))  # ten held-out fields


def _ms_per_call(plan, I, E, torch, calls=30, warmup=3):
    """GPU time per call over back-to-back calls (what a time-stepping caller sees); one run."""
    out = torch.empty(plan.n, dtype=torch.float32, device="cuda")
    for _ in range(warmup):
        plan.evaluate(I, E, out=out)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(calls):
        plan.evaluate(I, E, out=out)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / calls


def test_gain_over_threshold(gpu_lib):
    import torch
    from paper_2112_10059_amd.train_selector import load_selector
    w, meta = load_selector()
    wl0 = gen.config2(seed=SEEDS[0], n_axis=128)
    learned = gpu_lib.Plan(wl0.xyz, wl0.gas, dict(src_rel=meta["base_src_rel"], e_abs=3e6), selector="learned",
                           selector_weights=w, selector_logit_threshold=meta["threshold"],
                           selector_fallback_rel=1e-4, **plan_kwargs(wl0))
    rule = gpu_lib.Plan(wl0.xyz, wl0.gas, dict(src_rel=1e-4, e_abs=3e6), **plan_kwargs(wl0))
    rows = []
    for seed in SEEDS:
        print(f"gain: held-out field seed {seed}", flush=True)
        wl = gen.config2(seed=seed, n_axis=128)
        I32, E32 = wl.I.astype(np.float32), wl.E.astype(np.float32)
        tI, tE = torch.tensor(I32, device="cuda"), torch.tensor(E32, device="cuda")
        S_l, st_l = learned.evaluate(tI, tE, stats=True)
        S_t, st_t = rule.evaluate(tI, tE, stats=True)
        tg = gen.sample_targets(np.arange(wl.n), wl.xyz, wl.head, k=300, seed=seed, head_cap=300)
        ref = photoionization(wl.xyz, I32.astype(np.float64), wl.gas, h=wl.h, targets=tg)
        e_l = rel_l2(S_l.double().cpu().numpy()[tg], ref.S_t)
        e_t = rel_l2(S_t.double().cpu().numpy()[tg], ref.S_t)
        # the two plans timed in turn, three runs each; the fastest run of each counts (a run that
        # met a transient stall of the device says nothing about the plan)
        ms_l, ms_t = float("inf"), float("inf")
        for _ in range(3):
            ms_l = min(ms_l, _ms_per_call(learned, tI, tE, torch))
            ms_t = min(ms_t, _ms_per_call(rule, tI, tE, torch))
        rows.append((seed, st_l["n_src"], st_t["n_src"], e_l, e_t, ms_l, ms_t, st_l["fell_back"]))
        print(f"  sources {st_l['n_src']} (rule {st_t['n_src']}), method rel-L2 {e_l:.3e} (rule {e_t:.3e}), "
              f"{ms_l:.4f} ms per call (rule {ms_t:.4f})", flush=True)
    learned.close()
    rule.close()
    r = np.array(rows, dtype=float)
    print(f"mean sources {r[:, 1].mean():.0f} vs {r[:, 2].mean():.0f}; largest method error {r[:, 3].max():.3e} vs "
          f"{r[:, 4].max():.3e}; ms per call {r[:, 5].sum() / len(r):.4f} vs {r[:, 6].sum() / len(r):.4f}", flush=True)
    assert np.all(r[:, 7] == 0), "the selector fell back on a held-out field"
    assert np.all(r[:, 3] <= 1e-3), "method error above 1e-3"
    assert np.all(r[:, 1] < r[:, 2]), "the selector kept as many sources as the rule"
    # the time the decisions cost is not recovered on this workload (every point is a target:
    # the call's time is set by the target-side passes, and 3 % fewer sources save little
    # there): the learned call takes about 8 % longer than the rule's; this bounds it at 15 %
    assert r[:, 5].sum() <= 1.15 * r[:, 6].sum()
