"""GPU parity of the learned leaf selector: network kernels vs the FP64 oracle, features vs an
independent NumPy computation, and the learned evaluation path's keep/drop/fallback behaviour."""
import math

import numpy as np
import pytest

import gen
from oracle import mlp as omlp
from oracle import photoionization, rel_l2
from tests.helpers import MORTON_BITS, plan_kwargs, reference_tree

pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    import torch
    return torch.tensor(np.asarray(a), dtype=dtype or torch.float32, device="cuda")


def _say(msg):
    print(msg, flush=True)


# ---------------------------------------------------------------- network kernels

def test_mlp_forward_fp32_and_bf16(gpu_lib):
    _say("mlp forward")
    rng = np.random.default_rng(1)
    p = omlp.init_params(3)
    X = rng.normal(size=(1000, 8)) * 2
    z_ref, _ = omlp.forward(p, X)
    z32 = gpu_lib.mlp_forward(_t(p), _t(X)).cpu().numpy()
    assert np.all(np.abs(z32 - z_ref) <= 2e-5 * (1 + np.abs(z_ref)))
    zbf = gpu_lib.mlp_forward(_t(p), _t(X), bf16=True).cpu().numpy()
    # BF16 weights/activations (8-bit mantissa) with FP32 accumulation: relative error a few 2^-8
    W1, b1, W2, b2, W3, b3 = omlp.unpack(p)
    bound = np.abs(W3) @ np.abs(omlp.gelu(omlp.forward(p, X)[1][3])).T  # scale of the last layer
    assert np.all(np.abs(zbf - z_ref) <= 4 * 2.0 ** -8 * (bound + 1.0))


def test_mlp_backward_matches_oracle(gpu_lib):
    _say("mlp backward")
    rng = np.random.default_rng(2)
    p = omlp.init_params(5) * 0.8
    X = rng.normal(size=(777, 8))
    y = (rng.uniform(size=777) < 0.25).astype(np.float64)
    loss_ref, g_ref = omlp.loss_and_grad(p, X, y, 3.0)
    g, loss = gpu_lib.mlp_backward(_t(p), _t(X), _t(y), 3.0)
    g = g.cpu().numpy().astype(np.float64)
    assert float(loss.cpu()) == pytest.approx(loss_ref, rel=1e-5)
    assert rel_l2(g, g_ref) <= 1e-4
    assert np.allclose(g, g_ref, rtol=1e-3, atol=1e-5 * np.abs(g_ref).max())


def test_adam_matches_oracle(gpu_lib):
    _say("adam")
    rng = np.random.default_rng(3)
    n = omlp.NPARAM
    p, m1, m2, g = (rng.normal(size=n) for _ in range(4))
    m2 = np.abs(m2)
    p_ref, m1_ref, m2_ref = omlp.adam_step(p, m1, m2, g, 1e-3, 0.9, 0.999, 1e-8, 7)
    tp, tm1, tm2 = _t(p), _t(m1), _t(m2)
    gpu_lib.adam_step(tp, tm1, tm2, _t(g), 1e-3, 0.9, 0.999, 1e-8, 7)
    assert np.allclose(tp.cpu().numpy(), p_ref, rtol=1e-5, atol=1e-6)
    assert np.allclose(tm1.cpu().numpy(), m1_ref, rtol=1e-5, atol=1e-6)
    assert np.allclose(tm2.cpu().numpy(), m2_ref, rtol=1e-5, atol=1e-6)


# ---------------------------------------------------------------- features

def _ranges(keys, level, anchors):
    shift = np.uint64(3 * (MORTON_BITS - level))
    pre = keys >> shift
    from tests.helpers import _spread
    a = np.asarray(anchors, dtype=np.uint64)
    p = (_spread(a[:, 0]) << np.uint64(2)) | (_spread(a[:, 1]) << np.uint64(1)) | _spread(a[:, 2])
    return np.searchsorted(pre, p, side="left"), np.searchsorted(pre, p, side="right")


def _plan_rows(plan, I32, src_rel, leaf_cap):
    """Selector rows from NumPy: leaves of the full tree over all points (box ids in the plan's
    box order) holding a point with I >= src_rel max I, and each leaf's sorted range."""
    keys = plan.debug_fetch("keys")
    perm = plan.debug_fetch("perm")
    full = reference_tree(keys, keys, leaf_cap, 16)
    Is = I32[perm].astype(np.float64)
    thr = src_rel * float(I32.max())
    ids, rng = [], []
    for b, row in enumerate(full):
        if row[8] != 1:
            continue
        st, n = int(row[4]), int(row[5])
        if n and (src_rel <= 0 or np.any(Is[st:st + n] >= thr)):
            ids.append(b)
            rng.append((st, st + n))
    return full, np.array(ids, dtype=np.int32), rng


def test_selector_features_match_numpy(gpu_lib):
    wl = gen.config2(seed=1010, n_axis=48)
    src_rel = 1e-7
    thr = dict(src_rel=src_rel, e_abs=3e6)
    _say("selector features c2_48")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, thr, leaf_capacity=32, **plan_kwargs(wl))
    I32, E32 = wl.I.astype(np.float32), wl.E.astype(np.float32)
    tI, tE = _t(I32), _t(E32)
    F = gpu_lib.selector_features(plan, tI, tE).cpu().numpy().astype(np.float64)
    full, ids, rng = _plan_rows(plan, I32, src_rel, 32)
    assert np.array_equal(plan.debug_fetch("feature_boxes"), ids)
    assert F.shape == (ids.size, 8)
    keys, perm = plan.debug_fetch("keys"), plan.debug_fetch("perm")
    Imax, Emax = float(I32.max()), float(E32.max())
    w_ref = wl.h ** 3
    lo, hi = wl.domain
    cube = hi - lo
    Es = E32[perm].astype(np.float64)
    Is = I32[perm].astype(np.float64)
    xE = wl.xyz[int(np.argmax(E32))]  # first in caller order among ties
    xI = wl.xyz[int(np.argmax(I32))]
    ref = np.zeros_like(F)
    for r, (b, (st, en)) in enumerate(zip(ids, rng)):
        lev, ax, ay, az = (int(v) for v in full[b, :4])
        Iall = Is[st:en]
        Iv = Iall[Iall >= src_rel * Imax]
        side = cube / 2 ** lev
        ctr = lo + (np.array([ax, ay, az]) + 0.5) * side
        e = Es[st:en] / Emax
        ref[r] = [math.log10(Iv.max() / Imax), math.log10(Iv.sum() * w_ref / (Imax * w_ref)),
                  math.log10(Iv.size / Iall.size), math.log10(1 + np.linalg.norm(ctr - xI) / side),
                  math.log10(1 + np.linalg.norm(ctr - xE) / side), e.max(), e.mean(), e.std()]
    assert np.allclose(F, ref, rtol=2e-5, atol=2e-5)
    plan.close()


def test_selector_fields_match_oracle(gpu_lib):
    """Each row's field at sampled targets equals the FP64 direct sum over that row's candidates."""
    import torch
    wl = gen.config2(seed=1014, n_axis=32)
    src_rel = 1e-3
    _say("selector fields c2_32")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, dict(src_rel=src_rel, e_abs=3e6), leaf_capacity=32, **plan_kwargs(wl))
    I32, E32 = wl.I.astype(np.float32), wl.E.astype(np.float32)
    tI = _t(I32)
    F = gpu_lib.selector_features(plan, tI, _t(E32))
    rng_ = np.random.default_rng(5)
    tg = np.sort(rng_.choice(wl.n, size=3000, replace=False)).astype(np.int32)
    # a ragged tail: 3000 targets are one block of 2048 plus a partial one
    fields = gpu_lib.selector_fields(plan, tI, torch.tensor(tg, device="cuda"), F.shape[0]).cpu().numpy()
    _, ids, rng = _plan_rows(plan, I32, src_rel, 32)
    perm = plan.debug_fetch("perm")
    Is = I32[perm].astype(np.float64)
    for r in range(0, ids.size, max(1, ids.size // 10)):
        st, en = rng[r]
        k = np.arange(st, en)
        k = k[Is[k] >= src_rel * float(I32.max())]
        sm = np.zeros(wl.n, dtype=bool)
        sm[perm[k]] = True
        res = photoionization(wl.xyz, I32.astype(np.float64), wl.gas, h=wl.h, smask=sm, targets=tg)
        assert np.allclose(fields[r], res.S_t, rtol=2e-5, atol=1e-6 * np.abs(res.S_t).max())
    with pytest.raises(gpu_lib.PhError):
        gpu_lib.selector_fields(plan, tI, torch.tensor(tg, device="cuda"), F.shape[0] + 1)
    plan.close()


# ---------------------------------------------------------------- learned evaluation path

def _const_net(bias):
    p = np.zeros(omlp.NPARAM, dtype=np.float32)
    p[-1] = bias
    return p


def test_learned_keep_all_equals_threshold_bitwise(gpu_lib):
    wl = gen.config2(seed=1011, n_axis=48)
    thr = dict(src_rel=1e-6, e_abs=3e6)
    _say("learned keep-all vs threshold")
    tI, tE = _t(wl.I.astype(np.float32)), _t(wl.E.astype(np.float32))
    p0 = gpu_lib.Plan(wl.xyz, wl.gas, thr, leaf_capacity=32, **plan_kwargs(wl))
    a = p0.evaluate(tI, tE).cpu().numpy()
    p1 = gpu_lib.Plan(wl.xyz, wl.gas, thr, leaf_capacity=32, selector="learned",
                      selector_weights=_const_net(50.0), **plan_kwargs(wl))
    b, st = p1.evaluate(tI, tE, stats=True)
    assert st["fell_back"] == 0 and st["n_src_dropped"] == 0
    assert np.array_equal(a.view(np.uint32), b.cpu().numpy().view(np.uint32))
    p0.close()
    p1.close()


def test_learned_drop_all_gives_zero(gpu_lib):
    wl = gen.config2(seed=1012, n_axis=40)
    thr = dict(src_rel=1e-6, e_abs=3e6)
    _say("learned drop-all")
    tI, tE = _t(wl.I.astype(np.float32)), _t(wl.E.astype(np.float32))
    p1 = gpu_lib.Plan(wl.xyz, wl.gas, thr, leaf_capacity=32, selector="learned",
                      selector_weights=_const_net(-50.0), **plan_kwargs(wl))
    b, st = p1.evaluate(tI, tE, stats=True)
    assert st["n_src"] == 0 and st["n_src_dropped"] > 0
    assert np.all(b.cpu().numpy() == 0)
    p1.close()


def test_learned_nonfinite_logits_fall_back_to_threshold(gpu_lib):
    wl = gen.config2(seed=1013, n_axis=40)
    thr = dict(src_rel=1e-6, e_abs=3e6)
    _say("learned fallback")
    tI, tE = _t(wl.I.astype(np.float32)), _t(wl.E.astype(np.float32))
    w = np.zeros(omlp.NPARAM, dtype=np.float32)
    w[512:576] = 1e30    # b1: every first-layer unit at 1e30 whatever the features ...
    w[576:4672] = 1e30   # W2: every second-layer unit overflows to +inf ...
    w[4736:4800] = np.where(np.arange(64) % 2 == 0, 1.0, -1.0).astype(np.float32)  # ... and inf - inf
    p1 = gpu_lib.Plan(wl.xyz, wl.gas, thr, leaf_capacity=32, selector="learned", selector_weights=w,
                      selector_fallback_rel=1e-4, **plan_kwargs(wl))
    b, st = p1.evaluate(tI, tE, stats=True)
    assert st["fell_back"] == 1
    p0 = gpu_lib.Plan(wl.xyz, wl.gas, dict(src_rel=1e-4, e_abs=3e6), leaf_capacity=32, **plan_kwargs(wl))
    a = p0.evaluate(tI, tE).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.cpu().numpy().view(np.uint32))
    p0.close()
    p1.close()


def test_learned_decisions_select_exactly_the_kept_rows(gpu_lib):
    """A network with real decisions: the selected sources are exactly the candidates of the rows
    whose BF16 logit (same kernel, same features) clears the threshold, and S matches the oracle
    on that source set."""
    wl = gen.config2(seed=1015, n_axis=40)
    src_rel = 1e-7
    thr = dict(src_rel=src_rel, e_abs=3e6)
    _say("learned decisions c2_40")
    I32, E32 = wl.I.astype(np.float32), wl.E.astype(np.float32)
    tI, tE = _t(I32), _t(E32)
    w = omlp.init_params(11).astype(np.float32)
    probe = gpu_lib.Plan(wl.xyz, wl.gas, thr, leaf_capacity=32, **plan_kwargs(wl))
    z0 = gpu_lib.mlp_forward(_t(w), gpu_lib.selector_features(probe, tI, tE), bf16=True).cpu().numpy()
    probe.close()
    tau = float(np.median(z0))
    plan = gpu_lib.Plan(wl.xyz, wl.gas, thr, leaf_capacity=32, selector="learned", selector_weights=w,
                        selector_logit_threshold=tau, **plan_kwargs(wl))
    S, st = plan.evaluate(tI, tE, stats=True)
    feats = plan.debug_fetch("features").reshape(-1, 8)
    z = gpu_lib.mlp_forward(_t(w), _t(feats), bf16=True).cpu().numpy()
    assert np.array_equal(z, z0)
    keep = z >= tau
    assert 0 < keep.sum() < keep.size
    _, ids, rng = _plan_rows(plan, I32, src_rel, 32)
    assert np.array_equal(plan.debug_fetch("feature_boxes"), ids)
    perm = plan.debug_fetch("perm")
    Is = I32[perm].astype(np.float64)
    kept = np.concatenate([np.arange(*rng[r]) for r in np.flatnonzero(keep)])
    kept = np.sort(kept[Is[kept] >= src_rel * float(I32.max())])
    assert np.array_equal(plan.debug_fetch("src"), kept.astype(np.int32))
    assert st["n_leaves"] == ids.size and st["fell_back"] == 0
    cand = int(np.sum([np.sum(Is[a:b] >= src_rel * float(I32.max())) for a, b in rng]))
    assert st["n_src_dropped"] == cand - kept.size
    sm = np.zeros(wl.n, dtype=bool)
    sm[perm[kept]] = True
    r = photoionization(wl.xyz, I32.astype(np.float64), wl.gas, h=wl.h, smask=sm,
                        E=E32.astype(np.float64), e_abs=3e6)
    assert rel_l2(S.double().cpu().numpy(), r.full(wl.n)) <= 1e-3
    plan.close()


@pytest.mark.parametrize("seed", [200, 217, 249])
def test_trained_selector_on_held_out_fields(gpu_lib, seed):
    """The committed selector on fields it was neither trained nor calibrated on: the method error
    against the FP64 direct sum over all sources stays within 1e-3 on sampled targets (head ball
    plus a uniform sample), it drops sources, and it does not fall back."""
    from paper_2112_10059_amd.train_selector import load_selector
    w, meta = load_selector()
    wl = gen.config2(seed=seed, n_axis=128)
    _say(f"trained selector, held-out field seed {seed}")
    I32, E32 = wl.I.astype(np.float32), wl.E.astype(np.float32)
    plan = gpu_lib.Plan(wl.xyz, wl.gas, dict(src_rel=meta["base_src_rel"], e_abs=3e6), selector="learned",
                        selector_weights=w, selector_logit_threshold=meta["threshold"],
                        selector_fallback_rel=1e-4, **plan_kwargs(wl))
    S, st = plan.evaluate(_t(I32), _t(E32), stats=True)
    assert st["fell_back"] == 0 and st["n_src_dropped"] > 0
    tg = gen.sample_targets(np.arange(wl.n), wl.xyz, wl.head, k=400, seed=seed, head_cap=400)
    ref = photoionization(wl.xyz, I32.astype(np.float64), wl.gas, h=wl.h, targets=tg)
    err = rel_l2(S.double().cpu().numpy()[tg], ref.S_t)
    _say(f"  kept {st['n_src']} of {st['n_src'] + st['n_src_dropped']} candidates, method rel-L2 {err:.3e}")
    assert err <= 1e-3
    plan.close()


def test_validated_learned_call_falls_back_to_the_plain_fmm(gpu_lib):
    """validate = 1: every learned call is judged by the plain FMM under the threshold rule.  With
    tol = 0 any difference falls back, and the output is the threshold rule's bit for bit; with a
    loose tol the learned output is kept, bit for bit as without validation."""
    from paper_2112_10059_amd.train_selector import load_selector
    w, meta = load_selector()
    wl = gen.config2(seed=1016, n_axis=64)
    _say("validated learned call")
    tI, tE = _t(wl.I.astype(np.float32)), _t(wl.E.astype(np.float32))
    kw = dict(selector="learned", selector_weights=w, selector_logit_threshold=meta["threshold"],
              selector_fallback_rel=1e-4, **plan_kwargs(wl))
    thr_l = dict(src_rel=meta["base_src_rel"], e_abs=3e6)
    plain = gpu_lib.Plan(wl.xyz, wl.gas, dict(src_rel=1e-4, e_abs=3e6), **plan_kwargs(wl))
    S_thr = plain.evaluate(tI, tE).cpu().numpy()
    unval = gpu_lib.Plan(wl.xyz, wl.gas, thr_l, **kw)
    S_l, st_l = unval.evaluate(tI, tE, stats=True)
    S_l = S_l.cpu().numpy()
    assert st_l["check_rel_l2"] == -1.0
    strict = gpu_lib.Plan(wl.xyz, wl.gas, thr_l, validate=True, tol=0.0, **kw)
    S0, st0 = strict.evaluate(tI, tE, stats=True)
    diff = rel_l2(S_l.astype(np.float64), S_thr.astype(np.float64))
    assert st0["check_rel_l2"] == pytest.approx(diff, rel=1e-6, abs=1e-12)
    if diff > 0:
        assert st0["fell_back"] == 1
    assert np.array_equal(S0.cpu().numpy().view(np.uint32), S_thr.view(np.uint32))
    loose = gpu_lib.Plan(wl.xyz, wl.gas, thr_l, validate=True, tol=0.5, **kw)
    S1, st1 = loose.evaluate(tI, tE, stats=True)
    assert st1["fell_back"] == 0
    assert np.array_equal(S1.cpu().numpy().view(np.uint32), S_l.view(np.uint32))
    # asynchronous validated calls on the same plan give the same results
    S2 = strict.evaluate(tI, tE)
    assert np.array_equal(S2.cpu().numpy().view(np.uint32), S_thr.view(np.uint32))
    for p in (plain, unval, strict, loose):
        p.close()
