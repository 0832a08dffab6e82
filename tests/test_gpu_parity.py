"""GPU parity of the HIP path (through the C ABI) against NumPy integer references and the FP64 oracle."""
import math

import numpy as np
import pytest

import gen
from oracle import photoionization, rel_l2, source_mask, target_mask
from tests.helpers import morton_keys, plan_kwargs, reference_tree

pytestmark = pytest.mark.gpu


def _tensor(a, dtype):
    import torch
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def _say(msg):
    print(msg, flush=True)


# ---------------------------------------------------------------- integer work: bit-exact

@pytest.mark.parametrize("cfg", ["c1", "c2_48"])
def test_morton_sort_bitexact(gpu_lib, cfg):
    wl = gen.config1() if cfg == "c1" else gen.config2(seed=1000, n_axis=48)
    _say(f"sort {cfg} n={wl.n}")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, wl.thresholds, **plan_kwargs(wl))
    lo, hi = wl.domain
    keys = morton_keys(wl.xyz, (lo, lo, lo), hi - lo)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(plan.debug_fetch("keys"), keys[order])
    assert np.array_equal(plan.debug_fetch("perm"), order.astype(np.int32))
    plan.close()


def test_morton_sort_ties_and_cloud(gpu_lib):
    """Point cloud with duplicated points: equal keys keep caller order (stable)."""
    rng = np.random.default_rng(4)
    xyz = rng.uniform(0, 1, size=(30_001, 3))
    xyz[1000:1100] = xyz[7]  # 100 copies of one point
    _say("sort cloud n=30001")
    plan = gpu_lib.Plan(xyz, gen.GAS_760, dict(src_rel=0.0), w=np.full(len(xyz), 1e-6), self_coeff=0.0,
                        cube_lo=(0, 0, 0), cube_size=1.0)
    keys = morton_keys(xyz, (0, 0, 0), 1.0)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(plan.debug_fetch("perm"), order.astype(np.int32))
    plan.close()


@pytest.mark.parametrize("src_rel,e_abs,e_rel", [(1e-4, 3e6, -1.0), (1e-3, -1.0, 0.005), (0.0, 1.2e7, -1.0)])
def test_selection_and_tree_bitexact(gpu_lib, src_rel, e_abs, e_rel):
    import torch
    wl = gen.config2(seed=1001, n_axis=48)
    thr = dict(src_rel=src_rel, e_abs=e_abs, e_applied=5e6, e_rel=e_rel)
    _say(f"selection/tree c2_48 thr={thr}")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, thr, **plan_kwargs(wl, leaf_capacity=32))
    I32 = wl.I.astype(np.float32)
    E32 = wl.E.astype(np.float32)
    S = plan.evaluate(_tensor(I32, torch.float32), _tensor(E32, torch.float32))
    torch.cuda.synchronize()
    perm = plan.debug_fetch("perm")
    smask = source_mask(I32.astype(np.float64), src_rel)
    tmask = target_mask(E32.astype(np.float64), e_abs, 5e6, e_rel)
    src_sorted = np.flatnonzero(smask[perm])
    tgt_sorted = np.flatnonzero(tmask[perm])
    assert np.array_equal(plan.debug_fetch("src"), src_sorted.astype(np.int32))
    assert np.array_equal(plan.debug_fetch("tgt"), tgt_sorted.astype(np.int32))
    keys = plan.debug_fetch("keys")
    lvl = plan.debug_fetch("level_start")
    ref = reference_tree(keys[src_sorted], keys[tgt_sorted], 32, len(lvl) - 2)
    got = plan.debug_fetch("boxes")
    # columns: level, ax, ay, az, s_first, s_cnt, t_first, t_cnt, parent, flags
    assert got.shape[0] == ref.shape[0]
    assert np.array_equal(got[:, :8], ref[:, :8])
    assert np.array_equal(got[:, 9] & 1, ref[:, 8])
    # inactive targets are exactly zero
    assert np.all(S.cpu().numpy()[~tmask] == 0)
    plan.close()


# ---------------------------------------------------------------- direct sum

@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_direct_c1(gpu_lib, precision, tol):
    import torch
    wl = gen.config1()
    _say(f"direct c1 {precision}")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, wl.thresholds, method="direct", precision=precision, **plan_kwargs(wl))
    dt = torch.float64 if precision == "fp64" else torch.float32
    Iin = wl.I if precision == "fp64" else wl.I.astype(np.float32).astype(np.float64)
    S = plan.evaluate(_tensor(Iin, dt)).double().cpu().numpy()
    ref = photoionization(wl.xyz, Iin, wl.gas, h=wl.h).full(wl.n)
    err = rel_l2(S, ref)
    _say(f"  rel-L2 = {err:.3e}")
    assert err <= tol
    # the library's own-cell coefficient (E1 closed form) matches the oracle's (quadrature)
    cs = plan.debug_fetch("c_self")[0]
    from oracle import cube_self_coefficient, gas_constants
    assert cs == pytest.approx(cube_self_coefficient(wl.h, gas_constants(wl.gas)), rel=1e-12)
    plan.close()


def test_direct_thresholded_c2_small(gpu_lib):
    import torch
    wl = gen.config2(seed=1002, n_axis=40)
    _say("direct c2_40 fp32 thresholds")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, wl.thresholds, method="direct", **plan_kwargs(wl))
    I32 = wl.I.astype(np.float32)
    S = plan.evaluate(_tensor(I32, torch.float32), _tensor(wl.E.astype(np.float32), torch.float32)).double().cpu().numpy()
    r = photoionization(wl.xyz, I32.astype(np.float64), wl.gas, h=wl.h, src_rel=1e-4,
                        E=wl.E.astype(np.float32).astype(np.float64), e_abs=3e6)
    assert rel_l2(S, r.full(wl.n)) <= 1e-6
    plan.close()


# ---------------------------------------------------------------- FMM

def test_fmm_fp64_c1(gpu_lib):
    import torch
    wl = gen.config1()
    _say("fmm c1 fp64 q=6")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, wl.thresholds, precision="fp64", leaf_capacity=27, **plan_kwargs(wl))
    S = plan.evaluate(_tensor(wl.I, torch.float64)).cpu().numpy()
    ref = photoionization(wl.xyz, wl.I, wl.gas, h=wl.h).full(wl.n)
    err = rel_l2(S, ref)
    _say(f"  rel-L2 = {err:.3e}")
    assert err <= 1e-6
    plan.close()


@pytest.mark.parametrize("q", [3, 4])
def test_fmm_fp32_c1(gpu_lib, q):
    import torch
    wl = gen.config1()
    _say(f"fmm c1 fp32 q={q}")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, wl.thresholds, precision="fp32", order_q=q, leaf_capacity=27,
                        **plan_kwargs(wl))
    I32 = wl.I.astype(np.float32)
    S = plan.evaluate(_tensor(I32, torch.float32)).double().cpu().numpy()
    ref = photoionization(wl.xyz, I32.astype(np.float64), wl.gas, h=wl.h).full(wl.n)
    err = rel_l2(S, ref)
    _say(f"  rel-L2 = {err:.3e}")
    assert err <= 1e-3
    plan.close()


def test_fmm_fp32_c2_small_adaptive(gpu_lib):
    import torch
    wl = gen.config2(seed=1003, n_axis=64)
    _say("fmm c2_64 fp32 thresholds")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, wl.thresholds, **plan_kwargs(wl))
    I32 = wl.I.astype(np.float32)
    E32 = wl.E.astype(np.float32)
    S, st = plan.evaluate(_tensor(I32, torch.float32), _tensor(E32, torch.float32), stats=True)
    S = S.double().cpu().numpy()
    _say(f"  stats {st}")
    r = photoionization(wl.xyz, I32.astype(np.float64), wl.gas, h=wl.h, src_rel=1e-4,
                        E=E32.astype(np.float64), e_abs=3e6)
    err = rel_l2(S, r.full(wl.n))
    _say(f"  rel-L2 = {err:.3e}")
    assert err <= 1e-3
    plan.close()


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-3), ("fp64", 1e-6)])
def test_fmm_threshold_c2_full_size(gpu_lib, precision, tol):
    """The benchmark's workload at its full size (128^3 streamer grid, seed 1000, the rule
    tau_s = 1e-4 of Sec. 3 eq. (18), targets |E| >= 3e6 V/m): the selected counts equal the
    oracle's masks, and S at sampled targets (3000 uniform, and up to 2000 within 1 mm of the
    head) matches the oracle over the same source set, at the bar of the precision."""
    import torch
    wl = gen.config2(seed=1000, n_axis=128)
    _say(f"threshold rule, 128^3, {precision}")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, wl.thresholds, precision=precision, **plan_kwargs(wl))
    I = wl.I.astype(np.float32) if precision == "fp32" else wl.I.astype(np.float64)
    E32 = wl.E.astype(np.float32)
    S, st = plan.evaluate(_tensor(I, torch.float32 if precision == "fp32" else torch.float64),
                          _tensor(E32, torch.float32), stats=True)
    S = S.double().cpu().numpy()
    smask = source_mask(I.astype(np.float64), wl.thresholds["src_rel"])
    tmask = target_mask(E32.astype(np.float64), wl.thresholds.get("e_abs", -1.0))
    assert st["n_src"] == int(smask.sum()) and st["n_tgt"] == int(tmask.sum())
    tg = gen.sample_targets(np.flatnonzero(tmask), wl.xyz, wl.head, k=3000, seed=11, head_cap=2000)
    ref = photoionization(wl.xyz, I.astype(np.float64), wl.gas, h=wl.h, smask=smask, targets=tg)
    err = rel_l2(S[tg], ref.S_t)
    _say(f"  rel-L2 on {tg.size} targets: {err:.3e}")
    assert err <= tol
    plan.close()


@pytest.mark.parametrize("n_axis,precision,tol,tol_quiet", [(128, "fp32", 1e-3, 1e-2), (128, "fp64", 1e-6, 2e-4),
                                                              (96, "fp32", 1e-3, 1e-2)])
def test_fmm_relative_rule_coarse_leaves(gpu_lib, n_axis, precision, tol, tol_quiet):
    """The relative field rule of Sec. 5 (|E| >= E_app + 0.005 (max|E| - E_app)) leaves few
    targets in the quiet parts of the field, so some target leaves stay coarse (more than 64
    grid points: the far field shares such a leaf's 64-point chunks among workgroups).  The
    test checks that such leaves occur, then S against the oracle over the same source set:
    at the bar of the precision on every target of the coarse leaves (up to 1500) together with
    2000 sampled ones, and on the coarse leaves' targets alone at tol_quiet.  There S is about
    1e-7 of its maximum and is all far field; its error, measured the same in the fine leaves
    around them, is the q = 4 lattice's (4e-5 to 6e-5 in FP64) and, in FP32, rounding raised
    by the check-to-equivalent solve (2e-3 to 3e-3).  A chunk left out or evaluated at the
    wrong cells gives errors of order 0.1 to 1.  On the 96^3 grid the coarse leaves hold 216 or
    1728 points: chunk groups that a leaf fills only in part."""
    import torch
    wl = gen.config2(seed=1000 if n_axis == 128 else 1096, n_axis=n_axis)  # 1000: the benchmark's field
    thr = dict(src_rel=1e-4, e_applied=5e6, e_rel=0.005)
    _say(f"relative rule, {n_axis}^3, {precision}")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, thr, precision=precision, **plan_kwargs(wl))
    I = wl.I.astype(np.float32) if precision == "fp32" else wl.I.astype(np.float64)
    E32 = wl.E.astype(np.float32)
    S, st = plan.evaluate(_tensor(I, torch.float32 if precision == "fp32" else torch.float64),
                          _tensor(E32, torch.float32), stats=True)
    S = S.double().cpu().numpy()
    smask = source_mask(I.astype(np.float64), thr["src_rel"])
    tmask = target_mask(E32.astype(np.float64), -1.0, thr["e_applied"], thr["e_rel"])
    assert st["n_src"] == int(smask.sum()) and st["n_tgt"] == int(tmask.sum())
    assert np.all(S[~tmask] == 0.0)
    # target leaves whose box holds more than 64 grid cells
    box = plan.debug_fetch("boxes")  # level, ax, ay, az, s_first, s_cnt, t_first, t_cnt, parent, flags
    cells = (n_axis >> box[:, 0]) ** 3
    coarse = np.flatnonzero(((box[:, 9] & 1) == 1) & (box[:, 7] > 0) & (box[:, 0] >= 2) & (cells > 64))
    assert coarse.size > 0
    perm, tgt = plan.debug_fetch("perm"), plan.debug_fetch("tgt")
    inside = np.concatenate([perm[tgt[box[b, 6]:box[b, 6] + box[b, 7]]] for b in coarse])
    _say(f"  {coarse.size} coarse target leaves (levels {sorted(set(box[coarse, 0].tolist()))}), "
         f"{inside.size} targets in them")
    rng = np.random.default_rng(5)
    inside = np.sort(rng.choice(inside, size=min(inside.size, 1500), replace=False))
    tg = np.union1d(inside, gen.sample_targets(np.flatnonzero(tmask), wl.xyz, wl.head, k=2000, seed=12,
                                               head_cap=500))
    ref = photoionization(wl.xyz, I.astype(np.float64), wl.gas, h=wl.h, smask=smask, targets=tg)
    err_in = rel_l2(S[inside], ref.S_t[np.searchsorted(tg, inside)])
    err = rel_l2(S[tg], ref.S_t)
    _say(f"  rel-L2 coarse leaves {err_in:.3e}, all sampled {err:.3e}")
    assert err <= tol and err_in <= tol_quiet
    plan.close()


def test_fmm_fp64_all_sources_c2_small(gpu_lib):
    """Plain FP64 FMM (every point a source and a target) on a 32^3 streamer grid: <= 1e-6."""
    import torch
    wl = gen.config2(seed=1004, n_axis=32)
    _say("fmm c2_32 fp64 all sources")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, dict(src_rel=0.0), precision="fp64", leaf_capacity=64, **plan_kwargs(wl))
    S = plan.evaluate(_tensor(wl.I, torch.float64)).cpu().numpy()
    ref = photoionization(wl.xyz, wl.I, wl.gas, h=wl.h).full(wl.n)
    err = rel_l2(S, ref)
    _say(f"  rel-L2 = {err:.3e}")
    assert err <= 1e-6
    plan.close()


def test_fmm_translation_chunks_match(gpu_lib, monkeypatch):
    """A small translation buffer (many source-box chunks) gives the same field to rounding."""
    import torch
    wl = gen.config2(seed=1005, n_axis=48)
    I32 = _tensor(wl.I.astype(np.float32), torch.float32)
    E32 = _tensor(wl.E.astype(np.float32), torch.float32)
    thr = dict(src_rel=1e-6, e_abs=3e6)
    _say("fmm c2_48 fp32 one chunk vs many chunks")
    p1 = gpu_lib.Plan(wl.xyz, wl.gas, thr, leaf_capacity=32, **plan_kwargs(wl))
    S1 = p1.evaluate(I32, E32).double().cpu().numpy()
    monkeypatch.setenv("PH_TRANSLATION_BUFFER_MB", "1")
    p2 = gpu_lib.Plan(wl.xyz, wl.gas, thr, leaf_capacity=32, **plan_kwargs(wl))
    S2 = p2.evaluate(I32, E32).double().cpu().numpy()
    assert rel_l2(S2, S1) < 1e-6
    r = photoionization(wl.xyz, wl.I.astype(np.float32).astype(np.float64), wl.gas, h=wl.h, src_rel=1e-6,
                        E=wl.E.astype(np.float32).astype(np.float64), e_abs=3e6)
    assert rel_l2(S2, r.full(wl.n)) <= 1e-3
    p1.close()
    p2.close()


def test_repeat_calls_bitwise_identical(gpu_lib):
    """No floating-point atomics: two identical calls give bitwise-identical output."""
    import torch
    wl = gen.config2(seed=1006, n_axis=48)
    plan = gpu_lib.Plan(wl.xyz, wl.gas, wl.thresholds, leaf_capacity=32, **plan_kwargs(wl))
    I32 = _tensor(wl.I.astype(np.float32), torch.float32)
    E32 = _tensor(wl.E.astype(np.float32), torch.float32)
    a = plan.evaluate(I32, E32).cpu().numpy()
    b = plan.evaluate(I32, E32).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    plan.close()
