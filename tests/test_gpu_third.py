"""Third adaptive strategy of Sec. 3 (the r_s skip) on a nonuniform cloud, where target leaves
have W lists (near boxes not adjacent to them): decisions and results against the oracle's
``third_strategy`` (exact FP64 sums over the same tree's boxes, built here in NumPy), the
W lists against the work counter, and the bound on what a skip changes."""
import numpy as np
import pytest

import gen
from oracle import rel_l2
from oracle.strategies import third_strategy
from tests.helpers import box_gap, plan_kwargs, reference_tree, w_lists

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _groups(plan, wl, smask, tmask, targets):
    """Per sampled target its leaf's group (or -1) and per group the W boxes' points and gaps,
    from the NumPy tree over the plan's sorted keys."""
    perm = plan.debug_fetch("perm")
    keys = plan.debug_fetch("keys")
    lvl = plan.debug_fetch("level_start")
    s_sorted = np.flatnonzero(smask[perm])
    t_sorted = np.flatnonzero(tmask[perm])
    rows = reference_tree(keys[s_sorted], keys[t_sorted], 64, len(lvl) - 2)
    W = w_lists(rows)
    lo, hi = wl.domain
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size, dtype=perm.dtype)
    tpos = np.searchsorted(t_sorted, inv[targets])
    leaves = [b for b in range(rows.shape[0]) if rows[b][8] == 1 and rows[b][7] > 0]
    first = np.array([rows[b][6] for b in leaves])
    order = np.argsort(first)
    leaf_of = np.array(leaves)[order][np.searchsorted(first[order], tpos, side="right") - 1]
    gid, groups = {}, []
    for b, A in W.items():
        gid[b] = len(groups)
        groups.append([(perm[s_sorted[rows[a][4]:rows[a][4] + rows[a][5]]], box_gap(rows[a], rows[b], lo, hi - lo))
                       for a in A])
    grp = np.array([gid.get(int(b), -1) for b in leaf_of], dtype=np.int64)
    m2p_targets = sum(len(A) * int(rows[b][7]) for b, A in W.items())
    return grp, groups, m2p_targets, inv


@pytest.mark.parametrize("precision,tol,r_s", [("fp32", 1e-3, 1e-4), ("fp32", 1e-3, 1e-2), ("fp64", 1e-6, 1e-4)])
def test_third_strategy_cloud(gpu_lib, precision, tol, r_s):
    import torch
    wl = gen.config3(seed=2004, n=120_000, src_rel=1e-4)
    thr = dict(src_rel=1e-4)
    dt = torch.float64 if precision == "fp64" else torch.float32
    Iin = wl.I if precision == "fp64" else wl.I.astype(np.float32).astype(np.float64)
    tI = torch.tensor(Iin, dtype=dt, device="cuda")
    _say(f"third strategy, {precision}, r_s {r_s:g}, cloud {wl.n}")
    q = 7 if precision == "fp64" else 4
    plan = gpu_lib.Plan(wl.xyz, wl.gas, dict(thr, r_s=r_s), precision=precision, order_q=q, **plan_kwargs(wl))
    S, st = plan.evaluate(tI, stats=True)
    S = S.double().cpu().numpy()
    flags = plan.debug_fetch("rs_skip")
    base = gpu_lib.Plan(wl.xyz, wl.gas, thr, precision=precision, order_q=q, **plan_kwargs(wl))
    S0 = base.evaluate(tI).double().cpu().numpy()
    smask = Iin >= 1e-4 * Iin.max()
    tmask = np.ones(wl.n, dtype=bool)
    tg = gen.sample_targets(np.arange(wl.n), wl.xyz, wl.head, k=1500, seed=8, head_radius=0.2, head_cap=500)
    grp, groups, m2p_targets, inv = _groups(plan, wl, smask, tmask, tg)
    # the W lists: the work counter holds W boxes x targets x lattice points
    assert st["work"]["m2p_evals"] == m2p_targets * q ** 3
    assert (grp >= 0).sum() > 0, "no sampled target has a W list"
    ref = third_strategy(wl.xyz, Iin, wl.gas, tg, grp, groups, r_s, w=wl.w, smask=smask)
    err = rel_l2(S[tg], ref.S_t)
    got = flags[inv[tg]] == 1
    g = grp >= 0
    ratio = ref.bound_t[g] / (r_s * ref.est_t[g])
    clear = np.abs(ratio - 1.0) > 10 * tol
    agree = (got[g] == ref.skipped[g])
    _say(f"  rel-L2 {err:.3e}; sampled targets with a W list {g.sum()}, skipped {got[g].sum()} (oracle "
         f"{ref.skipped[g].sum()}), decisions agree on {agree[clear].sum()} of {clear.sum()} clear cases")
    assert err <= tol
    assert np.all(agree[clear])
    # a skip changes S by at most r_s relative (what the FMM drops is the W terms it would add)
    drop = (S0 - S)[tg][g] / S0[tg][g]
    assert np.all(drop >= 0) and np.all(drop <= r_s * 1.01 + 1e-6)
    assert np.all(drop[~got[g]] == 0)
    assert np.all(S[tg][~g] == S0[tg][~g])
    plan.close()
    base.close()
