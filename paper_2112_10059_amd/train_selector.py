"""Train the learned leaf selector on synthetic streamer fields with the library's own GPU kernels.

The selector decides, per leaf of the plan's tree that holds sources of the threshold rule
(Sec. 3 eq. (18): I >= base_src_rel I_max), whether the leaf's sources enter the
photoionization sum: it can only remove whole leaves from the rule's source set, which also
removes their boxes from the near field and the multipole passes.

Recipe:
  * fields: the seeded streamer generator (head + channel on the uniform grid); seeds
    [0, n_train) train, [n_train, n_train + n_cal) calibrate the decision threshold;
  * references per field: S (every point a source) and S_rule (the rule's sources) from the
    plain FP64 FMM; S_0 = S - S_rule is what the rule itself leaves out;
  * rows: the plan leaves holding the rule's sources, with their features
    (ph_selector_features); per row b its field S_b at every target (ph_selector_fields, in
    chunks of targets), the Gram matrix G[b, b'] = <S_b, S_b'> and c[b] = <S_0, S_b>.  All
    fields are non-negative, and dropping a set D of rows makes the method error exactly
    ||S_0 + sum_D S_b|| (squared: ||S_0||^2 + 2 sum_D c + sum_{D x D} G);
  * labels: rows are dropped one at a time, always the one that raises that error the least,
    while it stays within label_budget ||S|| (1 = keep);
  * network 8 -> 64 -> 64 -> 1 (exact-erf GELU), BCE with logits, positive weight
    n_drop / n_keep, Adam; features standardised on the training rows and the standardisation
    folded into the first layer, so inference takes raw features;
  * decision threshold: the largest logit threshold at which the method error of the dropped
    rows stays within gate_budget ||S|| on every calibration field, with the BF16 logits that
    the evaluation path computes.

Output: a text file (header lines with the metadata, then the 4801 parameters in the C ABI's
layout, one per line) read by ``load_selector``.

Usage (GPU):  python -m paper_2112_10059_amd.train_selector --out paper_2112_10059_amd/selector_c2.txt
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import binding as B

NIN, NHID = 8, 64
NPARAM = B.MLP_NPARAM
DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_c2.txt")


def keep_labels(G: np.ndarray, c: np.ndarray, d0: float, s_norm: float, budget: float) -> np.ndarray:
    """1 = keep.  Rows are dropped one at a time, always the one whose drop raises the squared
    error d0 + 2 sum_D c + sum_{D x D} G the least (ties: lowest index), while the error stays
    <= budget * s_norm (the running sums make each step O(rows))."""
    G = np.asarray(G, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    m = G.shape[0]
    diag = np.diag(G).copy()
    acc = c.copy()  # <S_0 + S_D, S_b> for every row b
    e2 = float(d0)
    lim = (budget * s_norm) ** 2
    dropped = np.zeros(m, dtype=bool)
    while True:
        rest = np.flatnonzero(~dropped)
        if rest.size == 0:
            break
        inc = diag[rest] + 2.0 * acc[rest]
        ok = e2 + inc <= lim
        if not ok.any():
            break
        j = rest[np.flatnonzero(ok)[np.argmin(inc[ok])]]
        e2 += diag[j] + 2.0 * acc[j]
        acc += G[:, j]
        dropped[j] = True
    lab = np.ones(m, dtype=np.float32)
    lab[dropped] = 0.0
    return lab


def he_init(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0.0, math.sqrt(2.0 / NIN), size=(NHID, NIN))
    W2 = rng.normal(0.0, math.sqrt(2.0 / NHID), size=(NHID, NHID))
    W3 = rng.normal(0.0, math.sqrt(1.0 / NHID), size=NHID)
    return np.concatenate([W1.ravel(), np.zeros(NHID), W2.ravel(), np.zeros(NHID), W3, [0.0]]).astype(np.float32)


def fold_standardisation(p: np.ndarray, mu: np.ndarray, sd: np.ndarray) -> np.ndarray:
    """Weights acting on raw x equal to p acting on (x - mu) / sd."""
    q = np.asarray(p, dtype=np.float64).copy()
    W1 = q[:NHID * NIN].reshape(NHID, NIN)
    b1 = q[NHID * NIN:NHID * NIN + NHID]
    W1f = W1 / sd[None, :]
    b1f = b1 - W1f @ mu
    q[:NHID * NIN] = W1f.ravel()
    q[NHID * NIN:NHID * NIN + NHID] = b1f
    return q.astype(np.float32)


def calibrate_threshold(fields, gate_budget: float) -> float:
    """Largest t such that on every field (z, G, c, d0, s_norm) the rows with logit < t leave a
    method error of at most gate_budget * s_norm (exact, from G, c and d0)."""
    best = math.inf
    for z, G, c, d0, s_norm in fields:
        order = np.argsort(z, kind="stable")
        acc = np.asarray(c, dtype=np.float64).copy()
        e2 = float(d0)
        lim = (gate_budget * s_norm) ** 2
        if e2 > lim:
            return -math.inf  # the rule alone is over the budget: keep every row
        for b in order:
            e2n = e2 + G[b, b] + 2.0 * acc[b]
            if e2n > lim:
                # rows strictly below z[b] are dropped: they are the prefix before b
                best = min(best, float(z[b]))
                break
            e2 = e2n
            acc += G[:, b]
    return best


def load_selector(path: str | None = None):
    """(weights float32[4801], meta dict) of a file written by this script."""
    path = path or DEFAULT_WEIGHTS
    meta, vals = {}, []
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                if line.startswith("# meta "):
                    meta = json.loads(line[len("# meta "):])
                continue
            if line.strip():
                vals.append(float(line))
    w = np.asarray(vals, dtype=np.float32)
    if w.size != NPARAM:
        raise ValueError(f"{path}: {w.size} parameters, expected {NPARAM}")
    return w, meta


def field_rows(plan, I, E, targets, S0, torch, chunk: int = 65536):
    """Features (rows x 8), Gram matrix G of the row fields over the targets, c = <S_0, S_b>."""
    F = B.selector_features(plan, I, E)
    m = F.shape[0]
    G = torch.zeros((m, m), dtype=torch.float64, device="cuda")
    c = torch.zeros(m, dtype=torch.float64, device="cuda")
    buf = torch.empty((max(m, 1), chunk), dtype=torch.float32, device="cuda")
    for t0 in range(0, targets.numel(), chunk):
        tc = targets[t0:t0 + chunk]
        Fc = B.selector_fields(plan, I, tc, m, ld=chunk, out=buf).double()
        G += Fc @ Fc.T
        c += Fc @ S0[t0:t0 + chunk]
    return F.cpu().numpy(), G.cpu().numpy(), c.cpu().numpy()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--n-train", type=int, default=180)
    ap.add_argument("--n-cal", type=int, default=20)
    ap.add_argument("--n-axis", type=int, default=128)
    ap.add_argument("--base-src-rel", type=float, default=1e-4)
    ap.add_argument("--label-budget", type=float, default=8e-4)
    ap.add_argument("--gate-budget", type=float, default=8.5e-4)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=7)
    a = ap.parse_args(argv)

    import torch
    import gen

    if not torch.cuda.is_available():
        raise SystemExit("train_selector needs a GPU")
    t0 = time.time()
    wl0 = gen.config2(seed=0, n_axis=a.n_axis)
    lo, hi = wl0.domain
    thr = dict(wl0.thresholds)
    thr["src_rel"] = a.base_src_rel
    geo = dict(h=wl0.h, w=wl0.w, cube_lo=(lo, lo, lo), cube_size=hi - lo)
    plan = B.Plan(wl0.xyz, wl0.gas, thr, **geo)
    p_all = B.Plan(wl0.xyz, wl0.gas, dict(src_rel=0.0), precision="fp64", **geo)
    p_rule = B.Plan(wl0.xyz, wl0.gas, dict(src_rel=a.base_src_rel), precision="fp64", **geo)
    rows, cals = [], []
    for s in range(a.n_train + a.n_cal):
        wl = wl0 if s == 0 else gen.config2(seed=s, n_axis=a.n_axis)
        I = torch.tensor(wl.I.astype(np.float32), device="cuda")
        E = torch.tensor(wl.E.astype(np.float32), device="cuda")
        plan.evaluate(I, E)
        # the call's own target set, in caller order
        targets = np.sort(plan.debug_fetch("perm")[plan.debug_fetch("tgt")]).astype(np.int64)
        I64 = torch.tensor(wl.I.astype(np.float32).astype(np.float64), device="cuda")
        S_all = p_all.evaluate(I64)
        S0 = (S_all - p_rule.evaluate(I64))[torch.tensor(targets, device="cuda")]
        s_norm = float(torch.linalg.norm(S_all[torch.tensor(targets, device="cuda")]))
        d0 = float(S0 @ S0)
        F, G, c = field_rows(plan, I, E, torch.tensor(targets.astype(np.int32), device="cuda"), S0, torch)
        y = keep_labels(G, c, d0, s_norm, a.label_budget)
        rows.append((F, y))
        if s >= a.n_train:
            cals.append((G, c, d0, s_norm))
        if s % 20 == 0 or s + 1 == a.n_train + a.n_cal:
            print(f"field {s}: {F.shape[0]} rows, keep {int(y.sum())}, rule error {math.sqrt(d0) / s_norm:.3e} "
                  f"({time.time() - t0:.0f} s)", flush=True)
    plan.close()
    p_all.close()
    p_rule.close()

    Xtr = np.concatenate([r[0] for r in rows[:a.n_train]]).astype(np.float64)
    ytr = np.concatenate([r[1] for r in rows[:a.n_train]]).astype(np.float32)
    mu = Xtr.mean(axis=0)
    sd = np.maximum(Xtr.std(axis=0), 1e-3)
    n_keep = float(ytr.sum())
    n_drop = float(ytr.size - n_keep)
    pos_weight = n_drop / max(n_keep, 1.0)
    print(f"training rows {ytr.size}: keep {int(n_keep)}, drop {int(n_drop)}, pos_weight {pos_weight:.3f}",
          flush=True)

    X = torch.tensor(((Xtr - mu) / sd).astype(np.float32), device="cuda")
    Y = torch.tensor(ytr, device="cuda")
    p = torch.tensor(he_init(a.seed), device="cuda")
    m1 = torch.zeros_like(p)
    m2 = torch.zeros_like(p)
    g = torch.empty_like(p)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    gen_t = torch.Generator(device="cpu").manual_seed(a.seed)
    step = 0
    for ep in range(a.epochs):
        order = torch.randperm(X.shape[0], generator=gen_t).to("cuda")
        tot, nb = 0.0, 0
        for i in range(0, X.shape[0], a.batch):
            idx = order[i:i + a.batch]
            xb, yb = X[idx].contiguous(), Y[idx].contiguous()
            B.mlp_backward(p, xb, yb, pos_weight, grad=g, loss=loss)
            step += 1
            B.adam_step(p, m1, m2, g, a.lr, 0.9, 0.999, 1e-8, step)
            tot += float(loss)
            nb += 1
        print(f"epoch {ep}: mean loss {tot / nb:.5f}", flush=True)

    pf = fold_standardisation(p.cpu().numpy(), mu, sd)
    wdev = torch.tensor(pf, device="cuda")
    cal, agree = [], []
    for (F, y), (G, c, d0, s_norm) in zip(rows[a.n_train:], cals):
        z = B.mlp_forward(wdev, torch.tensor(F, device="cuda"), bf16=True).cpu().numpy().astype(np.float64)
        cal.append((z, G, c, d0, s_norm))
        agree.append(y)
    tau = calibrate_threshold(cal, a.gate_budget)
    if not math.isfinite(tau):
        tau = 1e30 if tau > 0 else -1e30
    kept, change, agreement = [], [], []
    for (z, G, c, d0, s_norm), y in zip(cal, agree):
        d = z < tau
        kept.append(float(np.mean(~d)))
        change.append(float(np.sqrt(d0 + 2.0 * c[d].sum() + G[np.ix_(d, d)].sum()) / s_norm))
        agreement.append(float(np.mean((~d) == (y > 0.5))))
    meta = dict(threshold=tau, base_src_rel=a.base_src_rel, label_budget=a.label_budget,
                gate_budget=a.gate_budget, n_train=a.n_train, n_cal=a.n_cal, n_axis=a.n_axis,
                epochs=a.epochs, batch=a.batch, lr=a.lr, seed=a.seed, pos_weight=pos_weight,
                feature_mean=mu.tolist(), feature_std=sd.tolist(),
                cal_kept_row_fraction=float(np.mean(kept)), cal_error_max=float(max(change)),
                cal_label_agreement=float(np.mean(agreement)))
    print("calibration:", json.dumps({k: meta[k] for k in ("threshold", "cal_kept_row_fraction",
                                                             "cal_error_max", "cal_label_agreement")}),
          flush=True)
    with open(a.out, "w") as f:
        f.write("# learned leaf selector: 8 -> 64 -> 64 -> 1 GELU network, parameters in the C ABI layout\n")
        f.write("# (W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3); keep a leaf iff logit >= threshold\n")
        f.write("# meta " + json.dumps(meta) + "\n")
        for v in pf:
            f.write(f"{float(v):.9e}\n")
    print(f"wrote {a.out} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    sys.exit(main())
