"""Train the learned leaf selector on synthetic streamer fields with the library's own GPU kernels.

The selector decides, per source leaf of the first-pass tree, whether the leaf's sources enter
the photoionization sum (adaptive source selection of Sec. 3 of the paper, made per leaf by
a network instead of a fixed relative threshold on I).

Recipe:
  * fields: the seeded streamer generator (head + channel on the uniform grid); seeds
    [0, n_train) train, [n_train, n_train + n_cal) calibrate the decision threshold;
  * rows: the source leaves of an evaluation with the candidate threshold base_src_rel;
    features from ph_selector_features;
  * contribution of leaf b: c_b = ||S_b|| / ||S|| over every active target (ph_selector_contrib
    over all targets, ||S|| from the same evaluation).  Every S_b is non-negative, so dropping a
    set D of leaves changes S by at most sum_{b in D} c_b in relative L2 (triangle inequality);
  * labels: drop the longest run of smallest c_b whose sum stays within label_budget (1 = keep);
  * network 8 -> 64 -> 64 -> 1 (exact-erf GELU), BCE with logits, positive weight
    n_drop / n_keep, Adam; features standardised on the training rows and the standardisation
    folded into the first layer, so inference takes raw features;
  * decision threshold: the largest logit threshold at which the bound sum_{dropped} c_b stays
    within gate_budget on every calibration field, taken with the BF16 forward pass that the
    evaluation path runs.

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


def keep_labels(c: np.ndarray, budget: float) -> np.ndarray:
    """1 = keep.  The smallest contributions are dropped while their running sum is <= budget."""
    c = np.asarray(c, dtype=np.float64)
    order = np.argsort(c, kind="stable")
    run = np.cumsum(c[order])
    n_drop = int(np.searchsorted(run, budget, side="right"))
    lab = np.ones(c.size, dtype=np.float32)
    lab[order[:n_drop]] = 0.0
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
    """Largest t such that, on every field, sum of c over rows with logit < t is <= gate_budget."""
    best = math.inf
    for z, c in fields:
        order = np.argsort(z, kind="stable")
        run = np.cumsum(c[order])
        over = np.flatnonzero(run > gate_budget)
        if over.size == 0:
            continue
        # rows strictly below z[order[k]] are dropped, k the first row that breaks the budget
        best = min(best, float(z[order[over[0]]]))
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


def _field_rows(plan, wl, label_budget, torch):
    I = torch.tensor(wl.I.astype(np.float32), device="cuda")
    E = torch.tensor(wl.E.astype(np.float32), device="cuda")
    S = plan.evaluate(I, E)
    F = B.selector_features(plan, I, E)
    # the evaluation's own target set, in caller order
    targets = np.sort(plan.debug_fetch("perm")[plan.debug_fetch("tgt")]).astype(np.int32)
    tdev = torch.tensor(targets, device="cuda")
    c = B.selector_contrib(plan, tdev, F.shape[0]).double().cpu().numpy()
    c = c / float(torch.linalg.vector_norm(S[tdev.long()].double()))
    return F.cpu().numpy(), c, keep_labels(c, label_budget)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--n-train", type=int, default=180)
    ap.add_argument("--n-cal", type=int, default=20)
    ap.add_argument("--n-axis", type=int, default=128)
    ap.add_argument("--base-src-rel", type=float, default=1e-7)
    ap.add_argument("--label-budget", type=float, default=5e-4)
    ap.add_argument("--gate-budget", type=float, default=8e-4)
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
    plan = B.Plan(wl0.xyz, wl0.gas, thr, h=wl0.h, w=wl0.w, cube_lo=(lo, lo, lo), cube_size=hi - lo)
    rows = []
    for s in range(a.n_train + a.n_cal):
        wl = wl0 if s == 0 else gen.config2(seed=s, n_axis=a.n_axis)
        F, c, y = _field_rows(plan, wl, a.label_budget, torch)
        rows.append((F, c, y))
        if s % 20 == 0 or s + 1 == a.n_train + a.n_cal:
            print(f"field {s}: {F.shape[0]} leaves, keep {int(y.sum())}, sum c {c.sum():.3f} "
                  f"({time.time() - t0:.0f} s)", flush=True)
    plan.close()

    Xtr = np.concatenate([r[0] for r in rows[:a.n_train]]).astype(np.float64)
    ytr = np.concatenate([r[2] for r in rows[:a.n_train]]).astype(np.float32)
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
    for F, c, y in rows[a.n_train:]:
        z = B.mlp_forward(wdev, torch.tensor(F, device="cuda"), bf16=True).cpu().numpy().astype(np.float64)
        cal.append((z, c))
    tau = calibrate_threshold(cal, a.gate_budget)
    if not math.isfinite(tau):
        tau = 1e30
    for (z, c), (_, _, y) in zip(cal, rows[a.n_train:]):
        agree.append(float(np.mean((z >= tau) == (y > 0.5))))
    kept = [float(np.mean(z >= tau)) for z, _ in cal]
    bound = [float(c[z < tau].sum()) for z, c in cal]
    meta = dict(threshold=tau, base_src_rel=a.base_src_rel, label_budget=a.label_budget,
                gate_budget=a.gate_budget, n_train=a.n_train, n_cal=a.n_cal, n_axis=a.n_axis,
                epochs=a.epochs, batch=a.batch, lr=a.lr, seed=a.seed, pos_weight=pos_weight,
                feature_mean=mu.tolist(), feature_std=sd.tolist(),
                cal_kept_leaf_fraction=float(np.mean(kept)), cal_bound_max=float(max(bound)),
                cal_label_agreement=float(np.mean(agree)))
    print("calibration:", json.dumps({k: meta[k] for k in ("threshold", "cal_kept_leaf_fraction",
                                                             "cal_bound_max", "cal_label_agreement")}),
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
