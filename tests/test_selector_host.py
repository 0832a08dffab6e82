"""Host logic of the selector training script against the oracle (no GPU)."""
import math

import numpy as np

from oracle import mlp as omlp
from paper_2112_10059_amd import train_selector as ts


def _fields(rng, m, nt=60):
    return rng.lognormal(-6, 2, size=(m, 1)) * rng.uniform(0, 1, size=(m, nt)) ** 3


def test_keep_labels_match_oracle_greedy_rule():
    rng = np.random.default_rng(0)
    for trial in range(40):
        m = int(rng.integers(1, 40))
        F = _fields(rng, m)
        F0 = rng.lognormal(-9, 1) * rng.uniform(0, 1, size=F.shape[1]) ** 2
        if trial % 5 == 0:
            F[: m // 3] = F[0]  # equal fields
        G, c, d0 = F @ F.T, F @ F0, float(F0 @ F0)
        s_norm = float(np.linalg.norm(F.sum(axis=0) + F0))
        budget = float(rng.choice([0.0, 1e-3, 1e-2, 1e-1, 10.0]))
        ours = ts.keep_labels(G, c, d0, s_norm, budget)
        ref = omlp.greedy_keep_labels(G, c, d0, s_norm, budget)
        assert np.array_equal(ours, ref.astype(np.float32))


def test_fold_standardisation_matches_oracle_forward():
    rng = np.random.default_rng(1)
    p = omlp.init_params(2).astype(np.float32)
    mu = rng.normal(size=8)
    sd = rng.uniform(0.1, 3.0, size=8)
    X = rng.normal(size=(200, 8)) * sd + mu
    z_std, _ = omlp.forward(p.astype(np.float64), (X - mu) / sd)
    z_fold, _ = omlp.forward(ts.fold_standardisation(p, mu, sd).astype(np.float64), X)
    assert np.allclose(z_fold, z_std, rtol=1e-5, atol=1e-5)


def test_calibrated_threshold_keeps_every_field_within_budget():
    rng = np.random.default_rng(2)
    fields, raw = [], []
    for _ in range(12):
        F = _fields(rng, 80)
        F0 = rng.lognormal(-9, 1) * rng.uniform(0, 1, size=F.shape[1]) ** 2
        z = rng.normal(size=80)
        S = F.sum(axis=0) + F0
        fields.append((z, F @ F.T, F @ F0, float(F0 @ F0), float(np.linalg.norm(S))))
        raw.append((z, F, F0))
    budget = 2e-2

    def err(z, F, F0, t):
        return np.linalg.norm(F0 + F[z < t].sum(axis=0)) / np.linalg.norm(F.sum(axis=0) + F0)

    t = ts.calibrate_threshold(fields, budget)
    assert math.isfinite(t)
    assert all(err(z, F, F0, t) <= budget * (1 + 1e-12) for z, F, F0 in raw)
    # the next larger logit breaks the budget on at least one field
    above = min(z[z > t].min() for z, _, _ in raw if np.any(z > t))
    assert any(err(z, F, F0, above + 1e-12) > budget for z, F, F0 in raw)
    # a field that never breaks the budget does not bind; one whose left-out field alone breaks
    # it keeps every row
    F = _fields(rng, 5)
    assert ts.calibrate_threshold([(np.zeros(5), F @ F.T, np.zeros(5), 0.0, 1e30)], 1e-3) == math.inf
    assert ts.calibrate_threshold([(np.zeros(5), F @ F.T, np.zeros(5), 1.0, 1.0)], 1e-3) == -math.inf


def test_weights_file_round_trip(tmp_path):
    p = omlp.init_params(3).astype(np.float32)
    path = tmp_path / "w.txt"
    with open(path, "w") as f:
        f.write('# meta {"threshold": 0.5}\n')
        for v in p:
            f.write(f"{float(v):.9e}\n")
    w, meta = ts.load_selector(str(path))
    assert meta["threshold"] == 0.5
    assert np.array_equal(w, p)
