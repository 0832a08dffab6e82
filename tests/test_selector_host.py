"""Host logic of the selector training script against the oracle (no GPU)."""
import math

import numpy as np

from oracle import mlp as omlp
from paper_2112_10059_amd import train_selector as ts


def test_keep_labels_match_oracle_budget_rule():
    rng = np.random.default_rng(0)
    for trial in range(50):
        c = rng.lognormal(-8, 3, size=rng.integers(1, 400))
        if trial % 5 == 0:
            c[: c.size // 3] = c[0]  # ties
        budget = float(rng.choice([0.0, 1e-4, 5e-4, 1e-2, 10.0]))
        ours = ts.keep_labels(c, budget)
        ref = omlp.budgeted_keep_labels(c, budget)
        assert np.array_equal(ours, ref.astype(np.float32))
        assert c[ours == 0].sum() <= budget


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
    fields = [(rng.normal(size=300), rng.lognormal(-9, 2, size=300)) for _ in range(20)]
    budget = 3e-3
    t = ts.calibrate_threshold(fields, budget)
    assert math.isfinite(t)
    assert all(c[z < t].sum() <= budget for z, c in fields)
    # the next larger logit would break the budget on at least one field
    above = min(z[z > t].min() for z, _ in fields if np.any(z > t))
    assert any(c[z < above + 1e-12].sum() > budget for z, c in fields)
    # nothing to drop within the budget -> threshold at -inf side never binds
    assert ts.calibrate_threshold([(np.zeros(3), np.ones(3))], 1e-3) == 0.0


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
