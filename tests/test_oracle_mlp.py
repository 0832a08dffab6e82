"""Pins of the FP64 selector-network oracle: central differences, GELU and BCE closed forms, Adam."""
import math

import numpy as np
import pytest
from scipy.special import erf

from oracle import mlp


def test_gelu_matches_erf_definition_and_derivative():
    x = np.linspace(-6, 6, 101)
    assert np.allclose(mlp.gelu(x), [0.5 * v * (1 + math.erf(v / math.sqrt(2))) for v in x], rtol=1e-14, atol=1e-15)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(x), fd, rtol=1e-7, atol=1e-9)


def test_bce_closed_form():
    z = np.array([-30.0, -2.0, 0.0, 1.5, 40.0])
    y = np.array([1.0, 0.0, 1.0, 1.0, 0.0])
    pw = 3.0
    sig = 1 / (1 + np.exp(-z))
    direct = -(pw * y * np.log(np.maximum(sig, 1e-300)) + (1 - y) * np.log(np.maximum(1 - sig, 1e-300)))
    # the extreme rows saturate the naive formula; compare on the finite ones and check the stable ones
    assert mlp.bce_with_logits(z[1:4], y[1:4], pw) == pytest.approx(direct[1:4].mean(), rel=1e-13)
    assert mlp.bce_with_logits(np.array([-30.0]), np.array([1.0]), pw) == pytest.approx(pw * 30.0, rel=1e-12)
    assert mlp.bce_with_logits(np.array([40.0]), np.array([0.0]), pw) == pytest.approx(40.0, rel=1e-12)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = mlp.init_params(1) * 0.7
    X = rng.normal(size=(37, 8))
    y = (rng.uniform(size=37) < 0.3).astype(float)
    _, g = mlp.loss_and_grad(p, X, y, 2.5)
    idx = rng.choice(mlp.NPARAM, size=120, replace=False)
    idx = np.concatenate([idx, [0, 511, 512, 575, 576, 4671, 4672, 4735, 4736, 4799, 4800]])
    h = 1e-6
    for k in idx:
        e = np.zeros(mlp.NPARAM)
        e[k] = h
        fd = (mlp.loss_and_grad(p + e, X, y, 2.5)[0] - mlp.loss_and_grad(p - e, X, y, 2.5)[0]) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-9), k


def test_layout_and_adam():
    p = np.arange(mlp.NPARAM, dtype=float)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    assert W1[0, 1] == 1 and b1[0] == 512 and W2[0, 0] == 576 and b2[0] == 4672 and W3[0] == 4736 and b3 == 4800
    assert np.array_equal(mlp.pack(W1, b1, W2, b2, W3, b3), p)
    # first Adam step moves every parameter by lr against the gradient sign (bias-corrected)
    g = np.linspace(-1, 1, mlp.NPARAM) + 1e-3
    q, m1, m2 = mlp.adam_step(np.zeros(mlp.NPARAM), np.zeros(mlp.NPARAM), np.zeros(mlp.NPARAM), g, 1e-2, 0.9, 0.999,
                              1e-12, 1)
    assert np.allclose(q, -1e-2 * np.sign(g), rtol=1e-6)


def test_budgeted_labels():
    c = np.array([0.5, 1e-4, 2e-4, 0.3, 3e-4, 0.2])
    lab = mlp.budgeted_keep_labels(c, 5e-4)
    # 1e-4 + 2e-4 = 3e-4 <= 5e-4; adding 3e-4 exceeds the budget
    assert lab.tolist() == [1, 0, 0, 1, 1, 1]
    assert mlp.budgeted_keep_labels(c, 0.0).tolist() == [1] * 6


def test_gram_labels_parallel_fields_reduce_to_the_triangle_rule():
    # identical directions: ||sum|| = sum of norms, so the rule is the running-sum rule
    rng = np.random.default_rng(3)
    c = rng.lognormal(-7, 2, size=40)
    G = np.outer(c, c)
    for budget in (1e-4, 1e-3, 1e-2):
        assert np.array_equal(mlp.budgeted_keep_labels_gram(G, 1.0, budget),
                              mlp.budgeted_keep_labels(c, budget))


def test_gram_labels_orthogonal_fields_drop_by_root_sum_of_squares():
    # disjoint supports: ||sum||^2 = sum of squared norms; hand-checked case
    c = np.array([3e-4, 1e-4, 0.5, 2e-4, 4e-4])
    G = np.diag(c ** 2)
    lab = mlp.budgeted_keep_labels_gram(G, 1.0, 4e-4)
    # sqrt(1e-8 + 4e-8 + 9e-8) = 3.74e-4 <= 4e-4; adding 4e-4 gives 5.48e-4
    assert lab.tolist() == [0, 0, 1, 0, 1]


def test_gram_labels_brute_force_on_explicit_fields():
    rng = np.random.default_rng(4)
    for trial in range(20):
        m, nt = int(rng.integers(2, 30)), 50
        F = rng.lognormal(-6, 2, size=(m, 1)) * rng.uniform(0, 1, size=(m, nt)) ** 3
        S = F.sum(axis=0)
        budget = float(rng.choice([1e-3, 1e-2, 1e-1]))
        lab = mlp.budgeted_keep_labels_gram(F @ F.T, np.linalg.norm(S), budget)
        drop = np.flatnonzero(lab == 0)
        # the dropped set changes S by at most the budget ...
        assert np.linalg.norm(F[drop].sum(axis=0)) <= budget * np.linalg.norm(S) * (1 + 1e-12)
        # ... and is the longest prefix in order of ||S_b|| with that property
        order = np.argsort(np.linalg.norm(F, axis=1), kind="stable")
        assert np.array_equal(np.sort(drop), np.sort(order[:drop.size]))
        if drop.size < m:
            nxt = order[:drop.size + 1]
            assert np.linalg.norm(F[nxt].sum(axis=0)) > budget * np.linalg.norm(S)


def test_greedy_labels_orthogonal_fields_hand_case():
    # disjoint supports, no field left out by the rule: the cheapest rows go first while the
    # root sum of squares stays within the budget
    c = np.array([3e-4, 1e-4, 0.5, 2e-4, 4e-4])
    lab = mlp.greedy_keep_labels(np.diag(c ** 2), np.zeros(5), 0.0, 1.0, 4e-4)
    assert lab.tolist() == [0, 0, 1, 0, 1]
    # with a left-out field of norm 3e-4 that overlaps nothing, only 1e-4 and 2e-4 still fit
    # (sqrt(9e-8 + 1e-8 + 4e-8) = 3.74e-4; adding 3e-4 gives 4.8e-4)
    lab = mlp.greedy_keep_labels(np.diag(c ** 2), np.zeros(5), 9e-8, 1.0, 4e-4)
    assert lab.tolist() == [1, 0, 1, 0, 1]
    # the left-out field alone over the budget: nothing is dropped
    assert mlp.greedy_keep_labels(np.diag(c ** 2), np.zeros(5), 1.0, 1.0, 4e-4).tolist() == [1] * 5


def test_greedy_labels_brute_force_on_explicit_fields():
    """From explicit non-negative fields: every greedy step is the cheapest, the final error is within
    the budget, and no remaining row could be dropped too."""
    rng = np.random.default_rng(8)
    for trial in range(15):
        m, nt = int(rng.integers(2, 14)), 40
        F = rng.lognormal(-6, 2, size=(m, 1)) * rng.uniform(0, 1, size=(m, nt)) ** 3
        F0 = rng.lognormal(-9, 1) * rng.uniform(0, 1, size=nt) ** 2
        S = F.sum(axis=0) + F0
        budget = float(rng.choice([1e-3, 1e-2, 1e-1]))
        lab = mlp.greedy_keep_labels(F @ F.T, F @ F0, float(F0 @ F0), np.linalg.norm(S), budget)
        drop = np.flatnonzero(lab == 0)
        lim = budget * np.linalg.norm(S)
        if drop.size:
            assert np.linalg.norm(F0 + F[drop].sum(axis=0)) <= lim * (1 + 1e-12)
        for b in np.flatnonzero(lab == 1):
            assert np.linalg.norm(F0 + F[drop].sum(axis=0) + F[b]) > lim * (1 - 1e-12)
        # replay: each step took the cheapest row among those that fit
        taken = []
        for _ in range(drop.size):
            rest = [b for b in range(m) if b not in taken]
            norms = [np.linalg.norm(F0 + F[taken + [b]].sum(axis=0)) for b in rest]
            nxt = rest[int(np.argmin(norms))]
            taken.append(nxt)
        assert sorted(taken) == sorted(drop.tolist())
