"""FP64 reference of the learned leaf selector network (oracle side, test infrastructure).

Network: 8 inputs -> 64 -> 64 -> 1 logit, exact-erf GELU after each hidden layer.
Parameter vector (4801 values, the C ABI's layout):
  W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3[1]     (row-major, out x in)
Loss: mean binary cross-entropy with logits, positive rows weighted by pos_weight:
  l(z, y) = -[pw y log sigmoid(z) + (1 - y) log(1 - sigmoid(z))].
Optimiser: Adam with bias correction.

Pins: central differences of the loss (tests), GELU against scipy's erf,
BCE against the explicit log-sigmoid formula.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

NIN, NHID = 8, 64
NPARAM = NHID * NIN + NHID + NHID * NHID + NHID + NHID + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + NHID * NIN].reshape(NHID, NIN); o += NHID * NIN
    b1 = p[o:o + NHID]; o += NHID
    W2 = p[o:o + NHID * NHID].reshape(NHID, NHID); o += NHID * NHID
    b2 = p[o:o + NHID]; o += NHID
    W3 = p[o:o + NHID]; o += NHID
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, W3, [b3]]).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def forward(p, X):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ W1.T + b1
    h1 = gelu(a1)
    a2 = h1 @ W2.T + b2
    h2 = gelu(a2)
    z = h2 @ W3 + b3
    return z, (X, a1, h1, a2, h2)


def bce_with_logits(z, y, pos_weight):
    z = np.asarray(z, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    # log sigmoid(z) = -log(1 + e^-z), log(1 - sigmoid(z)) = -z - log(1 + e^-z), stably
    ls = -np.logaddexp(0.0, -z)
    l1s = -np.logaddexp(0.0, z)
    return float(np.mean(-(pos_weight * y * ls + (1.0 - y) * l1s)))


def loss_and_grad(p, X, y, pos_weight):
    """Mean weighted BCE and its gradient with respect to the packed parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    z, (X, a1, h1, a2, h2) = forward(p, X)
    y = np.asarray(y, dtype=np.float64)
    m = X.shape[0]
    s = 1.0 / (1.0 + np.exp(-z))
    dz = (pos_weight * y * (s - 1.0) + (1.0 - y) * s) / m
    dW3 = h2.T @ dz
    db3 = dz.sum()
    dh2 = np.outer(dz, W3)
    da2 = dh2 * gelu_grad(a2)
    dW2 = da2.T @ h1
    db2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * gelu_grad(a1)
    dW1 = da1.T @ X
    db1 = da1.sum(axis=0)
    return bce_with_logits(z, y, pos_weight), pack(dW1, db1, dW2, db2, dW3, db3)


def adam_step(p, m1, m2, g, lr, b1, b2, eps, step):
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    mh = m1 / (1 - b1 ** step)
    vh = m2 / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m1, m2


def init_params(seed: int = 0):
    """He-style initialisation (normal, std sqrt(2 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, np.sqrt(2.0 / NIN), size=(NHID, NIN))
    W2 = rng.normal(0, np.sqrt(2.0 / NHID), size=(NHID, NHID))
    W3 = rng.normal(0, np.sqrt(1.0 / NHID), size=NHID)
    return pack(W1, np.zeros(NHID), W2, np.zeros(NHID), W3, 0.0)


def budgeted_keep_labels(contrib, budget):
    """Keep/drop labels of source leaves from their contributions c_b (norm fractions).

    The smallest contributions are dropped while their sum stays <= budget; since every
    leaf's field is non-negative, the dropped field's norm is at most that sum
    (triangle inequality).  Returns 1 = keep, 0 = drop.
    """
    c = np.asarray(contrib, dtype=np.float64)
    order = np.argsort(c, kind="stable")
    cs = np.cumsum(c[order])
    ndrop = int(np.searchsorted(cs, budget, side="right"))
    lab = np.ones(c.size, dtype=np.float64)
    lab[order[:ndrop]] = 0.0
    return lab


def budgeted_keep_labels_gram(G, s_norm, budget):
    """Keep/drop labels of source leaves from the Gram matrix of their fields at the targets.

    G[b, b'] = <S_b, S_b'> over the targets; s_norm = ||S|| over the same targets.  Leaves are
    taken in increasing order of ||S_b|| = sqrt(G[b, b]) and dropped while the norm of the sum
    of the dropped fields, sqrt(sum over b, b' in D of G[b, b']), stays <= budget * s_norm: the
    exact change of S that dropping D causes.  Returns 1 = keep, 0 = drop.
    """
    G = np.asarray(G, dtype=np.float64)
    order = np.argsort(np.sqrt(np.maximum(np.diag(G), 0.0)), kind="stable")
    dropped = []
    for b in order:
        trial = dropped + [int(b)]
        if np.sqrt(G[np.ix_(trial, trial)].sum()) > budget * s_norm:
            break
        dropped = trial
    lab = np.ones(G.shape[0], dtype=np.float64)
    lab[dropped] = 0.0
    return lab


def greedy_keep_labels(G, c, d0, s_norm, budget):
    """Keep/drop labels of the learned selector's rows under one error budget (test infrastructure).

    The rows are the source leaves of the threshold rule's source set (Sec. 3 eq. (18)); the
    points the rule itself leaves out have the field S_0 at the targets, and row b the field
    S_b.  Inputs: G[b, b'] = <S_b, S_b'>, c[b] = <S_0, S_b>, d0 = ||S_0||^2 over the targets,
    and s_norm = ||S|| of every source.  Dropping a set D of rows makes the error
    ||S_0 + sum_{b in D} S_b||, whose square is d0 + 2 sum_D c + sum_{D x D} G.  Rows are dropped
    one at a time, each time the row whose drop raises that square the least (ties: the lowest
    index), while the error stays <= budget * s_norm.  Returns 1 = keep, 0 = drop.
    """
    G = np.asarray(G, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    m = G.shape[0]
    lim = (budget * s_norm) ** 2

    def err2(D):
        D = list(D)
        return float(d0) + 2.0 * c[D].sum() + G[np.ix_(D, D)].sum()

    dropped = []
    while True:
        best, best_e = None, None
        for b in range(m):
            if b in dropped:
                continue
            e = err2(dropped + [b])
            if e <= lim and (best_e is None or e < best_e):
                best, best_e = b, e
        if best is None:
            break
        dropped.append(best)
    lab = np.ones(m, dtype=np.float64)
    lab[dropped] = 0.0
    return lab
