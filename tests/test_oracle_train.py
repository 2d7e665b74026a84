"""CPU pins of the oracle's training step (softmax(W phi + b) with
cross-entropy on the McKernel features), independent of its formulas:
closed forms, invariants and central finite differences in FP64."""
import numpy as np
import pytest

import workloads


def _setup(orc, batch=6, d=13, E=2, C=4, seed=5):
    rng = np.random.default_rng(seed)
    x = workloads.normal(batch, d, seed=seed)
    n = orc.padded_dim(d)
    p = orc.params(77, n, E, 1.5)
    B = p["B"].astype(np.float64)
    G = p["G"].astype(np.float64)
    S = p["S64"].copy()
    perm = p["perm"]
    W = rng.standard_normal((C, 2 * n * E)) * 0.5
    b = rng.standard_normal(C) * 0.1
    y = rng.integers(0, C, batch)
    return x.astype(np.float64), y, W, b, B, perm, G, S


def _loss(orc, x, y, W, b, B, perm, G, S):
    return orc.train_step(x, y, W, b, B, perm, G, S)["loss"]


def test_zero_classifier_loss_is_log_classes(orc):
    x, y, W, b, B, perm, G, S = _setup(orc)
    out = orc.train_step(x, y, np.zeros_like(W), np.zeros_like(b), B, perm, G, S)
    assert out["loss"] == pytest.approx(np.log(W.shape[0]), rel=1e-15)
    # uniform softmax: d loss / d b = (1/C - onehot) summed over rows / batch
    C = W.shape[0]
    expect = (np.full(C, 1.0 / C) * len(y) - np.bincount(y, minlength=C)) / len(y)
    np.testing.assert_allclose(out["db"], expect, rtol=0, atol=1e-15)


def test_softmax_gradient_rows_sum_to_zero(orc):
    rng = np.random.default_rng(1)
    lg = rng.standard_normal((9, 7)) * 3
    y = rng.integers(0, 7, 9)
    loss, dl = orc.softmax_xent(lg, y)
    np.testing.assert_allclose(dl.sum(axis=1), 0.0, atol=1e-16)
    # against the definition with log-sum-exp written out
    ref = np.mean([np.log(np.sum(np.exp(lg[i]))) - lg[i, y[i]] for i in range(9)])
    assert loss == pytest.approx(ref, rel=1e-14)


@pytest.mark.parametrize("which", ["W", "b", "x", "B", "G", "S"])
def test_gradients_match_central_differences(orc, which):
    x, y, W, b, B, perm, G, S = _setup(orc)
    args = {"x": x, "W": W, "b": b, "B": B, "G": G, "S": S}
    out = orc.train_step(x, y, W, b, B, perm, G, S)
    grad = {"x": out["dx"], "W": out["dW"], "b": out["db"], "B": out["dB"], "G": out["dG"], "S": out["dS"]}[which]
    rng = np.random.default_rng(hash(which) % 1000)
    a = args[which]
    def central(idx, h):
        ap, am = a.copy(), a.copy()
        ap[idx] += h
        am[idx] -= h
        kw = dict(args)
        kw[which] = ap
        lp = _loss(orc, kw["x"], y, kw["W"], kw["b"], kw["B"], perm, kw["G"], kw["S"])
        kw[which] = am
        lm = _loss(orc, kw["x"], y, kw["W"], kw["b"], kw["B"], perm, kw["G"], kw["S"])
        return (lp - lm) / (2 * h)

    h = 1e-3
    for _ in range(6):
        idx = tuple(rng.integers(0, s) for s in a.shape)
        fd1 = central(idx, h)
        assert fd1 == pytest.approx(grad[idx], rel=2e-3, abs=1e-8), (which, idx)
        # Richardson: the O(h^2) error of the central difference cancels
        fd = (4 * central(idx, h / 2) - fd1) / 3
        assert fd == pytest.approx(grad[idx], rel=1e-6, abs=1e-10), (which, idx)


def test_sgd_step_decreases_loss(orc):
    x, y, W, b, B, perm, G, S = _setup(orc, batch=16)
    out = orc.train_step(x, y, W, b, B, perm, G, S)
    lr = 0.05
    nxt = orc.train_step(x - lr * out["dx"] * 0, y, W - lr * out["dW"], b - lr * out["db"],
                         B - lr * out["dB"], perm, G - lr * out["dG"], S - lr * out["dS"])
    assert nxt["loss"] < out["loss"]
