"""Pins of the FP64 gate-network oracle (brute force and closed forms)."""
import numpy as np
import pytest

from oracle import mlp


def _data(n=40, seed=1):
    rng = np.random.default_rng(seed)
    F = rng.normal(size=(n, 12))
    y = (rng.random(n) < 0.3).astype(float)
    return F, y


def test_backward_matches_central_differences():
    """Analytic backward against FP64 central differences (step 1e-6)."""
    F, y = _data()
    p = mlp.init_params(3, mu=np.zeros(12), sigma=np.ones(12))
    p[mlp.OFF["b1"]:mlp.OFF["b1"] + 64] = 0.05  # keep ReLU kinks away from the sample points
    p[mlp.OFF["b2"]:mlp.OFF["b2"] + 64] = 0.05
    _, g = mlp.loss_and_grad(p, F, y, pos_weight=3.0)
    rng = np.random.default_rng(7)
    idx = np.concatenate([rng.choice(np.nonzero(mlp.TRAINABLE)[0], 60, replace=False), [mlp.OFF["b3"]]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss_and_grad(pp, F, y, 3.0)[0] - mlp.loss_and_grad(pm, F, y, 3.0)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])
    # padded inputs and the fixed slots get no gradient
    assert np.all(g[~mlp.TRAINABLE] == 0)
    assert np.all(g[mlp.OFF["W1"] + 12 * 64:mlp.OFF["W1"] + 16 * 64] == 0)


def test_loss_closed_forms():
    """All-zero weights: z = b3, loss = mean w log(1 + exp(-+b3))."""
    F, y = _data(8)
    p = np.zeros(mlp.N_PARAM)
    p[mlp.OFF["b3"]] = 0.7
    loss, g = mlp.loss_and_grad(p, F, y, pos_weight=2.0)
    w = np.where(y > 0.5, 2.0, 1.0)
    ref = np.mean(w * np.where(y > 0.5, np.log1p(np.exp(-0.7)), np.log1p(np.exp(0.7))))
    assert loss == pytest.approx(ref, rel=1e-14)
    assert g[mlp.OFF["b3"]] == pytest.approx(np.mean(w * (1 / (1 + np.exp(-0.7)) - y)), rel=1e-14)


def test_bf16_rounding_is_round_to_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -9, -2.5, 3.0e38])
    r = mlp.bf16(x)
    assert r[0] == 1.0
    # 1+2^-8 is a tie between 1 and 1+2^-7 -> even mantissa (1.0)
    assert r[1] == 1.0
    assert r[2] == 1.0 + 2 ** -7  # above the tie -> up
    assert r[3] == 1.0            # below the tie -> down
    assert r[4] == -2.5


def test_adam_first_step_is_lr_sign():
    """First Adam step moves every trainable weight by lr * sign(g) (bias-corrected)."""
    p = mlp.init_params(0)
    g = np.random.default_rng(2).normal(size=mlp.N_PARAM) * mlp.TRAINABLE
    m, v = np.zeros(mlp.N_PARAM), np.zeros(mlp.N_PARAM)
    p1 = mlp.adam_step(p.copy(), g, m, v, 1, 1e-3)
    d = (p1 - p)[mlp.TRAINABLE]
    assert np.allclose(d, -1e-3 * np.sign(g[mlp.TRAINABLE]), rtol=1e-4)
    assert np.all(p1[~mlp.TRAINABLE] == p[~mlp.TRAINABLE])
