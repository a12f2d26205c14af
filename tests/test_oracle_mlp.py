"""Pins for the oracle MLP (CPU only)."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp


def test_bf16_round_matches_torch():
    rng = np.random.Generator(np.random.PCG64(1))
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-8, 8, 4000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, -1e-40]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(x), ref)


def test_gelu_values():
    # GELU(z) = z Phi(z); Phi(1) = 0.841344746068543, Phi(-1) = 0.158655253931457
    assert mlp.gelu(np.array([1.0]))[0] == pytest.approx(0.841344746068543, abs=1e-14)
    assert mlp.gelu(np.array([-1.0]))[0] == pytest.approx(-0.158655253931457, abs=1e-14)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    z = np.linspace(-4, 4, 17)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(z), fd, atol=1e-8)


def _batch(B, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = np.abs(rng.normal(size=(B, mlp.D_IN))) * 0.1
    bt = rng.uniform(0, 2 * np.pi, B)
    gt = rng.uniform(0, np.pi, B)
    return x, bt, gt


def test_exact_backward_vs_finite_differences():
    params = mlp.init_params(3)
    x, bt, gt = _batch(6, 4)

    def L(pr):
        return mlp.loss_and_dout(mlp.forward_exact(pr, x), bt, gt)[0]

    _, dout = mlp.loss_and_dout(mlp.forward_exact(params, x), bt, gt)
    g = mlp.backward_exact(params, x, dout)
    rng = np.random.Generator(np.random.PCG64(9))
    h = 1e-6
    for key in ("W1", "b1", "W2", "b2", "W3", "b3"):
        for _ in range(6):
            idx = tuple(int(rng.integers(0, s)) for s in params[key].shape)
            pp = {k: v.copy() for k, v in params.items()}
            pm = {k: v.copy() for k, v in params.items()}
            pp[key][idx] += h
            pm[key][idx] -= h
            fd = (L(pp) - L(pm)) / (2 * h)
            assert g[key][idx] == pytest.approx(fd, abs=1e-9, rel=1e-5)


def test_bf16_backward_close_to_exact():
    params = mlp.init_params(5)
    x, bt, gt = _batch(64, 6)
    o, cache = mlp.forward(params, x)
    o_exact = mlp.forward_exact(params, x)
    np.testing.assert_allclose(o, o_exact, atol=3e-2)
    _, dout = mlp.loss_and_dout(o, bt, gt)
    g = mlp.backward(params, cache, dout)
    ge = mlp.backward_exact(params, x, dout)
    for k in g:
        a, b = g[k].ravel(), ge[k].ravel()
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
        assert cos > 0.999, k


def test_adam_first_step_is_signed_lr():
    """With zero moments, bias correction makes step 1 equal lr * g/(|g|+eps')."""
    params = {"w": np.array([1.0, -2.0, 3.0])}
    grads = {"w": np.array([0.5, -4.0, 1e-3])}
    state = {}
    mlp.adam_step(params, grads, state, lr=0.01, eps=0.0)
    np.testing.assert_allclose(params["w"], [1.0 - 0.01, -2.0 + 0.01, 3.0 - 0.01], atol=1e-15)


def test_features_layout():
    hist = np.array([2, 5, 1, 0])
    x = mlp.features(hist, 3, 4.0 / 3.0, 16)
    assert x.shape == (131,)
    np.testing.assert_allclose(x[:4], [2 / 8, 5 / 8, 1 / 8, 0])
    assert not x[4:128].any()
    assert x[128] == 3 / 24 and x[129] == pytest.approx(4.0 / 24.0) and x[130] == pytest.approx(4 / 6)


def test_angle_map_and_loss_gradient():
    rng = np.random.Generator(np.random.PCG64(2))
    o = rng.normal(size=(5, 2))
    bt = rng.uniform(0, 2 * np.pi, 5)
    gt = rng.uniform(0, np.pi, 5)
    beta, gamma = mlp.angles(o)
    assert np.all((beta > 0) & (beta < 2 * math.pi) & (gamma > 0) & (gamma < math.pi))
    loss, dout = mlp.loss_and_dout(o, bt, gt)
    h = 1e-7
    for i in range(5):
        for j in range(2):
            op, om = o.copy(), o.copy()
            op[i, j] += h
            om[i, j] -= h
            fd = (mlp.loss_and_dout(op, bt, gt)[0] - mlp.loss_and_dout(om, bt, gt)[0]) / (2 * h)
            assert dout[i, j] == pytest.approx(fd, abs=1e-8)


def test_adam_constant_gradient_moves_lr_per_step():
    """With the same gradient g at every step, the moments are m_t = (1 - b1^t) g
    and v_t = (1 - b2^t) g^2, so the bias-corrected m-hat = g and v-hat = g^2 at
    every t: each step moves every parameter by exactly lr * sign(g) (eps = 0).
    A wrong moment recursion or a bias correction that does not use t fails."""
    params = {"w": np.array([1.0, -2.0, 3.0, 0.25])}
    grads = {"w": np.array([0.5, -4.0, 1e-3, -7.0])}
    state = {}
    lr = 0.01
    for t in range(1, 13):
        mlp.adam_step(params, grads, state, lr=lr, b1=0.9, b2=0.999, eps=0.0)
        expect = np.array([1.0, -2.0, 3.0, 0.25]) - t * lr * np.sign(grads["w"])
        np.testing.assert_allclose(params["w"], expect, rtol=0, atol=1e-13)
    assert state["t"] == 12


def test_adam_two_steps_hand_computed():
    """Scalar parameter 0.5, gradients 1 then -2, lr 0.1, b1 0.9, b2 0.999, eps 0.
    Step 1: m = 0.1, v = 0.001, m-hat = 1, v-hat = 1, so w = 0.4.
    Step 2: m = 0.09 - 0.2 = -0.11, v = 0.000999 + 0.004 = 0.004999,
    m-hat = -0.11 / 0.19 = -11/19, v-hat = 0.004999 / 0.001999 = 4999/1999,
    step = 0.1 * (11/19) / sqrt(4999/1999) = 0.0366103527035846 (by hand with
    exact fractions), so w = 0.4366103527035846."""
    params = {"w": np.array([0.5])}
    state = {}
    mlp.adam_step(params, {"w": np.array([1.0])}, state, lr=0.1, b1=0.9, b2=0.999, eps=0.0)
    assert params["w"][0] == pytest.approx(0.4, abs=1e-15)
    mlp.adam_step(params, {"w": np.array([-2.0])}, state, lr=0.1, b1=0.9, b2=0.999, eps=0.0)
    assert state["m_w"][0] == pytest.approx(-0.11, abs=1e-16)
    assert state["v_w"][0] == pytest.approx(0.004999, abs=1e-17)
    assert params["w"][0] == pytest.approx(0.4366103527035846, abs=1e-15)


def test_loss_value_hand_computed_batch_of_two():
    """o = [[0, 0], [ln 3, -ln 3]]: sigmoids 1/2, 1/2 and 3/4, 1/4, so
    (beta, gamma) = (pi, pi/2) and (3 pi/2, pi/4). Targets (pi/2, pi/2) and
    (pi, 0): the normalized errors are (1/4, 0) and (1/4, 1/4), the loss is the
    batch mean of (1/16, 1/8) = 3/32, and dL/do = 2 r sig (1 - sig) / 2:
    [[1/16, 0], [3/64, 3/64]]."""
    o = np.array([[0.0, 0.0], [math.log(3.0), -math.log(3.0)]])
    loss, dout = mlp.loss_and_dout(o, np.array([math.pi / 2, math.pi]), np.array([math.pi / 2, 0.0]))
    assert loss == pytest.approx(3.0 / 32.0, abs=1e-15)
    np.testing.assert_allclose(dout, [[1.0 / 16.0, 0.0], [3.0 / 64.0, 3.0 / 64.0]], rtol=0, atol=1e-15)
