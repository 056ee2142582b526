"""Pins of the warm-start network oracle: bf16 rounding against torch's
conversion and hand-checked ties, forward pass and gradients against torch
autograd in float64, gradients against central differences, Adam's first
step against its closed form, and the size of the bf16 effect."""

import numpy as np
import pytest
import torch

import synth
from oracle import mlp as omlp


def test_bf16_rounding_ties_and_library():
    # spacing of bfloat16 at 1 is 2^-7; halfway cases go to the even significand
    assert omlp.bf16(1 + 2 ** -8) == 1.0
    assert omlp.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6
    assert omlp.bf16(-(1 + 2 ** -8)) == -1.0
    assert omlp.bf16(1 + 2 ** -8 + 2 ** -20) == 1 + 2 ** -7
    assert omlp.bf16(0.0) == 0.0
    rng = np.random.default_rng(0)
    v = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(omlp.bf16(v.astype(np.float64)), want)


def _torch_net(p, H, O):
    W1, b1, W2, b2, W3, b3 = [torch.tensor(a, dtype=torch.float64, requires_grad=True)
                              for a in omlp.unpack(p, H, O)]
    return [W1, b1, W2, b2, W3, b3]


@pytest.mark.parametrize("H,O,n", [(32, 5, 3), (64, 40, 17)])
def test_forward_and_gradient_match_autograd(H, O, n):
    p = synth.mlp_init(H, O, seed=H + O).astype(np.float64)
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, n)
    t = rng.normal(size=(n, O)) * 0.3
    W1, b1, W2, b2, W3, b3 = _torch_net(p, H, O)
    xt = torch.tensor(x)[:, None]
    h1 = torch.tanh(xt @ W1[None, :] + b1)
    h2 = torch.tanh(h1 @ W2.T + b2)
    y = h2 @ W3.T + b3
    loss = ((y - torch.tensor(t)) ** 2).mean()
    loss.backward()
    want_g = np.concatenate([a.grad.numpy().ravel() for a in (W1, b1, W2, b2, W3, b3)])
    got_y, _ = omlp.forward(p, x, H, O, bf16_inputs=False)
    got_l, got_g = omlp.loss_grad(p, x, t, H, O, bf16_inputs=False)
    np.testing.assert_allclose(got_y, y.detach().numpy(), rtol=1e-13, atol=1e-14)
    assert abs(got_l - loss.item()) < 1e-14
    np.testing.assert_allclose(got_g, want_g, rtol=1e-11, atol=1e-15)


def test_gradient_matches_central_differences():
    H, O, n = 16, 3, 4
    p = synth.mlp_init(H, O, seed=9).astype(np.float64)
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, n)
    t = rng.normal(size=(n, O))
    _, g = omlp.loss_grad(p, x, t, H, O, bf16_inputs=False)
    eps = 1e-6
    for k in rng.choice(p.size, 40, replace=False):
        pp, pm = p.copy(), p.copy()
        pp[k] += eps
        pm[k] -= eps
        fd = (omlp.loss_grad(pp, x, t, H, O, False)[0] - omlp.loss_grad(pm, x, t, H, O, False)[0]) / (2 * eps)
        assert abs(fd - g[k]) < 1e-8 + 1e-6 * abs(g[k])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    q, m, v = omlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1, 1e-2)
    # bias-corrected moments equal g and g^2 on the first step
    np.testing.assert_allclose(q, p - 1e-2 * g / (np.abs(g) + omlp.EPS), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_bf16_effect_is_within_rounding():
    H, O, n = 64, 20, 10
    p = synth.mlp_init(H, O, seed=4).astype(np.float64)
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, n)
    t = rng.normal(size=(n, O)) * 0.2
    l64, g64 = omlp.loss_grad(p, x, t, H, O, bf16_inputs=False)
    l16, g16 = omlp.loss_grad(p, x, t, H, O, bf16_inputs=True)
    assert abs(l16 - l64) < 2 ** -7 * l64
    assert np.linalg.norm(g16 - g64) < 2 ** -6 * np.linalg.norm(g64)
    assert not np.array_equal(g16, g64)


def test_training_fits_a_smooth_curve():
    H, O = 32, 4
    p = synth.mlp_init(H, O, seed=6).astype(np.float64)
    x = np.linspace(0, 1, 12)
    t = np.stack([np.sin(2 * x), x ** 2, np.cos(3 * x) * 0.5, 0.3 - x], axis=1)
    p2, losses, _ = omlp.train(p, x, t, H, O, 400, 3e-3)
    assert losses[-1] < 0.02 * losses[0]
