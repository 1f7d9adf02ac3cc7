"""Pins of the oracle's Adam update (the optimiser the paper trains with,
Sec. 4.1 and 4.2), against closed forms and an independent implementation."""
import numpy as np
import torch

import oracle as O


def test_constant_gradient_moves_by_lr_each_step():
    # with a constant gradient the bias-corrected moments are g and g^2
    # exactly, so each step moves every weight by lr * g / (|g| + eps)
    rng = np.random.default_rng(0)
    W0 = [rng.standard_normal((5, 3)), rng.standard_normal((4, 1))]
    g = [rng.standard_normal(w.shape) for w in W0]
    m = [np.zeros_like(w) for w in W0]
    v = [np.zeros_like(w) for w in W0]
    W = W0
    lr, eps = 1e-2, 1e-8
    for t in range(1, 8):
        W, m, v = O.adam(W, g, m, v, t, lr, eps=eps)
        for w, w0, gg in zip(W, W0, g):
            np.testing.assert_allclose(w, w0 - t * lr * gg / (np.abs(gg) + eps), rtol=1e-12, atol=1e-14)


def test_zero_gradient_keeps_weights_and_decays_moments():
    W = [np.ones((3, 2))]
    m = [np.full((3, 2), 0.5)]
    v = [np.full((3, 2), 0.25)]
    W1, m1, v1 = O.adam(W, [np.zeros((3, 2))], m, v, 1, 1e-3, beta1=0.9, beta2=0.999, eps=1e-8)
    np.testing.assert_array_equal(m1[0], 0.9 * m[0])
    np.testing.assert_array_equal(v1[0], 0.999 * v[0])
    # a zero gradient still moves W by the decayed first moment
    assert np.all(W1[0] < W[0])


def test_matches_torch_adam():
    # torch.optim.Adam (an independent implementation) on the same tensors
    rng = np.random.default_rng(1)
    W = [rng.standard_normal((6, 4)), rng.standard_normal((7,))]
    params = [torch.tensor(w, dtype=torch.float64, requires_grad=True) for w in W]
    opt = torch.optim.Adam(params, lr=3e-3, betas=(0.85, 0.995), eps=1e-7)
    m = [np.zeros_like(w) for w in W]
    v = [np.zeros_like(w) for w in W]
    for t in range(1, 6):
        g = [rng.standard_normal(w.shape) for w in W]
        for p, gg in zip(params, g):
            p.grad = torch.tensor(gg, dtype=torch.float64)
        opt.step()
        W, m, v = O.adam(W, g, m, v, t, 3e-3, beta1=0.85, beta2=0.995, eps=1e-7)
        for p, w in zip(params, W):
            np.testing.assert_allclose(p.detach().numpy(), w, rtol=1e-13, atol=1e-15)
