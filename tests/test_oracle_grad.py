"""Pins of the oracle's weight gradient dL/dW (the reverse pass of the step).

References: central finite differences of the loss in double precision
(coordinates and random directions), exactness of finite differences for the
last layer of a Poisson net (the loss is quadratic there), PyTorch CPU
float64 autograd through nested derivatives of an independently written
HRKAN, and additivity of the reverse pass over point shards.
"""
import numpy as np
import pytest
import torch

import oracle as O
from conftest import relerr
from paper_2409_14248_amd import workloads as WL
from test_oracle_jets import torch_hrkan


def small_problem(kind, widths=(2, 4, 3, 1), G=5, n_int=60, n_bc=16, seed=0, std=0.4):
    net = WL.Net(widths, G=G)
    rng = np.random.default_rng(seed)
    Ws = [rng.standard_normal(s) * std for s in net.weight_shapes()]
    if kind == WL.POISSON2D:
        x_int, x_bc, g = WL.poisson_points(n_int, n_bc, rng)
        pde = WL.Pde(WL.POISSON2D)
    else:
        x_int, x_bc, g = WL.burgers_points(n_int, n_bc, rng)
        pde = WL.Pde(WL.BURGERS1D, nu=0.05)
    return net, pde, Ws, x_int, x_bc, g


def loss_of(net, pde, Ws, x_int, x_bc, g):
    return O.step(net, pde, Ws, x_int, x_bc, g)["loss"][0]


def central(f, h):
    """Central difference with one Richardson step (error O(h^4))."""
    d = lambda t: (f(t) - f(-t)) / (2 * t)
    return (4 * d(h / 2) - d(h)) / 3


@pytest.mark.parametrize("kind", [WL.POISSON2D, WL.BURGERS1D])
def test_gradient_coordinates_fd(kind):
    net, pde, Ws, xi, xb, g = small_problem(kind)
    gW = O.step(net, pde, Ws, xi, xb, g)["gW"]
    rng = np.random.default_rng(3)
    h = 1e-4
    for l, W in enumerate(Ws):
        flat = rng.choice(W.size, size=min(12, W.size), replace=False)
        for f in flat:
            def shifted(t):
                Wt = [w.copy() for w in Ws]
                Wt[l].flat[f] += t
                return loss_of(net, pde, Wt, xi, xb, g)
            fd = central(shifted, h)
            scale = max(1e-3, np.max(np.abs(gW[l])))
            assert abs(fd - gW[l].flat[f]) < 1e-6 * scale, (l, f, fd, gW[l].flat[f])


@pytest.mark.parametrize("kind", [WL.POISSON2D, WL.BURGERS1D])
def test_gradient_directional_fd(kind):
    net, pde, Ws, xi, xb, g = small_problem(kind, seed=7)
    gW = O.step(net, pde, Ws, xi, xb, g)["gW"]
    rng = np.random.default_rng(9)
    h = 1e-4
    for _ in range(4):
        V = [rng.standard_normal(w.shape) for w in Ws]
        nrm = np.sqrt(sum(np.sum(v * v) for v in V))
        V = [v / nrm for v in V]
        fd = central(lambda t: loss_of(net, pde, [w + t * v for w, v in zip(Ws, V)], xi, xb, g), h)
        an = sum(np.sum(a * v) for a, v in zip(gW, V))
        assert abs(fd - an) < 1e-6 * max(1.0, abs(an))


def test_poisson_last_layer_quadratic_fd_exact():
    # For Poisson the loss is a quadratic function of the last layer's
    # weights, so a central difference with a large step is exact.
    net, pde, Ws, xi, xb, g = small_problem(WL.POISSON2D, seed=2)
    gW = O.step(net, pde, Ws, xi, xb, g)["gW"]
    h = 0.5
    L = len(Ws) - 1
    for f in range(0, Ws[L].size, 3):
        Wp = [w.copy() for w in Ws]
        Wm = [w.copy() for w in Ws]
        Wp[L].flat[f] += h
        Wm[L].flat[f] -= h
        fd = (loss_of(net, pde, Wp, xi, xb, g) - loss_of(net, pde, Wm, xi, xb, g)) / (2 * h)
        assert abs(fd - gW[L].flat[f]) < 1e-11 * max(1.0, abs(fd))


@pytest.mark.parametrize("kind", [WL.POISSON2D, WL.BURGERS1D])
def test_gradient_matches_torch_autograd(kind):
    net, pde, Ws, xi, xb, g = small_problem(kind, widths=(2, 3, 3, 1), seed=5)
    res = O.step(net, pde, Ws, xi, xb, g)
    X = torch.tensor(xi, requires_grad=True)
    Wt = [torch.tensor(w, requires_grad=True) for w in Ws]
    u = torch_hrkan(net, Wt, X)
    gr = torch.autograd.grad(u.sum(), X, create_graph=True)[0]
    ux, uy = gr[:, 0], gr[:, 1]
    uxx = torch.autograd.grad(ux.sum(), X, create_graph=True)[0][:, 0]
    if kind == WL.POISSON2D:
        uyy = torch.autograd.grad(uy.sum(), X, create_graph=True)[0][:, 1]
        Xd = X.detach()
        r = uxx + uyy + 2 * np.pi ** 2 * torch.sin(np.pi * Xd[:, 0]) * torch.sin(np.pi * Xd[:, 1])
    else:
        r = uy + u * ux - pde.nu * uxx
    ub = torch_hrkan(net, Wt, torch.tensor(xb))
    L = pde.alpha * torch.mean(r ** 2) + torch.mean((ub - torch.tensor(g)) ** 2)
    assert abs(L.item() - res["loss"][0]) < 1e-12 * abs(L.item())
    grads = torch.autograd.grad(L, Wt)
    for a, b in zip(res["gW"], grads):
        assert relerr(a, b.numpy()) < 1e-11


def test_reverse_pass_is_additive_over_point_shards():
    net, pde, Ws, xi, xb, g = small_problem(WL.BURGERS1D, n_int=80, seed=4)
    seed = np.random.default_rng(1).standard_normal((5, 80))
    full = O.backward(net, Ws, xi, seed)
    a = O.backward(net, Ws, xi[:33], np.ascontiguousarray(seed[:, :33]))
    b = O.backward(net, Ws, xi[33:], np.ascontiguousarray(seed[:, 33:]))
    for f, x, y in zip(full, a, b):
        assert relerr(f, x + y) < 1e-14


def test_layer_backward_matches_network_backward():
    net, pde, Ws, xi, xb, g = small_problem(WL.POISSON2D, widths=(2, 5, 4, 1), n_int=40, seed=8)
    seed = np.random.default_rng(2).standard_normal((5, 40))
    full = O.backward(net, Ws, xi, seed)
    _, blocks = O.forward(net, Ws, xi, all_jets=True)
    ybar = seed.reshape(5, 1, 40)
    for l in range(len(Ws) - 1, -1, -1):
        zbar, gW = O.layer_backward(net, l, Ws[l], blocks[l], ybar)
        assert relerr(gW, full[l]) < 1e-13
        ybar = zbar
