"""Pins of the oracle's jets above second order and of the linear PDE of any
order (Sec. 3: a PDE with a fifth-derivative term is handled by a larger HR
order m, such as 6; the derivatives of the basis then stay non-zero and
smooth).

References used, none of them the oracle's formulas:
- PyTorch CPU float64 nested autograd (up to five nested gradients per
  coordinate) on an independently written HRKAN forward;
- exact rational arithmetic: a one-layer network whose output along x is a
  weighted sum of basis functions, differentiated as expanded polynomials;
- consistency across jet orders (the order-2 slots of an order-5 run);
- the manufactured solution sin(pi x) sin(pi y), whose derivatives of any
  order come from the complex exponential, and the Poisson residual as the
  linear PDE with two second-derivative terms;
- the whole loss and its weight gradient by torch autograd, and central
  differences of the oracle's own loss.
"""
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle as O
from conftest import relerr
from test_oracle_basis import exact_hr
from test_oracle_jets import rand_weights, torch_hrkan
from paper_2409_14248_amd import workloads as WL
from paper_2409_14248_amd.workloads import LINEAR2D, POISSON2D, Net, Pde


def torch_jets_n(net, Ws, x, n):
    """[u, d^k u/dx^k (k = 1..n), d^k u/dy^k (k = 1..n)] by nested autograd."""
    X = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    Wt = [torch.tensor(w, dtype=torch.float64, requires_grad=True) for w in Ws]
    u = torch_hrkan(net, Wt, X)
    out = [u]
    for axis in (0, 1):
        d = u
        for _ in range(n):
            d = torch.autograd.grad(d.sum(), X, create_graph=True)[0][:, axis]
            out.append(d)
    return X, Wt, out


HIGH_NETS = [
    Net((2, 3, 1), G=5, m=6, order=3),
    Net((2, 3, 1), G=5, m=6, order=4),
    Net((2, 4, 3, 1), G=6, m=6, order=4),
    Net((2, 2, 2, 1), G=4, m=7, order=5),
    Net((2, 3, 2, 1), G=5, m=6, order=5),
]


@pytest.mark.parametrize("net", HIGH_NETS)
def test_high_order_jets_match_torch_autograd(net):
    Ws = rand_weights(net, 21)
    x = np.random.default_rng(6).uniform(-1, 1, size=(61, 2))
    u = O.forward(net, Ws, x)
    assert u.shape == (1 + 2 * net.order, 61)
    _, _, ref = torch_jets_n(net, Ws, x, net.order)
    for slot, r in enumerate(ref):
        r = r.detach().numpy()
        assert relerr(u[slot], r) < 1e-10, (slot, relerr(u[slot], r))


def test_order_two_slots_inside_an_order_five_run():
    net5 = Net((2, 4, 3, 1), G=6, m=6, order=5)
    net2 = Net((2, 4, 3, 1), G=6, m=6)
    Ws = rand_weights(net5, 3)
    x = np.random.default_rng(7).uniform(-1, 1, size=(200, 2))
    u5 = O.forward(net5, Ws, x)
    u2 = O.forward(net2, Ws, x)
    # order 2: U, X, XX, Y, YY; order 5: U, X1..X5, Y1..Y5
    for s2, s5 in [(0, 0), (1, 1), (2, 2), (3, 6), (4, 7)]:
        assert relerr(u5[s5], u2[s2]) < 1e-13, (s2, s5)


def test_single_layer_exact_rationals():
    """[2,1] with weights only on input 0: d^k u/dx^k = sum_b W_b v_b^(k)(x)
    exactly; the y-derivatives are zero."""
    net = Net((2, 1), G=4, m=6, order=5)
    nb = net.n_basis
    wx = [Fraction(3 * b - 5, 4) for b in range(nb)]
    W = np.zeros((2 * nb, 1))
    W[:nb, 0] = [float(w) for w in wx]
    h = Fraction(2, net.G)
    xs = [Fraction(-13, 16), Fraction(-1, 8), Fraction(5, 32), Fraction(11, 16), Fraction(29, 32)]
    x = np.array([[float(v), 0.3] for v in xs])
    u = O.forward(net, [W], x)
    for p, xv in enumerate(xs):
        for k in range(6):
            ref = Fraction(0)
            for b in range(nb):
                s = -1 + (b - net.k) * h
                e = -1 + (b + 1) * h
                ref += wx[b] * exact_hr(net.m, s, e, xv, k)
            scale = max(1.0, float(abs(ref)), float((Fraction(2) / (4 * h)) ** k) * 10)
            assert abs(u[k, p] - float(ref)) <= 1e-12 * scale, (p, k, u[k, p], float(ref))
        for k in range(1, 6):
            assert u[5 + k, p] == 0.0


def sin_jets(x, n):
    """Jets of u* = sin(pi x) sin(pi y) up to order n: d^k sin(pi t) =
    Im((i pi)^k exp(i pi t))."""
    def d(k, t):
        return np.imag((1j * np.pi) ** k * np.exp(1j * np.pi * t))
    X, Y = x[:, 0], x[:, 1]
    out = [np.sin(np.pi * X) * np.sin(np.pi * Y)]
    out += [d(k, X) * np.sin(np.pi * Y) for k in range(1, n + 1)]
    out += [np.sin(np.pi * X) * d(k, Y) for k in range(1, n + 1)]
    return np.array(out)


@pytest.mark.parametrize("order,c0,cx,cy", [
    (4, 0.0, (0, 0, 0, 1), (0, 0, 0, 1)),
    (5, 0.5, (0, 0, 0, 0, 1), (1,)),
    (3, -2.0, (1, 0, 3), (0, 2, -1)),
    (5, 1.0, (0.5, -1, 0.25, 2, -0.125), (1, 1, 1, 1, 1)),
])
def test_linear_residual_vanishes_at_the_manufactured_solution(order, c0, cx, cy):
    pde = Pde(LINEAR2D, alpha=0.3, c0=c0, cx=cx, cy=cy)
    x = np.random.default_rng(8).uniform(-1, 1, size=(300, 2))
    j = sin_jets(x, order)
    xb = np.array([[-1.0, 0.2], [1.0, -0.7], [0.4, -1.0], [-0.3, 1.0]])
    ub = np.sin(np.pi * xb[:, 0]) * np.sin(np.pi * xb[:, 1])
    r, loss, si, sb = O.residual(pde, x, j, ub, np.zeros(4), order=order)
    scale = np.pi ** order * 10
    assert np.abs(r).max() < 1e-12 * scale
    assert loss[0] < 1e-20 * scale ** 2
    # seeds of a linear residual: 2 alpha r / n times each coefficient
    rng = np.random.default_rng(9)
    jr = j + rng.standard_normal(j.shape)
    r, loss, si, sb = O.residual(pde, x, jr, ub, np.zeros(4), order=order)
    coef = [c0] + list(cx) + [0] * (order - len(cx)) + list(cy) + [0] * (order - len(cy))
    for q in range(1 + 2 * order):
        assert np.allclose(si[q], 2 * 0.3 * r / 300 * coef[q], rtol=1e-13, atol=0)


def test_linear_with_two_second_derivatives_is_poisson():
    """u_xx + u_yy = f with f from sin(pi x) sin(pi y) is Sec. 4.1's Poisson
    problem: the same residual, loss and seeds."""
    lin = Pde(LINEAR2D, alpha=0.05, cx=(0, 1), cy=(0, 1))
    poi = Pde(POISSON2D, alpha=0.05)
    rng = np.random.default_rng(10)
    x = rng.uniform(-1, 1, size=(500, 2))
    j = rng.standard_normal((5, 500))
    ub, g = rng.standard_normal(40), rng.standard_normal(40)
    a = O.residual(lin, x, j, ub, g)
    b = O.residual(poi, x, j, ub, g)
    for u, v in zip(a, b):
        assert np.allclose(u, v, rtol=1e-12, atol=1e-12)


def torch_linear_loss(net, pde, Ws, x_int, x_bc, g_bc):
    X, Wt, jets = torch_jets_n(net, Ws, x_int, net.order)
    n = net.order
    f = torch.tensor(O_free_source(pde, x_int), dtype=torch.float64)
    r = pde.c0 * jets[0]
    for k in range(1, n + 1):
        cxk = pde.cx[k - 1] if k - 1 < len(pde.cx) else 0.0
        cyk = pde.cy[k - 1] if k - 1 < len(pde.cy) else 0.0
        r = r + cxk * jets[k] + cyk * jets[n + k]
    r = r - f
    ub = torch_hrkan(net, Wt, torch.tensor(x_bc, dtype=torch.float64))
    loss = pde.alpha * (r * r).mean() + ((ub - torch.tensor(g_bc)) ** 2).mean()
    gW = torch.autograd.grad(loss, Wt)
    return float(loss.detach()), [g.numpy() for g in gW]


def O_free_source(pde, x):
    """The linear operator applied to sin(pi x) sin(pi y), from sin_jets."""
    n = max(len(pde.cx), len(pde.cy), 1)
    j = sin_jets(x, n)
    f = pde.c0 * j[0]
    for k in range(1, n + 1):
        if k - 1 < len(pde.cx):
            f = f + pde.cx[k - 1] * j[k]
        if k - 1 < len(pde.cy):
            f = f + pde.cy[k - 1] * j[n + k]
    return f


@pytest.mark.parametrize("name", ["linear_o4", "linear_o5"])
def test_high_order_step_matches_torch_autograd(name):
    wl = WL.WORKLOADS[name]
    pr = WL.make_problem(wl, n_int=96, n_bc=16)
    out = O.step(pr.net, pr.pde, pr.W, pr.x_int, pr.x_bc, pr.g_bc)
    loss, gW = torch_linear_loss(pr.net, pr.pde, pr.W, pr.x_int, pr.x_bc, pr.g_bc)
    assert abs(out["loss"][0] - loss) <= 1e-10 * abs(loss)
    for a, b in zip(out["gW"], gW):
        assert relerr(a, b) < 1e-9, relerr(a, b)


def test_high_order_gradient_against_central_differences():
    """Directional central differences of the oracle's own loss, order 4 with
    m = 6 (C^5 basis: the loss is C^1 in W and its second derivative only
    jumps where a hidden input crosses a knot)."""
    wl = WL.WORKLOADS["linear_o4"]
    pr = WL.make_problem(wl, n_int=256, n_bc=32)
    out = O.step(pr.net, pr.pde, pr.W, pr.x_int, pr.x_bc, pr.g_bc)
    gnorm = np.sqrt(sum(float((g * g).sum()) for g in out["gW"]))
    rng = np.random.default_rng(12)
    h = 1e-6
    for _ in range(3):
        V = [rng.standard_normal(w.shape) for w in pr.W]
        nv = np.sqrt(sum(float((v * v).sum()) for v in V))
        V = [v / nv for v in V]
        lp = O.step(pr.net, pr.pde, [w + h * v for w, v in zip(pr.W, V)], pr.x_int, pr.x_bc, pr.g_bc)["loss"][0]
        lm = O.step(pr.net, pr.pde, [w - h * v for w, v in zip(pr.W, V)], pr.x_int, pr.x_bc, pr.g_bc)["loss"][0]
        fd = (lp - lm) / (2 * h)
        an = sum(float((g * v).sum()) for g, v in zip(out["gW"], V))
        assert abs(fd - an) <= 1e-6 * gnorm, (fd, an, gnorm)


def test_pde_above_the_jet_order_is_refused():
    pr = WL.make_problem(WL.WORKLOADS["linear_o5"], n_int=16, n_bc=8)
    low = Net(pr.net.widths, G=pr.net.G, m=pr.net.m, order=4)
    with pytest.raises(AssertionError):
        O.step(low, pr.pde, pr.W, pr.x_int, pr.x_bc, pr.g_bc)
    with pytest.raises(AssertionError):
        O.residual(pr.pde, pr.x_int, np.zeros((9, 16)), np.zeros(8), np.zeros(8), order=4)

