"""Pins of the oracle's residuals, losses and seeds (Sec. 4.1 Eq. 3 with its
loss; Sec. 4.2 Eq. 5 and 6 with its loss).

References: manufactured exact solutions whose residual is zero, the
closed-form loss of the zero network, and finite differences of the loss
with respect to the jets (which fixes every seed's sign and factor).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2409_14248_amd import workloads as WL

GOLD = os.path.join(os.path.dirname(__file__), "golden", "loss_at_zero_weights.json")


def poisson_truth_jets(x):
    # u = sin(pi x) sin(pi y), the closed-form solution of Sec. 4.1
    X, Y = x[:, 0], x[:, 1]
    sx, sy = np.sin(np.pi * X), np.sin(np.pi * Y)
    cx, cy = np.cos(np.pi * X), np.cos(np.pi * Y)
    p = np.pi
    return np.stack([sx * sy, p * cx * sy, -p * p * sx * sy, p * sx * cy, -p * p * sx * sy])


def burgers_wave_jets(x, nu, adv, a=0.7, c=0.2):
    # v = c - a tanh(a (x - c t) / (2 nu)) solves v_t + v v_x = nu v_xx;
    # u = v / adv then solves u_t + adv u u_x = nu u_xx.
    X, T = x[:, 0], x[:, 1]
    k = a / (2 * nu)
    th = np.tanh(k * (X - c * T))
    s2 = 1 - th ** 2
    v = c - a * th
    vx = -a * k * s2
    vxx = 2 * a * k * k * th * s2
    vt = a * k * c * s2
    return np.stack([v, vx, vxx, vt, np.zeros_like(v)]) / adv


def test_poisson_manufactured_residual_is_zero():
    x = np.random.default_rng(0).uniform(-1, 1, size=(500, 2))
    jets = poisson_truth_jets(x)
    r, loss, _, _ = O.residual(WL.Pde(WL.POISSON2D), x, jets, np.zeros(3), np.zeros(3))
    assert np.max(np.abs(r)) < 1e-12
    assert loss[1] < 1e-25


@pytest.mark.parametrize("nu,adv", [(0.01 / math.pi, 1.0), (0.05, 1.0), (0.001 / 16, 0.25)])
def test_burgers_travelling_wave_residual_is_zero(nu, adv):
    x = np.stack([np.random.default_rng(1).uniform(-1, 1, 400),
                  np.random.default_rng(2).uniform(0, 1, 400)], 1)
    jets = burgers_wave_jets(x, nu, adv, a=0.02 if nu < 1e-3 else 0.7)
    r, _, _, _ = O.residual(WL.Pde(WL.BURGERS1D, nu, adv=adv), x, jets, np.zeros(1), np.zeros(1))
    scale = np.max(np.abs(jets[3]))
    assert np.max(np.abs(r)) < 1e-12 * max(1.0, scale)


def test_loss_of_zero_network_poisson_grid():
    with open(GOLD) as f:
        g = json.load(f)["poisson_32x32"]
    wl = WL.WORKLOADS["poisson_c1"]
    pr = WL.make_problem(wl)
    W0 = [np.zeros_like(w) for w in pr.W]
    res = O.step(pr.net, pr.pde, W0, pr.x_int, pr.x_bc, pr.g_bc)
    assert abs(res["loss"][0] - g["L"]) < 1e-13 * g["L"]
    assert abs(res["loss"][1] - g["L_pde"]) < 1e-13 * g["L_pde"]
    assert res["loss"][2] == 0.0
    for gw in res["gW"]:
        assert np.all(gw == 0.0)


def test_loss_of_zero_network_burgers_layout():
    with open(GOLD) as f:
        g = json.load(f)["burgers_2048ic_2048bc"]
    wl = WL.WORKLOADS["burgers_c2"]
    pr = WL.make_problem(wl, n_int=512)
    W0 = [np.zeros_like(w) for w in pr.W]
    res = O.step(pr.net, pr.pde, W0, pr.x_int, pr.x_bc, pr.g_bc)
    assert abs(res["loss"][0] - g["L"]) < 1e-14
    assert res["loss"][1] == 0.0
    assert abs(res["loss"][2] - g["L_bc"]) < 1e-14
    # the zero network's gradient vanishes: hidden jets are zero and the
    # initial-line misfit -sin(pi x) is antisymmetric on a symmetric grid
    for gw in res["gW"]:
        assert np.max(np.abs(gw)) < 1e-15


@pytest.mark.parametrize("kind", [WL.POISSON2D, WL.BURGERS1D])
def test_seeds_are_loss_derivatives(kind):
    rng = np.random.default_rng(4)
    n_int, n_bc = 7, 5
    x = rng.uniform(-1, 1, size=(n_int, 2))
    jets = rng.standard_normal((5, n_int))
    u_bc = rng.standard_normal(n_bc)
    g_bc = rng.standard_normal(n_bc)
    pde = WL.Pde(kind, nu=0.037, alpha=0.05, adv=0.8)
    _, loss, si, sb = O.residual(pde, x, jets, u_bc, g_bc)
    h = 1e-6
    used = [2, 4] if kind == WL.POISSON2D else [0, 1, 2, 3]
    for q in range(5):
        for p in range(n_int):
            jp = jets.copy(); jp[q, p] += h
            jm = jets.copy(); jm[q, p] -= h
            fd = (O.residual(pde, x, jp, u_bc, g_bc)[1][0] - O.residual(pde, x, jm, u_bc, g_bc)[1][0]) / (2 * h)
            assert abs(fd - si[q, p]) < 1e-8 * max(1.0, abs(fd)), (q, p)
            if q not in used:
                assert si[q, p] == 0.0
    for p in range(n_bc):
        up = u_bc.copy(); up[p] += h
        um = u_bc.copy(); um[p] -= h
        fd = (O.residual(pde, x, jets, up, g_bc)[1][0] - O.residual(pde, x, jets, um, g_bc)[1][0]) / (2 * h)
        assert abs(fd - sb[p]) < 1e-8


def test_loss_definition_weights():
    # L = alpha L_pde + L_bc with means over each point set
    rng = np.random.default_rng(6)
    x = rng.uniform(-1, 1, size=(10, 2))
    jets = rng.standard_normal((5, 10))
    pde = WL.Pde(WL.POISSON2D, alpha=0.05)
    r, loss, _, _ = O.residual(pde, x, jets, np.array([0.5, -0.5]), np.zeros(2))
    assert abs(loss[2] - 0.25) < 1e-15
    assert abs(loss[1] - np.mean(r ** 2)) < 1e-14 * loss[1]
    assert abs(loss[0] - (0.05 * loss[1] + loss[2])) < 1e-14 * loss[0]
