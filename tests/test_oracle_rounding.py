"""Pins of the oracle's rounding model against conversions it does not share.

The rounding model (hro_set_rounding) only sizes the error that FP32 / BF16
storage alone causes on a network; the FP32 and BF16 gates of the GPU tests
are built on it. Each of its primitives is pinned here:
- every rounding of a value (feature, stored jet or bar, bar as the split
  operand, bar as the second operand) against torch's float64 -> float32 and
  float32 -> bfloat16 casts (round to nearest, ties to even);
- the FP32 accumulation step against the exact sum computed with rationals
  and rounded once to FP32 by hand, including a case where rounding to double
  first and then to FP32 gives another result;
- the bar roundings where the reverse pass uses them: on a one-row layer the
  weight gradient and the input bar reduce to a product of two rounded values
  that torch computes independently.
"""
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle as O
from paper_2409_14248_amd.workloads import Net


def _values():
    rng = np.random.default_rng(11)
    v = np.concatenate([
        rng.standard_normal(400) * 10.0 ** rng.integers(-30, 30, 400),
        [0.0, -0.0, 1.0, -1.0, 3.0e38, -3.0e38, 1e-40, -1e-42, np.inf, -np.inf],
        # ties of the BF16 grid: half-way between two BF16 neighbours
        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 2.0 ** -20 * (1.0 + 2.0 ** -8)],
        # ties of the FP32 grid, reached from double
        [1.0 + 2.0 ** -24, 1.0 + 3 * 2.0 ** -24],
    ])
    return v


def _torch_f32(v):
    return torch.tensor(v, dtype=torch.float64).float()


def _torch_bf16(v):
    return _torch_f32(v).to(torch.bfloat16).float()


def _torch_split2(v):
    f = _torch_f32(v)
    hi = f.to(torch.bfloat16).float()
    lo = (f - hi).to(torch.bfloat16).float()
    return hi.double() + lo.double()


def _model(what, vals):
    return np.array([O.model_round(what, x) for x in vals])


def _same(a, b):
    return np.array_equal(np.asarray(a, np.float64), np.asarray(b, np.float64), equal_nan=True)


def test_exact_mode_rounds_nothing():
    v = _values()
    for what in range(4):
        assert _same(_model(what, v), v), what
    assert O.model_acc(1.0, 1.0 / 3.0, 3.0) == 1.0 + (1.0 / 3.0) * 3.0


def test_fp32_mode_roundings():
    v = _values()
    f32 = _torch_f32(v).double().numpy()
    with O.rounding("f32"):
        assert _same(_model(O.MODEL_FEATURE, v), f32)
        assert _same(_model(O.MODEL_STORE, v), f32)
        # bars enter the FP32 contractions as stored (already FP32)
        assert _same(_model(O.MODEL_BAR_SPLIT, v), v)
        assert _same(_model(O.MODEL_BAR_HI, v), v)


@pytest.mark.parametrize("split", [1, 2])
def test_bf16_mode_roundings(split):
    v = _values()
    f32 = _torch_f32(v).double().numpy()
    hi = _torch_bf16(v).double().numpy()
    sp = hi if split == 1 else _torch_split2(v).numpy()
    with O.rounding("bf16", split):
        assert _same(_model(O.MODEL_FEATURE, v), sp)
        assert _same(_model(O.MODEL_STORE, v), f32)
        assert _same(_model(O.MODEL_BAR_SPLIT, v), sp)
        assert _same(_model(O.MODEL_BAR_HI, v), hi)


def _f32_bits(x):
    return int(np.array([x], dtype=np.float32).view(np.uint32)[0])


def _round_f32(q: Fraction) -> float:
    """Exact rational -> nearest FP32 value, ties to the even significand."""
    c = np.float32(float(q))
    cands = [np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))]
    best = None
    for x in cands:
        d = abs(Fraction(float(x)) - q)
        key = (d, _f32_bits(x) & 1)
        if best is None or key < best[0]:
            best = (key, float(x))
    return best[1]


def test_fp32_accumulation_step_is_one_rounding():
    rng = np.random.default_rng(5)
    trip = rng.standard_normal((2000, 3))
    trip[:, 0] *= 10.0 ** rng.integers(-6, 6, 2000)
    trip = trip.astype(np.float32).astype(np.float64)     # operands held in FP32
    # acc + w a just below the half-way point of two FP32 neighbours: one
    # rounding goes down, rounding to double first lands on the half-way
    # point and then rounds to even, upwards
    crafted = [(1.0 + 2.0 ** -23, 1.0 + 2.0 ** -23, 2.0 ** -24 * (1.0 - 2.0 ** -23)),
               (1.0, 2.0 ** -12, 2.0 ** -12), (-3.0, 1.5, 2.0)]
    with O.rounding("f32"):
        for acc, w, a in list(map(tuple, trip)) + crafted:
            exact = Fraction(acc) + Fraction(w) * Fraction(a)
            assert O.model_acc(acc, w, a) == _round_f32(exact), (acc, w, a)
    acc, w, a = crafted[0]
    assert float(np.float32(acc + w * a)) != _round_f32(Fraction(acc) + Fraction(w) * Fraction(a))


@pytest.mark.parametrize("split", [1, 2])
def test_bar_roundings_inside_the_reverse_pass(split):
    """A layer whose only non-zero weight is 1 at row (input 0, basis 4):
    the weight gradient of that row is the rounded feature times the bar's
    high BF16 piece, and the value bar of input 0 is the bar as the split
    operand times v'(z), stored in FP32."""
    net = Net((2, 1), G=5)
    s, e = O.supports(net)
    nb = O.n_basis(net)
    W = np.zeros((2 * nb, 1))
    W[4, 0] = 1.0
    n = 64
    rng = np.random.default_rng(8)
    z = rng.uniform(s[4] + 0.05, e[4] - 0.05, n)
    zin = np.zeros((5, 2, n))
    zin[0, 0] = z
    zin[0, 1] = 5.0           # outside every support: input 1 adds nothing
    ybar = np.zeros((5, 1, n))
    ybar[0, 0] = rng.standard_normal(n) * 10.0 ** rng.integers(-3, 3, n)
    phi = np.array([O.basis(4, s[4], e[4], v, 1) for v in z])
    feat = torch.tensor(phi[:, 0]).float()
    if split == 1:
        feat_r = feat.to(torch.bfloat16).double()
        bar_sp = _torch_bf16(ybar[0, 0]).double()
    else:
        feat_r = _torch_split2(phi[:, 0])
        bar_sp = _torch_split2(ybar[0, 0])
    bar_hi = _torch_bf16(ybar[0, 0]).double()
    for p in range(n):
        with O.rounding("bf16", split):
            zbar, gW = O.layer_backward(net, 0, W, zin[:, :, p:p + 1], ybar[:, :, p:p + 1])
        want_g = (feat_r[p] * bar_hi[p]).item()
        assert gW[4, 0] == want_g, p
        want_zbar = float(np.float32((bar_sp[p] * phi[p, 1]).item()))
        assert zbar[0, 0, 0] == want_zbar, p
