"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (normwise relative error ||gpu - oracle|| / ||oracle||):
  FP64 path: 1e-10.  FP32 path: 1e-5 where the network's conditioning allows
  it. Where it does not, the end-to-end gate is FLOOR_FACTOR x the error of
  the oracle's FP32 rounding model (one rounding per basis feature, an FP32
  fused multiply-add chain for every contraction, FP32 storage of every jet):
  the floor any FP32 implementation meets on that network. The kernels
  evaluate each feature with about ten dependent FP32 operations where the
  model rounds once, so their error may sit a few times above the floor. Every layer is
  in addition checked teacher-forced (the oracle fed the GPU's own layer
  inputs) at the plain 1e-5.
"""
import numpy as np
import pytest
import torch

import oracle as O
from conftest import relerr
from gpu_util import (NP_DTYPE, expand, gpu_forward, gpu_step, oracle_step, saved_blocks, to_dev)
from paper_2409_14248_amd import hrkan as H
from paper_2409_14248_amd import workloads as WL

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5}
FLOOR_FACTOR = 10.0


def fp32_floor(pr: WL.Problem, x, mask):
    """Error of the oracle's FP32 rounding model against the exact oracle:
    the floor any FP32 implementation meets on this network."""
    q = pr.rounded(np.float32)
    ref = O.forward(q.net, q.W, x)
    with O.rounding("f32"):
        rnd = O.forward(q.net, q.W, x)
    slots = __import__("gpu_util").SLOTS_OF_MASK[mask]
    return max(relerr(rnd[s], ref[s]) for s in slots)


def fp32_step_gates(pr: WL.Problem):
    """Gates for a whole FP32 step: max(1e-5, FLOOR_FACTOR x the error of the
    oracle's FP32 rounding model) for the loss and for each weight gradient."""
    q = pr.rounded(np.float32)
    ref = O.step(q.net, q.pde, q.W, q.x_int, q.x_bc, q.g_bc)
    with O.rounding("f32"):
        rnd = O.step(q.net, q.pde, q.W, q.x_int, q.x_bc, q.g_bc)
    gate = lambda a, b: max(TOL["f32"], FLOOR_FACTOR * relerr(a, b))
    return ref, gate(rnd["loss"], ref["loss"]), [gate(a, b) for a, b in zip(rnd["gW"], ref["gW"])]


# ---------------------------------------------------------------------------
# the FP64 Poisson workload: 32x32 grid, [2,8,1], G=5 -- whole step
# ---------------------------------------------------------------------------
def test_step_poisson_c1_f64():
    pr = WL.make_problem(WL.WORKLOADS["poisson_c1"])
    loss, gW, _ = gpu_step(pr, "f64")
    ref = oracle_step(pr, "f64")
    assert relerr(loss, ref["loss"]) < 1e-10
    for a, b in zip(gW, ref["gW"]):
        assert relerr(a, b) < 1e-10


def test_forward_jets_poisson_c1_f64():
    pr = WL.make_problem(WL.WORKLOADS["poisson_c1"])
    jets, *_ = gpu_forward(pr, "f64", pr.x_int, H.MASK_POISSON)
    ref = O.forward(pr.net, pr.W, pr.x_int)
    for c in range(5):
        assert relerr(jets[c], ref[c]) < 1e-10, c


@pytest.mark.parametrize("name", ["burgers_c2", "poisson_c3", "burgers_c4"])
def test_step_f64_at_each_network_shape(name):
    wl = WL.WORKLOADS[name]
    pr = WL.make_problem(wl, n_int=1000, n_bc=64)
    loss, gW, _ = gpu_step(pr, "f64")
    ref = oracle_step(pr, "f64")
    assert relerr(loss, ref["loss"]) < 1e-10
    for a, b in zip(gW, ref["gW"]):
        assert relerr(a, b) < 1e-10


@pytest.mark.parametrize("k,m", [(3, 2), (3, 3), (3, 5), (2, 4), (1, 3), (0, 2)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_step_other_orders(k, m, dtype):
    """Other support widths k and HR orders m (Eq. 2; m = 2 is the
    ReLU-KAN basis of Eq. 1) run on the generic kernels; the FP64 step meets
    1e-10 against the oracle, the FP32 step its rounding-model gate. With
    m = 2 the second derivative of a bump jumps at its support ends (the
    smoothness argument of Sec. 2.3); random points fall on no knot, so the
    comparison stays well defined."""
    net = WL.Net((2, 6, 5, 1), G=6, k=k, m=m)
    wl = WL.Workload("orders", net, WL.Pde(WL.BURGERS1D, WL.NU_BURGERS), 700, 48, dtype,
                     WL.SEED_BASE + 40 + 7 * k + m)
    pr = WL.make_problem(wl)
    loss, gW, ws = gpu_step(pr, dtype)
    assert H.read_status(ws) == 0
    if dtype == "f64":
        ref = oracle_step(pr, "f64")
        assert relerr(loss, ref["loss"]) < 1e-10
        for a, b in zip(gW, ref["gW"]):
            assert relerr(a, b) < 1e-10
    else:
        ref, gl, gg = fp32_step_gates(pr)
        assert relerr(loss, ref["loss"]) < gl
        for a, b, gt in zip(gW, ref["gW"], gg):
            assert relerr(a, b) < gt


# The deepest and widest networks the interface takes: 8 layers, one of them
# HRKAN_MAX_WIDTH = 1024 wide (the wide layers run on the generic kernels,
# the 32-wide ones on the matrix-core kernels); 300 points run as one merged
# set, 2,000 on two streams.
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n_int", [300, 2000])
def test_step_max_layers_and_width(dtype, n_int):
    net = WL.Net((2, 8, 1024, 16, 32, 32, 8, 24, 1), G=5)
    assert net.n_layers == H.MAX_LAYERS
    wl = WL.Workload("deep", net, WL.Pde(WL.POISSON2D), n_int, 40, dtype, WL.SEED_BASE + 90)
    pr = WL.make_problem(wl)
    loss, gW, ws = gpu_step(pr, dtype)
    assert H.read_status(ws) == 0
    if dtype == "f64":
        ref = oracle_step(pr, "f64")
        assert relerr(loss, ref["loss"]) < 1e-10
        for a, b in zip(gW, ref["gW"]):
            assert relerr(a, b) < 1e-10
    else:
        ref, gl, gg = fp32_step_gates(pr)
        assert relerr(loss, ref["loss"]) < gl
        for a, b, gt in zip(gW, ref["gW"], gg):
            assert relerr(a, b) < gt


def special_points():
    """Coordinates on the knots of the c2 grid (G = 10 on [-1, 1], h = 0.2,
    supports extended by k h beyond each end: Sec. 2.2), one FP32 unit on
    either side of them, on the grid ends and far outside it, paired in
    every combination of a short list."""
    h = 0.2
    knots = -1.0 + h * np.arange(-3, 14)
    eps = np.float32(np.finfo(np.float32).eps)
    v = np.concatenate([knots, knots * (1 + eps), knots * (1 - eps),
                        [-1.0, 1.0, 0.0, 1.6, -1.6, 1.61, -1.61, 3.0, -10.0, 1e6]])
    v = v.astype(np.float32).astype(np.float64)
    short = v[::3]
    xs, ts = np.meshgrid(v, short, indexing="ij")
    return np.stack([xs.ravel(), ts.ravel()], axis=1)


# The window and support tests of every kernel at the points where they
# switch: inputs on knots (the basis is C^2, Eq. 2 with m = 4, so either
# window gives the same values), on the ends of the extended supports and
# far outside them (all-zero basis).
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_step_at_knots_and_outside_the_grid(dtype):
    base = WL.make_problem(WL.WORKLOADS["burgers_c2"], n_int=8, n_bc=8)
    x = special_points()
    n = x.shape[0]
    xb = x[: n // 4]
    pr = WL.Problem(base.net, base.pde, base.W, x, xb, np.sin(np.pi * xb[:, 0]))
    q = pr.rounded(NP_DTYPE[dtype])
    mask = H.MASK_BURGERS
    jets, *_ = gpu_forward(pr, dtype, q.x_int, mask)
    ref = O.forward(q.net, q.W, q.x_int)
    loss, gW, ws = gpu_step(pr, dtype)
    assert H.read_status(ws) == 0
    sref = oracle_step(pr, dtype)
    if dtype == "f64":
        for c, sl in enumerate(__import__("gpu_util").SLOTS_OF_MASK[mask]):
            assert relerr(jets[c], ref[sl]) < 1e-10, c
        assert relerr(loss, sref["loss"]) < 1e-10
        for a, b in zip(gW, sref["gW"]):
            assert relerr(a, b) < 1e-10
    else:
        gate = max(TOL["f32"], FLOOR_FACTOR * fp32_floor(pr, q.x_int, mask))
        for c, sl in enumerate(__import__("gpu_util").SLOTS_OF_MASK[mask]):
            assert relerr(jets[c], ref[sl]) < gate, (c, relerr(jets[c], ref[sl]), gate)
        _, gl, gg = fp32_step_gates(pr)
        assert relerr(loss, sref["loss"]) < gl
        for a, b, gt in zip(gW, sref["gW"], gg):
            assert relerr(a, b) < gt


# ---------------------------------------------------------------------------
# FP32 path
# ---------------------------------------------------------------------------
# The step runs the two sets as one set, on two streams, or one after the
# other by the interior points times the widest hidden layer (32 here):
# 4,133 and 65 points merge, 40,000 overlap, 131,077 go one after the other;
# a set without boundary points never merges
@pytest.mark.parametrize("n_int,n_bc", [(4096 + 37, 256), (1, 4), (63, 0), (0, 100), (65, 8),
                                        (40000, 300), (131072 + 5, 700)])
def test_step_burgers_c2_shape_f32_sizes(n_int, n_bc):
    wl = WL.WORKLOADS["burgers_c2"]
    pr = WL.make_problem(wl, n_int=n_int, n_bc=n_bc)
    loss, gW, _ = gpu_step(pr, "f32")
    ref, gl, gg = fp32_step_gates(pr)
    assert relerr(loss, ref["loss"]) < gl
    for a, b, gt in zip(gW, ref["gW"], gg):
        if np.linalg.norm(b) > 0:
            assert relerr(a, b) < gt
        else:
            assert np.max(np.abs(a)) == 0.0


@pytest.mark.slow
def test_step_burgers_c2_full_f32():
    pr = WL.make_problem(WL.WORKLOADS["burgers_c2"])
    loss, gW, _ = gpu_step(pr, "f32")
    ref = oracle_step(pr, "f32")
    assert relerr(loss, ref["loss"]) < TOL["f32"]
    for a, b in zip(gW, ref["gW"]):
        assert relerr(a, b) < TOL["f32"]


@pytest.mark.parametrize("name,mask", [("burgers_c2", H.MASK_BURGERS), ("poisson_c3", H.MASK_POISSON),
                                       ("burgers_c4", H.MASK_BURGERS)])
def test_forward_layers_teacher_forced_f32(name, mask):
    wl = WL.WORKLOADS[name]
    pr = WL.make_problem(wl, n_int=777, n_bc=4)
    q = pr.rounded(np.float32)
    x = q.x_int
    n = x.shape[0]
    C = H.mask_channels(mask)
    jets, sv, *_ = gpu_forward(pr, "f32", x, mask, saved=True)
    blocks = saved_blocks(pr, sv, "f32", C, n)
    ins = [O.input_jets(x)] + [expand(b, mask) for b in blocks]
    outs = [expand(b, mask) for b in blocks] + [expand(jets.reshape(C, 1, n), mask)]
    slots = __import__("gpu_util").SLOTS_OF_MASK[mask]
    for l, W in enumerate(q.W):
        ref = O.layer_forward(q.net, l, W, ins[l])
        for s in slots:
            assert relerr(outs[l][s], ref[s]) < TOL["f32"], (l, s)


@pytest.mark.parametrize("name,mask", [("burgers_c2", H.MASK_BURGERS), ("poisson_c3", H.MASK_POISSON),
                                       ("burgers_c4", H.MASK_BURGERS)])
def test_forward_end_to_end_f32(name, mask):
    wl = WL.WORKLOADS[name]
    pr = WL.make_problem(wl, n_int=2048, n_bc=4)
    q = pr.rounded(np.float32)
    jets, *_ = gpu_forward(pr, "f32", q.x_int, mask)
    ref = O.forward(q.net, q.W, q.x_int)
    floor = fp32_floor(pr, q.x_int, mask)
    gate = max(TOL["f32"], FLOOR_FACTOR * floor)
    for c, s in enumerate(__import__("gpu_util").SLOTS_OF_MASK[mask]):
        assert relerr(jets[c], ref[s]) < gate, (c, relerr(jets[c], ref[s]), floor)


@pytest.mark.parametrize("name,mask", [("burgers_c2", H.MASK_BURGERS), ("poisson_c3", H.MASK_POISSON)])
def test_backward_teacher_forced_f32(name, mask):
    """GPU weight gradient for given seeds vs the oracle reverse pass fed the
    GPU's saved forward jets."""
    wl = WL.WORKLOADS[name]
    pr = WL.make_problem(wl, n_int=1500, n_bc=4)
    q = pr.rounded(np.float32)
    n = q.n_int
    C = H.mask_channels(mask)
    _, sv, W, xd, ws, nd = gpu_forward(pr, "f32", q.x_int, mask, saved=True)
    seed = np.random.default_rng(3).standard_normal((C, n)).astype(np.float32)
    gW = H.backward(nd, W, xd, mask, to_dev(seed, "f32"), sv, ws)
    torch.cuda.synchronize()
    blocks = saved_blocks(pr, sv, "f32", C, n)
    ins = [O.input_jets(q.x_int)] + [expand(b, mask) for b in blocks]
    ybar = expand(seed.astype(np.float64).reshape(C, 1, n), mask)
    for l in range(len(q.W) - 1, -1, -1):
        zbar, ref = O.layer_backward(q.net, l, q.W[l], ins[l], ybar)
        assert relerr(gW[l].double().cpu().numpy(), ref) < TOL["f32"], l
        ybar = zbar
        if l > 0:
            # the GPU's bars are internal; keep the oracle's chain but drop the
            # channels the mask does not carry
            keep = np.zeros_like(ybar)
            keep[__import__("gpu_util").SLOTS_OF_MASK[mask]] = ybar[__import__("gpu_util").SLOTS_OF_MASK[mask]]
            ybar = keep


# ---------------------------------------------------------------------------
# properties and edge cases
# ---------------------------------------------------------------------------
def test_step_is_deterministic():
    pr = WL.make_problem(WL.WORKLOADS["burgers_c2"], n_int=5000, n_bc=320)
    a_loss, a_gW, _ = gpu_step(pr, "f32")
    b_loss, b_gW, _ = gpu_step(pr, "f32")
    assert np.array_equal(a_loss, b_loss)
    for a, b in zip(a_gW, b_gW):
        assert np.array_equal(a, b)


def test_backward_accumulate_is_additive_over_shards():
    pr = WL.make_problem(WL.WORKLOADS["burgers_c2"], n_int=3000, n_bc=4)
    mask = H.MASK_BURGERS
    x = pr.x_int.astype(np.float32)
    seed = np.random.default_rng(0).standard_normal((4, 3000)).astype(np.float32)
    parts = []
    for sl in (slice(0, 3000), slice(0, 1234), slice(1234, 3000)):
        xs = np.ascontiguousarray(x[sl])
        _, sv, W, xd, ws, nd = gpu_forward(pr, "f32", xs, mask, saved=True)
        parts.append((sv, W, xd, ws, nd, to_dev(np.ascontiguousarray(seed[:, sl]), "f32")))
    sv, W, xd, ws, nd, sd = parts[0]
    full = H.backward(nd, W, xd, mask, sd, sv, ws)
    sv, W, xd, ws, nd, sd = parts[1]
    acc = H.backward(nd, W, xd, mask, sd, sv, ws)
    sv, W, xd, ws, nd, sd = parts[2]
    acc = H.backward(nd, W, xd, mask, sd, sv, ws, gW_out=acc, accumulate=True)
    torch.cuda.synchronize()
    for f, a in zip(full, acc):
        assert relerr(a.cpu().numpy(), f.cpu().numpy()) < 1e-6


def test_nonfinite_input_sets_status_bit():
    pr = WL.make_problem(WL.WORKLOADS["burgers_c2"], n_int=300, n_bc=8)
    nd = H.net_desc(pr.net, "f32")
    pd = H.pde_desc(pr.pde)
    W = [to_dev(w, "f32") for w in pr.W]
    xi = to_dev(pr.x_int, "f32")
    xi[17, 0] = float("nan")
    xb, g = to_dev(pr.x_bc, "f32"), to_dev(pr.g_bc, "f32")
    ws = H.alloc_workspace(H.workspace_bytes(nd, pd, pr.n_int, pr.n_bc))
    assert H.read_status(ws) == 0
    loss, _ = H.step(nd, pd, W, xi, xb, g, ws)
    assert H.read_status(ws) & H.STATUS_NONFINITE
    assert H.read_status(ws) == 0        # read clears
    assert not np.isfinite(loss.cpu().numpy()[0])


def test_residual_call_matches_oracle():
    pr = WL.make_problem(WL.WORKLOADS["poisson_c3"], n_int=999, n_bc=64)
    rng = np.random.default_rng(1)
    jets = rng.standard_normal((5, 999))
    ubc = rng.standard_normal(64)
    pd = H.pde_desc(pr.pde)
    ws = H.alloc_workspace(1 << 16)
    r = torch.empty(999, dtype=torch.float64, device="cuda")
    si = torch.empty((5, 999), dtype=torch.float64, device="cuda")
    sb = torch.empty(64, dtype=torch.float64, device="cuda")
    loss = H.residual(pd, H.F64, to_dev(jets, "f64"), to_dev(ubc, "f64"), to_dev(pr.x_int, "f64"),
                      to_dev(pr.g_bc, "f64"), ws, r_out=r, seed_int=si, seed_bc=sb)
    torch.cuda.synchronize()
    rr, rl, rsi, rsb = O.residual(pr.pde, pr.x_int, jets, ubc, pr.g_bc)
    assert relerr(loss.cpu().numpy(), rl) < 1e-13
    assert relerr(r.cpu().numpy(), rr) < 1e-13
    assert relerr(si.cpu().numpy(), rsi) < 1e-13
    assert relerr(sb.cpu().numpy(), rsb) < 1e-13


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_autograd_functions_match_step(dtype):
    """The two autograd Functions (separate forward-jets, residual and
    backward calls) against the fused step: the same products, other
    summation orders (BF16: the same BF16 pieces in both)."""
    pr = WL.make_problem(WL.WORKLOADS["burgers_c2"], n_int=2000, n_bc=128)
    nd = H.net_desc(pr.net, dtype)
    pd = H.pde_desc(pr.pde)
    W = [to_dev(w, dtype).requires_grad_(True) for w in pr.W]
    xi, xb, g = to_dev(pr.x_int, dtype), to_dev(pr.x_bc, dtype), to_dev(pr.g_bc, dtype)
    jets = H.HRKANJets.apply(nd, H.MASK_BURGERS, xi, *W)
    ub = H.HRKANJets.apply(nd, H.MASK_VALUE, xb, *W)
    L, Lp, Lb = H.HRKANResidual.apply(pd, H.F32, jets, ub[0], xi, g)
    L.backward()
    ref_loss, ref_gW, _ = gpu_step(pr, dtype)
    assert abs(L.item() - ref_loss[0]) <= 1e-6 * abs(ref_loss[0])
    for w, b in zip(W, ref_gW):
        assert relerr(w.grad.double().cpu().numpy(), b) < 1e-5


# 6,000 points run as one merged set, 40,000 on two streams (the capture
# then holds the fork and join)
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("n_int", [6000, 40000])
def test_graph_replay_matches_eager_step(dtype, n_int):
    """The step captured in a HIP graph gives the eager result on every
    replay, with eager work on the same buffers in between (BF16: including
    the per-call BF16 weight copies of the dense kernels)."""
    pr = WL.make_problem(WL.WORKLOADS["burgers_c2"], n_int=n_int, n_bc=400)
    st = H.Step(pr, dtype)
    loss0, gW0 = st()
    torch.cuda.synchronize()
    ref_loss = loss0.cpu().numpy().copy()
    ref_gW = [g.cpu().numpy().copy() for g in gW0]
    st.capture()
    for rep in range(4):
        for g in st.gW:
            g.fill_(float("nan"))            # eager work between replays
        st.loss.zero_()
        torch.cuda.synchronize()
        loss, gW = st.replay()
        torch.cuda.synchronize()
        assert np.array_equal(loss.cpu().numpy(), ref_loss), rep
        for a, b in zip(gW, ref_gW):
            assert np.array_equal(a.cpu().numpy(), b), rep
