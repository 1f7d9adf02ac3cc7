"""Edge cases of the tile-coherent FP32 kernels and of the point ordering
that precedes them, against the FP64 oracle.

The tile-coherent kernels take the FP32 hidden layers with 64 or 128
outputs (and the first layer of such networks); a step orders each point
set along a Z-order curve first when its sets run separately (more than
2^20 interior points x widest hidden layer). Covered here on [2,64,64,1]
and [2,128,128,1] networks: point counts that leave ragged tiles, fewer
points than one tile, empty sets, every set schedule (merged, two streams,
one after the other), inputs on the knots, one FP32 unit beside them and
far outside the grid (an all-zero basis), duplicated points, a NaN input,
and determinism of the ordered step.

Gate: max(1e-5, 3 x floor), the floor being the error of the oracle's FP32
rounding model on the same inputs; jets also max-scaled element-wise.
"""
import numpy as np
import pytest

import oracle as O
from conftest import check, maxerr, relerr
from gpu_util import SLOTS_OF_MASK, gpu_forward, gpu_step, to_dev
from paper_2409_14248_amd import hrkan as H
from paper_2409_14248_amd import workloads as WL
from test_gpu_parity import check_step_f32

pytestmark = pytest.mark.gpu

NETS = {64: WL.Net((2, 64, 64, 1), G=16), 128: WL.Net((2, 128, 128, 1), G=20)}


def problem(width, n_int, n_bc, seed=0):
    wl = WL.Workload(f"tc{width}", NETS[width], WL.Pde(WL.BURGERS1D, WL.NU_BURGERS), n_int, n_bc, "f32",
                     WL.SEED_BASE + 60 + seed)
    return WL.make_problem(wl)


# (n_int, n_bc): ragged tiles; fewer than 16 points; empty sets; at width 64
# merged up to 16,384 interior points, two streams up to 65,536, then one
# after the other (the last two ordered along the curve)
SIZES = [(4096 + 37, 256), (1, 4), (15, 0), (0, 100), (17, 4), (40000 + 3, 2048), (70000 + 5, 4096)]


@pytest.mark.parametrize("n_int,n_bc", SIZES)
def test_step_sizes_width64(n_int, n_bc):
    pr = problem(64, n_int, n_bc)
    print(f"[case] [2,64,64,1] {n_int}+{n_bc}", flush=True)
    loss, gW, ws = gpu_step(pr, "f32")
    assert H.read_status(ws) == 0
    check_step_f32(f"w64 {n_int}+{n_bc}", pr, loss, gW, literal=False)


@pytest.mark.parametrize("n_int,n_bc", [(3000 + 7, 192), (15, 4), (40000 + 11, 1024)])
def test_step_sizes_width128(n_int, n_bc):
    pr = problem(128, n_int, n_bc)
    print(f"[case] [2,128,128,1] {n_int}+{n_bc}", flush=True)
    loss, gW, ws = gpu_step(pr, "f32")
    assert H.read_status(ws) == 0
    check_step_f32(f"w128 {n_int}+{n_bc}", pr, loss, gW, literal=False)


def special_points(G):
    """Knots of the G-interval grid on [-1, 1] (supports extended by 3
    intervals each side), one FP32 unit either side of them, the grid ends
    and points far outside, paired in every combination of a short list."""
    h = 2.0 / G
    knots = -1.0 + h * np.arange(-3, G + 4)
    eps = np.float32(np.finfo(np.float32).eps)
    v = np.concatenate([knots, knots * (1 + eps), knots * (1 - eps),
                        [-1.0, 1.0, 0.0, 1.6, -1.6, 1.61, -1.61, 3.0, -10.0, 1e6]])
    v = v.astype(np.float32).astype(np.float64)
    xs, ts = np.meshgrid(v, v[::3], indexing="ij")
    return np.stack([xs.ravel(), ts.ravel()], axis=1)


@pytest.mark.parametrize("width", [64, 128])
def test_knots_and_outside_the_grid(width):
    """Forward jets (element-wise) and the step at the special points; the
    interior set is repeated to pass the two-set size, so that it is
    ordered along the curve, with duplicated points."""
    base = problem(width, 8, 8)
    x = special_points(NETS[width].G)
    reps = max(1, (17000 * 64 // width) // x.shape[0] + 1)
    xi = np.concatenate([x] * reps)[:: 1]
    xb = x[: x.shape[0] // 4]
    pr = WL.Problem(base.net, base.pde, base.W, xi, xb, np.sin(np.pi * xb[:, 0]))
    q = pr.rounded(np.float32)
    mask = H.MASK_BURGERS
    jets, *_ = gpu_forward(pr, "f32", x, mask)
    ref = O.forward(q.net, q.W, x)
    with O.rounding("f32"):
        rnd = O.forward(q.net, q.W, x)
    for c, s in enumerate(SLOTS_OF_MASK[mask]):
        check(f"w{width} knots jet{s} norm", relerr(jets[c], ref[s]), 1e-5, relerr(rnd[s], ref[s]))
        check(f"w{width} knots jet{s} max", maxerr(jets[c], ref[s]), 1e-5, maxerr(rnd[s], ref[s]))
    print(f"[case] w{width} knots step {pr.n_int}+{pr.n_bc}", flush=True)
    loss, gW, ws = gpu_step(pr, "f32")
    assert H.read_status(ws) == 0
    check_step_f32(f"w{width} knots step", pr, loss, gW, literal=False)


def test_nan_input_on_the_ordered_path_sets_status_bit():
    pr = problem(64, 40000, 1024)
    nd = H.net_desc(pr.net, "f32")
    pd = H.pde_desc(pr.pde)
    W = [to_dev(w, "f32") for w in pr.W]
    xi = to_dev(pr.x_int, "f32")
    xi[12345, 1] = float("nan")
    xb, g = to_dev(pr.x_bc, "f32"), to_dev(pr.g_bc, "f32")
    ws = H.alloc_workspace(H.workspace_bytes(nd, pd, pr.n_int, pr.n_bc))
    assert H.read_status(ws) == 0
    loss, _ = H.step(nd, pd, W, xi, xb, g, ws)
    assert H.read_status(ws) & H.STATUS_NONFINITE
    assert not np.isfinite(loss.cpu().numpy()[0])


def test_ordered_step_is_deterministic():
    pr = problem(128, 40000 + 11, 1024, seed=3)
    a_loss, a_gW, _ = gpu_step(pr, "f32")
    b_loss, b_gW, _ = gpu_step(pr, "f32")
    assert np.array_equal(a_loss, b_loss)
    for a, b in zip(a_gW, b_gW):
        assert np.array_equal(a, b)
