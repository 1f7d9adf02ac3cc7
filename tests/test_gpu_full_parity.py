"""Full-size parity of the training step with the FP64 oracle: the loss and
every weight gradient, plus the output jets and the residual element-wise.

The loss is alpha times the mean squared residual plus the mean squared
boundary misfit (Sec. 4.1, Sec. 4.2), so every interior point enters every
weight gradient. Sizes:
- Poisson [2,64,64,64,1], G = 16: its whole set, 262,144 interior + 16,384
  boundary points, FP32;
- Burgers [2,128,128,128,1], G = 20: one GPU's share of its 1,048,576-point
  set when the step is spread over four, 262,144 interior + 16,384 boundary
  points (the same seeded distribution), FP32 and BF16 with S = 2 and S = 3.
  Each hidden-layer weight gradient there spans many point slices, so its
  FP64 reduction of slices runs as at the full size, and the FP32 one runs
  with the XCD-aware block order (112 slices) of the full-size step.

Gates: FP32 max(1e-5, 3 x floor), the floor being the error of the oracle's
FP32 rounding model on the same inputs (on these networks it exceeds 1e-5 for
any FP32 implementation); BF16 the literal 2e-2, S = 3 against the oracle on
the FP32 master weights, S = 2 against the oracle on the BF16-rounded weights
that its kernels multiply. Each oracle run is made once per module.
"""
import numpy as np
import pytest
import torch

import oracle as O
from conftest import check, maxerr, relerr
from gpu_util import SLOTS_OF_MASK, bf16_round, gpu_step, to_dev
from paper_2409_14248_amd import hrkan as H
from paper_2409_14248_amd import workloads as WL

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL_F32, TOL_BF16, FACTOR = 1e-5, 2e-2, 3.0
C4_SHARE = (262144, 16384)

_cache = {}


def _problem(name):
    if name == "burgers_c4":
        return WL.make_problem(WL.WORKLOADS[name], n_int=C4_SHARE[0], n_bc=C4_SHARE[1])
    return WL.make_problem(WL.WORKLOADS[name])


def _oracle(name, which):
    """which: "exact" (FP32 inputs), "f32" (FP32 rounding model) or "bf16w"
    (exact, weights rounded to BF16). Computed once, printed with its time."""
    key = (name, which)
    if key not in _cache:
        import time
        q = _problem(name).rounded(np.float32)
        t = time.time()
        if which == "exact":
            out = O.step(q.net, q.pde, q.W, q.x_int, q.x_bc, q.g_bc)
        elif which == "f32":
            with O.rounding("f32"):
                out = O.step(q.net, q.pde, q.W, q.x_int, q.x_bc, q.g_bc)
        else:
            out = O.step(q.net, q.pde, [bf16_round(w) for w in q.W], q.x_int, q.x_bc, q.g_bc)
        print(f"[oracle] {name} {which}: {q.n_int}+{q.n_bc} points in {time.time() - t:.1f} s "
              f"({O.num_threads()} threads)", flush=True)
        _cache[key] = out
    return _cache[key]


@pytest.mark.parametrize("name", ["poisson_c3", "burgers_c4"])
def test_full_size_step_f32(name):
    pr = _problem(name)
    print(f"[case] {name} f32 step, {pr.n_int}+{pr.n_bc} points", flush=True)
    loss, gW, ws = gpu_step(pr, "f32")
    assert H.read_status(ws) == 0
    del ws
    ref, rnd = _oracle(name, "exact"), _oracle(name, "f32")
    check(f"{name} full f32 loss", relerr(loss, ref["loss"]), TOL_F32, relerr(rnd["loss"], ref["loss"]), FACTOR)
    for l, (a, b, c) in enumerate(zip(gW, ref["gW"], rnd["gW"])):
        check(f"{name} full f32 gW{l}", relerr(a, b), TOL_F32, relerr(c, b), FACTOR)


@pytest.mark.parametrize("name", ["poisson_c3", "burgers_c4"])
def test_full_size_jets_and_residual_f32(name):
    """Output jets at every interior point and the residual, normwise and
    max-scaled element-wise."""
    pr = _problem(name)
    q = pr.rounded(np.float32)
    mask = H.pde_mask(pr.pde)
    nd = H.net_desc(pr.net, "f32")
    pd = H.pde_desc(pr.pde)
    W = [to_dev(w, "f32") for w in pr.W]
    ws = H.alloc_workspace(H.workspace_bytes(nd, pd, q.n_int, q.n_bc))
    xi, xb, g = to_dev(q.x_int, "f32"), to_dev(q.x_bc, "f32"), to_dev(q.g_bc, "f32")
    jets = H.forward_jets(nd, W, xi, mask, ws)
    ub = H.forward_jets(nd, W, xb, H.MASK_VALUE, ws)
    r = torch.empty(q.n_int, dtype=torch.float32, device="cuda")
    H.residual(pd, H.F32, jets, ub[0], xi, g, ws, r_out=r)
    torch.cuda.synchronize()
    jets = jets.double().cpu().numpy()
    r = r.double().cpu().numpy()
    ref, rnd = _oracle(name, "exact"), _oracle(name, "f32")
    for c, s in enumerate(SLOTS_OF_MASK[mask]):
        check(f"{name} full jet{s} norm", relerr(jets[c], ref["jets"][s]), TOL_F32,
              relerr(rnd["jets"][s], ref["jets"][s]), FACTOR)
        check(f"{name} full jet{s} max", maxerr(jets[c], ref["jets"][s]), TOL_F32,
              maxerr(rnd["jets"][s], ref["jets"][s]), FACTOR)
    check(f"{name} full r norm", relerr(r, ref["r"]), TOL_F32, relerr(rnd["r"], ref["r"]), FACTOR)
    check(f"{name} full r max", maxerr(r, ref["r"]), TOL_F32, maxerr(rnd["r"], ref["r"]), FACTOR)


@pytest.mark.parametrize("S", [3, 2])
def test_full_size_step_bf16_burgers_c4(S):
    pr = _problem("burgers_c4")
    print(f"[case] burgers_c4 bf16 S={S} step, {pr.n_int}+{pr.n_bc} points", flush=True)
    loss, gW, ws = gpu_step(pr, "bf16", S)
    assert H.read_status(ws) == 0
    del ws
    ref = _oracle("burgers_c4", "exact" if S == 3 else "bf16w")
    lab = f"burgers_c4 share bf16 S{S} W={'f32' if S == 3 else 'bf16'}"
    check(f"{lab} loss", relerr(loss, ref["loss"]), TOL_BF16)
    for l, (a, b) in enumerate(zip(gW, ref["gW"])):
        check(f"{lab} gW{l}", relerr(a, b), TOL_BF16)
