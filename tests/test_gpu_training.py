"""The training loop the paper runs (Adam, Sec. 4.1 and 4.2) on the HIP path:
the fused Adam update against the oracle's Adam, a captured epoch (step and
update in one HIP graph) against eager epochs, and the paper's own Poisson
and Burgers instances through the step against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from conftest import relerr
from gpu_util import gpu_step, to_dev
from paper_2409_14248_amd import hrkan as H
from paper_2409_14248_amd import workloads as WL
from test_gpu_parity import check_step_f32

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype,tol", [("f32", 2e-6), ("f64", 1e-13)])
def test_adam_matches_oracle(dtype, tol):
    net = WL.Net((2, 32, 32, 1), G=10)
    nd = H.net_desc(net, dtype)
    rng = np.random.default_rng(5)
    W = [rng.standard_normal(s) * 0.1 for s in net.weight_shapes()]
    np_dt = np.float32 if dtype == "f32" else np.float64
    W = [w.astype(np_dt).astype(np.float64) for w in W]
    Wd = [to_dev(w, dtype) for w in W]
    md = [torch.zeros_like(w) for w in Wd]
    vd = [torch.zeros_like(w) for w in Wd]
    t = torch.zeros(1, dtype=torch.int64, device="cuda")
    m = [np.zeros_like(w) for w in W]
    v = [np.zeros_like(w) for w in W]
    for step in range(1, 4):
        g = [(rng.standard_normal(w.shape) * 10.0 ** rng.uniform(-4, 1)).astype(np_dt).astype(np.float64) for w in W]
        H.adam(nd, Wd, [to_dev(a, dtype) for a in g], md, vd, t, 1e-2, (0.9, 0.999), 1e-8)
        W, m, v = O.adam(W, g, m, v, step, 1e-2, 0.9, 0.999, 1e-8)
        torch.cuda.synchronize()
        for a, b in zip(Wd, W):
            assert relerr(a.double().cpu().numpy(), b) < tol, step
        for a, b in zip(md + vd, m + v):
            assert relerr(a.double().cpu().numpy(), b) < tol, step
    assert int(t.item()) == 3


# the paper's Poisson instance runs its step as one merged set; 40,000
# Burgers points run the two point sets on two streams inside the graph
@pytest.mark.parametrize("name,n_int", [("poisson_paper", None), ("burgers_c2", 40000)])
def test_trainer_graph_replays_match_eager_epochs(name, n_int):
    """Twenty epochs replayed from one captured graph give bit for bit the
    weights of twenty eager epochs (the step count lives in device memory)."""
    pr = WL.make_problem(WL.WORKLOADS[name], n_int=n_int, n_bc=(1000 if n_int else None))
    a = H.Trainer(pr, "f32", lr=1e-2)
    ha = a.run(20, graph=False, record_every=5)
    b = H.Trainer(pr, "f32", lr=1e-2)
    hb = b.run(20, graph=True, record_every=5)
    torch.cuda.synchronize()
    for wa, wb in zip(a.step.W, b.step.W):
        assert torch.equal(wa, wb)
    assert ha == hb
    assert int(b.t.item()) == 20
    assert ha[19][0] < ha[0][0]          # the loss went down


@pytest.mark.parametrize("name", ["poisson_paper", "burgers_paper"])
def test_paper_instances_step_matches_oracle(name):
    pr = WL.make_problem(WL.WORKLOADS[name])
    loss, gW, ws = gpu_step(pr, "f32")
    assert H.read_status(ws) == 0
    check_step_f32(f"{name} f32", pr, loss, gW, literal=True)
