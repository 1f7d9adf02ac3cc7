"""The batched step (hrkan_plan_*): many Burgers instances of one network
shape, each with its own weights, viscosity and point counts, run as one
HIP graph launch over a concatenated point axis.

Each instance's loss and gradient must equal what the single-instance step
(hrkan_step) gives for that instance alone, within FP32 summation-order
differences (the two paths slice the weight-gradient sums differently), and
one instance is checked against the FP64 oracle at the FP32 gate.
"""
import numpy as np
import pytest
import torch

import oracle as O
from conftest import check, relerr
from gpu_util import gpu_step
from paper_2409_14248_amd import hrkan as H
from paper_2409_14248_amd import workloads as WL

pytestmark = pytest.mark.gpu

SAME_STEP_TOL = 2e-5


def _instances(n, lo=200, hi=5000):
    return WL.batched_instances(WL.WORKLOADS["burgers_batched_c5"], n_instances=n, lo=lo, hi=hi)


def _check_against_single_steps(plan, probs):
    torch.cuda.synchronize()
    loss = plan.loss.cpu().numpy()
    for q, pr in enumerate(probs):
        ls, gW, _ = gpu_step(pr, "f32")
        assert relerr(loss[q], ls) <= SAME_STEP_TOL, (q, loss[q], ls)
        for l, g in enumerate(plan.layer_grads(q, pr.net)):
            assert relerr(g.double().cpu().numpy(), gW[l]) <= SAME_STEP_TOL, (q, l)


def test_batched_step_matches_single_instance_steps():
    probs = _instances(7)
    # an instance whose counts are not multiples of anything, and a tiny one
    probs[2] = WL.make_problem(WL.WORKLOADS["burgers_c2"], n_int=1001, n_bc=4, seed=77,
                               pde=WL.Pde(WL.BURGERS1D, 0.004))
    probs[5] = WL.make_problem(WL.WORKLOADS["burgers_c2"], n_int=3, n_bc=4, seed=78,
                               pde=WL.Pde(WL.BURGERS1D, 0.05))
    plan = H.Plan(probs)
    plan.execute()
    _check_against_single_steps(plan, probs)
    tp, blocks = plan.config()
    assert tp in (1024, 2048, 4096) and blocks > 0
    assert H.read_status(plan.ws) == 0


def test_batched_instance_matches_oracle():
    probs = _instances(3, lo=2000, hi=3000)
    plan = H.Plan(probs)
    plan.execute()
    torch.cuda.synchronize()
    q = probs[1].rounded(np.float32)
    ref = O.step(q.net, q.pde, q.W, q.x_int, q.x_bc, q.g_bc)
    check("batched 3-instance inst1 loss", relerr(plan.loss[1].cpu().numpy(), ref["loss"]), 1e-5)
    for l, g in enumerate(plan.layer_grads(1, q.net)):
        check(f"batched 3-instance inst1 gW{l}", relerr(g.double().cpu().numpy(), ref["gW"][l]), 1e-5)


@pytest.mark.slow
def test_full_batched_plan_against_oracle():
    """The 256-instance Burgers batch (nu log-uniform in [1e-3, 1e-1], interior
    counts uniform in [4,096, 65,536], boundary counts 1/16 of them), with the
    first instance set to the smallest count of that range and the last to
    the largest: those two, the instance with the most and the one with the
    fewest drawn points against the FP64 oracle at the literal 1e-5."""
    wl = WL.WORKLOADS["burgers_batched_c5"]
    probs = WL.batched_instances(wl)
    assert len(probs) == 256
    for q, n in ((0, 4096), (255, 65536)):
        probs[q] = WL.make_problem(wl, n_int=n, n_bc=n // 16, seed=wl.seed + 1000 * (q + 1), pde=probs[q].pde)
    print(f"[case] full batched plan: {sum(p.n_int for p in probs)} interior points", flush=True)
    plan = H.Plan(probs)
    plan.execute()
    torch.cuda.synchronize()
    assert H.read_status(plan.ws) == 0
    sizes = [p.n_int for p in probs[1:255]]
    picks = sorted({0, 255, 1 + int(np.argmin(sizes)), 1 + int(np.argmax(sizes))})
    for q in picks:
        r = probs[q].rounded(np.float32)
        ref = O.step(r.net, r.pde, r.W, r.x_int, r.x_bc, r.g_bc)
        lab = f"batched c5 inst{q} ({r.n_int}+{r.n_bc}, nu {r.pde.nu:.2e})"
        check(f"{lab} loss", relerr(plan.loss[q].cpu().numpy(), ref["loss"]), 1e-5)
        for l, g in enumerate(plan.layer_grads(q, r.net)):
            check(f"{lab} gW{l}", relerr(g.double().cpu().numpy(), ref["gW"][l]), 1e-5)
    plan.close()


def test_batched_replays_are_identical_and_follow_weight_updates():
    probs = _instances(5)
    plan = H.Plan(probs)
    plan.execute()
    torch.cuda.synchronize()
    l1, g1 = plan.loss.clone(), plan.gW.clone()
    plan.execute()
    torch.cuda.synchronize()
    assert torch.equal(l1, plan.loss) and torch.equal(g1, plan.gW)
    # a step of plain gradient descent on every instance, then the next step
    with torch.no_grad():
        plan.W -= 1e-3 * plan.gW
    plan.execute()
    torch.cuda.synchronize()
    new = []
    for q, pr in enumerate(probs):
        Ws, o = [], 0
        for r, c in pr.net.weight_shapes():
            Ws.append(plan.W[q, o:o + r * c].reshape(r, c).double().cpu().numpy())
            o += r * c
        new.append(WL.Problem(pr.net, pr.pde, Ws, pr.x_int, pr.x_bc, pr.g_bc))
    _check_against_single_steps(plan, new)


def test_autotune_cache_is_written_and_reused(tmp_path, monkeypatch):
    """The first plan of a kind of batch times the candidates and stores the
    winner under its key; a second plan of the same kind reads it (no
    timing) and gives the same step bit for bit; a batch in another point
    bucket is tuned anew."""
    import json
    cache = tmp_path / "autotune.json"
    monkeypatch.setenv("HRKAN_AUTOTUNE_CACHE", str(cache))
    probs = _instances(5)
    p1 = H.Plan(probs)
    c1, ms1 = p1.autotune_info()
    assert not c1 and ms1 > 0
    doc = json.loads(cache.read_text())
    assert doc["hrkan_autotune"] == 1 and len(doc["entries"]) == 1
    key = next(iter(doc["entries"]))
    print(f"[autotune] key {key}: {doc['entries'][key]}", flush=True)
    assert "|w=2,32,32,1|G=10|k=3|m=4|" in key and "|inst=2^3|" in key
    assert doc["entries"][key]["slice_pts"] == p1.config()[0]
    p2 = H.Plan(probs)
    c2, ms2 = p2.autotune_info()
    assert c2 and ms2 == pytest.approx(ms1, rel=1e-5)
    assert p2.config() == p1.config()
    p1.execute()
    p2.execute()
    torch.cuda.synchronize()
    assert torch.equal(p1.loss, p2.loss) and torch.equal(p1.gW, p2.gW)
    p3 = H.Plan(_instances(5, lo=20000, hi=30000))
    assert not p3.autotune_info()[0]
    assert len(json.loads(cache.read_text())["entries"]) == 2
    for p in (p1, p2, p3):
        p.close()
    # an empty value turns the cache off
    monkeypatch.setenv("HRKAN_AUTOTUNE_CACHE", "")
    p4 = H.Plan(probs)
    assert not p4.autotune_info()[0]
    p4.close()


@pytest.mark.parametrize("S", [2, 3])
def test_bf16_batched_plan_against_oracle(S):
    """BF16 plans (block-sparse kernels, S product terms, FP32 master
    weights) against the FP64 oracle at the literal 2e-2: on the master
    weights for S = 3, on the BF16-rounded weights for S = 2 (only their high
    piece enters the products)."""
    from gpu_util import bf16_round
    probs = _instances(4, lo=2000, hi=6000)
    plan = H.Plan(probs, dtype="bf16", bf16_split=S)
    plan.execute()
    torch.cuda.synchronize()
    assert H.read_status(plan.ws) == 0
    loss = plan.loss.cpu().numpy()
    for q in (0, 3):
        qq = probs[q].rounded(np.float32)
        W = qq.W if S == 3 else [bf16_round(w) for w in qq.W]
        ref = O.step(qq.net, qq.pde, W, qq.x_int, qq.x_bc, qq.g_bc)
        check(f"bf16 plan S{S} instance {q} loss", relerr(loss[q], ref["loss"]), 2e-2)
        for l, g in enumerate(plan.layer_grads(q, probs[q].net)):
            check(f"bf16 plan S{S} instance {q} gW{l}", relerr(g.double().cpu().numpy(), ref["gW"][l]), 2e-2)
    plan.close()
