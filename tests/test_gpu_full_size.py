"""Full-size launches checked on sampled points.

The benchmark workloads at their full point counts run through
hrkan_forward_jets. Those are the forward kernels and tile shapes of the
step: c2 with 65,536 interior points, c3 with 262,144, c4 with 1,048,576.
A point's output jets depend on that point alone (Sec. 3: every point goes
through the same layers). So the oracle computes them for a seeded sample
of points, and the launch's outputs at those points are compared with it.
The first and last points are always in the sample.

Gates are those of the small-size tests, taken over the sample (normwise
per channel):
- FP32: max(1e-5, 3 x the oracle's FP32 rounding floor);
- BF16 (S = 2): the literal 2e-2 against the oracle on the BF16-rounded
  weights that the S = 2 kernels multiply.
"""
import numpy as np
import pytest

import oracle as O
from conftest import check, relerr
from gpu_util import SLOTS_OF_MASK, bf16_round, to_dev
from paper_2409_14248_amd import hrkan as H
from paper_2409_14248_amd import workloads as WL

pytestmark = pytest.mark.gpu

SAMPLE = 64
TOL = {"f32": 1e-5, "bf16": 2e-2}
FLOOR_FACTOR = 3.0


def sample_points(n, seed):
    rng = np.random.default_rng(seed)
    idx = rng.choice(np.arange(1, n - 1), SAMPLE - 2, replace=False)
    return np.sort(np.concatenate([[0, n - 1], idx]))


@pytest.mark.parametrize("name,dtype", [("burgers_c2", "bf16"), ("poisson_c3", "f32"),
                                        ("burgers_c4", "f32"), ("burgers_c4", "bf16")])
def test_full_size_forward_jets_at_sampled_points(name, dtype):
    pr = WL.make_problem(WL.WORKLOADS[name])
    q = pr.rounded(np.float32)
    mask = H.pde_mask(pr.pde)
    nd = H.net_desc(pr.net, dtype, 2)
    pd = H.pde_desc(pr.pde)
    W = [to_dev(w, "f32") for w in pr.W]
    ws = H.alloc_workspace(H.workspace_bytes(nd, pd, pr.n_int, 0))
    jets = H.forward_jets(nd, W, to_dev(pr.x_int, "f32"), mask, ws)
    idx = sample_points(pr.n_int, WL.SEED_BASE + 77)
    got = jets[:, idx].double().cpu().numpy()
    del jets, ws
    xs = q.x_int[idx]
    if dtype == "f32":
        ref = O.forward(q.net, q.W, xs)
        with O.rounding("f32"):
            rnd = O.forward(q.net, q.W, xs)
    else:
        ref = O.forward(q.net, [bf16_round(w) for w in q.W], xs)
    for c, slot in enumerate(SLOTS_OF_MASK[mask]):
        err = relerr(got[c], ref[slot])
        if dtype == "f32":
            check(f"{name} full sampled f32 jet{slot}", err, TOL["f32"], relerr(rnd[slot], ref[slot]), FLOOR_FACTOR)
        else:
            check(f"{name} full sampled bf16 S2 W=bf16 jet{slot}", err, TOL["bf16"])


def _step(pr, dtype, x_int, x_bc, g_bc):
    nd = H.net_desc(pr.net, dtype, 2)
    pd = H.pde_desc(pr.pde)
    W = [to_dev(w, "f32") for w in pr.W]
    xi, xb, g = to_dev(x_int, "f32"), to_dev(x_bc, "f32"), to_dev(g_bc, "f32")
    ws = H.alloc_workspace(H.workspace_bytes(nd, pd, len(x_int), len(x_bc)))
    loss, gW = H.step(nd, pd, W, xi, xb, g, ws)
    out = loss.cpu().numpy().copy(), [t.double().cpu().numpy() for t in gW]
    del ws
    return out


# The loss is alpha times the mean of the squared residuals plus the mean of
# the squared boundary misfits (Sec. 4.1, Sec. 4.2), so on a point set split
# into two halves of equal counts, L(all) = (L(half 1) + L(half 2)) / 2, and
# the same holds for its gradient: an identity of the full-size launch that a
# dropped slice, a wrong normalisation or a point range read twice breaks.
@pytest.mark.parametrize("name,dtype", [("poisson_c3", "f32"), ("burgers_c4", "f32"), ("burgers_c4", "bf16")])
def test_full_size_step_is_the_mean_of_its_halves(name, dtype):
    pr = WL.make_problem(WL.WORKLOADS[name])
    hi, hb = pr.n_int // 2, pr.n_bc // 2
    assert 2 * hi == pr.n_int and 2 * hb == pr.n_bc
    rng = np.random.default_rng(WL.SEED_BASE + 78)
    pi, pb = rng.permutation(pr.n_int), rng.permutation(pr.n_bc)
    la, ga = _step(pr, dtype, pr.x_int, pr.x_bc, pr.g_bc)
    l1, g1 = _step(pr, dtype, pr.x_int[pi[:hi]], pr.x_bc[pb[:hb]], pr.g_bc[pb[:hb]])
    l2, g2 = _step(pr, dtype, pr.x_int[pi[hi:]], pr.x_bc[pb[hb:]], pr.g_bc[pb[hb:]])
    assert relerr(la, (l1 + l2) / 2) < 1e-5, (la, l1, l2)
    for l, (a, b, c) in enumerate(zip(ga, g1, g2)):
        assert relerr(a, (b + c) / 2) < 1e-4, (l, relerr(a, (b + c) / 2))
