"""Finite-difference check of the HIP path's FP64 gradient on the Poisson
network [2,64,64,64,1], G = 16 (Sec. 4.1's problem at the larger network).

The loss L(W) = alpha L_pde + L_bc is evaluated by the same HIP step, in FP64,
at W +- h V; central differences with h = 1e-4 are compared with the
gradient the step returns:
  * directional: (L(W + hV) - L(W - hV)) / 2h against <gW, V> for 8 seeded
    random unit directions V (all layers at once), on the full point set;
  * coordinate: 64 seeded weights per layer, on a smaller point set.
Smoothness: the residual holds second-derivative jets, which depend on a
weight of an earlier layer through v'' of the later layers' inputs; with
m = 4 the basis of Eq. 2 is C^3, so v'' is only C^1 and the loss is C^1 in W,
its second derivative jumping wherever a point's hidden input crosses a
knot. A central difference D(h) is then accurate to O(h) times those jumps
rather than O(h^2). The FP64 oracle's own central differences on the same
sampled weights of this large network (inv_w = 4 per layer scales each
second-derivative jet by 16) are off its exact gradient by up to 7.5e-4 of
the layer's largest gradient entry at h = 1e-4 and 1.5e-6 at h = 1e-6
(first layer; 1.1e-5 and 1.9e-8 for the second), while sums over many
weights along a direction average the kinks out. The coordinate check
therefore allows 3e-3 (h = 1e-4) and 1e-5 (h = 1e-6) of the largest entry,
about 4 and 7 times those measured errors.
"""
import numpy as np
import pytest
import torch

from gpu_util import to_dev
from paper_2409_14248_amd import hrkan as H
from paper_2409_14248_amd import workloads as WL

pytestmark = pytest.mark.gpu

H_FD = 1e-4


def _setup(n_int=None, n_bc=None):
    pr = WL.make_problem(WL.WORKLOADS["poisson_c3"], n_int=n_int, n_bc=n_bc)
    nd = H.net_desc(pr.net, "f64")
    pd = H.pde_desc(pr.pde)
    W = [to_dev(w, "f64") for w in pr.W]
    xi, xb, g = to_dev(pr.x_int, "f64"), to_dev(pr.x_bc, "f64"), to_dev(pr.g_bc, "f64")
    ws = H.alloc_workspace(H.workspace_bytes(nd, pd, pr.n_int, pr.n_bc))
    loss_buf = torch.empty(3, dtype=torch.float64, device="cuda")
    gW_buf = [torch.empty_like(w) for w in W]

    def loss_at(Wx):
        H.step(nd, pd, Wx, xi, xb, g, ws, loss_out=loss_buf, gW_out=gW_buf)
        return float(loss_buf[0].item())

    loss, gW = H.step(nd, pd, W, xi, xb, g, ws)
    torch.cuda.synchronize()
    return pr, W, loss_at, [t.clone() for t in gW]


def test_directional_fd_full_c3_points():
    pr, W, loss_at, gW = _setup()
    rng = np.random.default_rng(WL.SEED_BASE + 31)
    for _ in range(8):
        V = [rng.standard_normal(w.shape) for w in pr.W]
        nrm = np.sqrt(sum(float((v * v).sum()) for v in V))
        V = [torch.as_tensor(v / nrm, device="cuda") for v in V]
        lp = loss_at([w + H_FD * v for w, v in zip(W, V)])
        lm = loss_at([w - H_FD * v for w, v in zip(W, V)])
        fd = (lp - lm) / (2 * H_FD)
        an = sum(float((gw * v).sum()) for gw, v in zip(gW, V))
        gnorm = np.sqrt(sum(float((gw * gw).sum()) for gw in gW))
        assert abs(fd - an) <= 1e-6 * gnorm, (fd, an, gnorm)


def test_coordinate_fd_sampled_weights():
    pr, W, loss_at, gW = _setup(n_int=8192, n_bc=512)
    rng = np.random.default_rng(WL.SEED_BASE + 32)
    for l, w in enumerate(W):
        flat = w.view(-1)
        gflat = gW[l].view(-1).cpu().numpy()
        gmax = float(np.abs(gflat).max())
        idx = rng.choice(flat.numel(), size=min(64, flat.numel()), replace=False)
        for k in idx:
            def central(h):
                Wp = [x.clone() for x in W]
                Wp[l].view(-1)[k] += h
                lp = loss_at(Wp)
                Wp[l].view(-1)[k] -= 2 * h
                lm = loss_at(Wp)
                return (lp - lm) / (2 * h)
            g_k = float(gflat[k])
            d4 = central(H_FD)
            assert abs(d4 - g_k) <= 5e-3 * abs(g_k) + 3e-3 * gmax, (l, int(k), d4, g_k)
            d6 = central(1e-6)
            assert abs(d6 - g_k) <= 1e-5 * abs(g_k) + 1e-5 * gmax, (l, int(k), d6, g_k)
