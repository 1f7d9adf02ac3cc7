"""Helpers of the GPU tests: move a seeded problem to the device in a run
dtype, run the HIP path through the C ABI, and run the oracle on the same
(rounded) inputs."""
import numpy as np
import torch

import oracle as O
from paper_2409_14248_amd import hrkan as H
from paper_2409_14248_amd import workloads as WL

NP_DTYPE = {"f64": np.float64, "f32": np.float32, "bf16": np.float32}


def to_dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=NP_DTYPE[dtype])).cuda()


def gpu_step(pr: WL.Problem, dtype: str, bf16_split: int = 2):
    nd = H.net_desc(pr.net, dtype, bf16_split)
    pd = H.pde_desc(pr.pde)
    W = [to_dev(w, dtype) for w in pr.W]
    xi, xb, g = to_dev(pr.x_int, dtype), to_dev(pr.x_bc, dtype), to_dev(pr.g_bc, dtype)
    ws = H.alloc_workspace(H.workspace_bytes(nd, pd, pr.n_int, pr.n_bc))
    loss, gW = H.step(nd, pd, W, xi, xb, g, ws)
    torch.cuda.synchronize()
    return loss.cpu().numpy(), [t.double().cpu().numpy() for t in gW], ws


def oracle_step(pr: WL.Problem, dtype: str):
    """Oracle on the inputs exactly as the run dtype holds them."""
    q = pr.rounded(NP_DTYPE[dtype])
    return O.step(q.net, q.pde, q.W, q.x_int, q.x_bc, q.g_bc)


def gpu_forward(pr: WL.Problem, dtype: str, x: np.ndarray, mask: int, saved: bool = False):
    nd = H.net_desc(pr.net, dtype)
    pd = H.pde_desc(pr.pde)
    W = [to_dev(w, dtype) for w in pr.W]
    xd = to_dev(x, dtype)
    n = x.shape[0]
    ws = H.alloc_workspace(H.workspace_bytes(nd, pd, n, 0))
    sv = None
    if saved:
        sv = torch.empty(max(H.saved_bytes(nd, n, mask), 4), dtype=torch.uint8, device="cuda")
    jets = H.forward_jets(nd, W, xd, mask, ws, saved=sv)
    torch.cuda.synchronize()
    return jets.double().cpu().numpy(), sv, W, xd, ws, nd


def saved_blocks(pr: WL.Problem, sv: torch.Tensor, dtype: str, C: int, n: int):
    """Split the saved buffer into per-layer [C][w_l][n] float64 arrays (l = 1..L-1)."""
    tdt = torch.float64 if dtype == "f64" else torch.float32
    flat = sv.view(tdt)
    out, off = [], 0
    for w in pr.net.widths[1:-1]:
        cnt = C * w * n
        out.append(flat[off:off + cnt].double().cpu().numpy().reshape(C, w, n))
        off += cnt
    return out


SLOTS_OF_MASK = {
    H.MASK_POISSON: [0, 1, 2, 3, 4],
    H.MASK_BURGERS: [0, 1, 2, 3],
    H.MASK_VALUE: [0],
}


def expand(jets_c: np.ndarray, mask: int) -> np.ndarray:
    """[C][...] channels of a mask -> the oracle's 5 slots (zeros elsewhere)."""
    out = np.zeros((5,) + jets_c.shape[1:])
    for c, s in enumerate(SLOTS_OF_MASK[mask]):
        out[s] = jets_c[c]
    return out


def bf16_round(a):
    """Round-to-nearest-even of FP32 values to the BF16 grid (as float64)."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
