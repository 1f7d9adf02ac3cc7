"""Training runs of the paper's instances on the HIP path: hrkan_step plus
hrkan_adam per epoch, replayed from one HIP graph.

    python -m paper_2409_14248_amd.train --workload poisson_paper --epochs 3000 --lr 1e-2

Prints one JSON line: wall time of the epochs (the graph replays, after a
one-time capture), the final loss and, for the Poisson instance, the test
MSE on the 100x100 grid against the manufactured solution
u = sin(pi x) sin(pi y) (Sec. 4.1). The paper does not state its learning
rate; the Burgers instance has no closed-form solution here.
"""
import argparse
import json
import math
import time

import numpy as np
import torch

from . import hrkan as H
from . import workloads as WL


def poisson_test_mse(tr: H.Trainer, side: int = 100):
    """MSE of the trained network against sin(pi x) sin(pi y) on a side x side
    grid spanning [-1,1]^2 (edges included), and that MSE relative to the
    mean square of the solution."""
    c = np.linspace(-1.0, 1.0, side)
    X, Y = np.meshgrid(c, c, indexing="ij")
    xy = np.stack([X.ravel(), Y.ravel()], 1)
    x = torch.as_tensor(xy, dtype=torch.float32, device="cuda").contiguous()
    pd = H.pde_desc(WL.Pde(WL.POISSON2D))
    ws = H.alloc_workspace(H.workspace_bytes(tr.step.nd, pd, xy.shape[0], 0))
    u = H.forward_jets(tr.step.nd, tr.step.W, x, H.MASK_VALUE, ws)[0].double().cpu().numpy()
    exact = np.sin(math.pi * xy[:, 0]) * np.sin(math.pi * xy[:, 1])
    mse = float(np.mean((u - exact) ** 2))
    return mse, mse / float(np.mean(exact ** 2))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="poisson_paper", choices=["poisson_paper", "burgers_paper"])
    ap.add_argument("--epochs", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=1e-2)
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--seed", type=int, default=None)
    args = ap.parse_args()
    wl = WL.WORKLOADS[args.workload]
    pr = WL.make_problem(wl, seed=args.seed)
    t0 = time.time()
    tr = H.Trainer(pr, args.dtype, lr=args.lr)
    tr.capture()
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    t1 = time.time()
    hist = tr.run(args.epochs, graph=True, record_every=max(1, args.epochs // 10))
    torch.cuda.synchronize()
    wall = time.time() - t1
    out = {"workload": args.workload, "epochs": args.epochs, "lr": args.lr, "dtype": args.dtype,
           "train_s": round(wall, 4), "setup_s": round(setup_s, 3),
           "ms_per_epoch": round(1e3 * wall / args.epochs, 4),
           "loss_first": hist[0], "loss_last": hist[args.epochs - 1],
           "loss_history": {str(k): v[0] for k, v in hist.items()}}
    if args.workload == "poisson_paper":
        mse, rel = poisson_test_mse(tr)
        out["test_mse"] = mse
        out["test_mse_relative_pct"] = 100.0 * rel
    print(json.dumps(out))


if __name__ == "__main__":
    main()
