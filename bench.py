#!/usr/bin/env python3
"""Benchmark of one HRKAN physics-informed training step on one MI355X.

A step is the whole hot path over one batch of synthetic collocation points:
forward jets at the interior and boundary points, residual and loss, and the
reverse pass to every weight (hrkan_step). Default workload: viscous Burgers
(nu = 0.01/pi) with a [2,128,128,128,1] HRKAN, G = 20, k = 3, m = 4,
1,048,576 interior + 65,536 initial/boundary points, inputs resident in HBM.
The headline is the FP32 step; the same step with BF16 products (S = 2 and
S = 3 BF16 terms per product, FP32 jets and accumulation) is timed beside it
on the same shapes. Each step is timed launched from the host and replayed
from a HIP graph, and the faster is reported (the JSON line names it and
gives both). Every timed variant also reports its error against the FP64
oracle on a step over the sample of the same points that the CPU baseline
times.

Prints ONE JSON line: interior collocation points per second over the timed
steps, the roofline position of the dominant kernel (its launches timed with
HIP events on the stream they run on; flops counted as the products the
method executes, the k+1 non-zero basis functions per input), and the CPU
oracle timed on the host cores on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PINN train-step collocation points/s (fwd jets+residual+bwd), bf16 vs fp32"

# MI355X published dense peaks (TFLOP/s) and HBM bandwidth (GB/s)
PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "hbm": 8000.0}

# the kernels and the launch sequence the counter summary was taken on
KERNEL_SRC = [os.path.join(ROOT, "paper_2409_14248_amd", "csrc", f) for f in ("kernels_tc.hip", "runtime.cpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_burgers_c4_f32.md")
TRAFFIC_RUN = ("burgers_c4", "f32")     # the workload and dtype those counters were taken on


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="burgers_c4")
    ap.add_argument("--dtype", default=None,
                    help="f64 | f32 | bf16 (default: FP32, or FP64 for an FP64 workload)")
    ap.add_argument("--bf16-split", type=int, default=2)
    ap.add_argument("--no-compare", action="store_true",
                    help="time only the headline dtype (no BF16 S = 2 / S = 3 steps beside FP32)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-points", type=int, default=2048,
                    help="interior points of each CPU oracle step of the baseline sample (the GPU step's "
                         "error figures are taken on the same sample)")
    ap.add_argument("--eager", action="store_true",
                    help="launch every kernel from the host instead of replaying a HIP graph")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 256 MiB device copy (calibrates HBM byte counters)")
    return ap.parse_args()


def layer_flops(net, C, n, live=False):
    """Algorithmic flops of each contraction of each layer for n points with C
    jet channels: 2*C*K*N per point, K = w_in * n_b (the dense basis-by-W
    product the method defines). live=True counts only the k+1 non-zero
    basis functions per input (K = w_in * (k+1)): the products the kernels
    execute."""
    out = {}
    for l in range(net.n_layers):
        K = net.widths[l] * ((net.k + 1) if live else net.n_basis)
        N = net.widths[l + 1]
        f = 2.0 * C * K * N * n
        out[f"fwd_l{l}"] = f
        out[f"dw_l{l}"] = f
        if l > 0:
            out[f"dx_l{l}"] = f
    return out


def kernel_flops(pr, C, live=False, merged=False):
    """Algorithmic flops of every profiled launch name: the interior set with
    C channels under the interior names and the boundary set with one channel
    under the _bc names; when the step runs the boundary points as more rows
    of the interior set (merged), the interior names carry both."""
    out = dict(layer_flops(pr.net, C, pr.n_int, live))
    for k, v in layer_flops(pr.net, 1, pr.n_bc, live).items():
        if merged:
            out[k] += v
        else:
            out[k + "_bc"] = v
    # a 1-output layer's weight gradient and input bars run as one launch
    for k in [k for k in out if k.startswith("dx_l")]:
        out["dwx" + k[2:]] = out["dw" + k[2:]] + out[k]
    return out


def traffic_record(kernel_name, launches_per_step, workload, dtype):
    """HBM bytes per launch of a kernel from the committed counter summary,
    if that summary was taken on this workload and the current kernel
    source; else None."""
    if (workload, dtype) != TRAFFIC_RUN:
        return None
    if not os.path.exists(TRAFFIC_FILE) or not all(os.path.exists(f) for f in KERNEL_SRC):
        return None
    txt = open(TRAFFIC_FILE).read()
    m = re.search(r"kernel source sha256:\s*([0-9a-f]{64})", txt)
    cur = hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SRC)).hexdigest()
    if not m or m.group(1) != cur:
        return None
    m = re.search(r"^\|\s*%s\s*\|\s*([0-9.eE+]+)\s*\|" % re.escape(kernel_name), txt, re.M)
    return float(m.group(1)) if m else None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def time_step(step, steps, warmup, eager_only):
    """Eager and graph-replayed timings of a step (ms per step)."""
    import torch

    def timed(fn, k):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record()
        for _ in range(k):
            fn()
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / k

    for _ in range(warmup):
        step()
    eager_ms = timed(step, steps)
    graph_ms = None
    if not eager_only:
        step.capture()
        for _ in range(warmup):
            step.replay()
        graph_ms = timed(step.replay, steps)
    launch = "hip_graph" if graph_ms is not None and graph_ms < eager_ms else "eager"
    ms = graph_ms if launch == "hip_graph" else eager_ms
    return ms, eager_ms, graph_ms, launch


def sample_problem(pr, n):
    """The first n interior and n/16 boundary points of a problem, same weights."""
    from paper_2409_14248_amd import workloads as WL
    n = min(n, pr.n_int)
    nb = min(max(n // 16, 4), pr.n_bc)
    return WL.Problem(pr.net, pr.pde, pr.W, pr.x_int[:n], pr.x_bc[:nb], pr.g_bc[:nb])


def cpu_baseline_leg(pr, dtype, args, want_bf16_weights):
    """The FP64 oracle, as it stands, timed on the host cores over whole steps
    on a bounded sample of the workload; its result on that sample is kept as
    the reference of the GPU error figures (and, for BF16 with S <= 2, one
    more oracle step with the weights rounded to BF16)."""
    import numpy as np
    import torch

    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O

    sub = sample_problem(pr, args.cpu_points)
    q = sub.rounded(np.float32 if dtype != "f64" else np.float64)
    t = time.time()
    reps = 0
    while True:
        master = O.step(q.net, q.pde, q.W, q.x_int, q.x_bc, q.g_bc)
        reps += 1
        el = time.time() - t
        if el >= args.cpu_seconds or reps >= 200:
            break
    cpu = {"value": round(reps * q.n_int / el, 1), "unit": "points/s", "cores": O.num_threads(),
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"{reps} whole FP64 step(s) of the {args.workload} network on its first {q.n_int} "
                     f"interior + {q.n_bc} boundary points in {el:.1f} s"}
    wb = None
    if want_bf16_weights:
        bw = [torch.tensor(w, dtype=torch.float32).to(torch.bfloat16).double().numpy() for w in q.W]
        wb = O.step(q.net, q.pde, bw, q.x_int, q.x_bc, q.g_bc)
    return cpu, sub, master, wb


def gpu_errors(sub, cases, master, wb):
    """Loss and weight-gradient errors of the GPU step on the sample against
    the oracle's: normwise relative error of the loss and the largest over
    the layers' gradients. cases: (label, dtype, S). For S <= 2 also against
    the oracle fed the BF16-rounded weights (the weights those kernels
    multiply)."""
    import numpy as np
    import torch

    from paper_2409_14248_amd import hrkan as H

    def rel(a, b):
        a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    out = {}
    for label, dtype, S in cases:
        st = H.Step(sub, dtype, S)
        loss, gW = st()
        torch.cuda.synchronize()
        loss = loss.cpu().numpy()
        gW = [g.double().cpu().numpy() for g in gW]
        e = {"sample": f"{sub.n_int}+{sub.n_bc} points",
             "err_loss": rel(loss, master["loss"]),
             "err_gW_max": max(rel(a, b) for a, b in zip(gW, master["gW"]))}
        if dtype == "bf16" and S <= 2 and wb is not None:
            e["err_loss_vs_bf16_weights"] = rel(loss, wb["loss"])
            e["err_gW_max_vs_bf16_weights"] = max(rel(a, b) for a, b in zip(gW, wb["gW"]))
        out[label] = {k: (float(f"{v:.4g}") if isinstance(v, float) else v) for k, v in e.items()}
        del st
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(how the step shards over several GPUs is described, not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2409_14248_amd import hrkan as H
    from paper_2409_14248_amd import workloads as WL

    wl = WL.WORKLOADS[args.workload]
    if wl.n_instances > 1:
        return bench_batched(args, wl)
    dtype = args.dtype or ("f64" if wl.dtype == "f64" else "f32")
    pr = WL.make_problem(wl)
    step = H.Step(pr, dtype, args.bf16_split)
    torch.cuda.synchronize()
    ms, eager_ms, graph_ms, launch = time_step(step, args.steps, args.warmup, args.eager)
    loss = step.loss.cpu().numpy()

    # per-kernel times: HIP events around every launch, in a pass of its own
    prof_steps = min(args.steps, 50)
    H.profile_enable(True)
    for _ in range(prof_steps):
        step()
    torch.cuda.synchronize()
    prof = H.profile_read()
    H.profile_enable(False)
    del step

    if args.calib_copy:
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    C = H.mask_channels(H.pde_mask(pr.pde))
    merged = pr.n_bc > 0 and "fwd_l0_bc" not in prof
    dense = kernel_flops(pr, C, merged=merged)
    live = kernel_flops(pr, C, live=True, merged=merged)
    total_ms = sum(v[1] for v in prof.values()) / prof_steps
    contraction = {k: v for k, v in prof.items() if k in dense}
    dname, (dcnt, dms) = max(contraction.items(), key=lambda kv: kv[1][1])
    per_launch_ms = dms / dcnt
    launches_per_step = dcnt / prof_steps
    f_dense = dense[dname] / launches_per_step
    f_live = live[dname] / launches_per_step
    peak = PEAK[dtype]
    achieved_live = f_live / (per_launch_ms * 1e-3) / 1e12
    achieved_dense = f_dense / (per_launch_ms * 1e-3) / 1e12
    roofline = {
        "bound": "mfma", "kernel": dname, "achieved": round(achieved_live, 3), "peak": peak,
        "unit": "TFLOP/s", "frac": round(achieved_live / peak, 4),
        "traffic": traffic_record(dname, launches_per_step, args.workload, dtype),
        "flops_per_launch": f_live, "launch_ms": round(per_launch_ms, 5),
        "kernel_share": round(dms / prof_steps / total_ms, 3),
        "achieved_dense_equivalent": round(achieved_dense, 3),
        "dense_equivalent_flops_per_launch": f_dense,
    }
    step_flops_live = sum(v for k, v in live.items() if not k.startswith("dwx"))

    # the same step with BF16 products on the same shapes
    compare = {}
    cases = [("f32" if dtype != "f64" else "f64", dtype, args.bf16_split)]
    if not args.no_compare and dtype == "f32" and pr.net.k == 3 and pr.net.m == 4:
        for S in (2, 3):
            st = H.Step(pr, "bf16", S)
            torch.cuda.synchronize()
            bms, beager, bgraph, blaunch = time_step(st, args.steps, args.warmup, args.eager)
            del st
            compare[f"bf16_s{S}"] = {
                "ms_per_step": round(bms, 5), "points_per_s": round(pr.n_int / (bms * 1e-3), 1),
                "speedup_vs_f32": round(ms / bms, 3), "launch": blaunch,
                "eager_ms_per_step": round(beager, 5),
                "graph_ms_per_step": None if bgraph is None else round(bgraph, 5),
            }
            cases.append((f"bf16_s{S}", "bf16", S))
    cpu, errors = None, {}
    if not args.no_cpu:
        want_wb = any(c[1] == "bf16" and c[2] <= 2 for c in cases)
        cpu, sub, master, wb = cpu_baseline_leg(pr, dtype, args, want_wb)
        errors = gpu_errors(sub, cases, master, wb)
    for k, v in compare.items():
        v["error_vs_oracle"] = errors.get(k)

    out = {
        "metric": METRIC,
        "value": round(pr.n_int / (ms * 1e-3), 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": args.workload, "pde": "poisson2d" if pr.pde.kind == 0 else "burgers1d",
            "widths": list(pr.net.widths), "G": pr.net.G, "k": pr.net.k, "m": pr.net.m,
            "n_int": pr.n_int, "n_bc": pr.n_bc,
            **({"bf16_split": args.bf16_split} if dtype == "bf16" else {}),
        },
        "launch": launch,
        "eager_ms_per_step": round(eager_ms, 5),
        "graph_ms_per_step": None if graph_ms is None else round(graph_ms, 5),
        "total_points_per_s": round((pr.n_int + pr.n_bc) / (ms * 1e-3), 1),
        "step_executed_tflops": round(step_flops_live / (ms * 1e-3) / 1e12, 3),
        "loss": [float(v) for v in loss],
        "error_vs_oracle": errors.get(cases[0][0]),
        **compare,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels_ms_per_step": {k: round(v[1] / prof_steps, 5) for k, v in sorted(prof.items())},
    }
    print(json.dumps(out))


def bench_batched(args, wl):
    """Batched instances: one plan (one HIP graph launch per step, FP32 or
    BF16 with --dtype bf16) against the plain step of the same dtype called
    once per instance."""
    import numpy as np
    import torch

    from paper_2409_14248_amd import hrkan as H
    from paper_2409_14248_amd import workloads as WL

    probs = WL.batched_instances(wl)
    n_int = sum(p.n_int for p in probs)
    n_bc = sum(p.n_bc for p in probs)
    dtype = args.dtype or "f32"
    if dtype == "f64":
        raise SystemExit("batched plans run f32 or bf16")
    t0 = time.time()
    plan = H.Plan(probs, dtype=dtype, bf16_split=args.bf16_split)
    torch.cuda.synchronize()
    create_s = time.time() - t0

    def timed(fn, k):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    for _ in range(args.warmup):
        plan.execute()
    ms = timed(plan.execute, args.steps)

    # the plain step, once per instance (eager launches, shared workspace)
    nd = H.net_desc(probs[0].net, dtype, args.bf16_split)
    ws = H.alloc_workspace(max(H.workspace_bytes(nd, H.pde_desc(p.pde), p.n_int, p.n_bc) for p in probs))
    dev = [([torch.as_tensor(w, dtype=torch.float32, device="cuda") for w in p.W],
            torch.as_tensor(p.x_int, dtype=torch.float32, device="cuda"),
            torch.as_tensor(p.x_bc, dtype=torch.float32, device="cuda"),
            torch.as_tensor(p.g_bc, dtype=torch.float32, device="cuda"), H.pde_desc(p.pde)) for p in probs]
    loss = torch.empty(3, dtype=torch.float64, device="cuda")
    gW = [torch.empty_like(w) for w in dev[0][0]]

    def looped():
        for W, xi, xb, g, pd in dev:
            H.step(nd, pd, W, xi, xb, g, ws, loss_out=loss, gW_out=gW)

    looped()
    loop_ms = timed(looped, max(1, args.steps // 10))

    # executed flops: the k+1 live basis rows per input (the dense-equivalent
    # count of every basis row is an extra key, not a roofline fraction)
    f_pt = sum(v for v in layer_flops(probs[0].net, 4, 1, live=True).values())
    f_bc = sum(v for v in layer_flops(probs[0].net, 1, 1, live=True).values())
    step_flops = f_pt * n_int + f_bc * n_bc
    achieved = step_flops / (ms * 1e-3) / 1e12
    d_pt = sum(v for v in layer_flops(probs[0].net, 4, 1).values())
    d_bc = sum(v for v in layer_flops(probs[0].net, 1, 1).values())
    dense = (d_pt * n_int + d_bc * n_bc) / (ms * 1e-3) / 1e12
    peak = PEAK["bf16" if dtype == "bf16" else "f32"]
    tp, blocks = plan.config()
    out = {
        "metric": METRIC,
        "value": round(n_int / (ms * 1e-3), 1),
        "unit": "points/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": args.workload, "instances": len(probs), "widths": list(probs[0].net.widths),
                   "G": probs[0].net.G, "n_int_total": n_int, "n_bc_total": n_bc,
                   "tile_points": tp, "blocks": blocks},
        "launch": "hip_graph (one per batched step)",
        "plan_create_s": round(create_s, 2),
        "looped_single_step_ms": round(loop_ms, 3),
        "looped_points_per_s": round(n_int / (loop_ms * 1e-3), 1),
        "speedup_vs_looped": round(loop_ms / ms, 3),
        "roofline": {"bound": "mfma", "kernel": "whole batched step (one graph)", "achieved": round(achieved, 3),
                     "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                     "traffic": None, "achieved_dense_equivalent": round(dense, 3)},
        "cpu_baseline": None,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
