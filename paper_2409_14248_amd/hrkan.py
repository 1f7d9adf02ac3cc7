"""Python binding of the HRKAN C ABI (include/hrkan.h).

Argument marshalling only: every step of the path runs in libhrkan.so's HIP
kernels. PyTorch supplies device memory (tensor.data_ptr()) and the current
HIP stream. There is no CPU fallback: if libhrkan.so is missing or cannot be
loaded, every call raises.

Names mirror the C calls: forward_jets, residual, backward, step,
plan_create / plan_execute. `HRKANJets` and `HRKANResidual` are
torch.autograd.Functions over the same calls, so that L.backward() runs the
hand-written adjoint instead of nested autograd.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import List, Optional, Sequence

import torch

from . import workloads as _wl

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhrkan.so")

MAX_LAYERS = 8
F64, F32, BF16 = 0, 1, 2
POISSON2D, BURGERS1D, LINEAR2D = 0, 1, 2
MAX_ORDER = 5
CH_U, CH_X, CH_XX, CH_Y, CH_YY = 1, 2, 4, 8, 16
CH_X3, CH_X4, CH_X5, CH_Y3, CH_Y4, CH_Y5 = 32, 64, 128, 256, 512, 1024
MASK_POISSON = CH_U | CH_X | CH_XX | CH_Y | CH_YY
MASK_BURGERS = CH_U | CH_X | CH_XX | CH_Y
MASK_VALUE = CH_U
STATUS_NONFINITE = 1

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_DEVICE, ERR_PLAN_MISMATCH, ERR_HOST_MEMORY = \
    0, -1, -2, -3, -4, -5, -6

EXPORTS = [
    "hrkan_net_init", "hrkan_pde_init", "hrkan_mask_channels", "hrkan_mask_of_orders", "hrkan_saved_bytes",
    "hrkan_workspace_bytes", "hrkan_forward_jets", "hrkan_residual", "hrkan_backward",
    "hrkan_step", "hrkan_step_static", "hrkan_adam", "hrkan_plan_workspace_bytes", "hrkan_plan_create", "hrkan_plan_execute",
    "hrkan_plan_config", "hrkan_plan_autotune_info", "hrkan_plan_destroy", "hrkan_read_status", "hrkan_status_string",
    "hrkan_last_error", "hrkan_version", "hrkan_profile_enable", "hrkan_profile_read",
]


class HrkanError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class NetDesc(ctypes.Structure):
    _fields_ = [
        ("n_layers", ctypes.c_int32),
        ("widths", ctypes.c_int32 * (MAX_LAYERS + 1)),
        ("G", ctypes.c_int32),
        ("k", ctypes.c_int32),
        ("m", ctypes.c_int32),
        ("lo", ctypes.c_double),
        ("hi", ctypes.c_double),
        ("dtype", ctypes.c_int32),
        ("bf16_split", ctypes.c_int32),
    ]


class PdeDesc(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("nu", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("adv", ctypes.c_double),
        ("c0", ctypes.c_double),
        ("cx", ctypes.c_double * MAX_ORDER),
        ("cy", ctypes.c_double * MAX_ORDER),
    ]


class Points(ctypes.Structure):
    _fields_ = [
        ("x_int", ctypes.c_void_p),
        ("n_int", ctypes.c_int64),
        ("x_bc", ctypes.c_void_p),
        ("n_bc", ctypes.c_int64),
        ("g_bc", ctypes.c_void_p),
    ]


_lib = None


def lib():
    """Load libhrkan.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HRKAN HIP library not built: {LIB_PATH} is missing "
                           "(run `python -m paper_2409_14248_amd.build_lib`)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
    P = ctypes.POINTER
    for name in EXPORTS:
        getattr(L, name).restype = ctypes.c_int
    L.hrkan_net_init.argtypes = [P(NetDesc)]
    L.hrkan_pde_init.argtypes = [P(PdeDesc), i32]
    L.hrkan_mask_channels.argtypes = [u32]
    L.hrkan_mask_of_orders.argtypes = [i32, i32]
    L.hrkan_saved_bytes.argtypes = [P(NetDesc), i64, u32, P(sz)]
    L.hrkan_workspace_bytes.argtypes = [P(NetDesc), P(PdeDesc), i64, i64, P(sz)]
    L.hrkan_forward_jets.argtypes = [P(NetDesc), P(vp), vp, i64, u32, vp, vp, vp, sz, vp]
    L.hrkan_residual.argtypes = [P(PdeDesc), i32, vp, vp, P(Points), vp, vp, vp, vp, vp, sz, vp]
    L.hrkan_backward.argtypes = [P(NetDesc), P(vp), vp, i64, u32, vp, vp, P(vp), i32, vp, sz, vp]
    L.hrkan_step.argtypes = [P(NetDesc), P(PdeDesc), P(vp), P(Points), vp, P(vp), vp, sz, vp]
    L.hrkan_step_static.argtypes = [P(NetDesc), P(PdeDesc), P(vp), P(Points), vp, P(vp), vp]
    L.hrkan_adam.argtypes = [P(NetDesc), P(vp), P(vp), P(vp), P(vp), vp, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double, ctypes.c_double, vp]
    L.hrkan_plan_workspace_bytes.argtypes = [P(NetDesc), i32, P(Points), P(sz)]
    L.hrkan_plan_create.argtypes = [P(vp), P(NetDesc), i32, P(PdeDesc), vp, P(Points), vp, vp, vp,
                                    sz, vp]
    L.hrkan_plan_execute.argtypes = [vp, vp]
    L.hrkan_plan_config.argtypes = [vp, P(i32), P(i32)]
    L.hrkan_plan_autotune_info.argtypes = [vp, P(i32), P(ctypes.c_double)]
    L.hrkan_plan_destroy.argtypes = [vp]
    L.hrkan_plan_destroy.restype = None
    L.hrkan_read_status.argtypes = [vp, sz, vp, P(u32)]
    L.hrkan_status_string.argtypes = [ctypes.c_int]
    L.hrkan_status_string.restype = ctypes.c_char_p
    L.hrkan_last_error.argtypes = []
    L.hrkan_last_error.restype = ctypes.c_char_p
    L.hrkan_mask_of_orders.restype = u32
    L.hrkan_version.argtypes = []
    L.hrkan_profile_enable.argtypes = [i32]
    L.hrkan_profile_read.argtypes = [ctypes.c_char_p, sz]
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != OK:
        L = lib()
        raise HrkanError(rc, f"{L.hrkan_status_string(rc).decode()}: {L.hrkan_last_error().decode()}")


# ---------------------------------------------------------------------------
# descriptors
# ---------------------------------------------------------------------------
DTYPES = {"f64": F64, "f32": F32, "bf16": BF16}
TORCH_DTYPE = {F64: torch.float64, F32: torch.float32, BF16: torch.float32}


def net_desc(net: _wl.Net, dtype="f32", bf16_split: int = 2) -> NetDesc:
    d = NetDesc()
    w = list(net.widths)
    d.n_layers = len(w) - 1
    for i, v in enumerate(w):
        d.widths[i] = int(v)
    d.G, d.k, d.m = int(net.G), int(net.k), int(net.m)
    d.lo, d.hi = float(net.lo), float(net.hi)
    d.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    d.bf16_split = int(bf16_split)
    return d


def pde_desc(pde: _wl.Pde) -> PdeDesc:
    p = PdeDesc()
    p.kind, p.nu, p.alpha, p.adv = int(pde.kind), float(pde.nu), float(pde.alpha), float(pde.adv)
    p.c0 = float(getattr(pde, "c0", 0.0))
    for k, v in enumerate(getattr(pde, "cx", ())):
        p.cx[k] = float(v)
    for k, v in enumerate(getattr(pde, "cy", ())):
        p.cy[k] = float(v)
    return p


def mask_of_orders(ox: int, oy: int) -> int:
    """The mask of the value and the derivatives of order 1..ox along x and
    1..oy along y."""
    m = lib().hrkan_mask_of_orders(int(ox), int(oy))
    if m == 0:
        raise HrkanError(ERR_INVALID_ARG, f"orders ({ox}, {oy}) outside 0..{MAX_ORDER}")
    return m


def pde_mask(pde) -> int:
    """Interior channel mask of a PDE (a workloads.Pde, or a kind for the
    Poisson and Burgers kinds)."""
    kind = pde if isinstance(pde, int) else int(pde.kind)
    if kind == POISSON2D:
        return MASK_POISSON
    if kind == BURGERS1D:
        return MASK_BURGERS
    return mask_of_orders(*pde.orders)


def mask_channels(mask: int) -> int:
    c = lib().hrkan_mask_channels(mask)
    if c < 0:
        check(c)
    return c


def array_dtype(nd: NetDesc) -> torch.dtype:
    return TORCH_DTYPE[nd.dtype]


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _ptr_array(ts: Sequence[torch.Tensor]):
    return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


def _dev(t: torch.Tensor, dtype: torch.dtype) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError("HRKAN arrays must be device tensors")
    if t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return t.contiguous()


def workspace_bytes(nd: NetDesc, pd: PdeDesc, n_int: int, n_bc: int) -> int:
    b = ctypes.c_size_t(0)
    check(lib().hrkan_workspace_bytes(ctypes.byref(nd), ctypes.byref(pd), int(n_int), int(n_bc),
                                      ctypes.byref(b)))
    return b.value


def saved_bytes(nd: NetDesc, n: int, mask: int) -> int:
    b = ctypes.c_size_t(0)
    check(lib().hrkan_saved_bytes(ctypes.byref(nd), int(n), int(mask), ctypes.byref(b)))
    return b.value


def alloc_workspace(nbytes: int, device=None) -> torch.Tensor:
    # torch's caching allocator returns 512-byte aligned blocks
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device or "cuda")
    assert t.data_ptr() % 256 == 0
    t[:256].zero_()          # device status word starts clear
    return t


# ---------------------------------------------------------------------------
# the four calls
# ---------------------------------------------------------------------------
def forward_jets(nd: NetDesc, W: Sequence[torch.Tensor], x: torch.Tensor, mask: int,
                 ws: torch.Tensor, jets_out: Optional[torch.Tensor] = None,
                 saved: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    dt = array_dtype(nd)
    x = _dev(x, dt)
    W = [_dev(w, dt) for w in W]
    n = x.shape[0]
    C = mask_channels(mask)
    if jets_out is None:
        jets_out = torch.empty((C, n), dtype=dt, device=x.device)
    check(lib().hrkan_forward_jets(ctypes.byref(nd), _ptr_array(W), _ptr(x), n, mask, _ptr(jets_out),
                                   _ptr(saved), _ptr(ws), ws.numel(), _stream(stream)))
    return jets_out


def residual(pd: PdeDesc, dtype: int, jets_int: torch.Tensor, u_bc: torch.Tensor,
             x_int: torch.Tensor, g_bc: torch.Tensor, ws: torch.Tensor,
             loss_out: Optional[torch.Tensor] = None, r_out: Optional[torch.Tensor] = None,
             seed_int: Optional[torch.Tensor] = None, seed_bc: Optional[torch.Tensor] = None,
             stream=None):
    pts = Points(x_int.data_ptr(), x_int.shape[0], None, u_bc.shape[0], g_bc.data_ptr())
    if loss_out is None:
        loss_out = torch.empty(3, dtype=torch.float64, device=jets_int.device)
    check(lib().hrkan_residual(ctypes.byref(pd), int(dtype), _ptr(jets_int), _ptr(u_bc),
                               ctypes.byref(pts), _ptr(r_out), _ptr(loss_out), _ptr(seed_int),
                               _ptr(seed_bc), _ptr(ws), ws.numel(), _stream(stream)))
    return loss_out


def backward(nd: NetDesc, W: Sequence[torch.Tensor], x: torch.Tensor, mask: int,
             seed: torch.Tensor, saved: Optional[torch.Tensor], ws: torch.Tensor,
             gW_out: Optional[List[torch.Tensor]] = None, accumulate: bool = False,
             stream=None) -> List[torch.Tensor]:
    dt = array_dtype(nd)
    W = [_dev(w, dt) for w in W]
    if gW_out is None:
        gW_out = [torch.empty_like(w) for w in W]
    check(lib().hrkan_backward(ctypes.byref(nd), _ptr_array(W), _ptr(x), x.shape[0], mask,
                               _ptr(seed), _ptr(saved), _ptr_array(gW_out), int(bool(accumulate)),
                               _ptr(ws), ws.numel(), _stream(stream)))
    return gW_out


def step(nd: NetDesc, pd: PdeDesc, W: Sequence[torch.Tensor], x_int: torch.Tensor,
         x_bc: torch.Tensor, g_bc: torch.Tensor, ws: torch.Tensor,
         loss_out: Optional[torch.Tensor] = None, gW_out: Optional[List[torch.Tensor]] = None,
         stream=None):
    """One training step; returns (loss[3] float64 device tensor, [gW_l])."""
    dt = array_dtype(nd)
    if loss_out is None:
        loss_out = torch.empty(3, dtype=torch.float64, device=x_int.device)
    if gW_out is None:
        gW_out = [torch.empty_like(w) for w in W]
    pts = Points(x_int.data_ptr(), x_int.shape[0], x_bc.data_ptr(), x_bc.shape[0], g_bc.data_ptr())
    check(lib().hrkan_step(ctypes.byref(nd), ctypes.byref(pd), _ptr_array(W), ctypes.byref(pts),
                           _ptr(loss_out), _ptr_array(gW_out), _ptr(ws), ws.numel(), _stream(stream)))
    return loss_out, gW_out


STATIC_SCRATCH_BYTES = 64 << 20


def step_static(nd: NetDesc, pd: PdeDesc, W: Sequence[torch.Tensor], x_int: torch.Tensor,
                x_bc: torch.Tensor, g_bc: torch.Tensor, loss_out: torch.Tensor,
                gW_out: List[torch.Tensor], stream=None):
    """hrkan_step_static: the step with the library's static device workspace
    (no allocation in the call; the caller passes every output buffer)."""
    pts = Points(x_int.data_ptr(), x_int.shape[0], x_bc.data_ptr(), x_bc.shape[0], g_bc.data_ptr())
    check(lib().hrkan_step_static(ctypes.byref(nd), ctypes.byref(pd), _ptr_array(W), ctypes.byref(pts),
                                  _ptr(loss_out), _ptr_array(gW_out), _stream(stream)))
    return loss_out, gW_out


def adam(nd: NetDesc, W: Sequence[torch.Tensor], gW: Sequence[torch.Tensor], m: Sequence[torch.Tensor],
         v: Sequence[torch.Tensor], step_dev: torch.Tensor, lr: float, betas=(0.9, 0.999), eps: float = 1e-8,
         stream=None) -> None:
    """Adam update of W in place (m, v: moment buffers; step_dev: device int64
    step count, advanced by the call)."""
    check(lib().hrkan_adam(ctypes.byref(nd), _ptr_array(W), _ptr_array(gW), _ptr_array(m), _ptr_array(v),
                           _ptr(step_dev), float(lr), float(betas[0]), float(betas[1]), float(eps),
                           _stream(stream)))


def profile_enable(on: bool = True) -> None:
    check(lib().hrkan_profile_enable(int(bool(on))))


def profile_read() -> dict:
    """{kernel name: (launches, total ms)} since profiling was enabled."""
    buf = ctypes.create_string_buffer(1 << 16)
    check(lib().hrkan_profile_read(buf, len(buf)))
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.split()
        out[name] = (int(cnt), float(ms))
    return out


def read_status(ws: torch.Tensor, stream=None) -> int:
    f = ctypes.c_uint32(0)
    check(lib().hrkan_read_status(_ptr(ws), ws.numel(), _stream(stream), ctypes.byref(f)))
    return f.value


# ---------------------------------------------------------------------------
# a reusable training step over resident device buffers
# ---------------------------------------------------------------------------
class Step:
    """Device-resident problem + workspace; __call__ runs one hrkan_step."""

    def __init__(self, problem: _wl.Problem, dtype="f32", bf16_split: int = 2, device="cuda"):
        self.nd = net_desc(problem.net, dtype, bf16_split)
        self.pd = pde_desc(problem.pde)
        dt = array_dtype(self.nd)
        to = lambda a: torch.as_tensor(a, dtype=dt).to(device).contiguous()
        self.W = [to(w) for w in problem.W]
        self.x_int, self.x_bc, self.g_bc = to(problem.x_int), to(problem.x_bc), to(problem.g_bc)
        self.ws = alloc_workspace(workspace_bytes(self.nd, self.pd, problem.n_int, problem.n_bc), device)
        self.loss = torch.empty(3, dtype=torch.float64, device=device)
        self.gW = [torch.empty_like(w) for w in self.W]

    def __call__(self, stream=None):
        return step(self.nd, self.pd, self.W, self.x_int, self.x_bc, self.g_bc, self.ws,
                    self.loss, self.gW, stream)

    def capture(self) -> "torch.cuda.CUDAGraph":
        """Record one step into a HIP graph (same kernels, same buffers);
        replay() then re-runs the step with a single graph launch."""
        self()                                    # eager first run: one-time kernel setup
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self()
        torch.cuda.synchronize()
        return self.graph

    def replay(self):
        self.graph.replay()
        return self.loss, self.gW


class Trainer:
    """Step plus Adam on resident buffers: run(epochs) trains the network on
    its collocation points; each epoch is one hrkan_step and one hrkan_adam,
    replayed from one HIP graph when graph=True."""

    def __init__(self, problem: _wl.Problem, dtype="f32", lr: float = 1e-2, betas=(0.9, 0.999),
                 eps: float = 1e-8, bf16_split: int = 2, device="cuda"):
        self.step = Step(problem, dtype, bf16_split, device)
        self.m = [torch.zeros_like(w) for w in self.step.W]
        self.v = [torch.zeros_like(w) for w in self.step.W]
        self.t = torch.zeros(1, dtype=torch.int64, device=device)
        self.lr, self.betas, self.eps = lr, betas, eps
        self.graph = None

    def epoch(self):
        loss, gW = self.step()
        adam(self.step.nd, self.step.W, gW, self.m, self.v, self.t, self.lr, self.betas, self.eps)
        return loss

    def capture(self):
        """Record one epoch (step and update) into a HIP graph; the weights,
        moments and step count it updates live in device memory."""
        saved = [w.clone() for w in self.step.W] + [a.clone() for a in self.m + self.v] + [self.t.clone()]
        self.epoch()                              # eager first run: one-time kernel setup
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.epoch()
        torch.cuda.synchronize()
        # undo the warm-up epoch
        n = len(self.step.W)
        for dst, src in zip(self.step.W + self.m + self.v + [self.t], saved):
            dst.copy_(src)
        torch.cuda.synchronize()
        return self.graph

    def run(self, epochs: int, graph: bool = True, record_every: int = 0):
        """Train for `epochs` epochs; returns the loss history {epoch: [L, L_pde, L_bc]}
        sampled every record_every epochs (and at the last)."""
        if graph and self.graph is None:
            self.capture()
        hist = {}
        for e in range(epochs):
            if graph:
                self.graph.replay()
            else:
                self.epoch()
            if (record_every and e % record_every == 0) or e == epochs - 1:
                hist[e] = self.step.loss.cpu().tolist()
        return hist


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------
class HRKANJets(torch.autograd.Function):
    """jets = HRKANJets.apply(nd, mask, x, *W): output jets [C][n] of the
    network at x; backward calls the hand-written adjoint (hrkan_backward),
    which recomputes the basis from the saved inner jets."""

    @staticmethod
    def forward(ctx, nd, mask, x, *W):
        n = x.shape[0]
        saved = torch.empty(max(saved_bytes(nd, n, mask), 4), dtype=torch.uint8, device=x.device)
        pd = PdeDesc(0, 0.0, 0.05, 1.0)
        ws = alloc_workspace(workspace_bytes(nd, pd, n, 0), x.device)
        jets = forward_jets(nd, W, x, mask, ws, saved=saved)
        ctx.nd, ctx.mask, ctx.saved, ctx.ws = nd, mask, saved, ws
        ctx.save_for_backward(x, *W)
        return jets

    @staticmethod
    def backward(ctx, gjets):
        x, *W = ctx.saved_tensors
        gW = backward(ctx.nd, W, x, ctx.mask, gjets.contiguous(), ctx.saved, ctx.ws)
        return (None, None, None, *gW)


class HRKANResidual(torch.autograd.Function):
    """L, L_pde, L_bc = HRKANResidual.apply(pd, dtype, jets_int, u_bc, x_int, g_bc);
    only L is differentiable; its backward returns the seeds dL/djets."""

    @staticmethod
    def forward(ctx, pd, dtype, jets_int, u_bc, x_int, g_bc):
        nblk = max(1, math.ceil((x_int.shape[0] + u_bc.shape[0]) / 256))
        ws = alloc_workspace(512 + 16 * nblk, jets_int.device)
        seed_int = torch.empty_like(jets_int)
        seed_bc = torch.empty_like(u_bc)
        loss = residual(pd, dtype, jets_int, u_bc, x_int, g_bc, ws, seed_int=seed_int, seed_bc=seed_bc)
        ctx.save_for_backward(seed_int, seed_bc)
        L, Lp, Lb = loss[0], loss[1], loss[2]
        ctx.mark_non_differentiable(Lp, Lb)
        return L.clone(), Lp.clone(), Lb.clone()

    @staticmethod
    def backward(ctx, gL, _gp, _gb):
        seed_int, seed_bc = ctx.saved_tensors
        g = gL.to(seed_int.dtype)
        return None, None, seed_int * g, seed_bc * g, None, None


# ---------------------------------------------------------------------------
# batched plans: many independent instances of one network, one graph launch
# ---------------------------------------------------------------------------
def _points_array(xs_int, xs_bc, gs_bc):
    arr = (Points * len(xs_int))()
    for q, (xi, xb, g) in enumerate(zip(xs_int, xs_bc, gs_bc)):
        arr[q] = Points(xi.data_ptr() if xi.numel() else None, xi.shape[0],
                        xb.data_ptr() if xb.numel() else None, xb.shape[0],
                        g.data_ptr() if g.numel() else None)
    return arr


def plan_workspace_bytes(nd: NetDesc, n_int: Sequence[int], n_bc: Sequence[int]) -> int:
    arr = (Points * len(n_int))()
    for q, (a, b) in enumerate(zip(n_int, n_bc)):
        arr[q] = Points(None, int(a), None, int(b), None)
    b = ctypes.c_size_t(0)
    check(lib().hrkan_plan_workspace_bytes(ctypes.byref(nd), len(n_int), arr, ctypes.byref(b)))
    return b.value


class Plan:
    """A batched step over instances of one network shape (hrkan_plan_*).

    Holds device copies of every instance's points, the packed weights
    W_packed [n_inst, n_params] (updated in place by the caller between
    steps), and the outputs loss [n_inst, 3] (float64) and gW [n_inst,
    n_params]. execute() is one HIP graph launch."""

    def __init__(self, problems: Sequence[_wl.Problem], device="cuda", stream=None, dtype="f32",
                 bf16_split: int = 2):
        net = problems[0].net
        self.nd = net_desc(net, dtype, bf16_split)
        self.n_inst = len(problems)
        to = lambda a, shape=None: torch.as_tensor(a, dtype=torch.float32, device=device).contiguous()
        self.x_int = [to(p.x_int) for p in problems]
        self.x_bc = [to(p.x_bc) for p in problems]
        self.g_bc = [to(p.g_bc) for p in problems]
        self.W = torch.stack([torch.cat([to(w).reshape(-1) for w in p.W]) for p in problems]).contiguous()
        self.gW = torch.empty_like(self.W)
        self.loss = torch.empty(self.n_inst, 3, dtype=torch.float64, device=device)
        self.pts = _points_array(self.x_int, self.x_bc, self.g_bc)
        pdes = (PdeDesc * self.n_inst)(*[pde_desc(p.pde) for p in problems])
        nbytes = ctypes.c_size_t(0)
        check(lib().hrkan_plan_workspace_bytes(ctypes.byref(self.nd), self.n_inst, self.pts,
                                               ctypes.byref(nbytes)))
        self.ws = alloc_workspace(nbytes.value, device)
        h = ctypes.c_void_p(None)
        check(lib().hrkan_plan_create(ctypes.byref(h), ctypes.byref(self.nd), self.n_inst, pdes,
                                      _ptr(self.W), self.pts, _ptr(self.loss), _ptr(self.gW), _ptr(self.ws),
                                      self.ws.numel(), _stream(stream)))
        self._h = h

    def execute(self, stream=None) -> None:
        check(lib().hrkan_plan_execute(self._h, _stream(stream)))

    def config(self):
        tp, bl = ctypes.c_int32(0), ctypes.c_int32(0)
        check(lib().hrkan_plan_config(self._h, ctypes.byref(tp), ctypes.byref(bl)))
        return tp.value, bl.value

    def autotune_info(self):
        """(configuration read from the autotune cache, its step time in ms)."""
        fc, ms = ctypes.c_int32(0), ctypes.c_double(0.0)
        check(lib().hrkan_plan_autotune_info(self._h, ctypes.byref(fc), ctypes.byref(ms)))
        return bool(fc.value), ms.value

    def layer_grads(self, q: int, net: _wl.Net) -> List[torch.Tensor]:
        """Instance q's gradient, split into the per-layer [w_l * n_b, w_{l+1}] arrays."""
        out, o = [], 0
        for r, c in net.weight_shapes():
            out.append(self.gW[q, o:o + r * c].reshape(r, c))
            o += r * c
        return out

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            lib().hrkan_plan_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
