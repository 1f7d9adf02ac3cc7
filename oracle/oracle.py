"""ctypes wrapper of the FP64 CPU oracle (hrkan_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark. It shares nothing with the GPU library and
is never a fallback for it.

Jet arrays are [S][width][n] float64 with S = 1 + 2n slots for jet order n
(net.order, 2 unless the net says otherwise): the value, d^k/dx0^k for
k = 1..n, then d^k/dx1^k; for n = 2 that is (value, d/dx0, d2/dx0^2, d/dx1,
d2/dx1^2). The output jets of the network are [S][n]. Weights of layer l are
[w_l * n_b, w_{l+1}] float64, row i*n_b + b.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hrkan_oracle.c")
_LIB = os.path.join(_HERE, "libhrkan_oracle.so")

MAX_LAYERS = 8
MAX_ORDER = 5
SLOTS = 5            # slots of the default jet order 2
POISSON2D = 0
BURGERS1D = 1
LINEAR2D = 2


def order_of(net) -> int:
    return int(getattr(net, "order", 2))


def slots(order: int) -> int:
    return 1 + 2 * int(order)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (strict IEEE double, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "hrkan_oracle.h"))
    ):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared",
             "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Net(ctypes.Structure):
    _fields_ = [
        ("n_layers", ctypes.c_int32),
        ("widths", ctypes.c_int32 * (MAX_LAYERS + 1)),
        ("G", ctypes.c_int32),
        ("k", ctypes.c_int32),
        ("m", ctypes.c_int32),
        ("lo", ctypes.c_double),
        ("hi", ctypes.c_double),
        ("order", ctypes.c_int32),
    ]


class _Pde(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("nu", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("adv", ctypes.c_double),
        ("c0", ctypes.c_double),
        ("cx", ctypes.c_double * MAX_ORDER),
        ("cy", ctypes.c_double * MAX_ORDER),
    ]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        i64 = ctypes.c_int64
        lib.hro_n_basis.argtypes = [P(_Net)]
        lib.hro_supports.argtypes = [P(_Net), _D, _D]
        lib.hro_basis.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int, _D]
        lib.hro_layer_forward.argtypes = [P(_Net), ctypes.c_int, _D, _D, i64, _D]
        lib.hro_layer_backward.argtypes = [P(_Net), ctypes.c_int, _D, _D, _D, i64, _D, _D]
        lib.hro_input_jets.argtypes = [_D, i64, ctypes.c_int, _D]
        lib.hro_forward.argtypes = [P(_Net), P(_D), _D, i64, _D, _D]
        lib.hro_residual.argtypes = [P(_Pde), ctypes.c_int, _D, _D, i64, _D, _D, i64, _D, _D, _D, _D]
        lib.hro_backward.argtypes = [P(_Net), P(_D), _D, i64, _D, P(_D)]
        lib.hro_step.argtypes = [P(_Net), P(_Pde), P(_D), _D, i64, _D, i64, _D, _D,
                                 P(_D), _D, _D, _D]
        lib.hro_num_threads.restype = ctypes.c_int
        lib.hro_set_rounding.argtypes = [ctypes.c_int, ctypes.c_int]
        lib.hro_set_rounding.restype = None
        lib.hro_model_round.argtypes = [ctypes.c_int, ctypes.c_double]
        lib.hro_model_round.restype = ctypes.c_double
        lib.hro_model_acc.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
        lib.hro_model_acc.restype = ctypes.c_double
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _net(net) -> _Net:
    n = _Net()
    w = list(net.widths)
    n.n_layers = len(w) - 1
    for i, v in enumerate(w):
        n.widths[i] = int(v)
    n.G, n.k, n.m = int(net.G), int(net.k), int(net.m)
    n.lo, n.hi = float(getattr(net, "lo", -1.0)), float(getattr(net, "hi", 1.0))
    n.order = order_of(net)
    return n


def _pde(pde) -> _Pde:
    p = _Pde()
    p.kind = int(pde.kind)
    p.nu = float(pde.nu)
    p.alpha = float(pde.alpha)
    p.adv = float(getattr(pde, "adv", 1.0))
    p.c0 = float(getattr(pde, "c0", 0.0))
    for k, v in enumerate(getattr(pde, "cx", ())):
        p.cx[k] = float(v)
    for k, v in enumerate(getattr(pde, "cy", ())):
        p.cy[k] = float(v)
    return p


def _wlist(Ws):
    Ws = [_f64(w) for w in Ws]
    arr = (_D * len(Ws))(*[_ptr(w) for w in Ws])
    return Ws, arr


class rounding:
    """Context manager enabling the oracle's rounding model (see
    hro_set_rounding): "f32", or "bf16" with `split` pieces per feature."""

    def __init__(self, mode: str, split: int = 1):
        self.mode = {"exact": 0, "f32": 1, "bf16": 2}[mode]
        self.split = split

    def __enter__(self):
        _load().hro_set_rounding(self.mode, self.split)
        return self

    def __exit__(self, *a):
        _load().hro_set_rounding(0, 1)


MODEL_FEATURE, MODEL_STORE, MODEL_BAR_SPLIT, MODEL_BAR_HI = 0, 1, 2, 3


def model_round(what: int, v: float) -> float:
    """One rounding of the current rounding model (see hro_model_round)."""
    return _load().hro_model_round(int(what), float(v))


def model_acc(acc: float, w: float, a: float) -> float:
    """One accumulation step acc + w * a of the current rounding model."""
    return _load().hro_model_acc(float(acc), float(w), float(a))


def num_threads() -> int:
    return _load().hro_num_threads()


def n_basis(net) -> int:
    return int(net.G) + int(net.k)


def supports(net):
    nb = n_basis(net)
    s = np.zeros(nb)
    e = np.zeros(nb)
    n = _net(net)
    _load().hro_supports(ctypes.byref(n), _ptr(s), _ptr(e))
    return s, e


def basis(m: int, s: float, e: float, z: float, nmax: int = 3) -> np.ndarray:
    out = np.zeros(nmax + 1)
    _load().hro_basis(int(m), float(s), float(e), float(z), int(nmax), _ptr(out))
    return out


def input_jets(x, order: int = 2) -> np.ndarray:
    x = _f64(x)
    n = x.shape[0]
    z = np.zeros((slots(order), 2, n))
    assert _load().hro_input_jets(_ptr(x), n, int(order), _ptr(z)) == 0
    return z


def layer_forward(net, layer: int, W, zin) -> np.ndarray:
    zin = _f64(zin)
    n = zin.shape[-1]
    wout = list(net.widths)[layer + 1]
    zout = np.zeros((slots(order_of(net)), wout, n))
    nn = _net(net)
    W = _f64(W)
    rc = _load().hro_layer_forward(ctypes.byref(nn), layer, _ptr(W), _ptr(zin), n, _ptr(zout))
    assert rc == 0
    return zout


def layer_backward(net, layer: int, W, zin, ybar, want_zbar: bool = True):
    zin = _f64(zin)
    ybar = _f64(ybar)
    n = zin.shape[-1]
    W = _f64(W)
    gW = np.zeros_like(W)
    zbar = np.zeros_like(zin) if want_zbar else None
    nn = _net(net)
    rc = _load().hro_layer_backward(ctypes.byref(nn), layer, _ptr(W), _ptr(zin), _ptr(ybar),
                                    n, _ptr(zbar), _ptr(gW))
    assert rc == 0
    return zbar, gW


def forward(net, Ws, x, all_jets: bool = False):
    """Output jets [S][n]; with all_jets, also the list of per-layer input jets."""
    x = _f64(x)
    n = x.shape[0]
    Ws, arr = _wlist(Ws)
    S = slots(order_of(net))
    u = np.zeros((S, n))
    widths = list(net.widths)
    blocks = None
    if all_jets:
        tot = sum(S * w * n for w in widths)
        blocks = np.zeros(tot)
    nn = _net(net)
    rc = _load().hro_forward(ctypes.byref(nn), arr, _ptr(x), n, _ptr(u), _ptr(blocks))
    assert rc == 0
    if not all_jets:
        return u
    out, o = [], 0
    for w in widths:
        out.append(blocks[o:o + S * w * n].reshape(S, w, n))
        o += S * w * n
    return u, out


def residual(pde, x_int, jets_int, u_bc, g_bc, order: int = 2):
    """(r [n_int], loss [3], seed_int [S][n_int], seed_bc [n_bc]) for output
    jets [S][n_int] of jet order `order`."""
    x_int = _f64(x_int)
    jets_int = _f64(jets_int)
    u_bc = _f64(u_bc)
    g_bc = _f64(g_bc)
    ni, nbc = x_int.shape[0], u_bc.shape[0]
    assert jets_int.shape[0] == slots(order)
    r = np.zeros(ni)
    loss = np.zeros(3)
    si = np.zeros((slots(order), ni))
    sb = np.zeros(nbc)
    p = _pde(pde)
    rc = _load().hro_residual(ctypes.byref(p), int(order), _ptr(x_int), _ptr(jets_int), ni, _ptr(u_bc),
                              _ptr(g_bc), nbc, _ptr(r), _ptr(loss), _ptr(si), _ptr(sb))
    assert rc == 0
    return r, loss, si, sb


def backward(net, Ws, x, seed):
    x = _f64(x)
    seed = _f64(seed)
    n = x.shape[0]
    Ws, arr = _wlist(Ws)
    gWs = [np.zeros_like(w) for w in Ws]
    garr = (_D * len(gWs))(*[_ptr(g) for g in gWs])
    nn = _net(net)
    rc = _load().hro_backward(ctypes.byref(nn), arr, _ptr(x), n, _ptr(seed), garr)
    assert rc == 0
    return gWs


def step(net, pde, Ws, x_int, x_bc, g_bc):
    """One full step: dict with loss [3], gW list, r, jets [S][n_int], u_bc."""
    x_int = _f64(x_int)
    x_bc = _f64(x_bc)
    g_bc = _f64(g_bc)
    ni, nbc = x_int.shape[0], x_bc.shape[0]
    Ws, arr = _wlist(Ws)
    gWs = [np.zeros_like(w) for w in Ws]
    garr = (_D * len(gWs))(*[_ptr(g) for g in gWs])
    loss = np.zeros(3)
    r = np.zeros(ni)
    jets = np.zeros((slots(order_of(net)), ni))
    ubc = np.zeros(nbc)
    nn = _net(net)
    p = _pde(pde)
    rc = _load().hro_step(ctypes.byref(nn), ctypes.byref(p), arr, _ptr(x_int), ni, _ptr(x_bc),
                          nbc, _ptr(g_bc), _ptr(loss), garr, _ptr(r), _ptr(jets), _ptr(ubc))
    assert rc == 0
    return {"loss": loss, "gW": gWs, "r": r, "jets": jets, "u_bc": ubc}


def adam(Ws, gWs, ms, vs, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """The Adam optimiser the paper trains with (Sec. 4.1, 4.2), in the
    update of Kingma and Ba: step t (1, 2, ...) with gradients gWs; returns
    new (Ws, ms, vs) as float64 arrays, one element at a time in plain
    numpy arithmetic."""
    out_w, out_m, out_v = [], [], []
    for w, g, m, v in zip(Ws, gWs, ms, vs):
        w, g, m, v = (np.asarray(a, dtype=np.float64) for a in (w, g, m, v))
        m = beta1 * m + (1.0 - beta1) * g
        v = beta2 * v + (1.0 - beta2) * g * g
        mhat = m / (1.0 - beta1 ** t)
        vhat = v / (1.0 - beta2 ** t)
        out_w.append(w - lr * mhat / (np.sqrt(vhat) + eps))
        out_m.append(m)
        out_v.append(v)
    return out_w, out_m, out_v
