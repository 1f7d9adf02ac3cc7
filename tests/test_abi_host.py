"""Host-side checks of the C ABI: the library loads, exports every function
declared in include/hrkan.h, and rejects invalid arguments with the
documented status codes before touching the device. No kernel runs here."""
import ctypes
import os
import re

import pytest

from paper_2409_14248_amd import hrkan as H
from paper_2409_14248_amd import workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hrkan.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hrkan_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    L = H.lib()
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(H.EXPORTS)
    assert L.hrkan_version() == 200


def test_status_strings():
    L = H.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.hrkan_status_string(code).decode() != "unknown status"


def nd_of(widths=(2, 8, 1), G=5, dtype="f32", **kw):
    return H.net_desc(WL.Net(tuple(widths), G=G, **kw), dtype)


def ws_bytes(nd, pd=None, n_int=100, n_bc=10):
    return H.workspace_bytes(nd, pd or H.pde_desc(WL.Pde(WL.POISSON2D)), n_int, n_bc)


def test_defaults():
    L = H.lib()
    nd = H.NetDesc()
    assert L.hrkan_net_init(ctypes.byref(nd)) == 0
    assert (nd.G, nd.k, nd.m, nd.lo, nd.hi) == (5, 3, 4, -1.0, 1.0)
    pd = H.PdeDesc()
    assert L.hrkan_pde_init(ctypes.byref(pd), H.BURGERS1D) == 0
    assert abs(pd.nu - 0.01 / 3.141592653589793) < 1e-18 and pd.alpha == 0.05 and pd.adv == 1.0


@pytest.mark.parametrize("mask,C", [(H.MASK_VALUE, 1), (H.MASK_BURGERS, 4), (H.MASK_POISSON, 5),
                                    (H.CH_U | H.CH_X | H.CH_Y, 3), (H.CH_U | H.CH_X | H.CH_XX, 3),
                                    (H.CH_U | H.CH_X, 2), (H.CH_U | H.CH_Y | H.CH_YY, 3),
                                    (H.CH_U | H.CH_X | H.CH_XX | H.CH_X3 | H.CH_X4 | H.CH_Y, 6),
                                    (H.CH_U | H.CH_X | H.CH_XX | H.CH_X3 | H.CH_X4 | H.CH_X5
                                     | H.CH_Y | H.CH_YY | H.CH_Y3 | H.CH_Y4 | H.CH_Y5, 11)])
def test_mask_channels(mask, C):
    assert H.mask_channels(mask) == C


@pytest.mark.parametrize("mask,code", [(H.CH_X, H.ERR_INVALID_ARG), (H.CH_X4 | H.CH_U, H.ERR_INVALID_ARG),
                                       (H.CH_U | H.CH_XX, H.ERR_INVALID_ARG),
                                       (H.CH_U | H.CH_Y | H.CH_Y3, H.ERR_INVALID_ARG),
                                       (H.CH_U | (1 << 11), H.ERR_INVALID_ARG)])
def test_bad_masks(mask, code):
    """U is required, the derivatives of a coordinate must be those of
    order 1..o, and only the defined bits may be set."""
    assert H.lib().hrkan_mask_channels(mask) == code


@pytest.mark.parametrize("ox,oy", [(0, 0), (2, 2), (2, 1), (4, 4), (5, 1), (0, 3), (5, 5)])
def test_mask_of_orders(ox, oy):
    m = H.mask_of_orders(ox, oy)
    assert H.mask_channels(m) == 1 + ox + oy
    assert H.lib().hrkan_mask_of_orders(6, 0) == 0
    assert H.lib().hrkan_mask_of_orders(0, -1) == 0
    if (ox, oy) == (2, 2):
        assert m == H.MASK_POISSON
    if (ox, oy) == (2, 1):
        assert m == H.MASK_BURGERS


def test_linear_pde_masks_and_bf16_refusal():
    """The linear kind's mask follows its highest non-zero coefficients; the
    BF16 kernels take at most second derivatives, so a BF16 network with a
    fourth-order PDE is refused, while FP32 and FP64 are accepted."""
    pde = WL.Pde(WL.LINEAR2D, cx=(0, 0, 0, 1), cy=(0, 0, 0, 1))
    assert H.pde_mask(pde) == H.mask_of_orders(4, 4)
    assert H.pde_mask(WL.Pde(WL.LINEAR2D, c0=1.0, cx=(1,), cy=(0, 0, 0, 0, 2))) == H.mask_of_orders(1, 5)
    pd = H.pde_desc(pde)
    b = ctypes.c_size_t(0)
    for dt, code in [(H.F64, H.OK), (H.F32, H.OK), (H.BF16, H.ERR_UNSUPPORTED)]:
        nd = nd_of((2, 32, 32, 1), G=10)
        nd.dtype, nd.bf16_split = dt, 2
        assert H.lib().hrkan_workspace_bytes(ctypes.byref(nd), ctypes.byref(pd), 100, 16, ctypes.byref(b)) == code
    # a linear PDE with second derivatives runs on BF16 like Poisson
    nd = nd_of((2, 32, 32, 1), G=10)
    nd.dtype, nd.bf16_split = H.BF16, 2
    pd2 = H.pde_desc(WL.Pde(WL.LINEAR2D, cx=(0, 1), cy=(0, 1)))
    assert H.lib().hrkan_workspace_bytes(ctypes.byref(nd), ctypes.byref(pd2), 100, 16, ctypes.byref(b)) == H.OK
    # non-finite coefficients are refused
    pd.cx[2] = float("inf")
    assert H.lib().hrkan_workspace_bytes(ctypes.byref(nd), ctypes.byref(pd), 100, 16, ctypes.byref(b)) == \
        H.ERR_INVALID_ARG


def test_workspace_grows_with_jet_order():
    """Interior regions are sized for max(5, C) channels."""
    nd = nd_of((2, 32, 32, 1), G=10)
    nd.dtype = H.F64
    b2, b5 = ctypes.c_size_t(0), ctypes.c_size_t(0)
    p2 = H.pde_desc(WL.Pde(WL.POISSON2D))
    p5 = H.pde_desc(WL.Pde(WL.LINEAR2D, cx=(0, 0, 0, 0, 1), cy=(0, 0, 0, 0, 1)))
    assert H.lib().hrkan_workspace_bytes(ctypes.byref(nd), ctypes.byref(p2), 4096, 256, ctypes.byref(b2)) == H.OK
    assert H.lib().hrkan_workspace_bytes(ctypes.byref(nd), ctypes.byref(p5), 4096, 256, ctypes.byref(b5)) == H.OK
    assert b5.value > b2.value


@pytest.mark.parametrize("mutate,code", [
    (lambda d: setattr(d, "n_layers", 0), H.ERR_INVALID_ARG),
    (lambda d: setattr(d, "n_layers", 9), H.ERR_INVALID_ARG),
    (lambda d: d.widths.__setitem__(0, 3), H.ERR_INVALID_ARG),
    (lambda d: d.widths.__setitem__(2, 2), H.ERR_INVALID_ARG),
    (lambda d: d.widths.__setitem__(1, 0), H.ERR_INVALID_ARG),
    (lambda d: setattr(d, "G", 0), H.ERR_INVALID_ARG),
    (lambda d: setattr(d, "m", 1), H.ERR_UNSUPPORTED),
    (lambda d: setattr(d, "k", 4), H.ERR_UNSUPPORTED),
    (lambda d: setattr(d, "hi", -2.0), H.ERR_INVALID_ARG),
    (lambda d: setattr(d, "lo", float("nan")), H.ERR_INVALID_ARG),
    (lambda d: setattr(d, "dtype", 7), H.ERR_INVALID_ARG),
    (lambda d: (setattr(d, "dtype", H.BF16), setattr(d, "bf16_split", 4)), H.ERR_INVALID_ARG),
    (lambda d: setattr(d, "G", 40), H.ERR_UNSUPPORTED),
    # BF16 runs only on the matrix-core kernels: k = 3, m = 4, hidden widths 32/64/128
    (lambda d: (setattr(d, "dtype", H.BF16), setattr(d, "bf16_split", 1)), H.ERR_UNSUPPORTED),
    (lambda d: (setattr(d, "dtype", H.BF16), d.widths.__setitem__(1, 32), setattr(d, "m", 2)),
     H.ERR_UNSUPPORTED),
])
def test_invalid_net_rejected(mutate, code):
    nd = nd_of()
    mutate(nd)
    b = ctypes.c_size_t(0)
    pd = H.pde_desc(WL.Pde(WL.POISSON2D))
    rc = H.lib().hrkan_workspace_bytes(ctypes.byref(nd), ctypes.byref(pd), 10, 10, ctypes.byref(b))
    assert rc == code, H.lib().hrkan_last_error()
    assert H.lib().hrkan_last_error().decode() != ""


def test_bf16_net_of_supported_shape_accepted():
    nd = nd_of((2, 32, 32, 1), G=10)
    nd.dtype, nd.bf16_split = H.BF16, 3
    b = ctypes.c_size_t(0)
    pd = H.pde_desc(WL.Pde(WL.BURGERS1D))
    assert H.lib().hrkan_workspace_bytes(ctypes.byref(nd), ctypes.byref(pd), 10, 10, ctypes.byref(b)) == H.OK
    assert b.value > 0


def test_workspace_grows_with_points_and_saved_bytes():
    nd = nd_of((2, 32, 32, 1), G=10)
    a = ws_bytes(nd, n_int=1000, n_bc=100)
    b = ws_bytes(nd, n_int=100000, n_bc=100)
    assert b > a > 0
    # saved jets: C * (32 + 32) * n floats for layers 1..2
    assert H.saved_bytes(nd, 1000, H.MASK_BURGERS) == 4 * 4 * 64 * 1000
    assert H.saved_bytes(H.net_desc(WL.Net((2, 8, 1), G=5), "f64"), 10, H.MASK_POISSON) == 8 * 5 * 8 * 10


class FakeDev:
    """Host pointers with plausible alignment: validation never dereferences."""

    def __init__(self, nbytes, offset=0):
        self.buf = ctypes.create_string_buffer(nbytes + 512)
        base = ctypes.addressof(self.buf)
        self.addr = (base + 255) // 256 * 256 + offset

    @property
    def p(self):
        return ctypes.c_void_p(self.addr)


def _fwd(nd, W, x, n, mask, out, saved, ws, wsb):
    return H.lib().hrkan_forward_jets(ctypes.byref(nd), W, x, n, mask, out, saved, ws, wsb, None)


def test_forward_argument_errors():
    nd = nd_of()
    need = ws_bytes(nd, n_int=64, n_bc=0)
    ws = FakeDev(need)
    w0, w1 = FakeDev(26 * 8 * 8), FakeDev(8 * 8 * 8)
    W = (ctypes.c_void_p * 2)(w0.addr, w1.addr)
    x, out = FakeDev(64 * 8), FakeDev(64 * 8 * 5)
    # NULL weights array / entry
    assert _fwd(nd, None, x.p, 64, H.MASK_POISSON, out.p, None, ws.p, need) == H.ERR_INVALID_ARG
    Wn = (ctypes.c_void_p * 2)(w0.addr, 0)
    assert _fwd(nd, Wn, x.p, 64, H.MASK_POISSON, out.p, None, ws.p, need) == H.ERR_INVALID_ARG
    # misaligned weight
    Wm = (ctypes.c_void_p * 2)(w0.addr + 2, w1.addr)
    assert _fwd(nd, Wm, x.p, 64, H.MASK_POISSON, out.p, None, ws.p, need) == H.ERR_INVALID_ARG
    # negative n, NULL x
    assert _fwd(nd, W, x.p, -1, H.MASK_POISSON, out.p, None, ws.p, need) == H.ERR_INVALID_ARG
    assert _fwd(nd, W, None, 64, H.MASK_POISSON, out.p, None, ws.p, need) == H.ERR_INVALID_ARG
    # workspace: NULL, misaligned, too small
    assert _fwd(nd, W, x.p, 64, H.MASK_POISSON, out.p, None, None, need) == H.ERR_INVALID_ARG
    ws_off = FakeDev(need, offset=64)
    assert _fwd(nd, W, x.p, 64, H.MASK_POISSON, out.p, None, ws_off.p, need) == H.ERR_INVALID_ARG
    assert _fwd(nd, W, x.p, 64, H.MASK_POISSON, out.p, None, ws.p, 100) == H.ERR_WORKSPACE
    # a mask with a gap in its derivative orders
    assert _fwd(nd, W, x.p, 64, H.CH_U | H.CH_YY, out.p, None, ws.p, need) == H.ERR_INVALID_ARG
    # a mask of more channels than the workspace was sized for (Poisson: 5)
    m44 = H.mask_of_orders(4, 4)
    assert _fwd(nd, W, x.p, 64, m44, out.p, None, ws.p, need) == H.ERR_WORKSPACE
    # n = 0 is a valid empty call that enqueues nothing
    assert _fwd(nd, W, x.p, 0, H.MASK_POISSON, out.p, None, ws.p, need) == H.OK


def test_step_and_residual_argument_errors():
    L = H.lib()
    nd = nd_of()
    pd = H.pde_desc(WL.Pde(WL.POISSON2D))
    need = ws_bytes(nd, pd, 64, 8)
    ws = FakeDev(need)
    w0, w1 = FakeDev(26 * 8 * 8), FakeDev(8 * 8 * 8)
    W = (ctypes.c_void_p * 2)(w0.addr, w1.addr)
    G = (ctypes.c_void_p * 2)(FakeDev(26 * 8 * 8).addr, FakeDev(64 * 8).addr)
    loss = FakeDev(24)
    xi, xb, g = FakeDev(64 * 8), FakeDev(8 * 8), FakeDev(8 * 4)
    pts = H.Points(xi.addr, 64, xb.addr, 8, g.addr)
    st = lambda nd_, pd_, pts_, loss_, wsb: L.hrkan_step(ctypes.byref(nd_), pd_, W, pts_, loss_, G, ws.p, wsb, None)
    assert st(nd, None, ctypes.byref(pts), loss.p, need) == H.ERR_INVALID_ARG
    bad = H.PdeDesc(5, 0.0, 0.05, 1.0)
    assert st(nd, ctypes.byref(bad), ctypes.byref(pts), loss.p, need) == H.ERR_INVALID_ARG
    nanp = H.PdeDesc(1, float("nan"), 0.05, 1.0)
    assert st(nd, ctypes.byref(nanp), ctypes.byref(pts), loss.p, need) == H.ERR_INVALID_ARG
    assert st(nd, ctypes.byref(pd), None, loss.p, need) == H.ERR_INVALID_ARG
    assert st(nd, ctypes.byref(pd), ctypes.byref(pts), None, need) == H.ERR_INVALID_ARG
    assert st(nd, ctypes.byref(pd), ctypes.byref(pts), loss.p, need - 256) == H.ERR_WORKSPACE
    neg = H.Points(xi.addr, -3, xb.addr, 8, g.addr)
    assert st(nd, ctypes.byref(pd), ctypes.byref(neg), loss.p, need) == H.ERR_INVALID_ARG
    nox = H.Points(None, 64, xb.addr, 8, g.addr)
    assert st(nd, ctypes.byref(pd), ctypes.byref(nox), loss.p, need) == H.ERR_INVALID_ARG
    # residual: bad dtype, NULL loss
    jets = FakeDev(64 * 8 * 5)
    r = lambda dt, loss_: L.hrkan_residual(ctypes.byref(pd), dt, jets.p, FakeDev(64).p, ctypes.byref(pts),
                                           None, loss_, None, None, ws.p, need, None)
    assert r(H.BF16, loss.p) == H.ERR_INVALID_ARG
    assert r(H.F32, None) == H.ERR_INVALID_ARG


def test_backward_argument_errors():
    L = H.lib()
    nd = nd_of((2, 4, 3, 1))
    need = ws_bytes(nd, n_int=64, n_bc=0)
    ws = FakeDev(need)
    W = (ctypes.c_void_p * 3)(*[FakeDev(4096).addr for _ in range(3)])
    G = (ctypes.c_void_p * 3)(*[FakeDev(4096).addr for _ in range(3)])
    x, seed = FakeDev(64 * 8), FakeDev(64 * 20)
    bw = lambda saved, gw: L.hrkan_backward(ctypes.byref(nd), W, x.p, 64, H.MASK_BURGERS, seed.p, saved,
                                            gw, 0, ws.p, need, None)
    assert bw(None, G) == H.ERR_INVALID_ARG          # saved required for L > 1
    assert bw(FakeDev(64).p, None) == H.ERR_INVALID_ARG


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(H, "_lib", None)
    monkeypatch.setattr(H, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        H.lib()


def test_plan_workspace_validation():
    nd = nd_of((2, 32, 32, 1), G=10)
    assert H.plan_workspace_bytes(nd, [5000, 300], [300, 20]) > 0
    # workspace grows with the points
    assert H.plan_workspace_bytes(nd, [50000, 300], [3000, 20]) > H.plan_workspace_bytes(nd, [5000, 300], [300, 20])
    with pytest.raises(H.HrkanError) as e:
        H.plan_workspace_bytes(nd, [], [])
    assert e.value.code == H.ERR_INVALID_ARG
    with pytest.raises(H.HrkanError) as e:
        H.plan_workspace_bytes(nd, [-1], [4])
    assert e.value.code == H.ERR_INVALID_ARG
    for bad in (nd_of((2, 32, 32, 1), G=10, dtype="f64"), nd_of((2, 8, 1), G=5)):
        with pytest.raises(H.HrkanError) as e:
            H.plan_workspace_bytes(bad, [100], [10])
        assert e.value.code == H.ERR_UNSUPPORTED


def test_plan_calls_reject_null_plan():
    L = H.lib()
    assert L.hrkan_plan_execute(None, None) == H.ERR_PLAN_MISMATCH
    assert L.hrkan_plan_config(None, None, None) == H.ERR_PLAN_MISMATCH
    assert L.hrkan_plan_autotune_info(None, None, None) == H.ERR_PLAN_MISMATCH
    L.hrkan_plan_destroy(None)


def test_adam_argument_errors():
    """hrkan_adam validates its pointers and hyper-parameters on the host."""
    net = WL.Net((2, 32, 32, 1), G=10)
    nd = H.net_desc(net, "f32")
    L = len(net.weight_shapes())
    fake = (ctypes.c_void_p * L)(*([0x10000] * L))      # aligned, never dereferenced
    null = (ctypes.c_void_p * L)(*([0] * L))
    t = ctypes.c_void_p(0x10000)

    def call(W=fake, g=fake, m=fake, v=fake, tdev=t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        return H.lib().hrkan_adam(ctypes.byref(nd), W, g, m, v, tdev, lr, b1, b2, eps, None)

    assert call(W=null) == H.ERR_INVALID_ARG
    assert call(v=null) == H.ERR_INVALID_ARG
    assert call(tdev=ctypes.c_void_p(0)) == H.ERR_INVALID_ARG
    assert call(tdev=ctypes.c_void_p(0x10004)) == H.ERR_INVALID_ARG     # misaligned counter
    assert call(lr=-1.0) == H.ERR_INVALID_ARG
    assert call(lr=float("nan")) == H.ERR_INVALID_ARG
    assert call(b1=1.0) == H.ERR_INVALID_ARG
    assert call(b2=-0.1) == H.ERR_INVALID_ARG
    assert call(eps=0.0) == H.ERR_INVALID_ARG
