"""Caller-owned workspace (qpgf_plan_workspace_bytes / qpgf_plan_set_workspace): a plan whose grids,
far slab and target scratch live in a torch buffer gives the same values as a plan that allocates
its own, allocates nothing while instances and calls stay within the sizes the workspace was made
for, refuses larger ones with QPGF_E_SIZE, and returns to its own arrays on request."""

import numpy as np
import pytest
import torch

from paper_1801_05977_amd import qpgf, workloads

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _pair(kind, prec, m, **kw):
    return qpgf.Plan(kind, prec, *m, **kw), qpgf.Plan(kind, prec, *m, **kw)


def _call(P, kind, k, a, x):
    if kind in (qpgf.KIND_G2D, qpgf.KIND_G2D_GRAD):
        return P(k, a[0], x=x)
    if kind == qpgf.KIND_G2D_HESS_DIFF:
        return P.hess_diff(k, k + 1.3, a[0], x)
    return P(k, a[0], a[1], x)


@pytest.mark.parametrize("kind,prec,m,dim,T,kw", [
    (qpgf.KIND_GD3D, qpgf.C128, (64, 64, 32), 3, 100_000, {}),       # binned gather: the scratch is used
    (qpgf.KIND_GD3D, qpgf.C64, (64, 64, 32), 3, 100_000, {}),
    (qpgf.KIND_MAXWELL3D, qpgf.C64, (32, 32, 16), 3, 80_000, {}),
    (qpgf.KIND_G2D_GRAD, qpgf.C128, (256, 64), 2, 50_000, {}),        # interleaved grid copy
    (qpgf.KIND_G2D, qpgf.C64, (256, 64), 2, 50_000, {}),              # node quads
    (qpgf.KIND_G2D, qpgf.C128, (256, 64), 2, 50_000, {"ring_interp": 1}),   # ring mask scratch
    (qpgf.KIND_G2D_HESS_DIFF, qpgf.C64, (256, 64), 2, 30_000, {}),
])
def test_workspace_plan_equals_own_plan(kind, prec, m, dim, T, kw):
    own, ws = _pair(kind, prec, m, **kw)
    kmax = 6.0
    buf = ws.use_workspace(kmax, T)
    assert buf.numel() == ws.workspace_bytes(kmax, T) and buf.data_ptr() % 256 == 0
    x = dev(workloads.targets(T, dim, seed=7))
    a = (0.21, -0.33)
    for k in (2.3, 4.6):   # the second-derivative differences also take k + 1.3 <= kmax
        g0 = _call(own, kind, k, a, x).cpu().numpy()
        g1 = _call(ws, kind, k, a, x).cpu().numpy()
        assert np.array_equal(g0, g1, equal_nan=True), k


def test_workspace_bounds_and_no_growth():
    kind, prec, m = qpgf.KIND_GD3D, qpgf.C128, (64, 64, 32)
    P = qpgf.Plan(kind, prec, *m)
    Tmax, kmax = 120_000, 5.0
    P.use_workspace(kmax, Tmax)
    x = dev(workloads.targets(Tmax, 3, seed=8))
    out = P.out_tensor(Tmax)
    P(1.1, 0.2, 0.1, x[:70_000], out[:70_000])                 # load the kernels once
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for k, T in ((4.99, Tmax), (3.0, 90_000), (5.0, Tmax)):     # larger slab and more targets than before
        P(k, 0.2, 0.1, x[:T], out[:T])
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    xs = dev(workloads.targets(Tmax + 1, 3, seed=9))
    with pytest.raises(qpgf.QpgfError) as e1:
        P(2.0, 0.2, 0.1, xs)
    with pytest.raises(qpgf.QpgfError) as e2:
        P(5.5, 0.2, 0.1, x[:1000])
    assert e1.value.status == 4 and e2.value.status == 4
    assert "workspace" in str(e1.value) and "workspace" in str(e2.value)
    # back to the plan's own arrays: larger instances and target counts work again
    P.use_workspace(None, None)
    g = P(5.5, 0.2, 0.1, xs).cpu().numpy()
    ref = qpgf.Plan(kind, prec, *m)(5.5, 0.2, 0.1, xs).cpu().numpy()
    assert np.array_equal(g, ref, equal_nan=True)


def test_workspace_argument_checks():
    P = qpgf.Plan(qpgf.KIND_GD3D, qpgf.C64, 32, 32, 16)
    L = qpgf.lib()
    n = P.workspace_bytes(3.0, 1000)
    buf = torch.empty(n + 512, dtype=torch.uint8, device="cuda")
    base = buf.data_ptr() + (-buf.data_ptr()) % 256
    import ctypes
    assert L.qpgf_plan_set_workspace(P._h, ctypes.c_void_p(base), n - 1, 3.0, 1000) == 4
    assert L.qpgf_plan_set_workspace(P._h, ctypes.c_void_p(base + 8), n, 3.0, 1000) == 1
    assert L.qpgf_plan_set_workspace(P._h, ctypes.c_void_p(base), n, float("inf"), 1000) == 1
    assert L.qpgf_plan_set_workspace(P._h, ctypes.c_void_p(base), n, 3.0, -1) == 1
    assert L.qpgf_plan_set_workspace(P._h, None, 5, 3.0, 1000) == 1
    # more modes or targets never need fewer bytes
    assert P.workspace_bytes(8.0, 1000) >= n and P.workspace_bytes(3.0, 10**6) > n
    assert L.qpgf_plan_set_workspace(P._h, ctypes.c_void_p(base), n, 3.0, 1000) == 0
    # the grids are gone until the next prepare
    with pytest.raises(qpgf.QpgfError):
        P.evaluate(dev(workloads.targets(10, 3, seed=1)))
    g = P(2.0, 0.1, 0.2, dev(workloads.targets(1000, 3, seed=2))).cpu().numpy()
    assert np.isfinite(g).all()
    del buf
