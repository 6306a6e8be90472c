"""qpgf_evaluate_noalloc (target scratch in the library's fixed device array) against qpgf_evaluate
(scratch the plan allocates) through the C ABI: the same values and flags, bit for bit, on two calls
in a row, the second with fewer targets; oversized calls are refused before any launch."""

import ctypes

import numpy as np
import pytest
import torch

from paper_1801_05977_amd import qpgf, workloads

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def _both(P, x):
    L = qpgf.lib()
    T = x.shape[0]
    outs = []
    for fn in (L.qpgf_evaluate_noalloc, L.qpgf_evaluate):
        out = P.out_tensor(T)
        flags = torch.full((T,), 255, dtype=torch.uint8, device="cuda")
        P._stream()
        st = fn(P._h, _vp(x), T, _vp(out), _vp(flags))
        assert st == 0, L.qpgf_last_error().decode()
        torch.cuda.synchronize()
        outs.append((out.cpu().numpy(), flags.cpu().numpy()))
    return outs


@pytest.mark.parametrize("kind,prec,m,dim,Ts,kw", [
    (qpgf.KIND_GD3D, qpgf.C64, (256, 256, 64), 3, (1_000_000, 300_000), {}),   # the headline shape
    (qpgf.KIND_GD3D, qpgf.C128, (64, 64, 32), 3, (200_000, 70_000), {}),
    (qpgf.KIND_MAXWELL3D, qpgf.C64, (32, 32, 16), 3, (100_000, 66_000), {}),
    (qpgf.KIND_GD3D, qpgf.C128, (64, 64, 32), 3, (5_000, 100), {}),             # below the binning threshold
    (qpgf.KIND_G2D, qpgf.C128, (256, 64), 2, (50_000, 20_000), {"ring_interp": 1}),
])
def test_noalloc_equals_evaluate(kind, prec, m, dim, Ts, kw):
    P = qpgf.Plan(kind, prec, *m, **kw)
    if dim == 3:
        P.prepare(3.7, 0.21, -0.33)
    else:
        P.prepare(3.7, 0.21)
    x = workloads.targets(Ts[0], dim, seed=11)
    for T in Ts:
        print(f"noalloc case kind={kind} prec={prec} m={m} T={T}", flush=True)
        (g0, f0), (g1, f1) = _both(P, dev(x[:T]))
        assert np.array_equal(f0, f1)
        assert np.array_equal(g0, g1, equal_nan=True)
        assert np.isfinite(g0).all()


def test_noalloc_refuses_what_does_not_fit():
    L = qpgf.lib()
    P = qpgf.Plan(qpgf.KIND_GD3D, qpgf.C64, 256, 256, 64)
    x = torch.zeros((2_000_000, 3), dtype=torch.float64, device="cuda")
    out = P.out_tensor(2_000_000)
    assert L.qpgf_evaluate_noalloc(P._h, _vp(x), 10, _vp(out), None) == 1     # not prepared
    P.prepare(3.7, 0.21, -0.33)
    st = L.qpgf_evaluate_noalloc(P._h, _vp(x), 2_000_000, _vp(out), None)
    msg = L.qpgf_last_error().decode()
    assert st == 4 and "at most" in msg, msg
    assert L.qpgf_evaluate_noalloc(P._h, _vp(x), -1, _vp(out), None) == 1
    assert L.qpgf_evaluate_noalloc(P._h, None, 10, _vp(out), None) == 1
