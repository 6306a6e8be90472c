"""GPU parity and accuracy of the higher-order 2D variant (sing_order 2 and 3, Remark 5.3):
the degree-2 and degree-3 terms of the logarithmic singularity removed as well.

Bars as for the other paths: complex128 <= 1e-10, complex64 <= 1e-5 in the parity measure
max_i |g_i - o_i| / max(|o_i|, RMS |o|); coefficient fills element by element.
"""

import ctypes
import math

import numpy as np
import pytest
import torch

import slabcheck
from oracle import highorder2d as ho
from oracle import method, truth
from paper_1801_05977_amd import qpgf, workloads

pytestmark = pytest.mark.gpu

A2 = 1.0 / (2.0 * math.sqrt(math.pi))
TOL = {qpgf.C128: 1e-10, qpgf.C64: 1e-5}
K, AL = 2.1, 0.3


def parity(g, o):
    g, o = np.asarray(g), np.asarray(o)
    s = np.sqrt(np.mean(np.abs(o) ** 2))
    return float(np.max(np.abs(g - o) / np.maximum(np.abs(o), s)))


def cen(a, axes):
    return np.fft.fftshift(a, axes=axes)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("order", [2, 3])
@pytest.mark.parametrize("prec", [qpgf.C128, qpgf.C64])
def test_ho_fill_and_grid_stages(prec, order):
    M1, M2 = 64, 32
    k, al = 5.3, 0.45
    P = qpgf.Plan(qpgf.KIND_G2D, prec, M1, M2, sing_order=order)
    ref_L = A2 * ho.lhat_ho(k, al, M1 // 2, M2 // 2, order)
    P.prepare(k, al, 0.0, stage=0)
    g = cen(P.field().cpu().numpy().reshape(M2, M1).T, (0, 1))
    tol = 1e-13 if prec == qpgf.C128 else 1e-7
    assert np.abs(g - ref_L).max() <= tol * np.abs(ref_L).max()
    # the removed part itself, against the oracle's E-hat (well above rounding of L-hat)
    P1 = qpgf.Plan(qpgf.KIND_G2D, prec, M1, M2)
    P1.prepare(k, al, 0.0, stage=0)
    g1 = cen(P1.field().cpu().numpy().reshape(M2, M1).T, (0, 1))
    ref_E = A2 * ho.ehat(k, al, M1 // 2, M2 // 2, order)
    if prec == qpgf.C128:
        assert np.abs((g1 - g) - ref_E).max() <= 1e-12 * np.abs(ref_E).max()
    P.prepare(k, al, 0.0, stage=2)
    g = cen(P.field().cpu().numpy().reshape(M2, M1).T, (0, 1))
    ref_G = method.grid_2d(ref_L / A2)
    tol = 1e-12 if prec == qpgf.C128 else 2e-6
    assert np.abs(g - ref_G).max() <= tol * np.abs(ref_G).max()


def _edge_targets():
    """Near and on the lattice point, in the cut-off ring, beyond the far slab, non-finite, x1
    outside the first cell."""
    pts = [[0.01, 0.003], [-0.05, 0.02], [0.25, -0.2], [0.3, 0.1], [2 * math.pi - 0.02, 0.05],
           [0.0, 0.0], [2 * math.pi, 0.0], [1.0, 1.5], [np.nan, 0.1], [0.5, np.inf],
           [1.3, 0.61], [-7.0, 0.003], [13.0, -0.0007], [math.pi, 0.59], [1e-4, -2e-4]]
    return np.array(pts, dtype=np.float64)


@pytest.mark.parametrize("order", [2, 3])
@pytest.mark.parametrize("prec", [qpgf.C128, qpgf.C64])
@pytest.mark.parametrize("shape,T", [((64, 32), 1_000), ((256, 64), 10_001), ((112, 32), 1_003)])
def test_ho_end_to_end(prec, order, shape, T):
    M1, M2 = shape
    x = np.vstack([workloads.targets(T, 2, seed=7), _edge_targets()])
    P = qpgf.Plan(qpgf.KIND_G2D, prec, M1, M2, sing_order=order)
    flags = torch.empty(len(x), dtype=torch.uint8, device="cuda")
    g = P(K, AL, 0.0, dev(x), flags=flags).cpu().numpy()
    fin = np.all(np.isfinite(x), axis=1)
    t = x[:, 0] - 2 * math.pi * np.floor((x[:, 0] + math.pi) / (2 * math.pi))
    on_lattice = fin & (np.hypot(t, x[:, 1]) == 0)
    ok_in = fin & ~on_lattice
    o = np.full(len(x), np.nan + 0j)
    o[ok_in] = ho.eval_g2d_ho(K, AL, x[ok_in], M1 // 2, M2 // 2, order)
    f = flags.cpu().numpy()
    np.testing.assert_array_equal((f & 8) != 0, ~fin)
    np.testing.assert_array_equal((f & 1) != 0, on_lattice)
    np.testing.assert_array_equal((f & 4) != 0, ok_in & (np.abs(x[:, 1]) >= slabcheck.limit(P.info)))
    bad = (f & 13) != 0
    assert np.all(np.isnan(g[bad]))
    assert parity(g[~bad], o[~bad]) <= TOL[prec]


def test_ho_order_one_is_the_default_path():
    x = dev(workloads.targets(2000, 2, seed=3))
    a = qpgf.Plan(qpgf.KIND_G2D, qpgf.C128, 128, 64)(K, AL, 0.0, x).cpu()
    b = qpgf.Plan(qpgf.KIND_G2D, qpgf.C128, 128, 64, sing_order=1)(K, AL, 0.0, x).cpu()
    assert torch.equal(a, b)


def test_ho_accuracy_near_the_lattice_point():
    """Against the series (1.2) at targets within 0.02 of the lattice point, complex128,
    512 x 256: removing the degree-2 and -3 terms takes the error down by orders of magnitude."""
    x = np.array([[0.0, 0.003], [0.001, 0.005], [-0.002, 0.008], [0.0, 0.012], [0.004, -0.02]])
    gt = truth.g2d(K, AL, x, max_terms=200_000_000)
    err = {}
    for order in (1, 2, 3):
        P = qpgf.Plan(qpgf.KIND_G2D, qpgf.C128, 512, 256, sing_order=order)
        err[order] = np.abs(P(K, AL, 0.0, dev(x)).cpu().numpy() - gt).max()
        P.close()
    assert err[1] > 1e-6
    assert err[2] < err[1] / 100
    assert err[3] < err[1] / 200 and err[3] < 3e-8


@pytest.mark.parametrize("prec", [qpgf.C128, qpgf.C64])
def test_ho_batched_equals_single_plans(prec):
    M2 = 64
    m1 = [256, 64, 512, 128]
    counts = [2000, 700, 3000, 1]
    t_off = np.concatenate([[0], np.cumsum(counts)])
    k, a = workloads.instances_2d(len(m1), 5, k_range=(1.0, 20.0), n2_max=32)
    x = workloads.targets(int(t_off[-1]), 2, seed=9)
    xd = dev(x)
    P = qpgf.Plan(qpgf.KIND_G2D, prec, max(m1), M2, sing_order=3)
    g = P.batched(k, a, m1, t_off, xd).cpu().numpy()
    # the higher-order tables' radial rule grows with the plan's grid, so the batched plan's
    # tables (largest x1 size) and a single plan's agree to quadrature rounding, not bitwise
    tol = 1e-13 if prec == qpgf.C128 else 1e-6
    for i, M in enumerate(m1):
        sl = slice(int(t_off[i]), int(t_off[i + 1]))
        Pi = qpgf.Plan(qpgf.KIND_G2D, prec, M, M2, sing_order=3)
        gi = Pi(k[i], a[i], 0.0, xd[sl].contiguous()).cpu().numpy()
        assert np.abs(g[sl] - gi).max() <= tol * np.abs(gi).max(), i
        Pi.close()
    sl = slice(int(t_off[0]), int(t_off[1]))
    o = ho.eval_g2d_ho(k[0], a[0], x[sl], m1[0] // 2, M2 // 2, 3)
    assert parity(g[sl], o) <= TOL[prec]


def test_ho_parameter_checks():
    L = qpgf.lib()
    for kind, dims, order in ((qpgf.KIND_G2D, (64, 32, 0), 0), (qpgf.KIND_G2D, (64, 32, 0), 4),
                              (qpgf.KIND_GD3D, (32, 32, 16), 2), (qpgf.KIND_G2D_GRAD, (64, 32, 0), 3)):
        p = qpgf.default_params(kind, qpgf.C128, *dims, sing_order=order)
        h = ctypes.c_void_p()
        assert L.qpgf_plan_create(ctypes.byref(p), ctypes.byref(h)) == 1, (kind, order)
