"""GPU parity of the 2D gradient path (Section 2.4.1) against the CPU oracle, through the C ABI.

Bars as for the other paths: complex128 <= 1e-10, complex64 <= 1e-5 in the
parity measure max_i |g_i - o_i| / max(|o_i|, RMS |o|), per component.
"""

import ctypes
import math

import numpy as np
import pytest
import torch

import slabcheck
from oracle import grad2d, method, truth
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


@pytest.mark.parametrize("prec", [qpgf.C128, qpgf.C64])
def test_grad2d_stages(prec):
    """Coefficients of both fields, their grids and the differentiated far slab, element by element."""
    M1, M2 = 64, 32
    P = qpgf.Plan(qpgf.KIND_G2D_GRAD, prec, M1, M2)
    assert P.info.n_fields == 2
    ref_L = [A2 * L for L in grad2d.lhat_grad_2d(K, AL, M1 // 2, M2 // 2)]
    P.prepare(K, AL, 0.0, stage=0)
    tol = 1e-13 if prec == qpgf.C128 else 1e-7
    for f in range(2):
        g = cen(P.field(0, f).cpu().numpy().reshape(M2, M1).T, (0, 1))
        assert np.abs(g - ref_L[f]).max() <= tol * np.abs(ref_L[f]).max(), f
    P.prepare(K, AL, 0.0, stage=2)
    tol = 1e-12 if prec == qpgf.C128 else 2e-6
    for f in range(2):
        g = cen(P.field(0, f).cpu().numpy().reshape(M2, M1).T, (0, 1))
        ref_G = method.grid_2d(ref_L[f] / A2)
        assert np.abs(g - ref_G).max() <= tol * np.abs(ref_G).max(), f
    # far slab: at its nodes the differentiated series (1.2) (x2 > 0)
    (si, pi), pts = slabcheck.nodes_2d(P.info, 60, seed=3)
    ref_F = truth.g2d_grad(K, AL, pts) * np.exp(-1j * AL * pts[:, 0])[:, None]
    for f in range(2):
        assert slabcheck.rel(slabcheck.slab_2d(P, f)[si, pi], ref_F[:, f]) <= tol, f


def _edge_targets(rng):
    """Near the lattice point and in the cut-off ring, on it, beyond the far slab, non-finite,
    both signs of x2 in the far branch, x1 outside the first cell."""
    pts = [[0.01, 0.003], [-0.05, 0.02], [0.25, -0.2], [0.3, 0.1], [2 * math.pi - 0.02, 0.05],
           [0.0, 0.0], [2 * math.pi, 0.0], [1.0, 1.5], [2.0, -3.0], [np.nan, 0.1], [0.5, np.inf],
           [1.3, 0.61], [1.3, -0.61], [-7.0, 0.9], [13.0, -0.95], [-20.0, 0.3], [math.pi, 0.59]]
    return np.array(pts, dtype=np.float64)


@pytest.mark.parametrize("prec", [qpgf.C128, qpgf.C64])
@pytest.mark.parametrize("shape,T", [((64, 32), 1_000), ((256, 64), 10_001), ((96, 32), 1_003)])
def test_grad2d_end_to_end(prec, shape, T):
    """Seeded uniform targets (ragged count) plus edge cases; flags exact, values to the parity bar."""
    M1, M2 = shape
    rng = np.random.default_rng(11)
    x = np.vstack([workloads.targets(T, 2, seed=3), _edge_targets(rng)])
    P = qpgf.Plan(qpgf.KIND_G2D_GRAD, prec, M1, M2)
    flags = torch.empty(len(x), dtype=torch.uint8, device="cuda")
    g = P(K, AL, 0.0, dev(x), flags=flags).cpu().numpy()
    assert g.shape == (len(x), 2)
    fin = np.all(np.isfinite(x), axis=1)
    o = np.full((len(x), 2), np.nan + 0j)
    with np.errstate(all="ignore"):
        o[fin] = grad2d.eval_g2d_grad(K, AL, x[fin], M1 // 2, M2 // 2)
    f = flags.cpu().numpy()
    z = np.abs(x[:, 1])
    t = x[:, 0] - 2 * math.pi * np.floor((x[:, 0] + math.pi) / (2 * math.pi))
    on_lattice = fin & (np.hypot(t, x[:, 1]) == 0)
    np.testing.assert_array_equal((f & 8) != 0, ~fin)
    np.testing.assert_array_equal((f & 2) != 0, fin & (z > 0.6))
    np.testing.assert_array_equal((f & 1) != 0, on_lattice)
    beyond = (f & 4) != 0
    assert np.all(beyond == (fin & (z >= slabcheck.limit(P.info))))
    bad = (f & 13) != 0
    assert np.all(np.isnan(g[bad]))
    ok = ~bad
    for p in range(2):
        assert parity(g[ok, p], o[ok, p]) <= TOL[prec], p


def test_grad2d_prepare_evaluate_split():
    """One preparation, two target sets: the same numbers as the combined call."""
    M1, M2 = 128, 32
    P = qpgf.Plan(qpgf.KIND_G2D_GRAD, qpgf.C128, M1, M2)
    xa = dev(workloads.targets(777, 2, seed=5))
    xb = dev(workloads.targets(1234, 2, seed=6))
    ga, gb = P(K, AL, 0.0, xa).cpu(), P(K, AL, 0.0, xb).cpu()
    P.prepare(K, AL)
    assert torch.equal(P.evaluate(xa).cpu(), ga)
    assert torch.equal(P.evaluate(xb).cpu(), gb)


def test_grad2d_kind_checks():
    L = qpgf.lib()
    Pg = qpgf.Plan(qpgf.KIND_G2D_GRAD, qpgf.C128, 64, 32)
    P0 = qpgf.Plan(qpgf.KIND_G2D, qpgf.C128, 64, 32)
    x = dev(workloads.targets(10, 2, seed=1))
    out = torch.empty((10, 2), dtype=torch.complex128, device="cuda")
    px, po = ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr())
    assert L.qpgf_g2d_grad(P0._h, K, AL, px, 10, po, None) == 1
    assert L.qpgf_g2d(Pg._h, K, AL, px, 10, po, None) == 1
    assert L.qpgf_g2d_grad(Pg._h, K, AL, px, -1, po, None) == 1
    assert L.qpgf_g2d_grad(Pg._h, K, AL, None, 10, po, None) == 1
    assert L.qpgf_g2d_grad(Pg._h, K, AL, None, 0, None, None) == 0
    with pytest.raises(qpgf.QpgfError):
        Pg.batched([K], [AL], [64], [0, 10], x)
    # Wood anomaly refused before any launch
    assert L.qpgf_g2d_grad(Pg._h, 1.0, 0.0, px, 10, po, None) == 2


def test_grad2d_accuracy_vs_series():
    """Against the differentiated eigenfunction series at |x2| >= 0.02 (complex128, 512 x 128).

    The method's own accuracy (the oracle gives the same numbers): the largest errors sit in
    the cut-off ring eps < r < 2 eps, where the O(1/r) part of h_p meets the steep C^8 cut-off.
    """
    x = workloads.targets(400, 2, seed=9)
    x = x[np.abs(x[:, 1]) >= 0.02]
    P = qpgf.Plan(qpgf.KIND_G2D_GRAD, qpgf.C128, 512, 128)
    g = P(K, AL, 0.0, dev(x)).cpu().numpy()
    gt = truth.g2d_grad(K, AL, x)
    e = np.abs(g - gt) / np.abs(gt)
    assert np.median(e) < 2e-7
    assert np.quantile(e, 0.99) < 1e-3
    assert e.max() < 5e-3
