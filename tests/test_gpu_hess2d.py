"""GPU parity of the second-derivative-difference path (Section 2.4.2) against the CPU oracle,
through the C ABI.  Bars as for the other paths: complex128 <= 1e-10, complex64 <= 1e-5 in the
parity measure max_i |g_i - o_i| / max(|o_i|, RMS |o|), per component.
"""

import ctypes
import math

import numpy as np
import pytest
import torch

import slabcheck
from oracle import hess2d, method, truth
from paper_1801_05977_amd import qpgf, workloads

pytestmark = pytest.mark.gpu

A2 = 1.0 / (2.0 * math.sqrt(math.pi))
TOL = {qpgf.C128: 1e-10, qpgf.C64: 1e-5}
K1, K2, AL = 2.1, 4.35, 0.3     # k2 away from Wood anomalies and special coefficients (min distance 0.27)


def parity(g, o):
    g, o = np.asarray(g), np.asarray(o)
    s = np.sqrt(np.mean(np.abs(o) ** 2))
    return float(np.max(np.abs(g - o) / np.maximum(np.abs(o), s)))


def cen(a, axes):
    return np.fft.fftshift(a, axes=axes)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("prec", [qpgf.C128, qpgf.C64])
def test_hess2d_stages(prec):
    """Coefficients of the three fields, their grids and the far slab, element by element."""
    M1, M2 = 64, 32
    P = qpgf.Plan(qpgf.KIND_G2D_HESS_DIFF, prec, M1, M2)
    assert P.info.n_fields == 3
    ref_L = [A2 * L for L in hess2d.lhat_hess_diff(K1, K2, AL, M1 // 2, M2 // 2)]
    P.prepare_hess_diff(K1, K2, AL, stage=0)
    tol = 1e-13 if prec == qpgf.C128 else 1e-7
    for f in range(3):
        g = cen(P.field(0, f).cpu().numpy().reshape(M2, M1).T, (0, 1))
        assert np.abs(g - ref_L[f]).max() <= tol * np.abs(ref_L[f]).max(), f
    P.prepare_hess_diff(K1, K2, AL, stage=2)
    tol = 1e-12 if prec == qpgf.C128 else 2e-6
    for f in range(3):
        g = cen(P.field(0, f).cpu().numpy().reshape(M2, M1).T, (0, 1))
        ref_G = method.grid_2d(ref_L[f] / A2)
        assert np.abs(g - ref_G).max() <= tol * np.abs(ref_G).max(), f
    # far slab: at its nodes the twice-differentiated series (1.2), k1 minus k2 (x2 > 0)
    (si, pi), pts = slabcheck.nodes_2d(P.info, 60, seed=4)
    ref_F = (truth.g2d_hess(K1, AL, pts) - truth.g2d_hess(K2, AL, pts)) * np.exp(-1j * AL * pts[:, 0])[:, None]
    for f in range(3):
        assert slabcheck.rel(slabcheck.slab_2d(P, f)[si, pi], ref_F[:, f]) <= tol, f


def _edge_targets():
    pts = [[0.01, 0.003], [-0.05, 0.02], [0.25, -0.2], [0.3, 0.1], [2 * math.pi - 0.02, 0.05],
           [0.0, 0.0], [2 * math.pi, 0.0], [1.0, 1.5], [2.0, -3.0], [np.nan, 0.1], [0.5, np.inf],
           [1.3, 0.61], [1.3, -0.61], [-7.0, 0.9], [13.0, -0.95], [-20.0, 0.3], [math.pi, 0.59]]
    return np.array(pts, dtype=np.float64)


@pytest.mark.parametrize("prec", [qpgf.C128, qpgf.C64])
@pytest.mark.parametrize("shape,T", [((64, 32), 1_000), ((256, 64), 10_001), ((80, 32), 1_003)])
def test_hess2d_end_to_end(prec, shape, T):
    """Seeded uniform targets (ragged count) plus edge cases; flags exact, values to the parity bar."""
    M1, M2 = shape
    x = np.vstack([workloads.targets(T, 2, seed=4), _edge_targets()])
    P = qpgf.Plan(qpgf.KIND_G2D_HESS_DIFF, prec, M1, M2)
    flags = torch.empty(len(x), dtype=torch.uint8, device="cuda")
    g = P.hess_diff(K1, K2, AL, dev(x), flags=flags).cpu().numpy()
    assert g.shape == (len(x), 3)
    fin = np.all(np.isfinite(x), axis=1)
    o = np.full((len(x), 3), np.nan + 0j)
    with np.errstate(all="ignore"):
        o[fin] = hess2d.eval_g2d_hess_diff(K1, K2, AL, x[fin], M1 // 2, M2 // 2)
    f = flags.cpu().numpy()
    t = x[:, 0] - 2 * math.pi * np.floor((x[:, 0] + math.pi) / (2 * math.pi))
    on_lattice = fin & (np.hypot(t, x[:, 1]) == 0)
    np.testing.assert_array_equal((f & 8) != 0, ~fin)
    np.testing.assert_array_equal((f & 2) != 0, fin & (np.abs(x[:, 1]) > 0.6))
    np.testing.assert_array_equal((f & 1) != 0, on_lattice)
    assert np.all(((f & 4) != 0) == (fin & (np.abs(x[:, 1]) >= slabcheck.limit(P.info))))
    bad = (f & 13) != 0
    assert np.all(np.isnan(g[bad]))
    ok = ~bad
    for p in range(3):
        assert parity(g[ok, p], o[ok, p]) <= TOL[prec], p


def test_hess2d_equal_wavenumbers_give_zero():
    """The degenerate instance k1 = k2: zero up to rounding (the two wavenumbers' quadrature terms
    are separate inlined computations, which the compiler may contract into FMAs differently)."""
    P = qpgf.Plan(qpgf.KIND_G2D_HESS_DIFF, qpgf.C128, 64, 32)
    x = dev(workloads.targets(513, 2, seed=8))
    scale = P.hess_diff(K1, K2, AL, x).abs().max().item()
    g = P.hess_diff(K1, K1, AL, x)
    assert g.abs().max().item() <= 1e-13 * scale


def test_hess2d_prepare_evaluate_split():
    P = qpgf.Plan(qpgf.KIND_G2D_HESS_DIFF, qpgf.C128, 128, 32)
    xa = dev(workloads.targets(777, 2, seed=5))
    xb = dev(workloads.targets(1234, 2, seed=6))
    ga, gb = P.hess_diff(K1, K2, AL, xa).cpu(), P.hess_diff(K1, K2, AL, xb).cpu()
    P.prepare_hess_diff(K1, K2, AL)
    assert torch.equal(P.evaluate(xa).cpu(), ga)
    assert torch.equal(P.evaluate(xb).cpu(), gb)


def test_hess2d_kind_checks():
    L = qpgf.lib()
    Ph = qpgf.Plan(qpgf.KIND_G2D_HESS_DIFF, qpgf.C128, 64, 32)
    P0 = qpgf.Plan(qpgf.KIND_G2D, qpgf.C128, 64, 32)
    x = dev(workloads.targets(10, 2, seed=1))
    out = torch.empty((10, 3), dtype=torch.complex128, device="cuda")
    px, po = ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr())
    assert L.qpgf_g2d_hess_diff(P0._h, K1, K2, AL, px, 10, po, None) == 1
    assert L.qpgf_prepare_hess_diff(P0._h, K1, K2, AL, 2) == 1
    assert L.qpgf_prepare(Ph._h, K1, AL, 0.0) == 1
    assert L.qpgf_prepare_stage(Ph._h, K1, AL, 0.0, 2) == 1
    assert L.qpgf_g2d(Ph._h, K1, AL, px, 10, po, None) == 1
    assert L.qpgf_prepare_hess_diff(Ph._h, K1, K2, AL, 3) == 1
    assert L.qpgf_g2d_hess_diff(Ph._h, K1, K2, AL, px, -1, po, None) == 1
    # a Wood anomaly of either wavenumber is refused before any launch
    assert L.qpgf_g2d_hess_diff(Ph._h, 1.0, K2, 0.0, px, 10, po, None) == 2
    assert L.qpgf_g2d_hess_diff(Ph._h, K2, 1.0, 0.0, px, 10, po, None) == 2
    with pytest.raises(ValueError):
        Ph(K1, AL, 0.0, x)
    p = qpgf.default_params(qpgf.KIND_G2D_HESS_DIFF, qpgf.C128, 64, 32, quad_q=192)
    h = ctypes.c_void_p()
    assert L.qpgf_plan_create(ctypes.byref(p), ctypes.byref(h)) == 1


@pytest.mark.parametrize("c_tilde", [1.0, 1.4])
def test_hess2d_accuracy_vs_series(c_tilde):
    """Against the twice-differentiated series at |x2| >= 0.02 (complex128, 512 x 128).

    The method's own accuracy (the oracle gives the same numbers).  T22 converges slowest:
    the Fourier series of d^2/dx2^2 of the truncated X K carries X'' K from the transition
    of X in c < |x2| < (c + c~)/2, so a wider transition (larger c~) helps it most.
    """
    x = workloads.targets(400, 2, seed=9)
    x = x[np.abs(x[:, 1]) >= 0.02]
    P = qpgf.Plan(qpgf.KIND_G2D_HESS_DIFF, qpgf.C128, 512, 128, c_tilde=c_tilde, far_h=c_tilde / 64,
                  far_zmax=c_tilde)
    g = P.hess_diff(K1, K2, AL, dev(x)).cpu().numpy()
    gt = truth.g2d_hess(K1, AL, x) - truth.g2d_hess(K2, AL, x)
    e = np.abs(g - gt) / np.abs(gt)
    assert e[:, 0].max() < 5e-3 and e[:, 1].max() < 5e-3
    if c_tilde == 1.0:
        assert np.median(e[:, 2]) < 5e-4 and np.quantile(e[:, 2], 0.99) < 8e-2
    else:
        assert np.median(e[:, 2]) < 2e-5 and np.quantile(e[:, 2], 0.99) < 2e-3 and e[:, 2].max() < 2e-2
