"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Stage checks compare coefficient fills, grids and far slabs element by element;
end-to-end checks compare G, G_d and the Maxwell tensor at seeded targets.
Bars: complex128 path max parity error <= 1e-10,
complex64 path <= 1e-5, where the parity error of a result set is
max_i |g_i - o_i| / max(|o_i|, s), s = RMS |o| over the set (a pointwise
relative error that does not blow up at isolated zeros of G).
"""

import math

import numpy as np
import pytest
import torch

import slabcheck
from oracle import method, truth
from paper_1801_05977_amd import qpgf, workloads

pytestmark = pytest.mark.gpu

A2 = 1.0 / (2.0 * math.sqrt(math.pi))
A3 = 1.0 / math.sqrt(8.0 * math.pi ** 2)
TOL = {qpgf.C128: 1e-10, qpgf.C64: 1e-5}


def parity(g, o):
    g, o = np.asarray(g), np.asarray(o)
    s = np.sqrt(np.mean(np.abs(o) ** 2))
    return float(np.max(np.abs(g - o) / np.maximum(np.abs(o), s)))


def cen(a, axes):
    """FFT order (index j mod M) -> centred order (index j + M/2) along the given axes."""
    return np.fft.fftshift(a, axes=axes)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


# ----------------------------------------------------------------------------- 2D stages

@pytest.mark.parametrize("prec", [qpgf.C128, qpgf.C64])
def test_fill2d_and_grid2d_stages(prec):
    M1, M2 = 64, 32
    k, al = 2.1, 0.3
    P = qpgf.Plan(qpgf.KIND_G2D, prec, M1, M2)
    ref_L = A2 * method.lhat_2d(k, al, M1 // 2, M2 // 2)
    P.prepare(k, al, 0.0, stage=0)
    g = cen(P.field().cpu().numpy().reshape(M2, M1).T, (0, 1))
    tol = 1e-13 if prec == qpgf.C128 else 1e-7
    assert np.abs(g - ref_L).max() <= tol * np.abs(ref_L).max()
    P.prepare(k, al, 0.0, stage=2)
    g = cen(P.field().cpu().numpy().reshape(M2, M1).T, (0, 1))
    ref_G = method.grid_2d(ref_L / A2)
    tol = 1e-12 if prec == qpgf.C128 else 2e-6
    assert np.abs(g - ref_G).max() <= tol * np.abs(ref_G).max()
    # far slab: at its nodes the series (1.2) itself, on its own grid of far_m1 >= 256 modes
    assert P.info.far_m1 == (512 if prec == qpgf.C128 else 256) and P.info.far_fields == 1
    assert P.info.far_points == (8 if prec == qpgf.C128 else 4)
    (si, pi), pts = slabcheck.nodes_2d(P.info, 60, seed=1)
    ref_F = truth.g2d(k, al, pts) * np.exp(-1j * al * pts[:, 0])
    assert slabcheck.rel(slabcheck.slab_2d(P)[si, pi], ref_F) <= tol


# ----------------------------------------------------------------------------- 3D stages

@pytest.mark.parametrize("prec", [qpgf.C128, qpgf.C64])
def test_fill3d_and_grid3d_stages(prec):
    M1, M2, M3 = 32, 64, 32
    k, a1, a2 = 3.7, 0.2, 0.35
    P = qpgf.Plan(qpgf.KIND_GD3D, prec, M1, M2, M3)
    ref_L = A3 * method.lhat_3d(k, a1, a2, M1 // 2, M2 // 2, M3 // 2)
    P.prepare(k, a1, a2, stage=0)
    g = cen(P.field().cpu().numpy().reshape(M3, M2, M1).transpose(2, 1, 0), (0, 1, 2))
    tol = 1e-13 if prec == qpgf.C128 else 1e-7
    assert np.abs(g - ref_L).max() <= tol * np.abs(ref_L).max()
    P.prepare(k, a1, a2, stage=2)
    g = cen(P.field().cpu().numpy().reshape(M3, M2, M1).transpose(2, 1, 0), (0, 1, 2))
    ref_G = method.grid_3d(ref_L / A3)
    tol = 1e-12 if prec == qpgf.C128 else 2e-6
    assert np.abs(g - ref_G).max() <= tol * np.abs(ref_G).max()
    # far slab: at its nodes the series (1.3) itself
    assert (P.info.far_m1, P.info.far_m2, P.info.far_fields) == (512, 512, 1)
    assert P.info.far_points == (8 if prec == qpgf.C128 else 4)
    idx, pts = slabcheck.nodes_3d(P.info, 30, seed=2)
    ref_F = truth.gd3d(k, a1, a2, pts) * np.exp(-1j * (a1 * pts[:, 0] + a2 * pts[:, 1]))
    assert slabcheck.rel(slabcheck.slab_3d(P)[idx], ref_F) <= tol


# ----------------------------------------------------------------------------- end to end

@pytest.mark.parametrize("prec", [qpgf.C128, qpgf.C64])
def test_g2d_small_workload(prec):
    """2D, k = 2.1, alpha = 0.3, 256 x-modes, 64 slices, 1e4 uniform targets, seed 0."""
    M1, M2, T = 256, 64, 10_000
    k, al = 2.1, 0.3
    x = workloads.targets(T, 2, seed=0)
    P = qpgf.Plan(qpgf.KIND_G2D, prec, M1, M2)
    flags = torch.empty(T, dtype=torch.uint8, device="cuda")
    g = P(k, al, 0.0, dev(x), flags=flags).cpu().numpy()
    o = method.eval_g2d(k, al, x, M1 // 2, M2 // 2)
    assert parity(g, o) <= TOL[prec]
    f = flags.cpu().numpy()
    np.testing.assert_array_equal((f & 2) != 0, np.abs(x[:, 1]) > 0.6)
    assert not np.any(f & 13)


def test_g2d_large_grid_row_major_path():
    """complex64 G on a grid whose node quads would outgrow L2 (2048 x 256): the gather reads the grid
    row by row; sampled targets against the oracle, wrapped rows included."""
    M1, M2 = 2048, 256
    k, al = 2.1, 0.3
    x = workloads.targets(100_000, 2, seed=12)
    P = qpgf.Plan(qpgf.KIND_G2D, qpgf.C64, M1, M2)
    g = P(k, al, 0.0, dev(x)).cpu().numpy()
    t = x[:, 0] - 2 * math.pi * np.floor((x[:, 0] + math.pi) / (2 * math.pi))
    wrap = np.nonzero(t > math.pi - 2 * (2 * math.pi / M1))[0]
    rng = np.random.default_rng(3)
    pick = np.concatenate([wrap[:50], rng.choice(len(x), 250, replace=False)])
    o = method.eval_g2d(k, al, x[pick], M1 // 2, M2 // 2)
    assert len(wrap) >= 50
    assert parity(g[pick], o) <= TOL[qpgf.C64]


@pytest.mark.parametrize("prec", [qpgf.C128, qpgf.C64])
@pytest.mark.parametrize("M1", [24, 80, 112, 96])
def test_g2d_mixed_radix_stages(prec, M1):
    """x1 sizes 2^a r (r = 3, 5, 7): coefficients and grid element by element; the far slab keeps a
    power-of-two mode count at least M1."""
    M2 = 32
    k, al = 2.1, 0.3
    P = qpgf.Plan(qpgf.KIND_G2D, prec, M1, M2)
    ref_L = A2 * method.lhat_2d(k, al, M1 // 2, M2 // 2)
    P.prepare(k, al, 0.0, stage=2)
    g = cen(P.field().cpu().numpy().reshape(M2, M1).T, (0, 1))
    ref_G = method.grid_2d(ref_L / A2)
    tol = 1e-12 if prec == qpgf.C128 else 2e-6
    assert np.abs(g - ref_G).max() <= tol * np.abs(ref_G).max()
    assert P.info.far_m1 == (512 if prec == qpgf.C128 else 256)


@pytest.mark.parametrize("prec", [qpgf.C128, qpgf.C64])
@pytest.mark.parametrize("M1", [768, 1280, 1792])
def test_g2d_mixed_radix_x1_sizes(prec, M1):
    """G on grids of 3, 5 and 7 times 256 x-nodes: seeded targets plus targets whose stencils wrap in x1,
    against the oracle; the far slab takes the next power of two of modes."""
    M2, T = 64, 20_001
    k, al = 2.1, 0.3
    x = workloads.targets(T, 2, seed=21)
    P = qpgf.Plan(qpgf.KIND_G2D, prec, M1, M2)
    g = P(k, al, 0.0, dev(x)).cpu().numpy()
    m = 1 << (M1 - 1).bit_length()
    assert P.info.far_m1 == m
    t = x[:, 0] - 2 * math.pi * np.floor((x[:, 0] + math.pi) / (2 * math.pi))
    wrap = np.nonzero((t > math.pi - 2 * (2 * math.pi / M1)) | (t < -math.pi + 2 * math.pi / M1))[0]
    rng = np.random.default_rng(5)
    pick = np.unique(np.concatenate([wrap[:40], rng.choice(len(x), 400, replace=False)]))
    assert len(wrap) >= 10
    o = method.eval_g2d(k, al, x[pick], M1 // 2, M2 // 2)
    assert parity(g[pick], o) <= TOL[prec]


@pytest.mark.parametrize("prec", [qpgf.C128, qpgf.C64])
@pytest.mark.parametrize("shape", [(64, 64, 32), (32, 128, 64)])
def test_gd3d_small(prec, shape):
    M1, M2, M3 = shape
    k, a1, a2 = 3.7, 0.2, 0.35
    T = 3000
    x = workloads.targets(T, 3, seed=2)
    P = qpgf.Plan(qpgf.KIND_GD3D, prec, M1, M2, M3)
    g = P(k, a1, a2, dev(x)).cpu().numpy()
    o = method.eval_gd3d(k, a1, a2, x, M1 // 2, M2 // 2, M3 // 2)
    assert parity(g, o) <= TOL[prec]


@pytest.mark.parametrize("prec", [qpgf.C128, qpgf.C64])
def test_maxwell3d_small(prec):
    M1, M2, M3 = 32, 32, 32
    k, a1, a2 = 5.3, 0.1, 0.4
    T = 2000
    x = workloads.targets(T, 3, seed=3)
    P = qpgf.Plan(qpgf.KIND_MAXWELL3D, prec, M1, M2, M3)
    g = P(k, a1, a2, dev(x)).cpu().numpy()
    o = method.eval_maxwell3d(k, a1, a2, x, M1 // 2, M2 // 2, M3 // 2)
    for comp in range(6):      # error per component, each with its own scale
        assert parity(g[:, comp], o[:, comp]) <= TOL[prec], comp


@pytest.mark.parametrize("prec", [qpgf.C128, qpgf.C64])
def test_maxwell_stages(prec):
    """Algorithm 4.1 step 1: the seven near fields L and L^{pq} = -c^p c^q L (pq = 11 22 33 12 13 23)
    element by element, and the far slab's six tensor entries against the series at its nodes."""
    M1, M2, M3 = 32, 32, 16
    k, a1, a2 = 5.3, 0.1, 0.4
    P = qpgf.Plan(qpgf.KIND_MAXWELL3D, prec, M1, M2, M3)
    assert (P.info.n_fields, P.info.far_fields) == (7, 6)
    assert P.info.far_m1 == 512
    L = method.lhat_3d(k, a1, a2, M1 // 2, M2 // 2, M3 // 2)
    refs = [A3 * L] + [A3 * m * L for m in method.maxwell_multipliers(a1, a2, M1 // 2, M2 // 2, M3 // 2)]
    P.prepare(k, a1, a2, stage=0)
    # the fill takes H(|xi|) from an 8-point Lagrange table of the radial transform (about 1e-13 of
    # the largest coefficient at k = 5.3); the oracle integrates H at every coefficient
    tol = 1e-12 if prec == qpgf.C128 else 1e-7
    for f in range(7):
        g = cen(P.field(0, f).cpu().numpy().reshape(M3, M2, M1).transpose(2, 1, 0), (0, 1, 2))
        assert np.abs(g - refs[f]).max() <= tol * np.abs(refs[f]).max(), f
    P.prepare(k, a1, a2, stage=2)
    tol = 1e-12 if prec == qpgf.C128 else 2e-6
    for f in range(7):
        g = cen(P.field(0, f).cpu().numpy().reshape(M3, M2, M1).transpose(2, 1, 0), (0, 1, 2))
        ref_G = method.grid_3d(refs[f] / A3)
        assert np.abs(g - ref_G).max() <= tol * np.abs(ref_G).max(), f
    idx, pts = slabcheck.nodes_3d(P.info, 12, seed=5)
    ref_F = truth.maxwell3d(k, a1, a2, pts) * np.exp(-1j * (a1 * pts[:, 0] + a2 * pts[:, 1]))[:, None]
    for f in range(6):
        assert slabcheck.rel(slabcheck.slab_3d(P, f)[idx], ref_F[:, f]) <= tol, f


@pytest.mark.parametrize("prec", [qpgf.C128, qpgf.C64])
@pytest.mark.parametrize("T", [2000, 70_000])
def test_maxwell3d_trace_option(prec, T):
    """maxwell_trace = 1: six near fields (no 33) and GG_33 = 2 G_d - GG_11 - GG_22, against the oracle's
    trace variant, in the unsorted and the tile-binned gathers (the oracle on a sample)."""
    M1, M2, M3 = 32, 32, 32
    k, a1, a2 = 5.3, 0.1, 0.4
    x = workloads.targets(T, 3, seed=31)
    P = qpgf.Plan(qpgf.KIND_MAXWELL3D, prec, M1, M2, M3, maxwell_trace=1)
    assert (P.info.n_fields, P.info.far_fields) == (6, 6)
    g = P(k, a1, a2, dev(x)).cpu().numpy()
    idx = np.random.default_rng(32).choice(T, 1500, replace=False)
    o = method.eval_maxwell3d(k, a1, a2, x[idx], M1 // 2, M2 // 2, M3 // 2, trace33=True)
    for comp in range(6):
        assert parity(g[idx, comp], o[:, comp]) <= TOL[prec], comp


@pytest.mark.parametrize("prec", [qpgf.C128, qpgf.C64])
@pytest.mark.parametrize("kind,shape", [(qpgf.KIND_GD3D, (64, 32, 32)), (qpgf.KIND_MAXWELL3D, (64, 32, 32)),
                                        (qpgf.KIND_GD3D, (128, 128, 64)), (qpgf.KIND_MAXWELL3D, (128, 128, 32))])
def test_binned_gather_large_target_count(prec, kind, shape):
    """T >= 65536 takes the binned path (targets sorted by grid tile, near and far tiles); includes
    targets beyond the far slab and on the lattice, whose flags must follow them.  The flags are
    checked for every target, the values against the oracle on a seeded sample of 2500 (the far
    ones against the series).  On 128 x 128 x 64 the 16 x 16 x 8 tiles would hold about 170 targets
    each, so the larger 32-node tiles are used; Maxwell on 128 x 128 x 32 (about 310 targets per
    tile) stages the seven fields one at a time."""
    (M1, M2, M3), T = shape, 120_001
    k, a1, a2 = 5.3, 0.1, 0.4
    x = workloads.targets(T, 3, seed=9, zmax=1.2)
    x[17] = [0.0, 2 * math.pi, 0.0]
    x[T - 1] = [4 * math.pi, 0.0, 0.0]
    P = qpgf.Plan(kind, prec, M1, M2, M3)
    flags = torch.empty(T, dtype=torch.uint8, device="cuda")
    g = P(k, a1, a2, dev(x), flags=flags).cpu().numpy()
    f = flags.cpu().numpy()
    z = np.abs(x[:, 2])
    beyond = z >= slabcheck.limit(P.info)
    on_lat = np.zeros(T, bool)
    on_lat[[17, T - 1]] = True
    np.testing.assert_array_equal(f, np.where(on_lat, 1, 0) | np.where(z > 0.6, 2, 0) | np.where(beyond, 4, 0))
    bad = (f & 5) != 0
    assert np.all(np.isnan(g[bad])) and np.all(np.isfinite(g[~bad]))
    rng = np.random.default_rng(19)
    idx = rng.choice(np.nonzero(~bad)[0], 2500, replace=False)
    st = method.prepare_3d(k, a1, a2, M1 // 2, M2 // 2, M3 // 2, maxwell=(kind == qpgf.KIND_MAXWELL3D))
    o = method.evaluate_3d(st, x[idx])
    gg = g[idx]
    if gg.ndim == 1:
        assert parity(gg, o) <= TOL[prec]
    else:
        for comp in range(6):
            assert parity(gg[:, comp], o[:, comp]) <= TOL[prec], comp


def test_prepare_then_evaluate_in_chunks_matches_single_call():
    M1, M2, M3 = 64, 64, 32
    k, a1, a2 = 3.7, 0.2, 0.35
    x = dev(workloads.targets(5000, 3, seed=5))
    P = qpgf.Plan(qpgf.KIND_GD3D, qpgf.C128, M1, M2, M3)
    whole = P(k, a1, a2, x)
    P.prepare(k, a1, a2)
    parts = torch.cat([P.evaluate(x[:1234].contiguous()), P.evaluate(x[1234:].contiguous())])
    assert torch.equal(whole, parts)
    again = P(k, a1, a2, x)
    assert torch.equal(whole, again)            # deterministic


def test_overlapped_binning_back_to_back_and_after_a_failed_prepare():
    """qpgf_gd3d bins the targets on a second stream while the grids are prepared.  Calls issued back to
    back on one plan (different targets, no host synchronisation), and a call after a preparation that
    failed (Wood anomaly), give exactly what the sequential prepare + evaluate path gives."""
    M = (64, 64, 32)
    xa = dev(workloads.targets(70_000, 3, seed=21))
    xb = dev(workloads.targets(90_000, 3, seed=22))
    P = qpgf.Plan(qpgf.KIND_GD3D, qpgf.C64, *M)
    ga = P(3.7, 0.2, 0.35, xa)
    gb = P(5.1, -0.3, 0.1, xb)
    with pytest.raises(qpgf.QpgfError) as e:
        P(1.25, 0.2, 0.35, xa)            # |alpha + (1, 0)| = 1.25: beta = 0
    assert e.value.status == 2
    gc = P(3.7, 0.2, 0.35, xa)
    Q = qpgf.Plan(qpgf.KIND_GD3D, qpgf.C64, *M)
    Q.prepare(3.7, 0.2, 0.35)
    ra = Q.evaluate(xa)
    Q.prepare(5.1, -0.3, 0.1)
    rb = Q.evaluate(xb)
    for g, r in ((ga, ra), (gb, rb), (gc, ra)):
        assert torch.equal(torch.isnan(g), torch.isnan(r))
        ok = ~torch.isnan(g)
        assert torch.equal(g[ok], r[ok])


# ----------------------------------------------------------------------------- edge cases

@pytest.mark.parametrize("prec", [qpgf.C128, qpgf.C64])
@pytest.mark.parametrize("T", [3000, 70_000])
def test_lattice_rmin_flags_and_values_3d(prec, T):
    """lattice_rmin > 0: targets within it of a lattice point give NaN and flag bit 0, targets just
    outside are evaluated (with the singular add-back) and match the oracle; both the unsorted and
    the tile-binned (T >= 65536) gathers."""
    M1, M2, M3 = 32, 32, 16
    k, a1, a2 = 3.7, 0.2, 0.35
    rmin = 1e-2
    x = workloads.targets(T, 3, seed=13)
    rng = np.random.default_rng(14)
    d = rng.normal(size=(40, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    cells = 2 * math.pi * rng.integers(-1, 3, (40, 2))
    rad = np.where(np.arange(40) % 2 == 0, 0.5 * rmin, 2 * rmin)
    x[:40, :2] = cells + rad[:, None] * d[:, :2]
    x[:40, 2] = rad * d[:, 2]
    P = qpgf.Plan(qpgf.KIND_GD3D, prec, M1, M2, M3, lattice_rmin=rmin)
    flags = torch.empty(T, dtype=torch.uint8, device="cuda")
    g = P(k, a1, a2, dev(x), flags=flags).cpu().numpy()
    f = flags.cpu().numpy()
    inside = np.zeros(T, bool)
    inside[:40:2] = True
    np.testing.assert_array_equal((f & 1) == 1, inside)
    assert np.all(np.isnan(g[inside])) and np.all(np.isfinite(g[~inside]))
    o = method.eval_gd3d(k, a1, a2, x[:2000], M1 // 2, M2 // 2, M3 // 2)
    sel = ~inside[:2000]
    assert parity(g[:2000][sel], o[sel]) <= TOL[prec]


def test_edge_targets_and_status_codes():
    M1, M2 = 64, 32
    k, al = 2.1, 0.3
    P = qpgf.Plan(qpgf.KIND_G2D, qpgf.C128, M1, M2)
    x = np.array([[0.0, 0.0],                 # lattice point: NaN, flag 1
                  [2 * math.pi, 0.0],         # lattice point one period over
                  [math.pi, 0.1],             # x1 = pi reduces to t = -pi
                  [-math.pi, 0.1],
                  [1.0, 0.6],                 # |x2| = c exactly: near
                  [1.0, 0.6000001],           # just far
                  [1.0, 1.5],                 # beyond the far slab: NaN, flag 4
                  [float("nan"), 0.2],        # non-finite: NaN, flag 8
                  [0.3, -0.25]])
    flags = torch.empty(len(x), dtype=torch.uint8, device="cuda")
    g = P(k, al, 0.0, dev(x), flags=flags).cpu().numpy()
    f = flags.cpu().numpy()
    assert list(f) == [1, 1, 0, 0, 0, 2, 6, 8, 0]
    assert np.isnan(g[[0, 1, 6, 7]]).all() and np.isfinite(g[[2, 3, 4, 5, 8]]).all()
    o = method.eval_g2d(k, al, x[[2, 3, 4, 5, 8]], M1 // 2, M2 // 2)
    assert parity(g[[2, 3, 4, 5, 8]], o) <= 1e-10
    # quasi-periodicity of the reduction: G(x1 + 2 pi) = e^{i 2 pi alpha} G(x1)
    np.testing.assert_allclose(g[2], np.exp(2j * math.pi * al) * g[3], rtol=1e-12)
    # T = 0 is a no-op
    P(k, al, 0.0, dev(np.zeros((0, 2))))
    # Wood anomaly: k = |alpha + 1| makes beta_1 = 0
    with pytest.raises(qpgf.QpgfError) as e:
        P(1.3, 0.3, 0.0, dev(x))
    assert e.value.status == 2
    # special coefficient beta_0 = pi (j2 = 1, c~ = 1) for k^2 = alpha^2 + pi^2: evaluated, not refused
    ks = math.sqrt(0.3 ** 2 + math.pi ** 2)
    gs = P(ks, 0.3, 0.0, dev(x[[2, 3, 4, 5, 8]])).cpu().numpy()
    os_ = method.eval_g2d(ks, 0.3, x[[2, 3, 4, 5, 8]], M1 // 2, M2 // 2)
    assert parity(gs, os_) <= 1e-10
    # wrong entry point for the plan kind
    P3 = qpgf.Plan(qpgf.KIND_GD3D, qpgf.C128, 32, 32, 32)
    with pytest.raises(qpgf.QpgfError) as e:
        qpgf._check(qpgf.lib().qpgf_g2d(P3._h, k, al, None, 0, None, None))
    assert e.value.status == 1


@pytest.mark.parametrize("k", [3.7, 7.3])
def test_gd3d_far_branch_next_to_c(k):
    """The far branch where it is hardest for the slab rule: |x3| just beyond c, where the
    evanescent terms of the series are largest, in the binned launch (7e4 targets).  At k = 3.7
    the complex128 far gather takes 7 points along x2 and x3, at k = 7.3 the slab's spacing is
    too coarse for that and it keeps 8.  The oracle sums the series (1.3) itself."""
    M1, M2, M3, T = 64, 64, 32, 70_000
    a1, a2 = 0.2, 0.35
    rng = np.random.default_rng(31)
    x = np.empty((T, 3))
    x[:, 0] = rng.uniform(0.0, 2 * math.pi, T)
    x[:, 1] = rng.uniform(0.0, 2 * math.pi, T)
    x[:, 2] = rng.choice([-1.0, 1.0], T) * rng.uniform(0.6 + 1e-9, 0.63, T)
    pick = rng.choice(T, 300, replace=False)
    o = truth.gd3d(k, a1, a2, x[pick])
    for prec in (qpgf.C128, qpgf.C64):
        P = qpgf.Plan(qpgf.KIND_GD3D, prec, M1, M2, M3)
        flags = torch.empty(T, dtype=torch.uint8, device="cuda")
        g = P(k, a1, a2, dev(x), flags=flags).cpu().numpy()
        assert np.all(flags.cpu().numpy() == 2)
        assert P.info.far_points_t == (4 if prec == qpgf.C64 else (7 if k < 5 else 8))
        err = parity(g[pick], o)
        print("far next to c", k, "c128" if prec == qpgf.C128 else "c64", err)
        # the slab's design error: about 1e-11 (complex128) and 1e-6 (complex64) of the series
        assert err <= (5e-11 if prec == qpgf.C128 else 5e-6)
        P.close()


@pytest.mark.parametrize("kind,prec,far_m", [
    (qpgf.KIND_GD3D, qpgf.C128, 256), (qpgf.KIND_GD3D, qpgf.C128, 2048),
    (qpgf.KIND_GD3D, qpgf.C64, 256), (qpgf.KIND_GD3D, qpgf.C64, 2048),
    (qpgf.KIND_MAXWELL3D, qpgf.C64, 256), (qpgf.KIND_MAXWELL3D, qpgf.C64, 2048)])
def test_far_slab_nodes_at_far_m(kind, prec, far_m):
    """The far slab at caller-set sizes: column tiles from 16 columns down to one, and at 2048 modes
    the Maxwell slab's unfused passes.  At sampled nodes it is the series (1.3) itself, the bands of
    dropped terms included (256 modes truncate the series at about e^-70 at these heights)."""
    k, a1, a2 = 3.7, 0.2, 0.35
    P = qpgf.Plan(kind, prec, 32, 32, 16, far_m=far_m)
    P.prepare(k, a1, a2, stage=2)
    assert (P.info.far_m1, P.info.far_m2) == (far_m, far_m)
    idx, pts = slabcheck.nodes_3d(P.info, 30 if kind == qpgf.KIND_GD3D else 12, seed=11)
    ph = np.exp(-1j * (a1 * pts[:, 0] + a2 * pts[:, 1]))
    tol = 1e-12 if prec == qpgf.C128 else 2e-6
    if kind == qpgf.KIND_GD3D:
        ref = truth.gd3d(k, a1, a2, pts) * ph
        assert slabcheck.rel(slabcheck.slab_3d(P)[idx], ref) <= tol
    else:
        ref = truth.maxwell3d(k, a1, a2, pts) * ph[:, None]
        for f in range(6):
            assert slabcheck.rel(slabcheck.slab_3d(P, f)[idx], ref[:, f]) <= tol, f
    P.close()


@pytest.mark.parametrize("kind,prec", [(qpgf.KIND_GD3D, qpgf.C128), (qpgf.KIND_GD3D, qpgf.C64),
                                       (qpgf.KIND_MAXWELL3D, qpgf.C64)])
def test_far_slab_reuse_bitwise(kind, prec):
    """The far slab's first transform leaves the bands that hold only terms past the cut unwritten
    and the second takes them as zero without reading them.  A plan whose slab still holds a
    wider band from a previous instance (same slab geometry: k 6.1 then 2.3) gives bitwise the
    slab and the values of a fresh plan."""
    M1, M2, M3, T = 64, 64, 32, 40_000
    rng = np.random.default_rng(47)
    x = np.empty((T, 3))
    x[:, 0] = rng.uniform(0.0, 2 * math.pi, T)
    x[:, 1] = rng.uniform(0.0, 2 * math.pi, T)
    x[:, 2] = rng.choice([-1.0, 1.0], T) * rng.uniform(0.6 + 1e-9, 1.0, T)
    xd = dev(x)
    used, fresh = qpgf.Plan(kind, prec, M1, M2, M3), qpgf.Plan(kind, prec, M1, M2, M3)
    used(6.1, 0.45, -0.3, xd)
    geom = (used.info.far_m1, used.info.far_m2, used.info.far_slices)
    g = used(2.3, 0.1, 0.2, xd).cpu().numpy()
    assert (used.info.far_m1, used.info.far_m2, used.info.far_slices) == geom
    ref = fresh(2.3, 0.1, 0.2, xd).cpu().numpy()
    assert np.array_equal(g.view(np.uint8), ref.view(np.uint8))
    for f in range(6 if kind == qpgf.KIND_MAXWELL3D else 1):
        a, b = used.field(1, f).cpu().numpy(), fresh.field(1, f).cpu().numpy()
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    used.close()
    fresh.close()


# ----------------------------------------------------------------------------- full size, sampled

@pytest.mark.timeout(900)
def test_gd3d_full_size_sampled():
    """3D G_d at the benchmark size: 256 x 256 modes, 64 slices, 1e7 targets.

    The GPU evaluates all 1e7 targets in the launch configuration the benchmark
    times; the oracle recomputes 400 of them (seeded sample, including the first
    and last target) from its own full-size coefficients and direct-DFT grid.
    """
    M1, M2, M3, T = 256, 256, 64, 10_000_000
    k, a1, a2 = 3.7, 0.2, 0.35
    x = workloads.targets(T, 3, seed=2)
    xd = dev(x)
    rng = np.random.default_rng(11)
    idx = np.unique(np.concatenate([[0, T - 1], rng.choice(T, 398, replace=False)]))
    outs = {}
    for prec in (qpgf.C128, qpgf.C64):
        P = qpgf.Plan(qpgf.KIND_GD3D, prec, M1, M2, M3)
        outs[prec] = P(k, a1, a2, xd)[torch.from_numpy(idx).cuda()].cpu().numpy()
        info = P.info
        P.close()
    o = method.eval_gd3d(k, a1, a2, x[idx], M1 // 2, M2 // 2, M3 // 2)
    assert parity(outs[qpgf.C128], o) <= TOL[qpgf.C128]
    assert parity(outs[qpgf.C64], o) <= TOL[qpgf.C64]


@pytest.mark.timeout(900)
def test_maxwell3d_full_size_sampled():
    """The Maxwell tensor at its benchmark size: k = 5.3, alpha = (0.1, 0.4), 512 x 512 modes, 32
    slices, 1e6 targets, both precisions, every component on its own scale.

    The GPU evaluates all 1e6 targets as the benchmark does; the oracle recomputes 400 of them
    (seeded, with the first and the last, plus targets inside the cut-off ring of a lattice
    point) from its own full-size coefficients of the seven fields."""
    M1, M2, M3, T = 512, 512, 32, 1_000_000
    k, a1, a2 = 5.3, 0.1, 0.4
    x = workloads.targets(T, 3, seed=3)
    rng = np.random.default_rng(12)
    ring = rng.normal(size=(12, 3))
    ring *= (rng.uniform(0.02, 0.38, 12) / np.linalg.norm(ring, axis=1))[:, None]
    x[:12] = ring + 2 * np.pi * rng.integers(-1, 2, (12, 1)) * np.array([1.0, 1.0, 0.0])
    idx = np.unique(np.concatenate([np.arange(12), [T - 1], rng.choice(T, 388, replace=False)]))
    xd = dev(x)
    outs = {}
    for prec in (qpgf.C128, qpgf.C64):
        P = qpgf.Plan(qpgf.KIND_MAXWELL3D, prec, M1, M2, M3)
        outs[prec] = P(k, a1, a2, xd)[torch.from_numpy(idx).cuda()].cpu().numpy()
        P.close()
    st = method.prepare_3d(k, a1, a2, M1 // 2, M2 // 2, M3 // 2, maxwell=True)
    o = method.evaluate_3d(st, x[idx])
    assert o.shape == (len(idx), 6)
    for prec in (qpgf.C128, qpgf.C64):
        errs = [parity(outs[prec][:, j], o[:, j]) for j in range(6)]
        print("maxwell full size", "c128" if prec == qpgf.C128 else "c64", errs)
        assert max(errs) <= TOL[prec], errs
