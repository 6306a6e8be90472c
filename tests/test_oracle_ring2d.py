"""Pins of the cut-off-ring option of the 2D oracle (``ring=True``: K interpolated for
targets with eps < r < 2 eps + 2 sqrt(2) h).

Independent routes: the eigenfunction series (1.2) for the accuracy it buys, and the
interpolation identity at grid nodes (where the stencil reproduces its node value, so
interpolating K or interpolating L and adding f Y back must agree).
"""

import math

import numpy as np
import pytest

from oracle import highorder2d as ho
from oracle import truth

K, AL = 2.1, 0.3


def _ring_targets(n, seed, lo=0.2, hi=0.45):
    rng = np.random.default_rng(seed)
    r = rng.uniform(lo, hi, n)
    th = rng.uniform(0, 2 * math.pi, n)
    x = np.column_stack([r * np.cos(th), r * np.sin(th)])
    return x[np.abs(x[:, 1]) >= 0.02]


@pytest.mark.parametrize("order", [1, 3])
def test_ring_agrees_with_plain_form_at_grid_nodes(order):
    N1, N2 = 64, 32
    h1, h2 = math.pi / N1, 1.0 / N2
    p = np.array([[5, 4], [-6, 5], [3, -9], [-2, -10], [7, 2]])        # r between 0.22 and 0.35
    x = p * [h1, h2]
    a = ho.eval_g2d_ho(K, AL, x, N1, N2, order)
    b = ho.eval_g2d_ho(K, AL, x, N1, N2, order, ring=True)
    assert np.all(ho.ring_zone(x[:, 0], x[:, 1], h1, h2))
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(a))


def test_ring_changes_only_ring_targets():
    N1, N2 = 64, 32
    h1, h2 = math.pi / N1, 1.0 / N2
    rng = np.random.default_rng(2)
    x = np.column_stack([rng.uniform(-math.pi, math.pi, 400), rng.uniform(-0.9, 0.9, 400)])
    a = ho.eval_g2d_ho(K, AL, x, N1, N2, 3)
    b = ho.eval_g2d_ho(K, AL, x, N1, N2, 3, ring=True)
    t = x[:, 0]
    near = np.abs(x[:, 1]) <= 0.6
    zone = near & ho.ring_zone(t, x[:, 1], h1, h2)
    assert zone.sum() > 5
    assert np.array_equal(a[~zone], b[~zone], equal_nan=True)
    # inside (eps, 2 eps) the target's own Y is fractional, so the two forms differ
    inner = zone & (np.hypot(t, x[:, 1]) < 0.4)
    assert inner.sum() > 3 and np.all(a[inner] != b[inner])


def test_ring_accuracy_against_the_series():
    """The ring's error falls by orders of magnitude and converges like the interpolation of a
    smooth function (about 16x per doubling of both axes)."""
    x = _ring_targets(120, seed=5)
    gt = truth.g2d(K, AL, x)
    err = {}
    for ring in (False, True):
        for N1, N2 in ((128, 64), (256, 128)):
            g = ho.eval_g2d_ho(K, AL, x, N1, N2, 3, ring=ring)
            err[ring, N1] = np.max(np.abs(g - gt) / np.abs(gt))
    assert err[True, 256] < err[False, 256] / 100
    assert err[True, 256] < 5e-6
    assert err[True, 256] < err[True, 128] / 10


# ----------------------------------------------------------------------------- the gradient (Section 2.4.1)

def test_grad_ring_agrees_with_plain_form_at_grid_nodes():
    from oracle import grad2d
    N1, N2 = 64, 32
    h1, h2 = math.pi / N1, 1.0 / N2
    p = np.array([[5, 4], [-6, 5], [3, -9], [-2, -10], [7, 2]])
    x = p * [h1, h2]
    a = grad2d.eval_g2d_grad(K, AL, x, N1, N2)
    b = grad2d.eval_g2d_grad(K, AL, x, N1, N2, ring=True)
    assert np.all(ho.ring_zone(x[:, 0], x[:, 1], h1, h2))
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(a))


def test_grad_ring_accuracy_against_the_series():
    from oracle import grad2d
    x = _ring_targets(120, seed=6, lo=0.15, hi=0.5)
    x = x[np.abs(x[:, 1]) <= 0.6]
    gt = truth.g2d_grad(K, AL, x)
    err = {}
    for ring in (False, True):
        for N1, N2 in ((128, 64), (256, 128)):
            g = grad2d.eval_g2d_grad(K, AL, x, N1, N2, ring=ring)
            err[ring, N1] = np.max(np.abs(g - gt) / np.abs(gt))
    assert err[True, 256] < err[False, 256] / 15
    assert err[True, 256] < 5e-5
    assert err[True, 256] < err[True, 128] / 8


# ----------------------------------------------------------------------------- second-derivative differences (Section 2.4.2)

def test_hess_ring_agrees_with_plain_form_at_grid_nodes():
    from oracle import hess2d
    N1, N2 = 64, 32
    h1, h2 = math.pi / N1, 1.0 / N2
    p = np.array([[5, 4], [-6, 5], [3, -9], [-2, -10], [7, 2]])
    x = p * [h1, h2]
    a = hess2d.eval_g2d_hess_diff(K, 4.35, AL, x, N1, N2)
    b = hess2d.eval_g2d_hess_diff(K, 4.35, AL, x, N1, N2, ring=True)
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(a))


def test_hess_ring_accuracy_against_the_series():
    from oracle import hess2d
    x = _ring_targets(100, seed=7, lo=0.15, hi=0.5)
    x = x[np.abs(x[:, 1]) <= 0.55]
    gt = truth.g2d_hess(K, AL, x) - truth.g2d_hess(4.35, AL, x)
    err = {}
    for ring in (False, True):
        for N1, N2 in ((128, 64), (256, 128)):
            g = hess2d.eval_g2d_hess_diff(K, 4.35, AL, x, N1, N2, ring=ring)
            err[ring, N1] = np.max(np.abs(g - gt) / np.abs(gt), axis=0)
    assert np.all(err[True, 256] < err[False, 256] / 15)
    assert np.all(err[True, 256] < 5e-5)
    assert np.all(err[True, 256] < err[True, 128] / 8)
