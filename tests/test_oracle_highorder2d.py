"""Pins of the higher-order 2D oracle (Remark 5.3: more of the logarithmic singularity removed).

Independent routes: scipy's Hankel function for the remainder K - f^(m) near the lattice
point, brute-force polar quadrature of the defining Fourier integral of the removed terms,
and the eigenfunction series (1.2) for the converged values.
"""

import math

import numpy as np
import pytest
from scipy.special import hankel1

from oracle import cutoffs as co
from oracle import highorder2d as ho
from oracle import method, truth

K, AL = 2.1, 0.3


def _remainder(r0, k, alpha, order):
    """max |K - f^(m) - (best cubic polynomial)| over an annulus r in [r0/2, r0] (Y = 1 there),
    K = e^{-i alpha t} (i/4) H0(k r) by scipy.  What is left is the non-analytic remainder."""
    th = np.linspace(0, 2 * math.pi, 64, endpoint=False) + 0.1
    R, TH = np.meshgrid(r0 * np.array([0.5, 0.6, 0.75, 0.9, 1.0]), th)
    r, th = R.ravel(), TH.ravel()
    t, z = r * np.cos(th), r * np.sin(th)
    Kx = np.exp(-1j * alpha * t) * 0.25j * hankel1(0, k * r)
    D = Kx - ho.f_removed(k, alpha, t, z, order)
    u, v = t / r0, z / r0                       # scaled, so the fit stays well conditioned
    M = np.column_stack([u ** a * v ** b for a in range(4) for b in range(4 - a)]).astype(complex)
    c, *_ = np.linalg.lstsq(M, D, rcond=None)
    return float(np.abs(D - M @ c).max())


@pytest.mark.parametrize("k,alpha", [(K, AL), (7.3, -0.45), (3.0, 1.3)])
def test_remainder_order_per_removed_degree(k, alpha):
    # K - f^(m) = analytic + O(r^{m+1} ln r): a decade in r takes ~10^{m+1} off the remainder
    # (a wrong sign or a dropped term of P_m leaves a lower power).
    for order, lo in ((1, 50), (2, 500), (3, 5000)):
        e2, e3 = _remainder(1e-2, k, alpha, order), _remainder(1e-3, k, alpha, order)
        assert e3 < e2 / lo, (order, e2, e3)
        assert e2 / e3 < 20 * lo, (order, e2, e3)


def test_order_one_is_algorithm_2_1():
    x = np.array([[0.1, 0.05], [-0.2, 0.3], [2.0, -0.4], [0.5, 0.8], [1.0, -0.9]])
    a = ho.eval_g2d_ho(K, AL, x, 32, 16, 1)
    b = method.eval_g2d(K, AL, x, 32, 16)
    assert np.array_equal(a, b)


def test_ehat_against_polar_quadrature():
    """E-hat^(3) = A2 int (f^(3) - f^(1)) e^{-i eta.x} dx by tensor quadrature in (r, theta)."""
    N1 = N2 = 8
    k, al = 5.0, 0.45
    E = ho.ehat(k, al, N1, N2, 3)
    A2 = 1.0 / (2.0 * math.sqrt(math.pi * co.C_TILDE))
    eps = co.EPS
    u, wu = method.gauss_legendre(0.0, 1.0, 300)            # r = eps u^2 on [0, eps]
    r0, w0 = eps * u * u, wu * 2 * eps * u
    r1, w1 = method.gauss_legendre(eps, 2 * eps, 300)
    r, w = np.concatenate([r0, r1]), np.concatenate([w0, w1])
    nth = 512
    th = 2 * math.pi * np.arange(nth) / nth
    R, TH = np.meshgrid(r, th, indexing="ij")
    t, z = R * np.cos(TH), R * np.sin(TH)
    g = ho.f_removed(k, al, t, z, 3) - ho.f_removed(k, al, t, z, 1)
    scale = np.abs(E).max()
    for j1, j2 in ((0, 0), (1, 0), (0, 1), (3, -2), (-7, 5), (7, 7), (-8, -8), (2, 3), (-8, 0), (0, -8)):
        ph = np.exp(-1j * (j1 * t + j2 * math.pi / co.C_TILDE * z)) * R * (2 * math.pi / nth)
        b = A2 * np.sum((g * ph).sum(1) * w)
        assert abs(E[j1 + N1, j2 + N2] - b) < 1e-12 * scale, (j1, j2)
    # order 2 keeps only the degree-2 terms: the difference is the degree-3 part
    g2 = ho.f_removed(k, al, t, z, 3) - ho.f_removed(k, al, t, z, 2)
    E2 = ho.ehat(k, al, N1, N2, 2)
    for j1, j2 in ((1, 0), (3, -2), (-7, 5)):
        ph = np.exp(-1j * (j1 * t + j2 * math.pi / co.C_TILDE * z)) * R * (2 * math.pi / nth)
        b = A2 * np.sum((g2 * ph).sum(1) * w)
        assert abs(E[j1 + N1, j2 + N2] - E2[j1 + N1, j2 + N2] - b) < 1e-12 * scale, (j1, j2)


def _near_source_targets():
    return np.array([[0.0, 0.003], [0.001, 0.005], [-0.002, 0.008], [0.0, 0.012], [0.004, -0.02]])


def test_higher_order_converges_faster_near_the_lattice_point():
    """Against the series (1.2): near the lattice point the remainder's coefficient tail
    sets the error; removing the degree-2 and -3 terms lowers it by orders of magnitude."""
    x = _near_source_targets()
    gt = truth.g2d(K, AL, x, max_terms=200_000_000)
    err = {}
    for order in (1, 3):
        for N1, N2 in ((128, 64), (256, 128)):
            g = ho.eval_g2d_ho(K, AL, x, N1, N2, order)
            err[order, N1] = np.abs(g - gt).max()
    assert err[3, 128] < err[1, 128] / 10
    assert err[3, 256] < err[1, 256] / 100
    assert err[3, 256] < 3e-8
    assert err[3, 256] < err[3, 128] / 16


def test_higher_order_elsewhere_no_worse():
    rng = np.random.default_rng(0)
    x = np.column_stack([rng.uniform(-math.pi, math.pi, 60),
                         rng.uniform(0.02, 0.55, 60) * rng.choice([-1.0, 1.0], 60)])
    x = np.vstack([x, [[1.0, 0.8], [-2.0, -0.7]]])                 # two far-branch targets
    gt = truth.g2d(K, AL, x)
    e1 = np.abs(ho.eval_g2d_ho(K, AL, x, 128, 64, 1) - gt) / np.abs(gt)
    e3 = np.abs(ho.eval_g2d_ho(K, AL, x, 128, 64, 3) - gt) / np.abs(gt)
    assert np.median(e3) <= 1.05 * np.median(e1) and e3.max() <= 1.05 * e1.max()
    assert np.array_equal(e1[-2:], e3[-2:])
