"""Pins of the gradient oracle (first derivatives of G, Section 2.4.1).

Each test compares the oracle with an independent route: the Hankel function of
scipy, brute-force polar quadrature of the defining Fourier integral, finite
differences of the pinned series for G, and the differentiated series itself.
"""

import math

import numpy as np
from scipy.special import hankel1

from oracle import cutoffs as co
from oracle import grad2d, method, truth

K2, AL2 = 2.1, 0.3


# ---------------------------------------------------------------- the singular parts h1, h2

def _annulus_residual(r0, k, alpha, printed_h2=False):
    """max |K_p - h_p - (best linear fit)| over an annulus r in [r0/2, r0], where
    K_p is e^{-i alpha x1} d/dx_p (i/4) H0(k|x|) by scipy's Hankel function."""
    th = np.linspace(0, 2 * math.pi, 48, endpoint=False) + 0.1
    R, TH = np.meshgrid(r0 * np.array([0.5, 0.7, 1.0]), th)
    r, th = R.ravel(), TH.ravel()
    t, z = r * np.cos(th), r * np.sin(th)
    dH = -(1j * k / 4) * hankel1(1, k * r) * np.exp(-1j * alpha * t)
    h1, h2 = grad2d.h_grad(k, alpha, t, z, printed_h2=printed_h2)
    out = []
    for D in (dH * t / r - h1, dH * z / r - h2):
        A = np.column_stack([np.ones_like(t), t, z]).astype(complex)
        c, *_ = np.linalg.lstsq(A, D, rcond=None)
        out.append(float(np.abs(D - A @ c).max()))
    return out


def test_h_grad_removes_the_hankel_singularity():
    # K_p - h_p = smooth + O(r^2 ln r): the non-linear remainder shrinks ~r^2 per decade.
    for k, al in ((K2, AL2), (7.3, -0.45)):
        e3, e4 = _annulus_residual(1e-3, k, al), _annulus_residual(1e-4, k, al)
        for a, b in zip(e3, e4):
            assert b < a / 40
        assert max(e4) < 1e-7 * max(1.0, k * k)


def test_h2_reading_x2_log_term():
    # As printed (x1 ln|x| in h2) the remainder keeps an |x| ln|x| term: ~10x per decade only.
    e3 = _annulus_residual(1e-3, K2, AL2, printed_h2=True)
    e4 = _annulus_residual(1e-4, K2, AL2, printed_h2=True)
    ours = _annulus_residual(1e-4, K2, AL2)
    assert e4[1] > e3[1] / 20
    assert e4[1] > 100 * ours[1]
    assert e4[0] == ours[0]                       # h1 is not affected


# ---------------------------------------------------------------- H-hat by brute force

def test_hhat_grad_against_polar_quadrature():
    """H-hat_{p,j} = A2 int h_p e^{-i eta.x} dx by tensor quadrature in (r, theta), no Bessel functions."""
    k, al, N1, N2 = K2, AL2, 8, 8
    H1, H2 = grad2d.hhat_grad_2d(k, al, N1, N2)
    A2 = 1.0 / (2.0 * math.sqrt(math.pi * co.C_TILDE))
    eps = co.EPS
    r0, w0 = method.gauss_legendre(0.0, eps, 300)
    r1, w1 = method.gauss_legendre(eps, 2 * eps, 300)
    r, w = np.concatenate([r0, r1]), np.concatenate([w0, w1])
    nth = 512
    th = 2 * math.pi * np.arange(nth) / nth
    R, TH = np.meshgrid(r, th, indexing="ij")
    t, z = R * np.cos(TH), R * np.sin(TH)
    h1, h2 = grad2d.h_grad(k, al, t, z)
    scale = max(np.abs(H1).max(), np.abs(H2).max())
    for j1, j2 in ((0, 0), (1, 0), (0, 1), (3, -2), (-7, 5), (7, 7), (-8, -8), (2, 3), (-8, 0), (0, -8)):
        E = np.exp(-1j * (j1 * t + j2 * math.pi / co.C_TILDE * z)) * R * (2 * math.pi / nth)
        b1 = A2 * np.sum((h1 * E).sum(1) * w)
        b2 = A2 * np.sum((h2 * E).sum(1) * w)
        assert abs(H1[j1 + N1, j2 + N2] - b1) < 1e-12 * scale, (j1, j2)
        assert abs(H2[j1 + N1, j2 + N2] - b2) < 1e-12 * scale, (j1, j2)


# ---------------------------------------------------------------- the differentiated series

def test_g2d_grad_series_against_finite_differences():
    x = np.array([[1.0, 0.3], [2.5, -0.7], [0.1, 0.05], [4.0, 0.9], [-0.3, -0.02]])
    g = truth.g2d_grad(K2, AL2, x)
    h = 1e-5
    for p, e in enumerate(np.eye(2)):
        fd = (truth.g2d(K2, AL2, x + h * e) - truth.g2d(K2, AL2, x - h * e)) / (2 * h)
        assert np.max(np.abs(g[:, p] - fd) / np.abs(g[:, p])) < 1e-7


def test_g2d_grad_series_symmetries():
    x = np.array([[1.0, 0.3], [2.5, 0.7], [0.1, 0.05]])
    g = truth.g2d_grad(K2, AL2, x)
    # quasi-periodic in x1
    gs = truth.g2d_grad(K2, AL2, x + [2 * math.pi, 0.0])
    assert np.allclose(gs, np.exp(2j * math.pi * AL2) * g, rtol=1e-12, atol=0)
    # G is even in x2: dG/dx1 even, dG/dx2 odd
    gm = truth.g2d_grad(K2, AL2, x * [1.0, -1.0])
    assert np.allclose(gm[:, 0], g[:, 0], rtol=1e-13, atol=0)
    assert np.allclose(gm[:, 1], -g[:, 1], rtol=1e-13, atol=0)


def test_far_branch_is_the_differentiated_series():
    # Section 2.4.1 / Algorithm 2.1 step 2b: beyond |x2| = c the derivatives are those of the series
    # (1.2) itself; at |x2| = c the target is near (the method's grid, which differs from the series).
    x = np.array([[0.3, 0.7], [2.0, -0.95], [5.0, 0.61], [1.1, -0.8]])
    np.testing.assert_array_equal(grad2d.eval_g2d_grad(K2, AL2, x, 64, 32), truth.g2d_grad(K2, AL2, x))
    xb = np.array([[0.3, 0.6], [0.3, -0.6]])
    assert np.all(grad2d.eval_g2d_grad(K2, AL2, xb, 64, 32) != truth.g2d_grad(K2, AL2, xb))


def test_g2d_grad_method_converges_to_truth():
    rng = np.random.default_rng(0)
    x = np.column_stack([rng.uniform(-math.pi, math.pi, 24),
                         rng.uniform(0.05, 0.55, 24) * rng.choice([-1.0, 1.0], 24)])
    # near the lattice point, inside and across the cut-off ring eps < r < 2 eps
    x = np.vstack([x, [[0.1, 0.06], [-0.2, -0.1], [0.05, 0.3], [0.0, 0.08], [0.27, -0.12]]])
    gt = truth.g2d_grad(K2, AL2, x)
    errs, meds = [], []
    for N1, N2 in ((64, 32), (128, 64)):
        g = grad2d.eval_g2d_grad(K2, AL2, x, N1, N2)
        e = np.abs(g - gt) / np.abs(gt)
        errs.append(e.max())
        meds.append(np.median(e))
    assert errs[0] < 0.5 and errs[1] < 5e-3 and errs[1] < errs[0] / 20
    assert meds[1] < 1e-4
