"""Pins of the second-derivative-difference oracle (T_pq for two wavenumbers, Section 2.4.2).

Independent routes: scipy's Hankel functions for the singular parts, brute-force polar
quadrature of the defining Fourier integral, finite differences of the (pinned) gradient
series, the Helmholtz equation, and the twice-differentiated series itself.
"""

import math

import numpy as np
from scipy.special import hankel1

from oracle import cutoffs as co
from oracle import hess2d, method, truth

K1, K2, AL = 2.1, 3.4, 0.3


def _d2_hankel(k, t, z):
    """d_p d_q H0(k r) for pq = 11, 12, 22 (H0' = -H1, H1' = (H0 - H2)/2)."""
    r = np.hypot(t, z)
    X = (t, z)
    H0, H1, H2 = (hankel1(n, k * r) for n in range(3))
    out = []
    for p, q in hess2d.PAIRS:
        d = 1.0 if p == q else 0.0
        out.append(-k * ((k / 2) * (H0 - H2) * X[p] * X[q] / r ** 2 + H1 * (d / r - X[p] * X[q] / r ** 3)))
    return out


def _annulus_residual(r0, k1, k2, alpha, printed_sign=False):
    """max |T_pq - h_pq - (best linear fit)| on the annulus r in [r0/2, r0], T_pq from Hankel functions."""
    th = np.linspace(0, 2 * math.pi, 48, endpoint=False) + 0.1
    R, TH = np.meshgrid(r0 * np.array([0.5, 0.7, 1.0]), th)
    r, th = R.ravel(), TH.ravel()
    t, z = r * np.cos(th), r * np.sin(th)
    e = np.exp(-1j * alpha * t)
    A, B = _d2_hankel(k1, t, z), _d2_hankel(k2, t, z)
    hs = hess2d.h_hess_diff(k1, k2, alpha, t, z, printed_sign=printed_sign)
    out = []
    for p in range(3):
        D = e * 0.25j * (A[p] - B[p]) - hs[p]
        M = np.column_stack([np.ones_like(t), t, z]).astype(complex)
        c, *_ = np.linalg.lstsq(M, D, rcond=None)
        out.append(float(np.abs(D - M @ c).max()))
    return out


def test_h_hess_diff_removes_the_hankel_singularity():
    # T_pq - h_pq = smooth + O(r^2 ln r): the non-linear remainder shrinks ~r^2 per decade.
    for k1, k2, al in ((K1, K2, AL), (6.0, 1.3, -0.45)):
        e3, e4 = _annulus_residual(1e-3, k1, k2, al), _annulus_residual(1e-4, k1, k2, al)
        for a, b in zip(e3, e4):
            assert b < a / 40
        assert max(e4) < 1e-8 * abs(k1 ** 4 - k2 ** 4)      # the remainder carries k^4 r^2 ln r


def test_sign_reading_of_the_singular_parts():
    # With the printed minus sign T - h keeps twice the singular part: the residual does not decay.
    ours = _annulus_residual(1e-4, K1, K2, AL)
    e3 = _annulus_residual(1e-3, K1, K2, AL, printed_sign=True)
    e4 = _annulus_residual(1e-4, K1, K2, AL, printed_sign=True)
    for p in range(3):
        assert e4[p] > 0.5 * e3[p] and e4[p] > 1e5 * ours[p]


def test_hhat_hess_diff_against_polar_quadrature():
    """H-hat_pq = A2 int h_pq e^{-i eta.x} dx by tensor quadrature in (r, theta), no Bessel functions."""
    N1 = N2 = 8
    H = hess2d.hhat_hess_diff(K1, K2, AL, N1, N2)
    A2 = 1.0 / (2.0 * math.sqrt(math.pi * co.C_TILDE))
    eps = co.EPS
    u, wu = method.gauss_legendre(0.0, 1.0, 300)            # r = eps u^2 on [0, eps]: ln r integrable to rounding
    r0, w0 = eps * u * u, wu * 2 * eps * u
    r1, w1 = method.gauss_legendre(eps, 2 * eps, 300)
    r, w = np.concatenate([r0, r1]), np.concatenate([w0, w1])
    nth = 512
    th = 2 * math.pi * np.arange(nth) / nth
    R, TH = np.meshgrid(r, th, indexing="ij")
    t, z = R * np.cos(TH), R * np.sin(TH)
    hs = hess2d.h_hess_diff(K1, K2, AL, t, z)
    scale = max(np.abs(h).max() for h in H)
    for j1, j2 in ((0, 0), (1, 0), (0, 1), (3, -2), (-7, 5), (7, 7), (-8, -8), (2, 3), (-8, 0), (0, -8)):
        E = np.exp(-1j * (j1 * t + j2 * math.pi / co.C_TILDE * z)) * R * (2 * math.pi / nth)
        for p in range(3):
            b = A2 * np.sum((hs[p] * E).sum(1) * w)
            assert abs(H[p][j1 + N1, j2 + N2] - b) < 1e-12 * scale, (p, j1, j2)


def test_g2d_hess_series_against_gradient_and_helmholtz():
    x = np.array([[1.0, 0.3], [2.5, -0.7], [0.1, 0.05], [-0.3, -0.02]])
    H = truth.g2d_hess(K1, AL, x)
    h = 1e-5
    for p, (i, j) in enumerate(hess2d.PAIRS):
        e = np.eye(2)[j]
        fd = (truth.g2d_grad(K1, AL, x + h * e)[:, i] - truth.g2d_grad(K1, AL, x - h * e)[:, i]) / (2 * h)
        assert np.max(np.abs(H[:, p] - fd) / np.abs(H[:, p])) < 1e-7
    G = truth.g2d(K1, AL, x)
    assert np.max(np.abs(H[:, 0] + H[:, 2] + K1 * K1 * G) / np.abs(H[:, 0])) < 1e-13
    Hm = truth.g2d_hess(K1, AL, x * [1.0, -1.0])
    assert np.allclose(Hm[:, [0, 2]], H[:, [0, 2]], rtol=1e-13, atol=0)
    assert np.allclose(Hm[:, 1], -H[:, 1], rtol=1e-13, atol=0)


def test_far_branch_is_the_twice_differentiated_series():
    # Section 2.4.2 / Algorithm 2.1 step 2b: beyond |x2| = c, the second derivatives of the series (1.2)
    # for both wavenumbers; at |x2| = c the target is near.
    x = np.array([[0.3, 0.7], [2.0, -0.95], [5.0, 0.61], [1.1, -0.8]])
    gt = truth.g2d_hess(K1, AL, x) - truth.g2d_hess(K2, AL, x)
    np.testing.assert_array_equal(hess2d.eval_g2d_hess_diff(K1, K2, AL, x, 64, 32), gt)
    xb = np.array([[0.3, 0.6], [0.3, -0.6]])
    gb = truth.g2d_hess(K1, AL, xb) - truth.g2d_hess(K2, AL, xb)
    assert np.all(hess2d.eval_g2d_hess_diff(K1, K2, AL, xb, 64, 32) != gb)


def test_hess_diff_method_converges_to_truth():
    rng = np.random.default_rng(0)
    x = np.column_stack([rng.uniform(-math.pi, math.pi, 24),
                         rng.uniform(0.05, 0.55, 24) * rng.choice([-1.0, 1.0], 24)])
    x = np.vstack([x, [[0.1, 0.06], [-0.2, -0.1], [0.05, 0.3], [0.0, 0.08], [0.27, -0.12]]])
    gt = truth.g2d_hess(K1, AL, x) - truth.g2d_hess(K2, AL, x)
    errs, meds = [], []
    for N1, N2 in ((64, 32), (128, 64)):
        g = hess2d.eval_g2d_hess_diff(K1, K2, AL, x, N1, N2)
        e = np.abs(g - gt) / np.abs(gt)
        errs.append(e.max(axis=0))
        meds.append(np.median(e, axis=0))
    # every component converges fast; T22 is limited by the x2 truncation X near |x2| = c
    assert np.all(errs[1] < errs[0] / 5) and np.all(meds[1] < meds[0] / 50)
    assert errs[1][0] < 1e-3 and errs[1][1] < 5e-3 and errs[1][2] < 3e-2
