"""Pins of the oracle at the special coefficients of Sections 2.1 / 3.1 (beta = -+ j pi / c~),
where the integration by parts behind (2.1) / (3.3) divides by zero and the coefficient is
taken from its defining integral (the paper's special-case formula) instead.

Routes: adaptive quadrature of the defining integrals, spherical quadrature of the 3D
singular part's transform, the integrated form away from the special point, and the
lattice sum at an exactly special instance.
"""

import math

import numpy as np
from scipy import integrate

from oracle import cutoffs as co
from oracle import method, truth

AL2 = 0.3
K2S = math.sqrt(AL2 ** 2 + math.pi ** 2)              # beta_{j1=0} = pi = J for j2 = 1: exactly special
A31, A32 = 0.2, 0.35
K3S = math.sqrt(A31 ** 2 + A32 ** 2 + math.pi ** 2)   # beta_{00} = pi = J for j3 = 1


def _cquad(f, a, b):
    re = integrate.quad(lambda x: f(x).real, a, b, limit=400, epsabs=1e-15, epsrel=1e-14)[0]
    im = integrate.quad(lambda x: f(x).imag, a, b, limit=400, epsabs=1e-15, epsrel=1e-14)[0]
    return re + 1j * im


def _defining(b, J, A):
    """A (i / (2 beta)) int_0^{c~} [e^{i(beta-J)x} + e^{i(beta+J)x}] X(x) dx (before any integration by parts)."""
    val = _cquad(lambda x: (np.exp(1j * (b - J) * x) + np.exp(1j * (b + J) * x)) * co.X(x), 0, 1)
    return A * 1j / (2 * b) * val


def test_khat_2d_at_special_coefficients():
    N1, N2 = 4, 3
    Kh = method.khat_2d(K2S, AL2, N1, N2)
    assert np.all(np.isfinite(Kh))
    A2 = 1 / (2 * math.sqrt(math.pi))
    for j1, j2 in ((0, 1), (0, -1), (1, 1), (-2, 0), (0, 0)):
        ref = _defining(truth.beta(K2S, AL2 + j1), j2 * math.pi, A2)
        assert abs(Kh[j1 + N1, j2 + N2] - ref) < 1e-12 * max(1, abs(ref)), (j1, j2)


def test_khat_3d_at_special_coefficients():
    N = 3
    Kh = method.khat_3d(K3S, A31, A32, N, N, N)
    assert np.all(np.isfinite(Kh))
    A3 = 1 / math.sqrt(8 * math.pi ** 2)
    for j in ((0, 0, 1), (0, 0, -1), (1, 0, 1), (0, 0, 0)):
        b = truth.beta(K3S, math.hypot(A31 + j[0], A32 + j[1]))
        ref = _defining(b, j[2] * math.pi, A3)
        assert abs(Kh[j[0] + N, j[1] + N, j[2] + N] - ref) < 1e-12 * max(1, abs(ref)), j


def test_direct_and_integrated_forms_agree_off_the_special_point():
    # |beta - J| = 0.05, outside the switch: the integration by parts of (2.1) and the direct integral
    a = AL2
    k = math.sqrt(a * a + (math.pi + 0.05) ** 2)
    b = truth.beta(k, np.array([a]))
    J = np.array([math.pi])
    Im, Ip = method.xprime_integrals(b, J)
    A2 = 1 / (2 * math.sqrt(math.pi))
    by_parts = method._coef_K(A2, k, b[:, None], J[None, :], a * a + J[None, :] ** 2 - k * k, Im, Ip)[0, 0]
    direct = A2 * 1j / (2 * b[0]) * (method.x_integral(b[0] - J[0]) + method.x_integral(b[0] + J[0]))
    assert abs(by_parts - direct) < 1e-13 * abs(direct)


def test_fhat_3d_at_special_coefficients_against_spherical_quadrature():
    # |xi| = k at the special coefficient: (1 - H)/(|xi|^2 - k^2) is 0/0 there
    N = 3
    Fh = method.fhat_3d(K3S, A31, A32, N, N, N)
    assert np.all(np.isfinite(Fh))
    A3 = 1 / math.sqrt(8 * math.pi ** 2)
    r, wr = method.gauss_legendre(0.0, 2 * co.EPS, 400)
    mu, wm = method.gauss_legendre(-1.0, 1.0, 200)
    for j in ((0, 0, 1), (0, 0, -1), (1, -2, 1)):
        xi = math.sqrt((A31 + j[0]) ** 2 + (A32 + j[1]) ** 2 + (j[2] * math.pi) ** 2)
        R, MU = np.meshgrid(r, mu, indexing="ij")
        integrand = np.exp(1j * K3S * R) / (4 * math.pi * R) * co.Y(R) * np.exp(-1j * xi * R * MU) * R * R
        ref = A3 * 2 * math.pi * np.sum(wr[:, None] * wm[None, :] * integrand)
        assert abs(Fh[j[0] + N, j[1] + N, j[2] + N] - ref) < 1e-11 * max(1, abs(ref)), j


def test_method_at_a_special_instance_converges_to_truth():
    rng = np.random.default_rng(3)
    x = np.stack([rng.uniform(0, 2 * math.pi, 16), rng.uniform(-1, 1, 16)], 1)
    x = x[np.abs(x[:, 1]) > 0.02]
    gt = truth.g2d(K2S, AL2, x)
    errs = []
    for N1, N2 in ((128, 32), (256, 64)):
        hf = 1.0 / N2
        g = method.eval_g2d(K2S, AL2, x, N1, N2)
        errs.append(np.max(np.abs(g - gt) / np.abs(gt)))
    assert errs[0] < 5e-3 and errs[1] < errs[0] / 4 and errs[1] < 1e-3
