"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these re-type an oracle formula: each compares the oracle with an
independent route to the same number (a different closed form, brute-force
quadrature of a defining integral, a different series, a PDE identity, or the
paper's own printed errors).
"""

import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import hankel1

from oracle import cutoffs as co
from oracle import method, truth

K2, AL2 = 2.1, 0.3                  # 2D instance of the small workload
K3, A31, A32 = 3.7, 0.2, 0.35       # 3D instance


# ---------------------------------------------------------------- cut-offs (Section 6: C^8)

def test_smoothstep_matches_binomial_closed_form():
    # I_u(9,9) equals the Bernstein sum sum_{j=9}^{17} C(17,j) u^j (1-u)^{17-j}.
    u = np.linspace(0.0, 1.0, 41)
    bern = sum(math.comb(17, j) * u ** j * (1 - u) ** (17 - j) for j in range(9, 18))
    np.testing.assert_allclose(co.smoothstep(u), bern, atol=1e-15)


def test_smoothstep_derivatives_by_finite_differences():
    u = np.linspace(0.05, 0.95, 19)
    h = 1e-5
    fd1 = (co.smoothstep(u + h) - co.smoothstep(u - h)) / (2 * h)
    np.testing.assert_allclose(co.smoothstep_d1(u), fd1, rtol=1e-8, atol=1e-9)
    fd2 = (co.smoothstep_d1(u + h) - co.smoothstep_d1(u - h)) / (2 * h)
    np.testing.assert_allclose(co.smoothstep_d2(u), fd2, rtol=1e-7, atol=1e-7)


def test_cutoff_plateaus_and_c8_contact():
    t = np.array([0.0, 0.3, 0.6, 0.8, 0.95, -0.5, -0.9])
    np.testing.assert_array_equal(co.X(t), [1, 1, 1, 0, 0, 1, 0])
    r = np.array([0.0, 0.1, 0.2, 0.4, 0.7])
    np.testing.assert_array_equal(co.Y(r), [1, 1, 1, 0, 0])
    # C^8 contact: S' ~ u^8 near 0 so S'(2u)/S'(u) -> 2^8.
    assert abs(co.smoothstep_d1(2e-6) / co.smoothstep_d1(1e-6) - 2 ** 8) < 0.01
    assert co.smoothstep(0.5) == pytest.approx(0.5, abs=1e-15)


# ---------------------------------------------------------------- the truth series (1.2), (1.3)

def test_beta_branch():
    a = np.array([-5.0, -2.0, 0.0, 1.5, 2.0, 7.0])
    b = truth.beta(K2, a)
    assert np.all(b.imag >= 0)
    np.testing.assert_allclose(b * b, K2 ** 2 - a ** 2, rtol=1e-14, atol=1e-14)
    assert np.all(b[np.abs(a) <= K2].real > 0)


def test_g2d_quasi_periodic_and_even():
    x = np.array([[0.4, 0.3], [2.0, -0.05], [-1.0, 0.7]])
    g = truth.g2d(K2, AL2, x)
    g_shift = truth.g2d(K2, AL2, x + [2 * math.pi, 0.0])
    np.testing.assert_allclose(g_shift, np.exp(2j * math.pi * AL2) * g, rtol=1e-13)
    np.testing.assert_allclose(truth.g2d(K2, AL2, x * [1, -1]), g, rtol=1e-14)


def test_g2d_helmholtz_residual():
    x0 = np.array([1.1, 0.35])
    h = 1e-3
    pts = np.array([x0, x0 + [h, 0], x0 - [h, 0], x0 + [0, h], x0 - [0, h]])
    g = truth.g2d(K2, AL2, pts)
    lap = (g[1] + g[2] + g[3] + g[4] - 4 * g[0]) / h ** 2
    assert abs(lap + K2 ** 2 * g[0]) / abs(K2 ** 2 * g[0]) < 1e-5


def test_g2d_eigen_equals_images_for_complex_k():
    # (1.1) and (1.2) are the same function; with Im k > 0 both converge fast.
    k = 2.1 + 0.9j
    x = np.array([[0.5, 0.2], [2.5, -0.4], [-1.0, 0.05]])
    eig = truth.g2d(k, AL2, x)
    img = truth.g2d_images(k, AL2, x, nmax=60)
    np.testing.assert_allclose(eig, img, rtol=1e-10)


def test_gd3d_quasi_periodic():
    x = np.array([[0.4, 1.3, 0.3], [2.0, -0.5, -0.2]])
    g = truth.gd3d(K3, A31, A32, x)
    g1 = truth.gd3d(K3, A31, A32, x + [2 * math.pi, 0, 0])
    g2 = truth.gd3d(K3, A31, A32, x + [0, -2 * math.pi, 0])
    np.testing.assert_allclose(g1, np.exp(2j * math.pi * A31) * g, rtol=1e-12)
    np.testing.assert_allclose(g2, np.exp(-2j * math.pi * A32) * g, rtol=1e-12)


def test_gd3d_eigen_equals_images_for_complex_k():
    k = 3.7 + 1.2j
    x = np.array([[0.3, 0.4, 0.3], [2.0, -1.0, -0.5]])
    eig = truth.gd3d(k, A31, A32, x)
    img = truth.gd3d_images(k, A31, A32, x, nmax=12)
    np.testing.assert_allclose(eig, img, rtol=1e-10)


def test_gd3d_helmholtz_residual():
    x0 = np.array([0.7, -0.4, 0.45])
    h = 2e-3
    offs = [np.zeros(3)] + [s * h * np.eye(3)[i] for i in range(3) for s in (1, -1)]
    g = truth.gd3d(K3, A31, A32, np.array([x0 + o for o in offs]))
    lap = (g[1:].sum() - 6 * g[0]) / h ** 2
    assert abs(lap + K3 ** 2 * g[0]) / abs(K3 ** 2 * g[0]) < 1e-5


def test_maxwell_hessian_by_finite_differences_and_divergence_free():
    x0 = np.array([0.7, -0.4, 0.45])
    h = 1e-3
    e = np.eye(3)
    hes = truth.gd3d_hessian(K3, A31, A32, x0[None])[0]
    idx = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (0, 2): 4, (1, 2): 5}
    for (p, q), i in idx.items():
        pts = np.array([x0 + h * e[p] + h * e[q], x0 + h * e[p] - h * e[q],
                        x0 - h * e[p] + h * e[q], x0 - h * e[p] - h * e[q]])
        g = truth.gd3d(K3, A31, A32, pts)
        fd = (g[0] - g[1] - g[2] + g[3]) / (4 * h * h)
        assert abs(fd - hes[i]) / abs(hes).max() < 1e-5, (p, q)
    # div GG = grad G + k^-2 grad(Lap G) = 0 away from the lattice.
    def tensor(x):
        t = truth.maxwell3d(K3, A31, A32, x[None])[0]
        T = np.empty((3, 3), complex)
        for (p, q), i in idx.items():
            T[p, q] = T[q, p] = t[i]
        return T
    div = np.zeros(3, complex)
    for p in range(3):
        div += (tensor(x0 + h * e[p])[p] - tensor(x0 - h * e[p])[p]) / (2 * h)
    scale = np.abs(tensor(x0)).max()
    assert np.abs(div).max() / scale < 1e-4


# ---------------------------------------------------------------- coefficient formulas

def _cquad(f, a, b):
    re = integrate.quad(lambda x: f(x).real, a, b, epsabs=1e-16, epsrel=1e-14, limit=400)[0]
    im = integrate.quad(lambda x: f(x).imag, a, b, epsabs=1e-16, epsrel=1e-14, limit=400)[0]
    return complex(re, im)


def test_maxwell_trace_identity():
    # GG_11 + GG_22 + GG_33 = 3 G_d + k^-2 Laplacian G_d = 2 G_d off the lattice (the Helmholtz
    # equation): the identity the method uses for GG_33, on the lattice sums themselves.
    x = np.array([[0.9, -0.7, 0.3], [2.0, 1.0, 0.8], [0.5, 0.4, -0.7], [4.0, 5.5, 0.05]])
    gg = truth.maxwell3d(K3, A31, A32, x)
    g = truth.gd3d(K3, A31, A32, x)
    assert np.max(np.abs(gg[:, 0] + gg[:, 1] + gg[:, 2] - 2 * g) / np.abs(g)) < 1e-11


def test_xprime_integrals_against_adaptive_quadrature():
    b = np.array([1.3, 0.0 + 4.0j, 3.7])
    J = np.array([0.0, math.pi, 7 * math.pi])
    Im, Ip = method.xprime_integrals(b, J)
    for i, bb in enumerate(b):
        for j, jj in enumerate(J):
            for sgn, got in ((-1, Im[i, j]), (1, Ip[i, j])):
                g = bb + sgn * jj
                ref = _cquad(lambda x: np.exp(1j * g * x) * co.dX(x), co.C, 0.5 * (co.C + co.C_TILDE))
                assert abs(got - ref) < 1e-13




def test_khat_2d_against_defining_integral():
    # K-hat_j = i/(4 sqrt(pi c~)) beta^-1 int_0^{c~} [e^{i(beta-J)x} + e^{i(beta+J)x}] X(x) dx
    # (Section 2.1, before the integration by parts that gives 2.1).
    N1, N2 = 4, 3
    Kh = method.khat_2d(K2, AL2, N1, N2)
    for j1 in (-4, -2, 0, 1, 3):
        for j2 in (-3, 0, 2):
            b = truth.beta(K2, AL2 + j1)
            J = j2 * math.pi
            val = _cquad(lambda x: (np.exp(1j * (b - J) * x) + np.exp(1j * (b + J) * x)) * co.X(x), 0, 1)
            ref = 1j / (4 * math.sqrt(math.pi)) / b * val
            assert abs(Kh[j1 + N1, j2 + N2] - ref) < 1e-12 * max(1, abs(ref))


def test_khat_3d_against_defining_integral():
    N = 3
    Kh = method.khat_3d(K3, A31, A32, N, N, N)
    for j in [(0, 0, 0), (1, -2, 1), (-3, 2, -2), (2, 2, 0)]:
        b = truth.beta(K3, math.hypot(A31 + j[0], A32 + j[1]))
        J = j[2] * math.pi
        val = _cquad(lambda x: (np.exp(1j * (b - J) * x) + np.exp(1j * (b + J) * x)) * co.X(x), 0, 1)
        ref = 1j / (2 * math.sqrt(8 * math.pi ** 2)) / b * val
        got = Kh[j[0] + N, j[1] + N, j[2] + N]
        assert abs(got - ref) < 1e-12 * max(1, abs(ref)), j


def _polar_coef(f, eta1, eta2, eps):
    """int f(x) e^{-i eta.x} dx over the disc |x| < 2 eps, polar Gauss-Legendre x trapezoid."""
    nth = 256
    th = 2 * math.pi * np.arange(nth) / nth
    s, ws = method.gauss_legendre(0.0, math.sqrt(2 * eps), 400)     # r = s^2 removes r ln r
    r = s * s
    R, TH = np.meshgrid(r, th, indexing="ij")
    x1, x2 = R * np.cos(TH), R * np.sin(TH)
    val = f(x1, x2, R) * np.exp(-1j * (eta1 * x1 + eta2 * x2)) * R * (2 * s)[:, None]
    return np.sum(ws[:, None] * val) * (2 * math.pi / nth)


def test_fhat_2d_against_brute_force_quadrature():
    # F-hat_{1,j} = int f1 phi_{-j}, f1 = -(1/2pi) ln|x| Y; f2 = x1 f1 (Section 2.2).
    N1, N2 = 6, 4
    F1, F2 = method.fhat_2d(N1, N2)
    A2 = 1 / (2 * math.sqrt(math.pi))
    f1 = lambda x1, x2, r: -np.log(r) * co.Y(r) / (2 * math.pi)
    f2 = lambda x1, x2, r: x1 * f1(x1, x2, r)
    for j1, j2 in [(0, 0), (1, 0), (0, 1), (-3, 2), (5, -4), (-6, 3)]:
        e1, e2 = j1, j2 * math.pi
        r1 = A2 * _polar_coef(f1, e1, e2, co.EPS)
        r2 = A2 * _polar_coef(f2, e1, e2, co.EPS)
        assert abs(F1[j1 + N1, j2 + N2] - r1) < 1e-11, (j1, j2)
        assert abs(F2[j1 + N1, j2 + N2] - r2) < 1e-11, (j1, j2)


def test_radial_H_is_one_on_the_sphere_rho_equals_k():
    # F-hat = A3 (1 - H)/(|xi|^2 - k^2) must stay finite at |xi| = k (F has compact support).
    for k in (1.0, 3.7, 12.5):
        assert abs(method.radial_H(k, np.array([k]))[0] - 1.0) < 1e-13


def test_fhat_3d_against_spherical_quadrature():
    # F-hat_j = A3 int e^{-i alpha.x'} e^{ik|x|}/(4 pi |x|) Y(|x|) e^{-i(j1 x1 + j2 x2 + J x3)} dx
    # computed in spherical coordinates about xi (no use of the Green-identity form 3.5).
    N = 3
    Fh = method.fhat_3d(K3, A31, A32, N, N, N)
    A3 = 1 / math.sqrt(8 * math.pi ** 2)
    r, wr = method.gauss_legendre(0.0, 2 * co.EPS, 400)
    mu, wm = method.gauss_legendre(-1.0, 1.0, 200)
    for j in [(0, 0, 0), (1, -2, 1), (-3, 2, -2), (2, 0, -3)]:
        xi = math.sqrt((A31 + j[0]) ** 2 + (A32 + j[1]) ** 2 + (j[2] * math.pi) ** 2)
        R, MU = np.meshgrid(r, mu, indexing="ij")
        integrand = np.exp(1j * K3 * R) / (4 * math.pi * R) * co.Y(R) * np.exp(-1j * xi * R * MU) * R * R
        ref = A3 * 2 * math.pi * np.sum(wr[:, None] * wm[None, :] * integrand)
        got = Fh[j[0] + N, j[1] + N, j[2] + N]
        assert abs(got - ref) < 1e-11 * max(1, abs(ref)), j


# ---------------------------------------------------------------- DFT and interpolation

def test_grid_2d_single_mode():
    N1, N2 = 8, 4
    L = np.zeros((2 * N1, 2 * N2), complex)
    L[3 + N1, -2 + N2] = 1.0
    g = method.grid_2d(L)
    p = np.arange(-N1, N1)[:, None] * math.pi / N1
    q = np.arange(-N2, N2)[None, :] * 1.0 / N2
    ref = np.exp(1j * (3 * p - 2 * math.pi * q)) / (2 * math.sqrt(math.pi))
    np.testing.assert_allclose(g, ref, atol=1e-14)


def test_grid_3d_single_mode():
    N = 4
    L = np.zeros((2 * N, 2 * N, 2 * N), complex)
    L[-1 + N, 2 + N, 3 + N] = 1.0
    g = method.grid_3d(L)
    x = np.arange(-N, N) * math.pi / N
    z = np.arange(-N, N) * 1.0 / N
    ref = np.exp(1j * (-x[:, None, None] + 2 * x[None, :, None] + 3 * math.pi * z[None, None, :]))
    np.testing.assert_allclose(g, ref / math.sqrt(8 * math.pi ** 2), atol=1e-14)


def test_lagrange_exact_on_cubics_and_nodes():
    f = np.linspace(0, 1, 11)
    w = method.lagrange4(f)
    nodes = np.array([-1.0, 0.0, 1.0, 2.0])
    for poly in ([1, 0, 0, 0], [0, 1, 0, 0], [2, -1, 3, 0.5], [0.3, 0, 0, -2]):
        P = np.polynomial.Polynomial(poly)
        np.testing.assert_allclose(w @ P(nodes), P(f), atol=1e-13)
    np.testing.assert_allclose(method.lagrange4(np.array([0.0, 1.0])), [[0, 1, 0, 0], [0, 0, 1, 0]], atol=1e-15)


# ---------------------------------------------------------------- whole chain vs truth

def test_g2d_method_converges_to_truth():
    rng = np.random.default_rng(7)
    x = np.stack([rng.uniform(0, 2 * math.pi, 16), rng.uniform(-1, 1, 16)], 1)
    x = x[np.abs(x[:, 1]) > 0.02]
    gt = truth.g2d(K2, AL2, x)
    errs = []
    for N1, N2 in ((128, 32), (256, 64)):
        g = method.eval_g2d(K2, AL2, x, N1, N2)
        errs.append(np.max(np.abs(g - gt) / np.abs(gt)))
    assert errs[0] < 5e-3
    assert errs[1] < errs[0] / 4 and errs[1] < 1e-3


@pytest.mark.slow
def test_gd3d_method_converges_to_truth():
    rng = np.random.default_rng(8)
    x = np.stack([rng.uniform(0, 2 * math.pi, 8), rng.uniform(0, 2 * math.pi, 8), rng.uniform(-1, 1, 8)], 1)
    x = x[np.abs(x[:, 2]) > 0.1]
    gt = truth.gd3d(K3, A31, A32, x)
    errs = []
    for N, N3 in ((16, 16), (32, 32)):
        g = method.eval_gd3d(K3, A31, A32, x, N, N, N3)
        errs.append(np.max(np.abs(g - gt) / np.abs(gt)))
    assert errs[1] < errs[0] / 4 and errs[1] < 2e-2


@pytest.mark.slow
def test_maxwell_method_against_truth():
    # Points outside the singular cut-off shell eps < r < 2 eps, where the
    # second derivatives of the truncated series converge at these N.
    x = np.array([[0.9, -0.7, 0.3], [2.0, 1.0, 0.8], [0.5, 0.4, -0.7]])
    gt = truth.maxwell3d(K3, A31, A32, x)
    rel = []
    for N in (32, 48):
        g = method.eval_maxwell3d(K3, A31, A32, x, N, N, N)
        rel.append((np.abs(g - gt).max(axis=1) / np.abs(gt).max(axis=1)).max())
    assert rel[1] < 2e-3 and rel[1] < rel[0] / 4


@pytest.mark.slow
def test_maxwell_trace_option_against_truth():
    # The trace variant (a Section 4 option, not Algorithm 4.1): GG_33 = 2 G_d - GG_11 - GG_22 in place
    # of the interpolated 33 field.  Away from the cut-off shell it converges to the lattice sums like
    # the seven-field path, its 33 entry agrees with that path's to the method's error, and its trace
    # is 2 G_d by construction.
    x = np.array([[0.9, -0.7, 0.3], [2.0, 1.0, 0.8], [0.5, 0.4, -0.7]])
    gt = truth.maxwell3d(K3, A31, A32, x)
    rel, d33 = [], []
    for N in (32, 48):
        g = method.eval_maxwell3d(K3, A31, A32, x, N, N, N, trace33=True)
        g7 = method.eval_maxwell3d(K3, A31, A32, x, N, N, N)
        rel.append((np.abs(g - gt).max(axis=1) / np.abs(gt).max(axis=1)).max())
        d33.append(np.max(np.abs(g[:, 2] - g7[:, 2]) / np.abs(gt).max(axis=1)))
        gd = method.eval_gd3d(K3, A31, A32, x, N, N, N)
        np.testing.assert_allclose(g[:, 0] + g[:, 1] + g[:, 2], 2 * gd, rtol=1e-12, atol=0)
    assert rel[1] < 2e-3 and rel[1] < rel[0] / 4
    assert d33[1] < 2e-3 and d33[1] < d33[0]


def test_far_branch_is_the_series():
    # Algorithms 2.1, 3.1, 4.1 step 2b: beyond |x_t| = c the series itself, (1.2), (1.3) and (1.3)
    # differentiated term by term; |x_t| = c exactly is near (R8).
    x = np.array([[0.3, 0.7], [2.0, -0.95], [5.0, 0.61]])
    np.testing.assert_array_equal(method.eval_g2d(K2, AL2, x, 32, 16), truth.g2d(K2, AL2, x))
    xb = np.array([[0.3, 0.6], [0.3, -0.6]])
    assert np.all(method.eval_g2d(K2, AL2, xb, 32, 16) != truth.g2d(K2, AL2, xb))
    x3 = np.array([[0.3, 1.1, 0.7], [2.0, -4.0, -0.95]])
    np.testing.assert_array_equal(method.eval_gd3d(K3, A31, A32, x3, 8, 8, 8), truth.gd3d(K3, A31, A32, x3))
    np.testing.assert_array_equal(method.eval_maxwell3d(K3, A31, A32, x3, 8, 8, 8), truth.maxwell3d(K3, A31, A32, x3))


# ---------------------------------------------------------------- the paper's printed errors

def _golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    return rows


def test_paper_table_points_2d_order_of_magnitude():
    """Tables 1-2 (Section 6.1.1): our error at the paper's points is within a decade.

    The paper's cut-offs and eps are unspecified, so only the decade is pinned;
    N >= 128, where both codes are past the pre-asymptotic range.
    """
    for tab, k, al, N, p, x1, x2, err in _golden("paper_tables_2d.txt"):
        k, al, N, x1, x2, err = float(k), float(al), int(N), float(x1), float(x2), float(err)
        x = np.array([[x1, x2]])
        g = method.eval_g2d(k, al, x, N, N)
        ours = abs(g[0] - truth.g2d(k, al, x)[0]) / abs(truth.g2d(k, al, x)[0])
        assert ours < 10 * err, (tab, N, p, ours, err)


def test_fhat_2d_radial_rule_converged_on_the_largest_tested_grid():
    # The ring integrals of F-hat (Section 2.2) carry J0(|eta| r), J1(|eta| r) over [eps, 2 eps]: ~33
    # oscillations at the corner |eta| = 1043 of the widest grid the tests use (2048 x 128).  The
    # oracle's 160-node rule must already sit at rounding there: doubling it moves no coefficient by
    # more than 1e-12 of the largest, while a 64-node rule is off by 2e-9 of it.
    F64 = method.fhat_2d(1024, 64, q=64)
    F160 = method.fhat_2d(1024, 64, q=160)
    F320 = method.fhat_2d(1024, 64, q=320)
    m = np.isfinite(F320[0])
    s = np.max(np.abs(F320[0][m]))
    for a, b in zip(F160, F320):
        assert np.max(np.abs(a[m] - b[m])) <= 1e-12 * s
    assert np.max(np.abs(F64[0][m] - F320[0][m])) > 1e-9 * s
