"""Exact quasi-periodic Green's functions by direct series summation.  TEST INFRASTRUCTURE ONLY.

Definitions followed (Section 1 of the paper):

* G(x)   2D, 2pi-periodic in x1, alpha-quasi-periodic: eigenfunction expansion
  (1.2), G = i/(4 pi) sum_n beta_n^-1 exp(i alpha_n x1 + i beta_n |x2|),
  alpha_n = alpha + n, beta_n = sqrt(k^2 - alpha_n^2) with Im beta_n >= 0.
* G_d(x) 3D, doubly periodic: expansion (1.3),
  G_d = i/(8 pi^2) sum beta^-1 exp(i alpha1_n1 x1 + i alpha2_n2 x2 + i beta |x3|).
* Maxwell tensor (1.4): GG = G_d I + k^-2 grad grad G_d, second derivatives
  taken term by term: d_p d_q multiplies a term by -xi_p xi_q with
  xi = (alpha1 + n1, alpha2 + n2, beta sgn x3).
* Image expansions (1.1) and its 3D analogue, used only for complex k
  (Im k > 0), where they converge exponentially; they pin the normalisation
  and branch of the eigenfunction expansions.

Truncation: every evanescent term is bounded by exp(-kappa |x_t|)/kappa with
kappa = sqrt(|xi_perp|^2 - k^2); the cut-off radius is chosen so that an
explicit bound on the whole discarded tail is below ``tol`` (absolute).
Points on the plane x_t = 0 are rejected (the series do not converge there
absolutely, Section 1).
"""

import math

import numpy as np
from scipy.special import hankel1


def beta(k, a):
    """beta = sqrt(k^2 - a^2) on the branch Im beta >= 0 (Section 1).

    For real k: sqrt(k^2-a^2) if |a| <= k, else i sqrt(a^2-k^2).
    For complex k with Im k > 0 the principal square root already has
    Im beta > 0.
    """
    a = np.asarray(a, dtype=np.float64)
    if np.iscomplexobj(k) and complex(k).imag != 0.0:
        return np.sqrt((k - a) * (k + a) + 0j)
    k = float(np.real(k))
    d = (k - np.abs(a)) * (k + np.abs(a))
    return np.where(d >= 0.0, np.sqrt(np.abs(d)) + 0j, 1j * np.sqrt(np.abs(d)))


# ----------------------------------------------------------------------------
# tail bounds
# ----------------------------------------------------------------------------

def _radius_2d(k, z, tol):
    """Smallest A with 2 e^{-kappa(A) z} / (kappa(A) (1 - e^{-z})) <= tol."""
    k = abs(k)
    A = k + 1.0
    for _ in range(1000):
        kap = math.sqrt(A * A - k * k)
        bound = 2.0 * math.exp(-kap * z) / (kap * (-math.expm1(-z)))
        if bound <= tol:
            return A
        A = max(A * 1.1, A + 1.0)
    raise ValueError("2D series: point too close to the plane x2 = 0")


def _radius_3d(k, z, tol, order):
    """Cut-off radius R for the 3D lattice sum with discarded tail <= tol.

    Lattice points xi_perp with |xi_perp| <= rho number at most
    pi (rho + 1/sqrt 2)^2.  For rho >= 2k, kappa >= (sqrt3/2) rho and
    kappa >= rho - k.  Summation by parts against that counting bound gives
    for the tail of f(rho) = rho^order e^{-kappa z}/kappa (order 0 or 2)
        B(R) = f_up(R) pi (R+0.71)^2 + int_R^inf 2 pi (rho+0.71) f_up d rho.
    """
    k = abs(k)
    R = max(2.0 * k, 2.0, 2.0 / z) + 1.0
    c = 2.0 / math.sqrt(3.0)
    for _ in range(400):
        e = math.exp(-(R - k) * z)
        if order == 0:
            integral = 2.0 * math.pi * 1.36 * c * e / z
            head = c * e / R * math.pi * (R + 0.71) ** 2
        else:
            integral = 2.0 * math.pi * 1.36 * c * e * (R * R / z + 2 * R / z ** 2 + 2 / z ** 3)
            head = c * e * R * math.pi * (R + 0.71) ** 2
        if integral + head <= tol:
            return R
        R *= 1.05
    raise ValueError("3D series: point too close to the plane x3 = 0")


# ----------------------------------------------------------------------------
# 2D: eigenfunction expansion (1.2)
# ----------------------------------------------------------------------------

def g2d(k, alpha, x, tol=1e-17, max_terms=2_000_000):
    """G(x) of (1.2) at targets x[T,2] (x2 != 0)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    out = np.empty(len(x), dtype=np.complex128)
    for i, (x1, x2) in enumerate(x):
        z = abs(x2)
        if z == 0.0:
            raise ValueError("2D series needs x2 != 0")
        A = _radius_2d(k, z, tol)
        n = np.arange(math.ceil(-A - alpha), math.floor(A - alpha) + 1, dtype=np.float64)
        if n.size > max_terms:
            raise ValueError("2D series: too many terms")
        an = alpha + n
        b = beta(k, an)
        out[i] = 1j / (4 * math.pi) * np.sum(np.exp(1j * an * x1 + 1j * b * z) / b)
    return out


def _radius_2d_grad(k, z, tol):
    """Smallest A >= k + 1 with 2 m(A) e^{-(A - k) z} / (1 - e^{-z}) <= tol, m(A) = A / sqrt(A^2 - k^2).

    Bounds the tail of the differentiated series: a term of |alpha_n| >= A has
    |alpha_n| / kappa_n <= m(A) and |beta_n| / kappa_n = 1, and e^{-kappa_n z} <= e^{-(|alpha_n| - k) z}.
    """
    k = abs(k)
    A = k + 1.0
    for _ in range(2000):
        m = A / math.sqrt(A * A - k * k)
        if 2.0 * m * math.exp(-(A - k) * z) / (-math.expm1(-z)) <= tol:
            return A
        A = max(A * 1.05, A + 1.0)
    raise ValueError("2D series: point too close to the plane x2 = 0")


def g2d_grad(k, alpha, x, tol=1e-17, max_terms=4_000_000):
    """(dG/dx1, dG/dx2) of (1.2) at targets x[T,2] (x2 != 0), differentiated term by term:
    d/dx1 multiplies a term by i alpha_n, d/dx2 by i beta_n sgn(x2)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    out = np.empty((len(x), 2), dtype=np.complex128)
    for i, (x1, x2) in enumerate(x):
        z = abs(x2)
        if z == 0.0:
            raise ValueError("2D series needs x2 != 0")
        A = _radius_2d_grad(k, z, tol)
        n = np.arange(math.ceil(-A - alpha), math.floor(A - alpha) + 1, dtype=np.float64)
        if n.size > max_terms:
            raise ValueError("2D series: too many terms")
        an = alpha + n
        b = beta(k, an)
        e = 1j / (4 * math.pi) * np.exp(1j * an * x1 + 1j * b * z) / b
        out[i, 0] = np.sum(1j * an * e)
        out[i, 1] = np.sign(x2) * np.sum(1j * b * e)
    return out


def _radius_2d_hess(k, z, tol):
    """Smallest A >= k + 1 whose tail bound for the twice-differentiated series is <= tol.

    A term of |alpha_n| = A + m >= A has alpha_n^2 / kappa_n, |alpha_n beta_n| / kappa_n and
    |beta_n|^2 / kappa_n all <= (A + m) m(A), m(A) = A / sqrt(A^2 - k^2), and
    e^{-kappa_n z} <= e^{-(A + m - k) z}; sum_m (A + m) q^m = A/(1 - q) + q/(1 - q)^2, q = e^{-z}.
    """
    k = abs(k)
    q = math.exp(-z)
    A = k + 1.0
    for _ in range(4000):
        m = A / math.sqrt(A * A - k * k)
        tail = 2.0 * m * math.exp(-(A - k) * z) * (A / (1 - q) + q / (1 - q) ** 2)
        if tail <= tol:
            return A
        A = max(A * 1.05, A + 1.0)
    raise ValueError("2D series: point too close to the plane x2 = 0")


def g2d_hess(k, alpha, x, tol=1e-17, max_terms=8_000_000):
    """(d11 G, d12 G, d22 G) of (1.2) at targets x[T,2] (x2 != 0), differentiated term by term:
    -alpha_n^2, -alpha_n beta_n sgn(x2), -beta_n^2."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    out = np.empty((len(x), 3), dtype=np.complex128)
    for i, (x1, x2) in enumerate(x):
        z = abs(x2)
        if z == 0.0:
            raise ValueError("2D series needs x2 != 0")
        A = _radius_2d_hess(k, z, tol)
        n = np.arange(math.ceil(-A - alpha), math.floor(A - alpha) + 1, dtype=np.float64)
        if n.size > max_terms:
            raise ValueError("2D series: too many terms")
        an = alpha + n
        b = beta(k, an)
        e = 1j / (4 * math.pi) * np.exp(1j * an * x1 + 1j * b * z) / b
        out[i, 0] = np.sum(-(an * an) * e)
        out[i, 1] = -np.sign(x2) * np.sum(an * b * e)
        out[i, 2] = np.sum(-(b * b) * e)
    return out


# ----------------------------------------------------------------------------
# 3D: eigenfunction expansion (1.3) and the Maxwell tensor (1.4)
# ----------------------------------------------------------------------------

def _lattice(a1, a2, R):
    n1 = np.arange(math.ceil(-R - a1), math.floor(R - a1) + 1, dtype=np.float64)
    n2 = np.arange(math.ceil(-R - a2), math.floor(R - a2) + 1, dtype=np.float64)
    x1, x2 = np.meshgrid(a1 + n1, a2 + n2, indexing="ij")
    keep = x1 * x1 + x2 * x2 <= R * R
    return x1[keep], x2[keep]


def _sum3d(k, a1, a2, x, tol, order, weights, max_terms, chunk=1 << 21):
    """Shared summation: over the lattice of beta^-1 e^{...} times weights(xi1,xi2,b,sgn)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    ncomp = weights(np.zeros(1), np.zeros(1), np.ones(1, complex), 1.0).shape[0]
    out = np.zeros((len(x), ncomp), dtype=np.complex128)
    for i, (x1, x2, x3) in enumerate(x):
        z = abs(x3)
        if z == 0.0:
            raise ValueError("3D series needs x3 != 0")
        R = _radius_3d(k, z, tol, order)
        if math.pi * (R + 1) ** 2 > max_terms:
            raise ValueError("3D series: too many terms (x3 too close to 0)")
        xi1, xi2 = _lattice(a1, a2, R)
        sg = 1.0 if x3 > 0 else -1.0
        acc = np.zeros(ncomp, dtype=np.complex128)
        for s in range(0, xi1.size, chunk):
            p, q = xi1[s:s + chunk], xi2[s:s + chunk]
            b = beta(k, np.sqrt(p * p + q * q))
            term = np.exp(1j * (p * x1 + q * x2 + b * z)) / b
            acc += weights(p, q, b, sg) @ term
        out[i] = 1j / (8 * math.pi ** 2) * acc
    return out


def gd3d(k, a1, a2, x, tol=1e-17, max_terms=4e8):
    """G_d(x) of (1.3) at targets x[T,3] (x3 != 0)."""
    w = lambda p, q, b, sg: np.ones((1, p.size))
    return _sum3d(k, a1, a2, x, tol, 0, w, max_terms)[:, 0]


MAXWELL_PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))   # 11,22,33,12,13,23


def gd3d_hessian(k, a1, a2, x, tol=1e-17, max_terms=4e8):
    """d_p d_q G_d for the six pairs 11,22,33,12,13,23, term by term."""
    def w(p, q, b, sg):
        xi = (p, q, b * sg)
        return np.stack([-(xi[i] * xi[j]) * np.ones(p.size) for i, j in MAXWELL_PAIRS])
    return _sum3d(k, a1, a2, x, tol, 2, w, max_terms)


def maxwell3d(k, a1, a2, x, tol=1e-17, max_terms=4e8):
    """Six unique entries (11,22,33,12,13,23) of GG = G_d I + k^-2 grad grad G_d (1.4)."""
    g = gd3d(k, a1, a2, x, tol, max_terms)
    h = gd3d_hessian(k, a1, a2, x, tol, max_terms)
    out = h / k ** 2
    out[:, :3] += g[:, None]
    return out


# ----------------------------------------------------------------------------
# image expansions (complex k only): (1.1) and its 3D analogue
# ----------------------------------------------------------------------------

def g2d_images(k, alpha, x, nmax):
    """(i/4) sum_n e^{i 2 pi alpha n} H0^(1)(k r_n), r_n = |x - (2 pi n, 0)|."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    n = np.arange(-nmax, nmax + 1, dtype=np.float64)
    r = np.sqrt((x[:, :1] - 2 * math.pi * n) ** 2 + x[:, 1:2] ** 2)
    return 0.25j * np.sum(np.exp(2j * math.pi * alpha * n) * hankel1(0, k * r), axis=1)


def gd3d_images(k, a1, a2, x, nmax):
    """sum_n e^{i 2 pi alpha.n} e^{i k r_n} / (4 pi r_n), r_n = |x - (2 pi n1, 2 pi n2, 0)|."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    n = np.arange(-nmax, nmax + 1, dtype=np.float64)
    n1, n2 = np.meshgrid(n, n, indexing="ij")
    n1, n2 = n1.ravel(), n2.ravel()
    out = np.empty(len(x), dtype=np.complex128)
    for i, (x1, x2, x3) in enumerate(x):
        r = np.sqrt((x1 - 2 * math.pi * n1) ** 2 + (x2 - 2 * math.pi * n2) ** 2 + x3 ** 2)
        out[i] = np.sum(np.exp(2j * math.pi * (a1 * n1 + a2 * n2)) * np.exp(1j * k * r) / (4 * math.pi * r))
    return out
