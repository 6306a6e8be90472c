"""The 2D G with more of its logarithmic singularity removed (Remark 5.3), computed
plainly in FP64.  TEST INFRASTRUCTURE ONLY.

The parity oracle of the library's higher-order 2D variant.  Near the lattice point
the only non-analytic part of K = e^{-i alpha x1} G is

    S(x) = -(1/2pi) ln r J0(k r) e^{-i alpha x1}

(the Bessel Y0 in (i/4) H0 carries ln(k r / 2) J0(k r); everything else in G and in the
other periodic images is analytic there).  Algorithm 2.1 removes the first two terms of
its Taylor factor, 1 - i alpha x1 (the functions f1 and f2 of Section 2.2), and leaves
-(1/2pi) ln r times terms of degree 2, whose Fourier coefficients fall like |eta|^-4:
the second-order convergence of Theorem 2.  Remark 5.3 points out that removing more
terms gives a higher order.  With t = x1 and m = 1, 2 or 3 this module removes

    f^(m) = -(1/2pi) ln r Y_eps(r) P_m(t, r),

    P_1 = 1 - i alpha t                                        (the paper's f1 - i alpha f2)
    P_2 = P_1 - (alpha^2/2) t^2 - (k^2/4) r^2
    P_3 = P_2 + i (alpha^3/6) t^3 + i (alpha k^2/4) t r^2,

the terms of degree <= m of J0(k r) e^{-i alpha t} = (1 - k^2 r^2/4 + ...)(1 - i alpha t
- alpha^2 t^2/2 + i alpha^3 t^3/6 - ...).  Then K - f^(m) = O(r^{m+1} ln r) near the
lattice point, its coefficients fall like |eta|^{-(m+3)}, and

    L-hat^(m) = K-hat - F-hat_1 + i alpha F-hat_2 - E-hat^(m),

E-hat^(m) the coefficients of the degree-2 and degree-3 terms.  The grid, the 16-point
stencil, the far branch and the phase are those of Algorithm 2.1; the add-back at a
target inside 2 eps is f^(m) in full.

E-hat^(m) by Hankel transforms (as for the derivative tables of Section 2.4): with the
plane-wave expansion, a radial g(r) times cos(n theta) has the coefficient
2 pi (-i)^n cos(n phi) int g(r) J_n(|eta| r) r dr, phi the angle of eta = (j1, j2 pi/c~), and

    t^2 ln r   = r^2 ln r (1 + cos 2 theta)/2,       r^2 ln r,
    t^3 ln r   = r^3 ln r (3 cos theta + cos 3 theta)/4,   t r^2 ln r = r^3 ln r cos theta,

so four radial integrals serve every (k, alpha):  T03 = int r^3 ln r Y J0,  T23 = int
r^3 ln r Y J2,  T14 = int r^4 ln r Y J1,  T34 = int r^4 ln r Y J3 (dr over [0, 2 eps]).

The cut-off ring (``ring=True``).  L = K - f Y_eps is smooth, but across eps < r < 2 eps it
carries the steep transition of Y_eps times the logarithm, and the 16-point stencil's error
there is far larger than anywhere else (Remark 5.6 traces the accuracy to the smoothness of
the cut-offs).  K itself is smooth in the ring.  So for a near target with r_lo < r < r_hi,
r_hi = 2 eps + 2 sqrt(2) h, r_lo = max(eps, eps/2 + 2 sqrt(2) h), h = max(h1, h2), the stencil
interpolates K = L + f Y at its nodes instead of L, and nothing is added back:
G = e^{i alpha x1} sum_ab w_a w_b (L + f Y)(node_ab).  Beyond r_hi every node has Y = 0 and
both forms coincide; below r_lo the paper's form is kept (there K is close to its
singularity, L is smooth; r_lo keeps every node of a zone target at least eps/2 from the
lattice point).  A node's position is its offset from the lattice point, (p1 h1, p2 h2)
with the stencil's own base indices.
"""

import math

import numpy as np
from scipy.special import jv

from . import cutoffs as co
from .grad2d import _radial_rules
from .method import ORACLE_Q, _reduce, _stencil, eval_g2d, grid_2d, lhat_2d

ORDERS = (1, 2, 3)


def poly(k, alpha, t, z, order):
    """P_m(t, r) above at cell points (t, z)."""
    t = np.asarray(t, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    r2 = t * t + z * z
    p = 1.0 - 1j * alpha * t
    if order >= 2:
        p = p - (alpha * alpha / 2) * t * t - (k * k / 4) * r2
    if order >= 3:
        p = p + 1j * (alpha ** 3 / 6) * t ** 3 + 1j * (alpha * k * k / 4) * t * r2
    return p


def f_removed(k, alpha, t, z, order, eps=co.EPS):
    """f^(m) = -(1/2pi) ln r Y_eps(r) P_m at cell points (t, z), r > 0."""
    t = np.asarray(t, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    r = np.hypot(t, z)
    return -np.log(r) * co.Y(r, eps) / (2 * math.pi) * poly(k, alpha, t, z, order)


def ehat(k, alpha, N1, N2, order, c_tilde=co.C_TILDE, eps=co.EPS, q=ORACLE_Q):
    """E-hat^(m): coefficients (basis of (2.1), A2 included) of the degree-2 and degree-3 terms of f^(m)."""
    A2 = 1.0 / (2.0 * math.sqrt(math.pi * c_tilde))
    e1 = np.arange(-N1, N1, dtype=np.float64)[:, None]
    e2 = (np.arange(-N2, N2, dtype=np.float64) * math.pi / c_tilde)[None, :]
    rho = np.sqrt(e1 ** 2 + e2 ** 2)
    phi = np.arctan2(e2 + 0 * e1, e1 + 0 * e2)
    out = np.zeros(rho.shape, dtype=np.complex128)
    if order < 2:
        return out
    r, w, Y = _radial_rules(float(rho.max()), eps, q)
    lr = np.log(r)
    rho_u, inv = np.unique(rho, return_inverse=True)
    T = np.empty((4, rho_u.size))
    for s in range(0, rho_u.size, 256):
        zz = rho_u[s:s + 256, None] * r[None, :]
        T[0, s:s + 256] = (jv(0, zz) * r ** 3 * lr * Y) @ w     # T03
        T[1, s:s + 256] = (jv(2, zz) * r ** 3 * lr * Y) @ w     # T23
        T[2, s:s + 256] = (jv(1, zz) * r ** 4 * lr * Y) @ w     # T14
        T[3, s:s + 256] = (jv(3, zz) * r ** 4 * lr * Y) @ w     # T34
    T03, T23, T14, T34 = (T[m][inv].reshape(rho.shape) for m in range(4))
    pi = math.pi
    ft_tt = pi * T03 - pi * np.cos(2 * phi) * T23                                  # t^2 ln r
    ft_rr = 2 * pi * T03                                                          # r^2 ln r
    ft_ttt = (2 * pi / 4) * (3 * (-1j) * np.cos(phi) * T14 + 1j * np.cos(3 * phi) * T34)   # t^3 ln r
    ft_trr = 2 * pi * (-1j) * np.cos(phi) * T14                                   # t r^2 ln r
    c = -1.0 / (2 * pi)
    out = out - (alpha * alpha / 2) * ft_tt - (k * k / 4) * ft_rr
    if order >= 3:
        out = out + 1j * (alpha ** 3 / 6) * ft_ttt + 1j * (alpha * k * k / 4) * ft_trr
    return A2 * c * out


def lhat_ho(k, alpha, N1, N2, order, c=co.C, c_tilde=co.C_TILDE, eps=co.EPS, q=ORACLE_Q):
    """L-hat^(m) = K-hat - F-hat_1 + i alpha F-hat_2 - E-hat^(m), shape [2N1, 2N2]."""
    return lhat_2d(k, alpha, N1, N2, c, c_tilde, eps, q) - ehat(k, alpha, N1, N2, order, c_tilde, eps, q)


def ring_bounds(h1, h2, eps=co.EPS):
    """(r_lo, r_hi) of the ring zone: r_hi = 2 eps + 2 sqrt(2) h, r_lo = max(eps, eps/2 + 2 sqrt(2) h),
    h = max(h1, h2); every node of a zone target's stencil (within 2 sqrt(2) h of it) then stays at
    least eps/2 from the lattice point, where K is singular."""
    reach = 2 * math.sqrt(2.0) * max(h1, h2)
    return max(eps, 0.5 * eps + reach), 2 * eps + reach


def ring_zone(t, z, h1, h2, eps=co.EPS):
    """Near targets whose stencil interpolates K (``ring=True``): r_lo < r < r_hi."""
    lo, hi = ring_bounds(h1, h2, eps)
    r = np.sqrt(t * t + z * z)
    return (r > lo) & (r < hi)


def eval_g2d_ho(k, alpha, x, N1, N2, order, c=co.C, c_tilde=co.C_TILDE, eps=co.EPS,
                q=ORACLE_Q, ring=False):
    """G at targets x[T,2] with f^(m) removed; order 1 is Algorithm 2.1 (far targets: the series).
    ``ring``: K interpolated in the cut-off ring (see above)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    M1, M2 = 2 * N1, 2 * N2
    h1, h2 = math.pi / N1, c_tilde / N2
    out = np.full(len(x), np.nan + 0j)
    near = np.abs(x[:, 1]) <= c
    if near.any():
        grid = grid_2d(lhat_ho(k, alpha, N1, N2, order, c, c_tilde, eps, q), c_tilde)
        t, _ = _reduce(x[near, 0])
        z = x[near, 1]
        i1, w1 = _stencil((t + math.pi) / h1, M1)
        i2, w2 = _stencil((z + c_tilde) / h2, M2)
        vals = grid[i1[:, :, None], i2[:, None, :]]
        L = np.einsum("ta,tb,tab->t", w1, w2, vals)
        g = L + f_removed(k, alpha, t, z, order, eps)
        if ring:
            zn = ring_zone(t, z, h1, h2, eps)
            if zn.any():
                # node offsets from the lattice point: base index floor(t / h) - 1 + a
                p1 = np.floor(t[zn] / h1)[:, None] - 1 + np.arange(4)
                p2 = np.floor(z[zn] / h2)[:, None] - 1 + np.arange(4)
                TN = (p1 * h1)[:, :, None] + 0 * p2[:, None, :]
                ZN = (p2 * h2)[:, None, :] + 0 * p1[:, :, None]
                fn = f_removed(k, alpha, TN, ZN, order, eps)
                g[zn] = np.einsum("ta,tb,tab->t", w1[zn], w2[zn], vals[zn] + fn)
        out[near] = np.exp(1j * alpha * x[near, 0]) * g
    if (~near).any():
        # beyond c nothing is removed: the series (1.2), as in Algorithm 2.1
        out[~near] = eval_g2d(k, alpha, x[~near], N1, N2, c, c_tilde, eps, q)
    return out
