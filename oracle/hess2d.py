"""Differences of second derivatives of the 2D G for two wavenumbers (Section 2.4.2),
computed plainly in FP64.  TEST INFRASTRUCTURE ONLY.

The parity oracle of the library's T_pq path.  With K_{pq} = e^{-i alpha x1} d_p d_q G
(periodic like K) and, for two wavenumbers k1, k2 and one alpha,

    T_pq = K^{(k1)}_pq - K^{(k2)}_pq,     pq in {11, 12, 22},

the Fourier coefficients are T-hat_pq = m_pq (K-hat^{(k1)} - K-hat^{(k2)}) with
m_11 = -(alpha + j1)^2, m_12 = -(alpha + j1) j2 pi/c~, m_22 = -(j2 pi/c~)^2.  The
k-independent 1/|x|^2 singularities of the second derivatives cancel in the difference;
what is left, the k^2 r^2 ln r term of (i/4) H0 differentiated twice and times
e^{-i alpha x1}, is removed as h_pq:

    h_11 = C (ln r / 2 - i alpha x1 ln r / 2 + x1^2/(2 r^2) - i alpha x1^3/(2 r^2)) Y(r)
    h_12 = C (x1 x2/(2 r^2) - i alpha x1^2 x2/(2 r^2)) Y(r)
    h_22 = C (ln r / 2 - i alpha x1 ln r / 2 + x2^2/(2 r^2) - i alpha x1 x2^2/(2 r^2)) Y(r)

with C = +(k1^2 - k2^2)/(2 pi).  Then L-hat_pq = T-hat_pq - H-hat_pq goes to the grid,
is interpolated with the 16-point stencil, h_pq is added back at the target and the
result multiplied by e^{i alpha x1}: d_p d_q G_{k1} - d_p d_q G_{k2}.

Steps (Section 2.4.2's order): K-hat of (2.1) for both wavenumbers (``method.khat_2d``),
the multipliers, H-hat_pq reduced to Hankel transforms (as in ``grad2d``: a radial
function times cos(n theta) or sin(n theta) has the coefficient 2 pi (-i)^n cos(n phi)
int g J_n(|eta| r) r dr), direct DFT grids, interpolation, add-back, phase.  Far branch:
the series (1.2) differentiated twice term by term, -alpha_n^2, -alpha_n beta_n sgn(x2),
-beta_n^2, for both wavenumbers.

Readings of Section 2.4.2 taken here:
* the constant of the singular parts is +(k1^2 - k2^2)/(2 pi): the first line of the
  expansion of T_11 has it, the second line and h_11, h_12, h_22 print a minus sign
  (with which T - h would keep twice the singular part; pinned against scipy's Hankel
  functions in the tests);
* the third of the three displayed second derivatives is d^2 G / dx2^2 (printed d x1 d x2);
* the O(|x|^2 ln|x|) terms are not removed (as in the paper).
"""

import math

import numpy as np
from scipy.special import jv

from . import cutoffs as co
from .grad2d import _radial_rules
from . import truth
from .method import ORACLE_Q, _reduce, _stencil, grid_2d, khat_2d
from .truth import beta

PAIRS = ((0, 0), (0, 1), (1, 1))     # 11, 12, 22


def h_hess_diff(k1, k2, alpha, t, z, eps=co.EPS, printed_sign=False):
    """(h_11, h_12, h_22) at cell points (t, z), r > 0.  ``printed_sign`` flips C (only to test the reading)."""
    t = np.asarray(t, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    r2 = t * t + z * z
    lr = 0.5 * np.log(r2)
    Y = co.Y(np.sqrt(r2), eps)
    C = (k1 * k1 - k2 * k2) / (2 * math.pi) * (-1.0 if printed_sign else 1.0)
    a = alpha
    h11 = C * (0.5 * lr - 0.5j * a * t * lr + t * t / (2 * r2) - 1j * a * t ** 3 / (2 * r2)) * Y
    h12 = C * (t * z / (2 * r2) - 1j * a * t * t * z / (2 * r2)) * Y
    h22 = C * (0.5 * lr - 0.5j * a * t * lr + z * z / (2 * r2) - 1j * a * t * z * z / (2 * r2)) * Y
    return h11, h12, h22


def hhat_hess_diff(k1, k2, alpha, N1, N2, c_tilde=co.C_TILDE, eps=co.EPS, q=ORACLE_Q):
    """H-hat_11, H-hat_12, H-hat_22 (coefficients of h_pq in the basis of (2.1)), each [2N1, 2N2]."""
    A2 = 1.0 / (2.0 * math.sqrt(math.pi * c_tilde))
    C = (k1 * k1 - k2 * k2) / (2 * math.pi)
    e1 = np.arange(-N1, N1, dtype=np.float64)[:, None]
    e2 = (np.arange(-N2, N2, dtype=np.float64) * math.pi / c_tilde)[None, :]
    rho = np.sqrt(e1 ** 2 + e2 ** 2)
    phi = np.arctan2(e2 + 0 * e1, e1 + 0 * e2)
    r, w, Y = _radial_rules(float(rho.max()), eps, q)
    lr = np.log(r)
    rho_u, inv = np.unique(rho, return_inverse=True)
    T = np.empty((6, rho_u.size))
    for s in range(0, rho_u.size, 256):
        zz = rho_u[s:s + 256, None] * r[None, :]
        J0, J1, J2, J3 = (jv(n, zz) for n in range(4))
        T[0, s:s + 256] = (J0 * r * lr * Y) @ w             # TL  = int ln r Y J0 r dr
        T[1, s:s + 256] = (J1 * r * r * lr * Y) @ w         # TA  = int ln r Y J1 r^2 dr
        T[2, s:s + 256] = (J0 * r * Y) @ w                  # TC0 = int Y J0 r dr
        T[3, s:s + 256] = (J2 * r * Y) @ w                  # TC2 = int Y J2 r dr
        T[4, s:s + 256] = (J1 * r * r * Y) @ w              # TD1 = int Y J1 r^2 dr
        T[5, s:s + 256] = (J3 * r * r * Y) @ w              # TD3 = int Y J3 r^2 dr
    TL, TA, TC0, TC2, TD1, TD3 = (T[m][inv].reshape(rho.shape) for m in range(6))
    cp, sp = np.cos(phi), np.sin(phi)
    c2, s2, c3, s3 = np.cos(2 * phi), np.sin(2 * phi), np.cos(3 * phi), np.sin(3 * phi)
    pi = math.pi
    ft_lnr = 2 * pi * TL                                         # ln r
    ft_tlnr = 2 * pi * (-1j) * cp * TA                           # t ln r = r ln r cos
    ft_tt = pi * TC0 - pi * c2 * TC2                             # t^2/r^2 = (1 + cos 2th)/2
    ft_tz = -pi * s2 * TC2                                       # t z/r^2 = sin 2th / 2
    ft_zz = pi * TC0 + pi * c2 * TC2                             # z^2/r^2 = (1 - cos 2th)/2
    ft_ttt = (2 * pi / 4) * (3 * (-1j) * cp * TD1 + 1j * c3 * TD3)   # t^3/r^2 = r (3 cos + cos 3th)/4
    ft_ttz = (2 * pi / 4) * ((-1j) * sp * TD1 + 1j * s3 * TD3)       # t^2 z/r^2 = r (sin + sin 3th)/4
    ft_tzz = (2 * pi / 4) * ((-1j) * cp * TD1 - 1j * c3 * TD3)       # t z^2/r^2 = r (cos - cos 3th)/4
    a = alpha
    H11 = A2 * C * (0.5 * ft_lnr - 0.5j * a * ft_tlnr + 0.5 * ft_tt - 0.5j * a * ft_ttt)
    H12 = A2 * C * (0.5 * ft_tz - 0.5j * a * ft_ttz)
    H22 = A2 * C * (0.5 * ft_lnr - 0.5j * a * ft_tlnr + 0.5 * ft_zz - 0.5j * a * ft_tzz)
    return H11, H12, H22


def multipliers(alpha, N1, N2, c_tilde=co.C_TILDE):
    xi1 = (alpha + np.arange(-N1, N1, dtype=np.float64))[:, None]
    J = (np.arange(-N2, N2, dtype=np.float64) * math.pi / c_tilde)[None, :]
    return -(xi1 * xi1) + 0 * J, -(xi1 * J), -(J * J) + 0 * xi1


def lhat_hess_diff(k1, k2, alpha, N1, N2, c=co.C, c_tilde=co.C_TILDE, eps=co.EPS, q=ORACLE_Q):
    """L-hat_pq = m_pq (K-hat^{(k1)} - K-hat^{(k2)}) - H-hat_pq for pq = 11, 12, 22."""
    dK = khat_2d(k1, alpha, N1, N2, c, c_tilde, q) - khat_2d(k2, alpha, N1, N2, c, c_tilde, q)
    H = hhat_hess_diff(k1, k2, alpha, N1, N2, c_tilde, eps, q)
    return [m * dK - h for m, h in zip(multipliers(alpha, N1, N2, c_tilde), H)]


def eval_g2d_hess_diff(k1, k2, alpha, x, N1, N2, c=co.C, c_tilde=co.C_TILDE, eps=co.EPS,
                       q=ORACLE_Q, ring=False):
    """(d11, d12, d22) of G_{k1} - G_{k2} at targets x[T,2] as [T, 3]; far targets (|x2| > c) take
    the series (1.2) differentiated twice term by term, for k1 minus for k2.

    ``ring``: in the cut-off ring (``highorder2d.ring_zone``) the stencil interpolates
    T_pq = L_pq + h_pq at its nodes instead of L_pq, and nothing is added back there (the
    reading of Remark 5.6 taken for G and its gradient)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    M1, M2 = 2 * N1, 2 * N2
    h1, h2 = math.pi / N1, c_tilde / N2
    grids = [grid_2d(L, c_tilde) for L in lhat_hess_diff(k1, k2, alpha, N1, N2, c, c_tilde, eps, q)]
    t, _ = _reduce(x[:, 0])
    x2 = x[:, 1]
    out = np.full((len(x), 3), np.nan + 0j)
    phase = np.exp(1j * alpha * x[:, 0])
    near = np.abs(x2) <= c
    if near.any():
        tn, zn = t[near], x2[near]
        i1, w1 = _stencil((tn + math.pi) / h1, M1)
        i2, w2 = _stencil((zn + c_tilde) / h2, M2)
        hs = h_hess_diff(k1, k2, alpha, tn, zn, eps)
        zone = np.zeros(len(tn), dtype=bool)
        if ring:
            from .highorder2d import ring_zone
            zone = ring_zone(tn, zn, h1, h2, eps)
        if zone.any():
            # node offsets from the lattice point: base index floor(t / h) - 1 + a
            p1 = np.floor(tn[zone] / h1)[:, None] - 1 + np.arange(4)
            p2 = np.floor(zn[zone] / h2)[:, None] - 1 + np.arange(4)
            hn = h_hess_diff(k1, k2, alpha, (p1 * h1)[:, :, None] + 0 * p2[:, None, :],
                             (p2 * h2)[:, None, :] + 0 * p1[:, :, None], eps)
        for p in range(3):
            vals = grids[p][i1[:, :, None], i2[:, None, :]]
            L = np.einsum("ta,tb,tab->t", w1, w2, vals)
            g = L + hs[p]
            if zone.any():
                g[zone] = np.einsum("ta,tb,tab->t", w1[zone], w2[zone], vals[zone] + hn[p])
            out[near, p] = phase[near] * g
    far = ~near
    if far.any():
        out[far] = truth.g2d_hess(k1, alpha, x[far]) - truth.g2d_hess(k2, alpha, x[far])
    return out
