"""First derivatives of the 2D Green's function by the FFT method (Section 2.4.1),
computed plainly in FP64.  TEST INFRASTRUCTURE ONLY.

The parity oracle of the library's gradient path.  With K = e^{-i alpha x1} G,

    K1 = i alpha K + dK/dx1 = e^{-i alpha x1} dG/dx1,    K2 = dK/dx2 = e^{-i alpha x1} dG/dx2,

both periodic like K, with Fourier coefficients i(alpha + j1) K-hat_j and
i j2 (pi / c~) K-hat_j.  Their singular parts h1, h2 (the leading terms of
e^{-i alpha x1} grad (i/4) H0(k|x|), cut off by Y_eps) are removed, so that

    L-hat_{p,j} = (multiplier_p) K-hat_j - H-hat_{p,j}

is transformed to the grid, interpolated with the same 16-point stencil as G,
and h_p is added back exactly at the target (then the phase e^{i alpha x1}).

Steps, in the order of Section 2.4.1:

1. K-hat_j of (2.1) (``method.khat_2d``) times the two multipliers.
2. H-hat_{p,j} = int h_p phi_{-j} over the cell.  h_p is a sum of radial
   functions times cos(n theta) or sin(n theta), n <= 3, so each coefficient
   reduces to Hankel transforms: the plane-wave expansion gives
       int g(r) cos(n theta) e^{-i eta.x} dx = 2 pi (-i)^n cos(n phi) int_0^inf g(r) J_n(|eta| r) r dr
   (sin likewise), phi the angle of eta = (j1, j2 pi / c~).  The radial integrals
   run over [0, eps] and [eps, 2 eps] (Y_eps = 1 on the first piece) with
   Gauss-Legendre rules fine enough for the highest |eta| of the grid.
3. Grid values by direct DFT sums (``method.grid_2d``).
4. Targets: reduction, near/far branch, 4 x 4 Lagrange interpolation, exact
   add-back of h_p, phase.  Far branch (|x2| > c): the series (1.2) differentiated
   term by term, i(alpha + n) for x1 and i beta_n sgn(x2) for x2.

Readings of Section 2.4.1 taken here:
* the second definition printed as K_1 = dK/dx2 is K_2;
* in h2 the logarithmic term is x2 ln|x| (the expansion of
  e^{-i alpha x1} d/dx2 (i/4) H0(k|x|) gives -(k^2/2) x2 ln|x|; the printed
  x1 ln|x| would leave a term of order |x| ln|x| in K2 - h2);
* the O(|x|^2 ln|x|) terms are not removed (as in the paper).
"""

import math

import numpy as np
from scipy.special import jv

from . import cutoffs as co
from . import truth
from .method import ORACLE_Q, _reduce, _stencil, gauss_legendre, grid_2d, khat_2d


def ring_zone(t, z, h1, h2, eps=co.EPS):
    """The cut-off ring of the ``ring`` option, as for G (``highorder2d.ring_zone``)."""
    from .highorder2d import ring_zone as rz
    return rz(t, z, h1, h2, eps)


# ----------------------------------------------------------------------------
# the singular parts h1, h2
# ----------------------------------------------------------------------------

def h_grad(k, alpha, t, z, eps=co.EPS, printed_h2=False):
    """(h1, h2) at cell points (t, z), r = |(t, z)| > 0 (Section 2.4.1).

    ``printed_h2`` uses x1 ln|x| in h2 as printed (only to test the reading).
    """
    t = np.asarray(t, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    r2 = t * t + z * z
    lr = 0.5 * np.log(r2)
    Y = co.Y(np.sqrt(r2), eps)
    c = -1.0 / (2.0 * math.pi)
    h1 = c * (-(k * k / 2) * t * lr + t / r2 - 1j * alpha * t * t / r2 - (alpha * alpha / 2) * t ** 3 / r2) * Y
    lz = t if printed_h2 else z
    h2 = c * (-(k * k / 2) * lz * lr + z / r2 - 1j * alpha * t * z / r2 - (alpha * alpha / 2) * t * t * z / r2) * Y
    return h1, h2


# ----------------------------------------------------------------------------
# H-hat_{p,j}
# ----------------------------------------------------------------------------

def _radial_rules(rho_max, eps, q):
    """Radial nodes/weights on [0, eps] and [eps, 2 eps], enough for |eta| <= rho_max: Gauss-Legendre,
    on [0, eps] in u with r = eps u^3 (the ln r factors of the integrands are then integrated to
    rounding; plain Gauss-Legendre leaves about 1e-10)."""
    n = max(q, int(math.ceil(rho_max * eps)) + 64)
    u, wu = gauss_legendre(0.0, 1.0, n)
    r0, w0 = eps * u ** 3, wu * 3 * eps * u * u
    r1, w1 = gauss_legendre(eps, 2 * eps, n)
    r = np.concatenate([r0, r1])
    w = np.concatenate([w0, w1])
    return r, w, co.Y(r, eps)


def hhat_grad_2d(k, alpha, N1, N2, c_tilde=co.C_TILDE, eps=co.EPS, q=ORACLE_Q):
    """H-hat_1 and H-hat_2 (coefficients of h1, h2 in the basis of (2.1)), shape [2N1, 2N2]."""
    A2 = 1.0 / (2.0 * math.sqrt(math.pi * c_tilde))
    c = -1.0 / (2.0 * math.pi)
    e1 = np.arange(-N1, N1, dtype=np.float64)[:, None]
    e2 = (np.arange(-N2, N2, dtype=np.float64) * math.pi / c_tilde)[None, :]
    rho = np.sqrt(e1 ** 2 + e2 ** 2)
    phi = np.arctan2(e2 + 0 * e1, e1 + 0 * e2)
    r, w, Y = _radial_rules(float(rho.max()), eps, q)
    lr = np.log(r)
    # the radial integrals depend on |eta| only: once per distinct |eta|
    rho_u, inv = np.unique(rho, return_inverse=True)
    T = np.empty((6, rho_u.size))
    for s in range(0, rho_u.size, 256):
        z = rho_u[s:s + 256, None] * r[None, :]
        J0, J1, J2, J3 = (jv(n, z) for n in range(4))
        T[0, s:s + 256] = (J1 * r * r * lr * Y) @ w         # TA  = int ln r Y J1 r^2 dr
        T[1, s:s + 256] = (J1 * Y) @ w                      # TB  = int Y J1 dr
        T[2, s:s + 256] = (J0 * r * Y) @ w                  # TC0 = int Y J0 r dr
        T[3, s:s + 256] = (J2 * r * Y) @ w                  # TC2 = int Y J2 r dr
        T[4, s:s + 256] = (J1 * r * r * Y) @ w              # TD1 = int Y J1 r^2 dr
        T[5, s:s + 256] = (J3 * r * r * Y) @ w              # TD3 = int Y J3 r^2 dr
    TA, TB, TC0, TC2, TD1, TD3 = (T[m][inv].reshape(rho.shape) for m in range(6))
    cs1, sn1 = np.cos(phi), np.sin(phi)
    two_pi = 2 * math.pi
    # h1 / c = -(k^2/2) r cos ln r + cos / r - i alpha (1 + cos 2th)/2 - (alpha^2/2) r (3 cos + cos 3th)/4
    f1 = (-(k * k / 2) * two_pi * (-1j) * cs1 * TA
          + two_pi * (-1j) * cs1 * TB
          - 1j * alpha * (math.pi * TC0 - math.pi * np.cos(2 * phi) * TC2)
          - (alpha * alpha / 2) * (two_pi / 4) * (3 * (-1j) * cs1 * TD1 + 1j * np.cos(3 * phi) * TD3))
    # h2 / c = -(k^2/2) r sin ln r + sin / r - i alpha sin 2th / 2 - (alpha^2/2) r (sin + sin 3th)/4
    f2 = (-(k * k / 2) * two_pi * (-1j) * sn1 * TA
          + two_pi * (-1j) * sn1 * TB
          - 1j * alpha * (-math.pi * np.sin(2 * phi) * TC2)
          - (alpha * alpha / 2) * (two_pi / 4) * ((-1j) * sn1 * TD1 + 1j * np.sin(3 * phi) * TD3))
    H1 = A2 * c * f1
    H2 = A2 * c * f2
    return H1, H2


def lhat_grad_2d(k, alpha, N1, N2, c=co.C, c_tilde=co.C_TILDE, eps=co.EPS, q=ORACLE_Q):
    """L-hat_{1,j} = i(alpha + j1) K-hat_j - H-hat_{1,j},  L-hat_{2,j} = i j2 (pi/c~) K-hat_j - H-hat_{2,j}."""
    K = khat_2d(k, alpha, N1, N2, c, c_tilde, q)
    H1, H2 = hhat_grad_2d(k, alpha, N1, N2, c_tilde, eps, q)
    m1 = 1j * (alpha + np.arange(-N1, N1, dtype=np.float64))[:, None]
    m2 = 1j * (np.arange(-N2, N2, dtype=np.float64) * math.pi / c_tilde)[None, :]
    return m1 * K - H1, m2 * K - H2


# ----------------------------------------------------------------------------
# evaluation
# ----------------------------------------------------------------------------

def eval_g2d_grad(k, alpha, x, N1, N2, c=co.C, c_tilde=co.C_TILDE, eps=co.EPS, q=ORACLE_Q,
                  ring=False):
    """(dG/dx1, dG/dx2) at targets x[T,2] as [T, 2]; far targets (|x2| > c) take the series (1.2)
    differentiated term by term.

    ``ring``: in the cut-off ring (``highorder2d.ring_zone``) the stencil interpolates
    K_p = L_p + h_p at its nodes instead of L_p, and nothing is added back there (the same
    reading of Remark 5.6 as for G: L_p carries the steep transition of Y_eps times the 1/r
    and logarithmic terms of h_p, K_p is smooth in the ring)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    M1, M2 = 2 * N1, 2 * N2
    h1, h2 = math.pi / N1, c_tilde / N2
    L1, L2 = lhat_grad_2d(k, alpha, N1, N2, c, c_tilde, eps, q)
    grids = (grid_2d(L1, c_tilde), grid_2d(L2, c_tilde))              # [p1, p2]
    t, _ = _reduce(x[:, 0])
    x2 = x[:, 1]
    out = np.full((len(x), 2), np.nan + 0j)
    phase = np.exp(1j * alpha * x[:, 0])
    near = np.abs(x2) <= c
    if near.any():
        tn, zn = t[near], x2[near]
        i1, w1 = _stencil((tn + math.pi) / h1, M1)
        i2, w2 = _stencil((zn + c_tilde) / h2, M2)
        hs = h_grad(k, alpha, tn, zn, eps)
        zone = ring_zone(tn, zn, h1, h2, eps) if ring else np.zeros(len(tn), dtype=bool)
        if zone.any():
            # node offsets from the lattice point: base index floor(t / h) - 1 + a
            p1 = np.floor(tn[zone] / h1)[:, None] - 1 + np.arange(4)
            p2 = np.floor(zn[zone] / h2)[:, None] - 1 + np.arange(4)
            hn = h_grad(k, alpha, (p1 * h1)[:, :, None] + 0 * p2[:, None, :],
                        (p2 * h2)[:, None, :] + 0 * p1[:, :, None], eps)
        for p in range(2):
            vals = grids[p][i1[:, :, None], i2[:, None, :]]
            L = np.einsum("ta,tb,tab->t", w1, w2, vals)
            g = L + hs[p]
            if zone.any():
                g[zone] = np.einsum("ta,tb,tab->t", w1[zone], w2[zone], vals[zone] + hn[p])
            out[near, p] = phase[near] * g
    far = ~near
    if far.any():
        out[far] = truth.g2d_grad(k, alpha, x[far])
    return out
