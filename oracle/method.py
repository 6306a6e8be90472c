"""The discrete FFT-based method, computed plainly in FP64.  TEST INFRASTRUCTURE ONLY.

This is the parity oracle: the same approximation as the library (Algorithms
2.1, 3.1 and 4.1 with the frozen parameter set below) but computed directly,
step by step in the paper's order:

1. Fourier coefficients of the periodised function K (eq. 2.1 in 2D, eq. 3.3
   in 3D), whose X'-integrals are evaluated by converged Gauss-Legendre
   quadrature and a matrix product (the "matrix computation" of Section 2.1).
2. Fourier coefficients of the removed singular part: F1, F2 in 2D
   (eqs. 2.4, 2.5; Phi-hat by radial Hankel quadrature) and F in 3D (eq. 3.5,
   the 3D integral reduced to a radial sine transform).
3. L-hat = K-hat - F-hat (eqs. 2.3 and the line after 3.5); Maxwell fields
   L-hat^{pq} = -c^p c^q L-hat (Section 4).
4. Grid values of the truncated series L_N by *direct* separable DFT sums
   (no FFT): L_N(x_p) = A sum_j L-hat_j exp(i pi j.p / N).
5. Targets: reduction to the cell (Alg. 2.1 step 2c / Alg. 3.1 step 2c),
   near/far branch on |x_t| <= c (step 2b), tensor-product 4-point Lagrange
   interpolation (the 16- and 64-point stencils of Sections 2.3 and 3.3), exact
   add-back of the singular part and the quasi-periodic phase.
   The far branch (|x_t| > c) sums the eigenfunction series itself, as step 2b
   of Algorithms 2.1, 3.1 and 4.1 prescribes: (1.2) for G, (1.3) for G_d and
   (1.3) differentiated term by term for the Maxwell tensor, each with its
   explicit tail bound (``truth``).
6. Maxwell (Algorithm 4.1): L_d and the six second-derivative fields
   L^{pq}, pq = 11, 22, 33, 12, 13, 23, each interpolated ("seven
   interpolation processes", Section 4).  ``trace33=True`` is the variant that
   drops the 33 field and takes GG_33 = 2 G_d - GG_11 - GG_22 from the trace
   (tr GG = 3 G_d + k^-2 Laplacian G_d = 2 G_d off the lattice); it is an
   option, not Algorithm 4.1.

Readings of the paper taken here (its silent or garbled points):
* cut-offs: C^8 smoothstep (see ``cutoffs``), c = 0.6, c~ = 1, eps = 0.2;
* the 3D basis is exp[i(j1 x1 + j2 x2 + j3 pi x3 / c~)] / sqrt(8 pi^2 c~)
  (Section 3.1 prints j1 x2 and drops the pi);
* eq. 3.2 has e^{i(beta + j3 pi/c~) x3} as its second exponential and 3.4
  has no stray i (they must agree with 3.3, which is consistent);
* bicubic / tricubic interpolation is the 4-point cubic Lagrange rule per
  axis (same stencil and O(h^4) order as the paper states);
* the final phase uses the original coordinates, G = e^{i alpha.x'} K(t)
  (Alg. 2.1 step 2e), so Alg. 3.1 step 2f returns G_d(x) and not G_d(t);
* grid sizes are independent per axis: M_i = 2 N_i.

Index conventions: coefficient arrays are indexed [j + N] (centred index j
shifted to start at 0), grid arrays [p + N] with x = p h, so index 0 is
x1 = -pi, x3 = -c~.
"""

import math

import numpy as np
from scipy.special import j0 as bessel_j0, j1 as bessel_j1

from . import cutoffs as co
from . import truth
from .truth import beta

ORACLE_Q = 160          # Gauss-Legendre nodes for every 1D integral


def gauss_legendre(a, b, q=ORACLE_Q):
    t, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (b - a) * t + 0.5 * (b + a), 0.5 * (b - a) * w


def lagrange4(f):
    """Cubic Lagrange basis at nodes -1, 0, 1, 2 evaluated at fraction f (shape [...,4])."""
    f = np.asarray(f, dtype=np.float64)
    nodes = (-1.0, 0.0, 1.0, 2.0)
    out = []
    for a in range(4):
        l = np.ones_like(f)
        for b in range(4):
            if b != a:
                l = l * (f - nodes[b]) / (nodes[a] - nodes[b])
        out.append(l)
    return np.stack(out, axis=-1)


def dft_matrix(N):
    """E[p + N, j + N] = exp(i pi j p / N) for centred j, p in [-N, N)."""
    j = np.arange(-N, N, dtype=np.float64)
    return np.exp(1j * math.pi * np.outer(j, j) / N)


# ----------------------------------------------------------------------------
# the X'-integrals of (2.1) / (3.3)
# ----------------------------------------------------------------------------

def xprime_integrals(b, J, c=co.C, c_tilde=co.C_TILDE, q=ORACLE_Q):
    """I(b - J) and I(b + J) with I(g) = int_0^{c~} e^{i g x} X'(x) dx, as [len(b), len(J)].

    X' vanishes outside [c, (c + c~)/2], so the integral runs over that interval.
    The factorisation e^{i(b -+ J)x} = e^{ibx} e^{-+iJx} turns both families into
    one matrix product (the "1D FFT and matrix computation" of Section 2.1).
    """
    x, w = gauss_legendre(c, 0.5 * (c + c_tilde), q)
    a = np.exp(1j * np.outer(b, x)) * (w * co.dX(x, c, c_tilde))     # [P, q]
    em = np.exp(-1j * np.outer(x, J))                                   # [q, M]
    return a @ em, a @ np.conj(em)


def _coef_K(A, k, b, J, lead_den, Im, Ip):
    """A [ 1/(|xi|^2 - k^2) + I(b-J)/(2b(J-b)) - I(b+J)/(2b(J+b)) ]  (eqs. 2.1, 3.3)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        return A * (1.0 / lead_den + Im / (2 * b * (J - b)) - Ip / (2 * b * (J + b)))


# The special coefficients beta = -+J of Sections 2.1 / 3.1, where the integration by parts
# behind (2.1) / (3.3) divides by zero (and loses digits close to it): there the coefficient
# is taken from the integral that defines it,
#     K-hat_j = A (i / (2 beta)) [ I0(beta - J) + I0(beta + J) ],   I0(g) = int_0^{c~} e^{igx} X(x) dx,
# which is the paper's special-case formula (its g = 0 term is int X) for every g.
SPECIAL_SWITCH = 1e-2


def x_integral(g, c=co.C, c_tilde=co.C_TILDE, q=ORACLE_Q):
    """I0(g) = int_0^{c~} e^{igx} X(x) dx for an array of g (X = 1 on [0, c], 0 beyond (c + c~)/2)."""
    x0, w0 = gauss_legendre(0.0, c, q)
    x1, w1 = gauss_legendre(c, 0.5 * (c + c_tilde), q)
    x = np.concatenate([x0, x1])
    w = np.concatenate([w0, w1 * co.X(x1, c, c_tilde)])
    g = np.asarray(g, dtype=np.complex128)
    return (np.exp(1j * g.ravel()[:, None] * x[None, :]) @ w).reshape(g.shape)


def _special(b, J):
    """Coefficients with a propagating beta within SPECIAL_SWITCH of |J|."""
    return (np.imag(b) == 0) & (np.abs(np.real(b) - np.abs(J)) < SPECIAL_SWITCH)


def _special_fix(K, A, b, J, c, c_tilde, q):
    m = _special(b, J)
    if m.any():
        bb, JJ = np.broadcast_to(b, m.shape)[m], np.broadcast_to(J, m.shape)[m]
        K[m] = A * (1j / (2 * bb)) * (x_integral(bb - JJ, c, c_tilde, q) + x_integral(bb + JJ, c, c_tilde, q))
    return K


# ----------------------------------------------------------------------------
# 2D (Section 2)
# ----------------------------------------------------------------------------

def khat_2d(k, alpha, N1, N2, c=co.C, c_tilde=co.C_TILDE, q=ORACLE_Q):
    """K-hat_j of (2.1) for j in S_N, shape [2N1, 2N2]."""
    A2 = 1.0 / (2.0 * math.sqrt(math.pi * c_tilde))
    a = alpha + np.arange(-N1, N1, dtype=np.float64)
    J = np.arange(-N2, N2, dtype=np.float64) * math.pi / c_tilde
    b = beta(k, a)
    Im, Ip = xprime_integrals(b, J, c, c_tilde, q)
    B, JJ = b[:, None], J[None, :]
    K = _coef_K(A2, k, B, JJ, a[:, None] ** 2 + JJ ** 2 - k * k, Im, Ip)
    return _special_fix(K, A2, B, JJ, c, c_tilde, q)


def phi1(r, eps=co.EPS):
    """Phi_1 = (2 + ln r) Y'(r)/r + Y''(r) ln r, i.e. Delta(ln r Y) away from 0 (Section 2.2)."""
    return (2.0 + np.log(r)) * co.dY(r, eps) / r + co.d2Y(r, eps) * np.log(r)


def fhat_2d(N1, N2, c_tilde=co.C_TILDE, eps=co.EPS, q=ORACLE_Q):
    """F-hat_1 and F-hat_2 of (2.4), (2.5) (and the j = 0 values), shape [2N1, 2N2].

    Phi-hat_j = int Phi(x) phi_{-j}(x) dx with the same basis as K-hat.  For the
    radial Phi_1: Phi-hat_1 = A2 2pi int Phi_1(r) J0(|eta| r) r dr, and for
    Phi_2 = x1 Phi_1 (its x1-moment): Phi-hat_2 = -i A2 2pi (j1/|eta|) int Phi_1 J1(|eta| r) r^2 dr,
    eta = (j1, j2 pi / c~).
    """
    A2 = 1.0 / (2.0 * math.sqrt(math.pi * c_tilde))
    j1 = np.arange(-N1, N1, dtype=np.float64)[:, None]
    J = (np.arange(-N2, N2, dtype=np.float64) * math.pi / c_tilde)[None, :]
    eta2 = j1 ** 2 + J ** 2
    eta = np.sqrt(eta2)
    r, w = gauss_legendre(eps, 2 * eps, q)
    wp = w * phi1(r, eps)
    F1 = np.empty((2 * N1, 2 * N2), dtype=np.complex128)
    F2 = np.empty_like(F1)
    for i in range(2 * N1):                           # one j1 row at a time (memory)
        e = eta[i][:, None] * r[None, :]
        i0 = (bessel_j0(e) * r) @ wp
        i1 = (bessel_j1(e) * r * r) @ wp
        with np.errstate(divide="ignore", invalid="ignore"):
            ph1 = A2 * 2 * math.pi * i0
            ph2 = -1j * A2 * 2 * math.pi * (j1[i, 0] / eta[i]) * i1
            f1 = (A2 + ph1 / (2 * math.pi)) / eta2[i]
            f2 = (-2j * j1[i, 0] * f1 + ph2 / (2 * math.pi)) / eta2[i]
        F1[i], F2[i] = f1, f2
    # j = 0 (Section 2.2): F1_0 = -A2 int_0^{2eps} t ln t Y(t) dt, F2_0 = 0.
    tq, tw = gauss_legendre(eps, 2 * eps, q)
    inner = eps * eps * (math.log(eps) / 2.0 - 0.25)      # int_0^eps t ln t dt (Y = 1 there)
    F1[N1, N2] = -A2 * (inner + np.sum(tw * tq * np.log(tq) * co.Y(tq, eps)))
    F2[N1, N2] = 0.0
    return F1, F2


def lhat_2d(k, alpha, N1, N2, c=co.C, c_tilde=co.C_TILDE, eps=co.EPS, q=ORACLE_Q, F=None):
    """L-hat = K-hat - F-hat_1 + i alpha F-hat_2 (2.3)."""
    F1, F2 = fhat_2d(N1, N2, c_tilde, eps, q) if F is None else F
    return khat_2d(k, alpha, N1, N2, c, c_tilde, q) - F1 + 1j * alpha * F2


def grid_2d(Lhat, c_tilde=co.C_TILDE):
    """L_N at the grid, [2N1, 2N2] indexed [p1 + N1, p2 + N2], by direct DFT sums."""
    M1, M2 = Lhat.shape
    A2 = 1.0 / (2.0 * math.sqrt(math.pi * c_tilde))
    return A2 * dft_matrix(M1 // 2) @ Lhat @ dft_matrix(M2 // 2).T


def _reduce(x):
    """x = 2 pi n + t with t in [-pi, pi) (Alg. 2.1 step 2c)."""
    n = np.floor((x + math.pi) / (2 * math.pi))
    return x - 2 * math.pi * n, n


def _stencil(u, M):
    """Base node floor(u), fraction, and the 4 wrapped node indices -1..2."""
    p0 = np.floor(u)
    f = u - p0
    idx = (p0.astype(np.int64)[:, None] + np.arange(-1, 3)[None, :]) % M
    return idx, lagrange4(f)


def eval_g2d(k, alpha, x, N1, N2, c=co.C, c_tilde=co.C_TILDE, eps=co.EPS, q=ORACLE_Q, F=None):
    """Algorithm 2.1 at targets x[T,2]; G_N(x).  Far targets (|x2| > c): the series (1.2)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    M1, M2 = 2 * N1, 2 * N2
    h1, h2 = math.pi / N1, c_tilde / N2
    t, _ = _reduce(x[:, 0])
    x2 = x[:, 1]
    out = np.full(len(x), np.nan + 0j)
    near = np.abs(x2) <= c
    # near: bicubic on L_N, then K_N = L_N + f1 - i alpha f2, G = e^{i alpha x1} K_N
    if near.any():
        grid = grid_2d(lhat_2d(k, alpha, N1, N2, c, c_tilde, eps, q, F), c_tilde)   # [p1, p2]
        tn, zn = t[near], x2[near]
        i1, w1 = _stencil((tn + math.pi) / h1, M1)
        i2, w2 = _stencil((zn + c_tilde) / h2, M2)
        vals = grid[i1[:, :, None], i2[:, None, :]]
        L = np.einsum("ta,tb,tab->t", w1, w2, vals)
        r = np.hypot(tn, zn)
        sing = -np.log(r) * co.Y(r, eps) / (2 * math.pi) * (1.0 - 1j * alpha * tn)
        out[near] = np.exp(1j * alpha * x[near, 0]) * (L + sing)
    far = ~near
    if far.any():
        # step 2b: |x2| > c takes the eigenfunction series (1.2)
        out[far] = truth.g2d(k, alpha, x[far])
    return out


# ----------------------------------------------------------------------------
# 3D (Section 3) and the Maxwell fields (Section 4)
# ----------------------------------------------------------------------------

def radial_H(k, rho, eps=co.EPS, q=ORACLE_Q, chunk=1 << 16):
    """H(rho) = rho^-1 int_eps^{2eps} e^{ikr} (2ik Y' + Y'') sin(rho r) dr;  H(0) = int (...) r dr.

    With g = e^{ikr}/(4 pi r), the integral in (3.5) is the 3D Fourier transform of
    the radial function g (2ik Y' + Y''), which reduces to this sine transform.
    """
    r, w = gauss_legendre(eps, 2 * eps, q)
    wg = w * np.exp(1j * k * r) * (2j * k * co.dY(r, eps) + co.d2Y(r, eps))
    rho = np.asarray(rho, dtype=np.float64)
    flat = rho.ravel()
    out = np.empty(flat.size, dtype=np.complex128)
    for s in range(0, flat.size, chunk):
        p = flat[s:s + chunk]
        with np.errstate(divide="ignore", invalid="ignore"):
            sn = np.where(p[:, None] > 0, np.sin(np.outer(p, r)) / p[:, None], r[None, :])
        out[s:s + chunk] = sn @ wg
    return out.reshape(rho.shape)


def _xi_3d(a1, a2, N1, N2, N3, c_tilde):
    xi1 = a1 + np.arange(-N1, N1, dtype=np.float64)
    xi2 = a2 + np.arange(-N2, N2, dtype=np.float64)
    J = np.arange(-N3, N3, dtype=np.float64) * math.pi / c_tilde
    rp2 = (xi1[:, None] ** 2 + xi2[None, :] ** 2).ravel()           # one entry per pencil (j1, j2)
    return rp2, J


def khat_3d(k, a1, a2, N1, N2, N3, c=co.C, c_tilde=co.C_TILDE, q=ORACLE_Q):
    """K-hat_dj of (3.3) (the corrected 3.2 integrated by parts), shape [2N1, 2N2, 2N3]."""
    A3 = 1.0 / math.sqrt(8 * math.pi ** 2 * c_tilde)
    rp2, J = _xi_3d(a1, a2, N1, N2, N3, c_tilde)
    b = beta(k, np.sqrt(rp2))
    Im, Ip = xprime_integrals(b, J, c, c_tilde, q)
    den = rp2[:, None] + J[None, :] ** 2 - k * k
    K = _coef_K(A3, k, b[:, None], J[None, :], den, Im, Ip)
    K = _special_fix(K, A3, b[:, None], J[None, :], c, c_tilde, q)
    return K.reshape(2 * N1, 2 * N2, 2 * N3)


def fhat_3d(k, a1, a2, N1, N2, N3, c_tilde=co.C_TILDE, eps=co.EPS, q=ORACLE_Q):
    """F-hat_j of (3.5): A3 (1 - H(|xi|)) / (|xi|^2 - k^2), shape [2N1, 2N2, 2N3]."""
    A3 = 1.0 / math.sqrt(8 * math.pi ** 2 * c_tilde)
    rp2, J = _xi_3d(a1, a2, N1, N2, N3, c_tilde)
    xi2 = rp2[:, None] + J[None, :] ** 2
    H = radial_H(k, np.sqrt(xi2), eps, q)
    with np.errstate(divide="ignore", invalid="ignore"):
        F = A3 * (1.0 - H) / (xi2 - k * k)
    # |xi| = k (the special coefficients): (1 - H)/(|xi|^2 - k^2) is 0/0 there; take the
    # radial form of the transform of e^{ikr} Y / (4 pi r) itself, (1/|xi|) int e^{ikr} Y sin(|xi| r) dr
    m = np.abs(np.sqrt(xi2) - k) < SPECIAL_SWITCH
    if m.any():
        rho = np.sqrt(xi2[m])
        r0, w0 = gauss_legendre(0.0, eps, q)
        r1, w1 = gauss_legendre(eps, 2 * eps, q)
        r = np.concatenate([r0, r1])
        w = np.concatenate([w0, w1]) * co.Y(r, eps) * np.exp(1j * k * r)
        F[m] = A3 * (np.sin(np.outer(rho, r)) @ w) / rho
    return F.reshape(2 * N1, 2 * N2, 2 * N3)


def lhat_3d(k, a1, a2, N1, N2, N3, c=co.C, c_tilde=co.C_TILDE, eps=co.EPS, q=ORACLE_Q):
    """L-hat_d = K-hat_d - F-hat (Algorithm 3.1 step 1b), shape [2N1, 2N2, 2N3]."""
    return (khat_3d(k, a1, a2, N1, N2, N3, c, c_tilde, q)
            - fhat_3d(k, a1, a2, N1, N2, N3, c_tilde, eps, q))


# The second-derivative fields of Algorithm 4.1: L^{pq} for pq = 11, 22, 33, 12, 13, 23 (the
# order of the Maxwell output).  TRACE_PAIRS is the option that drops the 33 field and takes
# GG_33 from the trace, GG_11 + GG_22 + GG_33 = 3 G_d + k^-2 Laplacian G_d = 2 G_d (the Helmholtz
# equation, off the lattice).
FIELD_PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
TRACE_PAIRS = ((0, 0), (1, 1), (0, 1), (0, 2), (1, 2))


def maxwell_multipliers(a1, a2, N1, N2, N3, c_tilde=co.C_TILDE, pairs=FIELD_PAIRS):
    """-c^p c^q for the given field pairs (Section 4), each [2N1,2N2,2N3]."""
    c1 = (a1 + np.arange(-N1, N1, dtype=np.float64))[:, None, None]
    c2 = (a2 + np.arange(-N2, N2, dtype=np.float64))[None, :, None]
    c3 = (np.arange(-N3, N3, dtype=np.float64) * math.pi / c_tilde)[None, None, :]
    cc = (c1, c2, c3)
    return [-(cc[p] * cc[q]) for p, q in pairs]


def grid_3d(Lhat, c_tilde=co.C_TILDE):
    """L_dN at the full grid [2N1,2N2,2N3] by direct separable DFT sums."""
    A3 = 1.0 / math.sqrt(8 * math.pi ** 2 * c_tilde)
    M1, M2, M3 = Lhat.shape
    g = np.tensordot(Lhat, dft_matrix(M3 // 2), axes=([2], [1]))      # [j1, j2, p3]
    g = np.tensordot(g, dft_matrix(M2 // 2), axes=([1], [1]))         # [j1, p3, p2]
    g = np.tensordot(g, dft_matrix(M1 // 2), axes=([0], [1]))         # [p3, p2, p1]
    return A3 * np.transpose(g, (2, 1, 0))


def _interp3(grids, i1, w1, i2, w2, i3, w3):
    """Tensor Lagrange over 64 nodes for each grid in ``grids``."""
    res = []
    for g in grids:
        v = g[i1[:, :, None, None], i2[:, None, :, None], i3[:, None, None, :]]
        res.append(np.einsum("ta,tb,tc,tabc->t", w1, w2, w3, v))
    return res


def _psi_derivs(k, r, eps):
    """psi = e^{ikr} Y(r)/(4 pi r) and its first two radial derivatives."""
    g = np.exp(1j * k * r) / (4 * math.pi * r)
    g1 = g * (1j * k - 1.0 / r)
    g2 = g * ((1j * k - 1.0 / r) ** 2 + 1.0 / r ** 2)
    y, y1, y2 = co.Y(r, eps), co.dY(r, eps), co.d2Y(r, eps)
    return g * y, g1 * y + g * y1, g2 * y + 2 * g1 * y1 + g * y2


def singular_part_3d(k, t, eps=co.EPS, pairs=FIELD_PAIRS):
    """The removed singular part F = psi (Section 3.2) at cell offsets t [T,3] and its second
    derivatives d_p d_q psi = psi'' t_p t_q / r^2 + psi' (delta_pq / r - t_p t_q / r^3) for the given
    pairs (the F^{pq} of Section 4): returns (psi [T], {pair: [T]})."""
    t = np.atleast_2d(np.asarray(t, dtype=np.float64))
    r = np.linalg.norm(t, axis=1)
    psi, d1, d2 = _psi_derivs(k, r, eps)
    hess = {}
    for p, q in pairs:
        tp, tq = t[:, p], t[:, q]
        hess[(p, q)] = d2 * tp * tq / r ** 2 + d1 * ((1.0 if p == q else 0.0) / r - tp * tq / r ** 3)
    return psi, hess


def prepare_3d(k, a1, a2, N1, N2, N3, maxwell=False, trace33=False, c=co.C, c_tilde=co.C_TILDE,
               eps=co.EPS, q=ORACLE_Q):
    """Algorithm 3.1 / 4.1 step 1: the near grids (L_d; for Maxwell also the six fields L^{pq},
    or five with ``trace33``)."""
    L = lhat_3d(k, a1, a2, N1, N2, N3, c, c_tilde, eps, q)
    pairs = TRACE_PAIRS if trace33 else FIELD_PAIRS
    fields = [L] + ([m * L for m in maxwell_multipliers(a1, a2, N1, N2, N3, c_tilde, pairs)] if maxwell else [])
    grids = [grid_3d(f, c_tilde) for f in fields]
    return dict(k=k, a1=a1, a2=a2, N=(N1, N2, N3), maxwell=maxwell, pairs=pairs if maxwell else (), c=c,
                c_tilde=c_tilde, eps=eps, grids=grids)


def evaluate_3d(st, x):
    """Algorithm 3.1 / 4.1 step 2 at targets x[T,3] against a prepared state.

    Returns G_d [T] or the Maxwell components [T,6] (11, 22, 33, 12, 13, 23).
    """
    k, a1, a2, c, c_tilde, eps = st["k"], st["a1"], st["a2"], st["c"], st["c_tilde"], st["eps"]
    N1, N2, N3 = st["N"]
    maxwell, pairs, grids = st["maxwell"], st["pairs"], st["grids"]
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    M1, M2, M3 = 2 * N1, 2 * N2, 2 * N3
    h1, h2, h3 = math.pi / N1, math.pi / N2, c_tilde / N3
    t1, n1 = _reduce(x[:, 0])
    t2, n2 = _reduce(x[:, 1])
    x3 = x[:, 2]
    T = len(x)
    out = np.full((T, 6 if maxwell else 1), np.nan + 0j)
    near = np.abs(x3) <= c
    if near.any():
        i1, w1 = _stencil((t1[near] + math.pi) / h1, M1)
        i2, w2 = _stencil((t2[near] + math.pi) / h2, M2)
        i3, w3 = _stencil((x3[near] + c_tilde) / h3, M3)
        Ls = _interp3(grids, i1, w1, i2, w2, i3, w3)
        tt = np.stack([t1[near], t2[near], x3[near]], axis=1)
        psi, hess = singular_part_3d(k, tt, eps, pairs)
        phase = np.exp(1j * (a1 * x[near, 0] + a2 * x[near, 1]))
        lat = np.exp(2j * math.pi * (a1 * n1[near] + a2 * n2[near]))
        # steps 2e/2g: G_d = e^{i alpha.x'} (L_dN + F); steps 2f/2h: d_p d_q G_d likewise with F^{pq}
        G = phase * Ls[0] + lat * psi
        if not maxwell:
            out[near, 0] = G
        else:
            dd = {}
            for f, pq in enumerate(pairs):
                dd[pq] = phase * Ls[f + 1] + lat * hess[pq]
            out[near] = _assemble(k, G, dd)
    far = ~near
    if far.any():
        # step 2b: |x3| > c takes the series (1.3), for Maxwell differentiated term by term
        xf = x[far]
        if not maxwell:
            out[far, 0] = truth.gd3d(k, a1, a2, xf)
        else:
            out[far] = truth.maxwell3d(k, a1, a2, xf)
    return out[:, 0] if not maxwell else out


def _assemble(k, G, dd):
    """GG_pq = delta_pq G_d + k^-2 d_p d_q G_d (eq. 4.1) in the order 11, 22, 33, 12, 13, 23; without a 33
    field (the trace option) GG_33 = 2 G_d - GG_11 - GG_22."""
    g11 = G + dd[(0, 0)] / k ** 2
    g22 = G + dd[(1, 1)] / k ** 2
    g33 = G + dd[(2, 2)] / k ** 2 if (2, 2) in dd else 2 * G - g11 - g22
    return np.stack([g11, g22, g33, dd[(0, 1)] / k ** 2, dd[(0, 2)] / k ** 2, dd[(1, 2)] / k ** 2], axis=1)


def smooth_3d(st, x):
    """The interpolated smooth part L_N(t) of Algorithm 3.1 step 2d at targets x [T,3] (near
    branch, |x3| <= c; NaN elsewhere), without the phase e^{i alpha.x'} or the add-back."""
    c, c_tilde = st["c"], st["c_tilde"]
    N1, N2, N3 = st["N"]
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    M1, M2, M3 = 2 * N1, 2 * N2, 2 * N3
    h1, h2, h3 = math.pi / N1, math.pi / N2, c_tilde / N3
    t1, _ = _reduce(x[:, 0])
    t2, _ = _reduce(x[:, 1])
    x3 = x[:, 2]
    out = np.full(len(x), np.nan + 0j)
    near = np.abs(x3) <= c
    if near.any():
        i1, w1 = _stencil((t1[near] + math.pi) / h1, M1)
        i2, w2 = _stencil((t2[near] + math.pi) / h2, M2)
        i3, w3 = _stencil((x3[near] + c_tilde) / h3, M3)
        out[near] = _interp3(st["grids"][:1], i1, w1, i2, w2, i3, w3)[0]
    return out


def eval_3d(k, a1, a2, x, N1, N2, N3, maxwell=False, trace33=False, c=co.C, c_tilde=co.C_TILDE,
            eps=co.EPS, q=ORACLE_Q):
    """Algorithm 3.1 (G_d, returns [T]) or Algorithm 4.1 (Maxwell, returns [T,6])."""
    st = prepare_3d(k, a1, a2, N1, N2, N3, maxwell, trace33, c, c_tilde, eps, q)
    return evaluate_3d(st, x)


def eval_gd3d(k, a1, a2, x, N1, N2, N3, **kw):
    return eval_3d(k, a1, a2, x, N1, N2, N3, maxwell=False, **kw)


def eval_maxwell3d(k, a1, a2, x, N1, N2, N3, trace33=False, **kw):
    return eval_3d(k, a1, a2, x, N1, N2, N3, maxwell=True, trace33=trace33, **kw)
