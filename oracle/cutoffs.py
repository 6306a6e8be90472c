"""Smooth cut-off functions X (Section 2.1) and Y_eps (Section 2.2).  TEST INFRASTRUCTURE ONLY.

The paper requires X(t) = 1 for |t| <= c, X(t) = 0 for |t| >= (c + c~)/2
(Section 2.1), Y_eps(t) = 1 on [0, eps] and 0 on [2 eps, inf) (Section 2.2),
and states in Section 6 that both are C^8.  It does not give their shape.
Reading used here: the transition is the smoothstep

    S(u) = I_u(9, 9)        (regularized incomplete beta function)

which rises from 0 at u = 0 to 1 at u = 1 and whose first 8 derivatives vanish
at both ends, so it joins the constant pieces in C^8.  Its derivative is the
Beta(9,9) density, S'(u) = u^8 (1-u)^8 / B(9,9), with 1/B(9,9) = 17!/(8! 8!).

    X(t)     = 1 - S((|t| - c) / w),   w = (c~ - c) / 2
    Y_eps(r) = 1 - S((r - eps) / eps)

Frozen method parameters (Section 6 fixes c = 0.6 and c~ = 1; eps is not
given, 0.2 is used).
"""

import math

import numpy as np
from scipy.special import betainc

C = 0.6          # near/far threshold c, Section 6
C_TILDE = 1.0    # periodisation half-length c~, Section 6
EPS = 0.2        # singular-part cut-off radius eps (paper: eps << 1; reading)

_INV_BETA_9_9 = math.factorial(17) / (math.factorial(8) ** 2)   # 1 / B(9, 9)


def smoothstep(u):
    """S(u) = I_u(9,9), clamped to 0 below u=0 and 1 above u=1."""
    u = np.clip(np.asarray(u, dtype=np.float64), 0.0, 1.0)
    return betainc(9.0, 9.0, u)


def smoothstep_d1(u):
    """S'(u): the Beta(9,9) density on (0,1), zero outside."""
    u = np.asarray(u, dtype=np.float64)
    inside = (u > 0.0) & (u < 1.0)
    uu = np.where(inside, u, 0.0)
    return np.where(inside, _INV_BETA_9_9 * uu ** 8 * (1.0 - uu) ** 8, 0.0)


def smoothstep_d2(u):
    """S''(u) = d/du [u^8 (1-u)^8] / B(9,9)."""
    u = np.asarray(u, dtype=np.float64)
    inside = (u > 0.0) & (u < 1.0)
    uu = np.where(inside, u, 0.0)
    d = 8.0 * uu ** 7 * (1.0 - uu) ** 8 - 8.0 * uu ** 8 * (1.0 - uu) ** 7
    return np.where(inside, _INV_BETA_9_9 * d, 0.0)


def X(t, c=C, c_tilde=C_TILDE):
    """Transverse cut-off X(t) of Section 2.1 (even in t)."""
    w = 0.5 * (c_tilde - c)
    return 1.0 - smoothstep((np.abs(t) - c) / w)


def dX(t, c=C, c_tilde=C_TILDE):
    """X'(t) for t >= 0 (the only side the coefficient integrals use)."""
    w = 0.5 * (c_tilde - c)
    return -smoothstep_d1((np.asarray(t) - c) / w) / w


def Y(r, eps=EPS):
    """Singular-part cut-off Y_eps(r) of Section 2.2."""
    return 1.0 - smoothstep((np.asarray(r) - eps) / eps)


def dY(r, eps=EPS):
    return -smoothstep_d1((np.asarray(r) - eps) / eps) / eps


def d2Y(r, eps=EPS):
    return -smoothstep_d2((np.asarray(r) - eps) / eps) / eps ** 2
