"""CPU FP64 reference of the surrogate network (test infrastructure only).

The surrogate models the smooth part L_d(x; k, alpha1, alpha2) that Algorithm 3.1
interpolates (K_d minus the singular part F, section 3, eq. 3.5), so that
G_d = e^{i alpha.x'} L_d(t) + e^{i 2 pi alpha.n} psi(t) with psi = e^{ikr} Y_eps(r) / (4 pi r)
added exactly (Algorithm 3.1 step 2e).  The network itself is this library's
design, not the paper's: 64 input features, four hidden layers of 256 with GELU,
a linear head to (Re, Im) of 10 L_d.

`forward` / `loss_and_grad` run in float64.  With ``bf16_ops=True`` they round the
same operands to bfloat16 (round to nearest even) that the matrix-core kernels
take in bfloat16: the features, the hidden weights, the hidden activations and
the back-propagated pre-activation gradients; every product and sum stays
float64.  The backward pass is pinned against central finite differences of the
float64 loss; the features against their periodicity.
"""

import math

import numpy as np
from scipy.special import erf

from . import method

D_IN, H, NOUT = 64, 256, 2
OUT_SCALE = 10.0            # the network predicts 10 L_d
C_NEAR, C_TILDE = 0.6, 1.0  # near region |x3| <= c, x3 period 2 c~


def layout():
    """Offsets of W0, b0, ..., W4, b4 in a member's flat parameter vector."""
    shapes = [(H, D_IN), (H,), (H, H), (H,), (H, H), (H,), (H, H), (H,), (NOUT, H), (NOUT,)]
    offs, o = [], 0
    for s in shapes:
        offs.append((o, s))
        o += int(np.prod(s))
    return offs, o


N_PARAM = layout()[1]


def unpack(p):
    offs, n = layout()
    p = np.asarray(p, dtype=np.float64)
    assert p.size == n
    return [p[o:o + int(np.prod(s))].reshape(s) for o, s in offs]


def bf16(a):
    """Round float32 values to bfloat16 (nearest even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(q, c=C_NEAR, c_tilde=C_TILDE):
    """The 64 features of queries q [B, 6] = (x1, x2, x3, k, alpha1, alpha2), float64."""
    q = np.asarray(q, dtype=np.float64)
    x1, x2, x3, k, a1, a2 = q.T
    t1 = x1 - 2 * math.pi * np.floor((x1 + math.pi) / (2 * math.pi))
    t2 = x2 - 2 * math.pi * np.floor((x2 + math.pi) / (2 * math.pi))
    cols = []
    for t in (t1, t2):
        for h in range(1, 9):
            cols += [np.cos(h * t), np.sin(h * t)]
    z = math.pi * x3 / c_tilde
    for h in range(1, 7):
        cols += [np.cos(h * z), np.sin(h * z)]
    r = np.sqrt(t1 ** 2 + t2 ** 2 + x3 ** 2)
    cols += [x3 / c, (k - 5.5) / 4.5, 2 * a1, 2 * a2]
    for arg in (k * t1, k * t2, k * x3, k * r, a1 * t1, a2 * t2, 2 * math.pi * a1, 2 * math.pi * a2):
        cols += [np.cos(arg), np.sin(arg)]
    F = np.stack(cols, axis=1)
    assert F.shape[1] == D_IN
    return F


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_d(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(p, q, bf16_ops=False):
    """Network output [B, 2] and the intermediates the backward pass needs."""
    rnd = bf16 if bf16_ops else (lambda a: np.asarray(a, dtype=np.float64))
    W = unpack(p)
    X = rnd(features(q))
    xs, zs = [X], []
    for l in range(4):
        Z = X @ rnd(W[2 * l]).T + W[2 * l + 1]
        zs.append(Z)
        X = rnd(gelu(Z))
        xs.append(X)
    out = X @ W[8].T + W[9]
    return out, (xs, zs)


def loss_and_grad(p, q, y, bf16_ops=False):
    """0.5 mean_b |out_b - y_b|^2 and its gradient, flat like p."""
    rnd = bf16 if bf16_ops else (lambda a: np.asarray(a, dtype=np.float64))
    W = unpack(p)
    out, (xs, zs) = forward(p, q, bf16_ops)
    B = out.shape[0]
    e = out - np.asarray(y, dtype=np.float64)
    loss = 0.5 * np.sum(e * e) / B
    dout = e / B
    g = [None] * 10
    g[8] = dout.T @ xs[4]
    g[9] = dout.sum(axis=0)
    dA = dout @ W[8]
    for l in range(3, -1, -1):
        dZ = dA * gelu_d(zs[l])
        dZr = rnd(dZ)
        g[2 * l] = dZr.T @ xs[l]
        g[2 * l + 1] = dZ.sum(axis=0)
        dA = dZr @ rnd(W[2 * l])
    return loss, np.concatenate([a.ravel() for a in g])


def init_params(seed):
    """He-uniform hidden weights, a small head, zero biases (any fixed draw serves the tests)."""
    rng = np.random.default_rng(seed)
    W = []
    for l in range(4):
        fan_in = D_IN if l == 0 else H
        b = math.sqrt(6.0 / fan_in)
        W += [rng.uniform(-b, b, (H, fan_in)), np.zeros(H)]
    W += [rng.uniform(-1, 1, (NOUT, H)) / math.sqrt(H), np.zeros(NOUT)]
    return np.concatenate([a.ravel() for a in W]).astype(np.float32).astype(np.float64)


def g_from_smooth(q, L, eps=0.2, c=C_NEAR):
    """G_d = e^{i alpha.x'} L + e^{i 2 pi alpha.n} psi(t) in the near region (Algorithm 3.1 step 2e);
    q [B, 6], L [B] complex; NaN where |x3| > c or the target sits on a lattice point."""
    q = np.asarray(q, dtype=np.float64)
    x1, x2, x3, k, a1, a2 = q.T
    t1, n1 = method._reduce(x1)
    t2, n2 = method._reduce(x2)
    r = np.sqrt(t1 ** 2 + t2 ** 2 + x3 ** 2)
    G = np.exp(1j * (a1 * x1 + a2 * x2)) * L
    lat = np.exp(2j * math.pi * (a1 * n1 + a2 * n2))
    rr = np.where(r > 0, r, 1.0)
    psi = method._psi_derivs(k, rr, eps)[0]
    G = G + np.where(r < 2 * eps, lat * psi, 0.0)
    return np.where((np.abs(x3) <= c) & (r > 0), G, np.nan + 0j)
