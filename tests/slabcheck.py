"""Far-slab node checks shared by the GPU stage tests (test infrastructure).

A far-slab value times the phase e^{i alpha.x'} is the eigenfunction series at that node
(Algorithms 2.1 / 3.1 / 4.1 step 2b), so sampled nodes are compared with the direct sum of the
series (``oracle.truth``): slice s lies at |x_t| = c - (P/2 - 1) h_f + s h_f (P = far_points), x1 node p (FFT order) at
2 pi p / far_m1 (centred p), likewise x2 in 3D.
"""

import math

import numpy as np

from oracle import truth


def _centred(p, m):
    return np.where(p < m // 2, p, p - m)


def nodes_2d(info, n, seed):
    """n sampled (slice, x1-node) pairs: indices into the [S][Mf1] slab and the node coordinates."""
    rng = np.random.default_rng(seed)
    s = rng.integers(0, info.far_slices, n)
    p = rng.integers(0, info.far_m1, n)
    x1 = 2 * math.pi * _centred(p, info.far_m1) / info.far_m1
    z = info.c - (info.far_points // 2 - 1) * info.far_h + s * info.far_h
    return (s, p), np.stack([x1, z], axis=1)


def nodes_3d(info, n, seed):
    rng = np.random.default_rng(seed)
    s = rng.integers(0, info.far_slices, n)
    q = rng.integers(0, info.far_m2, n)
    p = rng.integers(0, info.far_m1, n)
    x1 = 2 * math.pi * _centred(p, info.far_m1) / info.far_m1
    x2 = 2 * math.pi * _centred(q, info.far_m2) / info.far_m2
    z = info.c - (info.far_points // 2 - 1) * info.far_h + s * info.far_h
    return (s, q, p), np.stack([x1, x2, z], axis=1)


def slab_2d(P, field=0):
    return P.field(which=1, field=field).cpu().numpy().reshape(P.info.far_slices, P.info.far_m1)


def slab_3d(P, field=0):
    i = P.info
    return P.field(which=1, field=field).cpu().numpy().reshape(i.far_slices, i.far_m2, i.far_m1)


def rel(g, o):
    return float(np.abs(g - o).max() / np.abs(o).max())


def limit(info):
    """Smallest |x_t| beyond the far slab (flag bit 2): the P slices from floor((z - z0)/hf) - (P/2 - 1)
    must stay below S, z0 = c - (P/2 - 1) hf, P = far_points."""
    return info.c + (info.far_slices - info.far_points + 1) * info.far_h
