"""The far slab's cut of negligible terms, checked on the host.

The slab drops every evanescent term (c/q) e^{-qz} of the series (1.3) with q z above a fixed
constant (q^2 = |xi|^2 - k^2, xi = (alpha1 + j1, alpha2 + j2)), deciding before any square root,
and leaves unwritten the columns (G_d) and rows (Maxwell) in which every term is dropped.  These
tests sum, in numpy, the magnitudes of every dropped term over the whole mode grid of real slab
geometries and compare them with the terms that are kept: the cut must sit far below FP64
rounding of the slab's values.  They also check that a column (row) flagged empty by its own
coordinate alone holds only dropped terms.
"""

import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
C3 = 1.0 / (8.0 * math.pi ** 2)   # the series (1.3): (i / 8 pi^2) beta^-1 e^{i beta z}


def cut_qz():
    src = open(os.path.join(ROOT, "paper_1801_05977_amd", "csrc", "qpgf_internal.h")).read()
    m = re.search(r"constexpr double kFarNegligibleQz = ([0-9.eE+-]+);", src)
    assert m, "the cut's constant is not where the library declares it"
    return float(m.group(1))


def modes(M1, M2, a1, a2):
    j1 = np.where(np.arange(M1) < M1 // 2, np.arange(M1), np.arange(M1) - M1)
    j2 = np.where(np.arange(M2) < M2 // 2, np.arange(M2), np.arange(M2) - M2)
    return (a1 + j1)[None, :], (a2 + j2)[:, None]


@pytest.mark.parametrize("k,a1,a2,M,z0", [
    (3.7, 0.2, 0.35, 512, 0.6 - 3 / 64),      # the 3D benchmark instance, complex128 slab, lowest slice
    (3.7, 0.2, 0.35, 512, 0.6 - 1 / 64),      # the same, complex64 slab (4-point rule)
    (9.5, -0.45, 0.1, 1024, 0.6 - 3 / 128),   # a large wavenumber: 1024^2 modes, spacing 1/128
    (1.0, 0.5, -0.5, 512, 0.6 - 3 / 64),      # a small one
])
def test_dropped_terms_are_negligible(k, a1, a2, M, z0):
    Q = cut_qz()
    x1, x2 = modes(M, M, a1, a2)
    r2 = x1 ** 2 + x2 ** 2
    d = r2 - k * k
    dropped = d * z0 * z0 > Q * Q
    assert dropped.mean() > 0.5   # most of the slab's modes are past the cut at these heights
    q = np.sqrt(np.where(dropped, d, 1.0))
    term = np.where(dropped, C3 * np.exp(-q * z0) / q, 0.0)
    prop = d < 0
    kept_max = np.max(C3 / np.sqrt(-d[prop]))   # the propagating terms c/p
    # the estimate 2 pi c e^{-Q} / z of the dropped sum (one mode per unit area; the lattice sum
    # is within a few per cent of it), and its size against the kept terms
    assert term.sum() <= 1.5 * 2 * math.pi * C3 * math.exp(-Q) / z0
    assert term.sum() <= 1e-19 * kept_max
    # the Maxwell entries multiply each term by at most 1 + |xi|^2 / k^2
    assert (term * (1.0 + r2 / (k * k))).sum() <= 1e-16 * kept_max


@pytest.mark.parametrize("k,a,z", [(3.7, 0.2, 0.553), (9.5, -0.45, 0.58), (3.7, 0.35, 1.0)])
def test_empty_band_holds_only_dropped_terms(k, a, z):
    """A column j1 with ((alpha1 + j1)^2 - k^2) z^2 past the cut holds no kept term for any j2."""
    Q = cut_qz()
    x1, x2 = modes(1024, 1024, a, 0.3)
    band_empty = (x1 ** 2 - k * k) * (z * z) > Q * Q            # per column
    elem_dropped = (x1 ** 2 + x2 ** 2 - k * k) * (z * z) > Q * Q  # per term
    assert band_empty.any() and not band_empty.all()
    assert np.all(elem_dropped[:, band_empty[0]])
