"""Seeded synthetic inputs shared by the tests and the benchmark.

This module holds no part of the method: it only draws targets and
(k, alpha) instances with NumPy's PCG64 generator, so that the GPU path and
the CPU oracle can be fed identical inputs.

Targets follow the paper's workloads (Section 6 evaluates fixed points in one
period cell; the benchmark uses many uniform points): uniform over one period
in the periodic coordinates and over [-1, 1] in the transverse one, rejecting
points within ``rmin`` of a lattice point (2 pi n, 0) / (2 pi n1, 2 pi n2, 0).
"""

import math

import numpy as np

TWO_PI = 2.0 * math.pi


def _lattice_distance(x):
    """Distance from each row of x (periodic coords first, transverse last) to the nearest lattice point."""
    per = x[:, :-1]
    red = per - TWO_PI * np.round(per / TWO_PI)
    return np.sqrt(np.sum(red * red, axis=1) + x[:, -1] ** 2)


def targets(T, dim, seed, rmin=1e-3, zmax=1.0):
    """T targets in [0, 2pi]^(dim-1) x [-zmax, zmax], at least rmin from the lattice.

    Draws in batches of T and keeps the first T accepted points, in draw order.
    Returned as a C-contiguous float64 array [T, dim].
    """
    rng = np.random.default_rng(seed)
    out = np.empty((0, dim))
    while len(out) < T:
        per = rng.uniform(0.0, TWO_PI, size=(T, dim - 1))
        tr = rng.uniform(-zmax, zmax, size=(T, 1))
        x = np.concatenate([per, tr], axis=1)
        out = np.concatenate([out, x[_lattice_distance(x) >= rmin]])
    return np.ascontiguousarray(out[:T])


def instances_2d(n, seed, k_range=(1.0, 20.0), a_range=(-0.5, 0.5), min_beta=1e-3, c_tilde=1.0,
                 special_tol=1e-6, n2_max=64):
    """n (k, alpha) pairs with every |k^2 - (alpha+j)^2|^(1/2) >= min_beta (away from Wood anomalies)
    and no |sqrt(k^2-(alpha+j)^2) - j2 pi/c~| below special_tol for |j2| <= n2_max."""
    rng = np.random.default_rng(seed)
    ks, als = [], []
    while len(ks) < n:
        k = rng.uniform(*k_range)
        a = rng.uniform(*a_range)
        j = np.arange(math.floor(-k - a) - 1, math.ceil(k - a) + 2)
        d = k * k - (a + j) ** 2
        if np.min(np.sqrt(np.abs(d))) < min_beta:
            continue
        prop = np.sqrt(d[d > 0])
        J = np.arange(0, n2_max + 1) * math.pi / c_tilde
        if prop.size and np.min(np.abs(prop[:, None] - J[None, :])) < special_tol:
            continue
        ks.append(k)
        als.append(a)
    return np.array(ks), np.array(als)


def x1_sizes_2d(n, seed, unit=256, most=8):
    """n x1 grid sizes unit * U{1..most} (with unit = 256: 256 .. 2048, the odd multiples taking the
    transforms' radix-3, -5 and -7 passes)."""
    rng = np.random.default_rng(seed)
    return [int(unit * v) for v in rng.integers(1, most + 1, n)]
