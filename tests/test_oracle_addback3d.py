"""Pins of the 3D near-lattice add-back (Algorithm 3.1 steps 2e-2f, Algorithm 4.1 steps 2e-2i).

The oracle adds back the removed singular part F = psi = e^{ikr} Y_eps(r) / (4 pi r) (Section 3.2)
and, for the Maxwell tensor, its second derivatives F^{pq} = d_p d_q psi (Section 4), with the
lattice phase e^{i 2 pi alpha.n} of the cell the target falls in (reading G6).  These tests pin
each piece against something other than its own formula:

* the second derivatives against fourth-order central differences of psi, inside r < eps and in the
  cut-off shell eps < r < 2 eps (where Y', Y'' enter);
* psi against the Helmholtz equation: inside r < eps, Delta psi + k^2 psi = 0;
* the whole chain next to lattice points of other cells (r < 2 eps, |x3| >= 0.08) against the lattice
  sum (1.3): the error must fall with N, which a sign or phase error in psi or in the lattice phase
  (an O(1) error at every N) would prevent;
* the paper's printed errors at P^3_4 = (0.03, 0.03, 0.1) (Tables 10 and 11), as far as the frozen
  cut-offs allow: with them the method trails the paper's by about one doubling of N.
"""

import math
import os

import numpy as np
import pytest

from oracle import method, truth

K, A1, A2 = 3.7, 0.2, 0.35
PAIRS = method.FIELD_PAIRS
HERE = os.path.dirname(os.path.abspath(__file__))


def _dirs(n, seed):
    d = np.random.default_rng(seed).normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


@pytest.mark.parametrize("r", [0.05, 0.15, 0.23, 0.29, 0.37])
def test_singular_hessian_by_finite_differences(r):
    t = r * _dirs(6, seed=int(100 * r))
    psi, hess = method.singular_part_3d(K, t, pairs=PAIRS)
    h = min(3e-4, 0.01 * r)
    e = np.eye(3)

    def f(pts):
        return method.singular_part_3d(K, pts, pairs=())[0]

    for (p, q) in PAIRS:
        if p == q:
            # f'' = (-f(2h) + 16 f(h) - 30 f(0) + 16 f(-h) - f(-2h)) / (12 h^2)
            fd = (-f(t + 2 * h * e[p]) + 16 * f(t + h * e[p]) - 30 * f(t) + 16 * f(t - h * e[p])
                  - f(t - 2 * h * e[p])) / (12 * h * h)
        else:
            def d1(pts):
                return (-f(pts + 2 * h * e[q]) + 8 * f(pts + h * e[q]) - 8 * f(pts - h * e[q])
                        + f(pts - 2 * h * e[q])) / (12 * h)
            fd = (-d1(t + 2 * h * e[p]) + 8 * d1(t + h * e[p]) - 8 * d1(t - h * e[p]) + d1(t - 2 * h * e[p])) / (12 * h)
        scale = max(np.abs(hess[(p, q)]).max(), np.abs(psi).max() / r ** 2)
        assert np.abs(hess[(p, q)] - fd).max() <= 1e-6 * scale, (r, p, q)


def test_singular_part_solves_helmholtz_inside_eps():
    # inside r < eps, Y = 1 and psi is the outgoing free-space Green's function: Delta psi = -k^2 psi
    t = np.vstack([r * _dirs(4, seed=7) for r in (0.03, 0.08, 0.15, 0.19)])
    psi, hess = method.singular_part_3d(K, t, pairs=PAIRS)
    lap = hess[(0, 0)] + hess[(1, 1)] + hess[(2, 2)]
    assert np.max(np.abs(lap + K * K * psi) / np.abs(K * K * psi)) < 1e-12
    # and it behaves like 1/(4 pi r) at the origin (the normalisation that cancels the lattice sum's pole)
    r = np.linalg.norm(t, axis=1)
    assert np.max(np.abs(psi * 4 * math.pi * r - np.exp(1j * K * r))) < 1e-14


# targets next to lattice points of other cells: r < eps and in the shell, |x3| >= 0.08
TP = 2 * math.pi
NEAR = np.array([[TP + 0.03, -TP + 0.03, 0.1],     # P^3_4 one cell over (r = 0.109)
                 [0.1, 0.05 - TP, 0.25],           # r = 0.274 (shell)
                 [2 * TP - 0.2, 0.1, -0.15],       # r = 0.269, x3 < 0
                 [-TP - 0.3, 0.1, 0.12],           # r = 0.338
                 [0.05, TP - 0.12, 0.08]])         # r = 0.153


@pytest.mark.slow
def test_gd3d_near_lattice_converges_to_the_lattice_sum():
    gt = truth.gd3d(K, A1, A2, NEAR)
    errs = []
    for N in (16, 32, 64):
        g = method.eval_gd3d(K, A1, A2, NEAR, N, N, N)
        errs.append(np.abs(g - gt) / np.abs(gt))
    # measured: max 0.31 / 0.094 / 0.0084
    assert errs[2].max() < 1e-2 and errs[2].max() < errs[0].max() / 20
    assert np.all(errs[2] < errs[0] / 4)


@pytest.mark.slow
def test_maxwell_near_lattice_addback_against_the_lattice_sum():
    # Algorithm 4.1 next to a lattice point of another cell, inside r < eps (Y' = Y'' = 0 there, so the
    # add-back is the exact Hessian of the outgoing Green's function, |d_p d_q psi| / k^2 ~ 5 here against
    # |GG| ~ 1.6): the error falls from N = 32 to 64 and stays far below the add-back's size, which a
    # sign or phase error in it would not.  (The slow convergence itself is the method's with the frozen
    # cut-offs: the 64-point stencils of the second-derivative fields reach into the steep cut-off shell.)
    x = np.array([[TP + 0.03, 0.03 - TP, 0.1]])
    gm = truth.maxwell3d(K, A1, A2, x)
    _, hs = method.singular_part_3d(K, x - [TP, -TP, 0.0], pairs=PAIRS)
    add = np.array([abs(hs[pq][0]) for pq in PAIRS]) / K ** 2
    errs = []
    for N in (32, 64):
        g = method.eval_maxwell3d(K, A1, A2, x, N, N, N)
        errs.append(np.abs(g - gm)[0])
    # measured: max 0.19 at N = 32, 0.063 at N = 64, against add-back entries of 0.9 .. 5
    assert np.all(errs[1] < 0.1 * add.max()) and errs[1].max() < 0.5 * errs[0].max()


def _golden_3d():
    path = os.path.join(HERE, "golden", "paper_tables_3d.txt")
    rows = []
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            tab, kind, k, a1, a2, N, x1, x2, x3, err = line.split()
            rows.append((tab, kind, float(k), float(a1), float(a2), int(N), float(x1), float(x2), float(x3),
                         float(err)))
    return rows


@pytest.mark.slow
def test_paper_tables_3d_gd_at_p34():
    """Tables 10 and 11 (Section 6.2.1), G_d at P^3_4 = (0.03, 0.03, 0.1), where r < eps.  The paper's
    cut-offs are unspecified; with the frozen ones (C^8 transitions, eps = 0.2) the error at 2N is within
    a decade of the paper's at N (measured ratios 3.3 and 2.7), and a sign or phase error in the add-back
    would be O(1)."""
    rows = [r for r in _golden_3d() if r[1] == "Gd"]
    paper = {(r[2], r[5]): r[9] for r in rows}
    for k, a1, a2 in sorted({(r[2], r[3], r[4]) for r in rows}):
        x = np.array([[rows[0][6], rows[0][7], rows[0][8]]])
        gt = truth.gd3d(k, a1, a2, x)[0]
        e64 = abs(method.eval_gd3d(k, a1, a2, x, 64, 64, 64)[0] - gt) / abs(gt)
        assert e64 < 10 * paper[(k, 32)], (k, e64, paper[(k, 32)])


@pytest.mark.slow
def test_paper_tables_3d_maxwell_at_p34():
    """Tables 22 and 23 (Section 6.3), the Maxwell tensor at P^3_4: the paper prints 9e-6 and 6e-6 at
    N = 64; with the frozen cut-offs the method's largest entry error there is 3e-2 and 4e-2 (GG_11 and
    GG_22; the stencils of their fields reach into the cut-off shell), three to four decades above the
    paper's.  Pinned: below 0.1 at N = 64 and falling from N = 32, i.e. no O(1) error in the add-back."""
    rows = [r for r in _golden_3d() if r[1] == "Mx"]
    for k, a1, a2 in sorted({(r[2], r[3], r[4]) for r in rows}):
        x = np.array([[rows[0][6], rows[0][7], rows[0][8]]])
        gt = truth.maxwell3d(k, a1, a2, x)[0]
        e = [np.max(np.abs(method.eval_maxwell3d(k, a1, a2, x, N, N, N)[0] - gt) / np.abs(gt)) for N in (32, 64)]
        assert e[1] < 0.1 and e[1] < e[0], (k, e)
