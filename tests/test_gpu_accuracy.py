"""Accuracy against the exact G_d (the lattice sum eq. 1.3, stored by tests/golden/make_truth_gd3d.py
at 2000 of the benchmark's targets) for the benchmark instance k = 3.7, alpha = (0.2, 0.35), at the
benchmark grid and refined grids.

The method's error is that of the truncated Fourier representation and the cubic interpolation
(sections 3 and 5); the parity tests compare with the oracle instead.  Error of a result set:
max_i |g_i - o_i| / max(|o_i|, s) with s the RMS of |o| (p50 / p99 / max reported).
"""

import os

import numpy as np
import pytest
import torch

from paper_1801_05977_amd import qpgf

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
K, A1, A2 = 3.7, 0.2, 0.35


def _truth():
    d = np.loadtxt(os.path.join(HERE, "golden", "truth_gd3d_k3.7.txt"))
    return d[:, 1:4].copy(), d[:, 4] + 1j * d[:, 5]


def _errors(g, o):
    s = np.sqrt(np.mean(np.abs(o) ** 2))
    e = np.abs(g - o) / np.maximum(np.abs(o), s)
    return np.percentile(e, 50), np.percentile(e, 99), e.max()


# grid -> bounds on (p99, max), both precisions; measured values on this sample are about half of these.
# 512 x 512 x 128 is the smallest of these grids whose p99 error is below 1e-6 (complex128).  The
# complex64 path adds its own rounding: the far branch sums 512 single-precision products per target,
# about 1e-6 of |G| at the 99th percentile, so its p99 bound is at least 1.5e-6.
GRIDS = [((256, 256, 64), (1.5e-3, 4e-3)), ((512, 512, 64), (1.5e-3, 3e-3)), ((256, 256, 128), (5e-6, 4e-3)),
         ((512, 512, 128), (1e-6, 5e-4)), ((1024, 1024, 256), (1e-6, 5e-5))]


@pytest.mark.timeout(600)
def test_accuracy_against_the_lattice_sum():
    x, o = _truth()
    xd = torch.from_numpy(x).cuda()
    rows = []
    for (M1, M2, M3), bound in GRIDS:
        for prec in (qpgf.C128, qpgf.C64):
            P = qpgf.Plan(qpgf.KIND_GD3D, prec, M1, M2, M3)
            g = P(K, A1, A2, xd).cpu().numpy().astype(np.complex128)
            p50, p99, mx = _errors(g, o)
            rows.append(((M1, M2, M3), "c128" if prec == qpgf.C128 else "c64", p50, p99, mx))
            print(f"\ngrid {M1}x{M2}x{M3} {rows[-1][1]:5s} p50 {p50:.2e} p99 {p99:.2e} max {mx:.2e}", flush=True)
            if prec == qpgf.C128:
                s_ = np.sqrt(np.mean(np.abs(o) ** 2))
                e = np.abs(g - o) / np.maximum(np.abs(o), s_)
                for i in np.argsort(e)[-3:]:
                    t = np.mod(x[i, :2] + np.pi, 2 * np.pi) - np.pi
                    print(f"   worst: err {e[i]:.1e} x3 {x[i, 2]:+.4f} |t| {np.hypot(*t):.4f} |G| {abs(o[i]):.2e}")
            p99_bound = bound[0] if prec == qpgf.C128 else max(bound[0], 1.5e-6)
            assert p99 <= p99_bound and mx <= bound[1], (M1, M2, M3, prec)
            P.close()
            del P
            torch.cuda.empty_cache()
    assert all(np.isfinite(r[4]) for r in rows)
