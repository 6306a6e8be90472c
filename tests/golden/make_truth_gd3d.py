"""Write truth_gd3d_k3.7.txt: the exact G_d (lattice sum eq. 1.3, oracle.truth) at a seeded sample
of the 3D benchmark targets (k = 3.7, alpha = (0.2, 0.35); 1e7 targets uniform in [0, 2pi]^2 x [-1, 1],
seed 2; 2000 of them drawn with seed 12 among those with |x3| >= 0.02, where the spectral series
converges within its term budget).  Calls only oracle/ and the seeded target generator.

    python tests/golden/make_truth_gd3d.py
"""

import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import truth  # noqa: E402
from paper_1801_05977_amd import workloads  # noqa: E402

K, A1, A2 = 3.7, 0.2, 0.35
T, N, TOL, ZMIN = 10_000_000, 2000, 1e-14, 0.02
OUT = os.path.join(HERE, "truth_gd3d_k3.7.txt")


def _one(row):
    return truth.gd3d(K, A1, A2, row[None, :], tol=TOL)[0]


def main():
    x = workloads.targets(T, 3, seed=2)
    ok = np.flatnonzero(np.abs(x[:, 2]) >= ZMIN)
    idx = np.sort(np.random.default_rng(12).choice(ok, N, replace=False))
    xs = x[idx]
    with Pool(int(os.environ.get("NPROC", "8"))) as pool:
        g = np.array(pool.map(_one, list(xs), chunksize=8))
    with open(OUT, "w") as f:
        f.write(f"# exact G_d, eq. 1.3 lattice sum (tail bound {TOL:g}); k={K} alpha=({A1},{A2})\n")
        f.write(f"# benchmark targets: workloads.targets(1e7, 3, seed=2), rows idx = sorted choice(seed 12) "
                f"among |x3| >= {ZMIN}\n")
        f.write("# idx x1 x2 x3 re im\n")
        for i, r, v in zip(idx, xs, g):
            f.write(f"{int(i)} {float(r[0])!r} {float(r[1])!r} {float(r[2])!r} {float(v.real)!r} {float(v.imag)!r}\n")


if __name__ == "__main__":
    main()
