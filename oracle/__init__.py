"""CPU FP64 oracle for the FFT-based quasi-periodic Green's function method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package; only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, constants or
tables with the HIP library: it is written independently from the paper
(Zhang & Zhang, "An FFT-based algorithm for efficient computation of Green's
functions for the Helmholtz and Maxwell's equations in periodic domains").

Two oracles live here:

* ``truth``  -- the exact Green's functions G (eq. 1.2), G_d (eq. 1.3) and the
  Maxwell tensor (eq. 1.4), summed directly from the eigenfunction expansions
  with explicit tail bounds, plus the image expansions (1.1) for complex k.
  It measures *accuracy*.
* ``method`` -- the same discrete approximation the library computes
  (Algorithms 2.1, 3.1 and 4.1 with the frozen parameter set), evaluated
  plainly: closed-form coefficients with converged quadrature, grid values by
  direct (non-FFT) DFT sums, tensor-product cubic Lagrange interpolation and
  the exact singular add-back.  It measures *parity*.

* ``grad2d`` -- the same for the first derivatives of the 2D G (Section
  2.4.1): differentiated coefficients, the singular parts h1, h2 and their
  Fourier coefficients by Hankel transforms, add-back at the target.

* ``hess2d`` -- the differences of second derivatives of the 2D G for two
  wavenumbers (Section 2.4.2), the same way.

* ``highorder2d`` -- the 2D G with the terms of degree 2 and 3 of the
  logarithmic singularity's Taylor factor removed as well (Remark 5.3).

``cutoffs`` holds the smooth cut-off functions X and Y_eps (Section 6 states
only that they are C^8; the reading used is documented there).
"""

from . import cutoffs, truth, method, grad2d, hess2d, highorder2d  # noqa: F401
