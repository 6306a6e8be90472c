"""qpgf: quasi-periodic Green's functions by the FFT-based method on MI355X (gfx950).

The compute path is the HIP shared library ``libqpgf.so`` built from ``csrc/``
(C ABI declared in ``include/qpgf.h``); ``qpgf.py`` is a thin ctypes binding
over it.  Importing the package does not load the library; the first call
into ``qpgf`` does, and fails loudly if it has not been built.
"""

__all__ = ["qpgf", "workloads"]
