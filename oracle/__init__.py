"""TEST INFRASTRUCTURE ONLY: the CPU reference ("oracle") for the free-space
Stokes sums of af Klinteberg, Shamshirgar & Tornberg (arXiv:1607.04808).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library shares no code with it.

Contents
--------
``direct``      FP64 C library (``direct.c``): direct sums of the three kernels
                (Section 2), truncated real-space sums (Section 3.2), Fourier
                parts in closed form, analytic gradients.
``se``          FP64 numpy implementation of the spectral Ewald steps
                (Sections 4-6): geometry, precompute of the mollified kernel,
                spreading, FFT, scaling, IFFT, quadrature.
"""
from . import direct  # noqa: F401
from . import se  # noqa: F401
