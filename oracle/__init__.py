"""Independent FP64 CPU oracle for the additive-kernel fast summation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_2404_17344_amd``) and never imports it.

Contents
--------
``direct``   -- plain O(N^2) sums of the windowed additive kernel and its
                l- and sigma-derivatives (C, OpenMP; ``direct.c``).
``fourier``  -- the paper's Fourier-side steps written out plainly in NumPy:
                continuous Fourier transforms of the kernels, periodised
                Fourier coefficients (analytic and sampled), the trigonometric
                sum of eq. (6) evaluated by brute force, the error bounds of
                Theorems 1-2 / Remarks 1-2, and the global sensitivity
                indices of Algorithm 1.
``nearfield`` -- the near-field corrected product for the Matern-1/2 kernel:
                image-free folded torus, Taylor-joint inner regularisation,
                coefficients of the regularised kernel by a DFT of samples,
                trigonometric sum plus a direct sum over close pairs.
"""
from .direct import oracle_direct, oracle_vjp, oracle_threads, build_oracle, lib_path  # noqa: F401
