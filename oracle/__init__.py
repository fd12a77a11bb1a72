"""CPU FP64 oracle of the Lippmann--Schwinger corrector solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
this package: only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark call it.  It is a plain, slow, deliberately unoptimised NumPy
implementation written from the paper (Brisard & Legoll, "Periodic
homogenization using the Lippmann--Schwinger formalism"):

* ``tensors``   -- Mandel notation helpers (oracle-private).
* ``green``     -- the periodic Green operator of Section 2.2.1 and its
                   truncated (eqs. 14/15 and the Nyquist rule of Section
                   3.2.1), filtered (Section 3.2.2), consistent (eq. 11) and
                   finite-difference (Section 3.2.3) discretisations.
* ``operator``  -- the discrete operator of eq. (13) applied with full complex
                   FFTs, and its right-hand side (eq. 9).
* ``dense``     -- the same system assembled in real space as the block
                   circulant matrix of eq. (12) with direct DFT sums (no FFT)
                   and solved with LAPACK; for grids of at most a few hundred
                   voxels.
* ``solvers``   -- textbook conjugate gradients and the basic fixed-point
                   scheme of Moulinec and Suquet.
* ``effective`` -- the homogenised matrix of Theorem 4 (A*_h p = A0 p + mean
                   of the polarisation).

Every function states the passage it follows.  Where the paper is silent the
reading adopted is stated in the docstring.
"""
