"""FP64 CPU oracle for MUFFIN and ADA-PT'ed MUFFIN (arXiv 1905.08468).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of the paper's method, written to check the GPU library.  Only
the test suite, the smoke check and the benchmark's CPU-baseline leg may
import it.  It shares no code with the GPU library (no kernels, tables,
filter generators or helpers); both only read the seeded inputs made by the
separate ``synth`` module.

Modules
-------
daubechies  Daubechies extremal-phase filters by spectral factorisation
            (mpmath, 60 digits).
operators   H_l / H_l^T (windowed linear convolution, direct and FFT forms),
            the union-of-Daubechies analysis operator W_s and its adjoint,
            the orthonormal DCT W_lambda and its adjoint.
muffin      weights, step sizes, power iteration, one MUFFIN iteration
            (Algs. 1-2), the derivative recursions (Algs. 3-4), PSURE-FDMC,
            SUGAR-FDMC and the ADA-PT loop (Alg. 5), the objective, the
            quality measures SNR and WMSE (Section 4.1).
visibility  the visibility-domain direct operator (exact Fourier sums at the
            bands' sample positions), its adjoint and point spread function.
unmix       per-pixel positivity-constrained least squares against chosen
            endmember spectra (the unmixing step of Section 4.3).

Every function states the passage of the paper it follows.  Functions whose
result no independent pin checks are marked "parity unpinned" in their
docstring.
"""
from .daubechies import daubechies_lowpass, daubechies_bank  # noqa: F401
from . import operators, muffin, unmix, visibility  # noqa: F401
