"""FP64 CPU oracle for the visibility-based binned bispectrum estimator.

Gill & Bharadwaj 2025 (arXiv:2506.10526), "A Visibility-based 21 cm Bispectrum
Estimator for Radio-interferometric Data".

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference that the HIP library is checked against.  Only the test suite,
`__graft_entry__.smoke()` and the `cpu_baseline` leg of `bench.py` may import
it; the product path (`paper_2506_10526_amd`) never does, and the oracle never
imports the product path or its compiled library.  The two share nothing but
the seeded input generator `paper_2506_10526_amd.synth`, which holds none of
the estimator's arithmetic.

Everything here is plain NumPy in float64 / complex128.  Library primitives
used as steps: numpy.fft (rfft2/irfft2/fft/irfftn) and numpy.matmul/einsum.

Modules
-------
bins        ring / shell binning and candidate triangles (Sec. 3.2, Fig. 1)
estimator   filtered fields, MABS and 3D estimators (Eqs. iFT, iFT_I, estimator_t)
brute       direct enumeration of closed grid triangles (Sec. 3.2)
theory      closed-form bispectrum of the quadratic field (Eq. mb1, Eq. bsana),
            N_nu sampling (Sec. 5, Fig. 2), route equivalence (Eq. dft)
generator   counter-based (Philox4x64-10) seeded cubes of the quadratic field (Sec. 4),
            the definition the GPU Monte Carlo generator is checked against
"""
from . import bins, estimator, brute, theory, generator  # noqa: F401
