"""FP64 CPU oracle for the PICO noise-map path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, calls or
links this package; only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the GPU path: its own Philox,
its own operators (numpy FFTs written literally as the centred orthonormal
transforms), its own conjugate gradients, its own estimator.

Every function follows the paper (Dalmaz et al., "Fast Voxelwise SNR
Estimation for Iterative MRI Reconstructions") and cites the section,
equation or algorithm it restates.  Floating point is float64 / complex128
throughout.

Pins (what each part is checked against, in tests/test_oracle_*.py):
  philox        numpy's library Philox4x64-10 (same round function, 64-bit
                constants); statistical moments of the derived probes.
  sense         closed-form SENSE variance for uniform undersampling vs the
                dense inverse built from the FFT operators; R=1 diagonal M;
                adjointness; whitening invariance.
  solvers       converged CG == LAPACK dense solve; power method == largest
                eigenvalue from LAPACK.
  pico          exact enumeration of all QPSK / Rademacher probes on tiny
                grids reproduces diag(Sigma); single-probe exactness at R=1;
                Re-part variance formulas; Tikhonov Loewner shrinkage.
  nufft         direct NUDFT adjointness; KB gridding within its error of the
                NUDFT; Toeplitz normal operator == NUDFT normal operator.
  wavelet       orthonormality of the derived db4 filters; perfect
                reconstruction; vanishing moments.
  cs            tangent vs central finite differences; tau=0 reduces to the
                linear unrolled map.
"""
from . import philox, sense, solvers, pico, nufft  # noqa: F401
