"""FP64 CPU oracle of the polyspectrum estimator -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It is written from the paper alone, shares no code with
the GPU library, and the GPU library never imports it.
"""
from .polyspec_oracle import (  # noqa: F401
    ESTIMATORS, average_with_error, c3opt3, chunk_count, chunk_frames, chunk_spectra,
    coefficients, coefficients_at, incomplete4, kstat2, kstat3, kstat4,
    kstat4_factorized, natural2, natural3, natural4, polyspectra, polyspectra_at,
    polyspectra_complex, polyspectra_interlaced, trispectrum_at,
    window,
)
