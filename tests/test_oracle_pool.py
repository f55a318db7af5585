"""The pooled oracle helper equals the oracle run in one process."""
import os
import sys

import numpy as np

import oracle as O
from paper_2505_01231_amd import synth

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from oracle_pool import polyspectra_pooled  # noqa: E402


def test_pooled_oracle_equals_single_process():
    N, Nf, m = 256, 40, 6
    z = synth.ar2_chi2(N * m * 7 + 11, seed=9)
    a = polyspectra_pooled(z, N, Nf, m, workers=3, window_kind="hann")
    b = O.polyspectra(z, N, Nf, m, window_kind="hann")
    assert a["n_chunks"] == b["n_chunks"] == 7
    for k in ("s2", "s3", "s4", "s2_err", "s3_err", "s4_err"):
        assert np.array_equal(a[k], b[k]), k
