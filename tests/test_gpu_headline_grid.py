"""The whole N_f = 2048 grid at the benchmark's frame length (N = 8192,
m = 10) on the first 2^22 samples of the benchmark record (51 chunks): S2, S3,
S4 and every error bar against the FP64 oracle, over every grid point, in all
three precisions (tolerance 1e-5, maximum over the grid normalised to the
spectrum's maximum magnitude).  The oracle runs chunk by chunk on a worker
pool (tests/oracle_pool.py)."""
import os
import sys

import numpy as np
import pytest

from paper_2505_01231_amd import synth

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from oracle_pool import polyspectra_pooled  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N, NF, M = 8192, 2048, 10
TOL = 1e-5


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def record_and_oracle():
    z = synth.ar2_chi2(1 << 22, seed=3)
    say("headline grid: oracle on 51 chunks")
    ref = polyspectra_pooled(z, N, NF, M, window_kind="acg")
    assert ref["n_chunks"] == 51
    return z, ref


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x2s"])
def test_headline_grid_full_parity(record_and_oracle, precision):
    from paper_2505_01231_amd import Plan
    z, ref = record_and_oracle
    dev = torch.device("cuda:0")
    say("headline grid", precision)
    with Plan(frame_len=N, n_freq=NF, m=M, window="acg", precision=precision) as p:
        out = p.execute(torch.from_numpy(z).to(dev))
        torch.cuda.synchronize()
        errs = {}
        for k in ("s2", "s3", "s4"):
            got = torch.view_as_complex(getattr(out, k)).cpu().numpy()[0]
            errs[k] = _rel(got, ref[k][0])
            errs[k + "_err"] = _rel(getattr(out, k + "_err").cpu().numpy()[0], ref[k + "_err"][0])
    say("  full-grid rel err", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= TOL, (precision, k, v)
