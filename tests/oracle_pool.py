"""The FP64 oracle over many chunks of one record on a pool of worker
processes (test infrastructure): one chunk per task, the per-chunk spectra
gathered in order and averaged by the oracle's own Section 4.2 function.
The workers are fresh interpreters that import only numpy and the oracle."""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np


def _one_chunk(args):
    import oracle as O
    z, N, Nf, m, kw = args
    out = O.polyspectra(np.asarray(z, dtype=np.float64), N, Nf, m, return_chunks=True, **kw)
    return out["chunks2"][0], out["chunks3"][0], out["chunks4"][0]


def polyspectra_pooled(z, N: int, Nf: int, m: int, workers: int | None = None, **kw) -> dict:
    """O.polyspectra(z, N, Nf, m, **kw) for S2, S3 and S4 of one channel,
    evaluated chunk by chunk in parallel."""
    import oracle as O
    n_chunks = O.chunk_count(len(z), N, m)
    span = N * m
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    per2 = per3 = per4 = None
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    os.environ.update({k: "1" for k in saved})
    try:
        with mp.get_context("spawn").Pool(workers) as pool:
            tasks = [(np.asarray(z[c * span:(c + 1) * span]), N, Nf, m, kw) for c in range(n_chunks)]
            for c, (a2, a3, a4) in enumerate(pool.imap(_one_chunk, tasks)):
                if per2 is None:
                    per2 = np.empty((n_chunks,) + a2.shape, np.complex128)
                    per3 = np.empty((n_chunks,) + a3.shape, np.complex128)
                    per4 = np.empty((n_chunks,) + a4.shape, np.complex128)
                per2[c], per3[c], per4[c] = a2, a3, a4
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    out = {"n_chunks": n_chunks}
    for key, per in (("s2", per2), ("s3", per3), ("s4", per4)):
        out[key], out[key + "_err"] = O.average_with_error(per)
        del per
    return out
