"""The allocation-free entry point ps_execute_static, called through the C
ABI: its outputs equal ps_execute's on the same records (same kernels and
work split, so bit for bit), on two calls in a row, the second with a
smaller input; records needing more than the static scratch are refused
before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest

from paper_2505_01231_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)


def _arrays(sp):
    return {k: getattr(sp, k).cpu().numpy() for k in ("s1", "s1_err", "s2", "s2_err", "s3", "s3_err", "s4", "s4_err")
            if getattr(sp, k) is not None}


def test_static_scratch_equals_execute():
    from paper_2505_01231_amd import Plan
    from paper_2505_01231_amd import _lib as L
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    lib = L.load()
    N, Nf, m = 1024, 160, 10
    z, _ = synth.mixed_channels(N * m * 37 + 555, seed=31)
    big = torch.from_numpy(z[:2].copy()).to(dev)
    with Plan(frame_len=N, n_freq=Nf, m=m, n_channels=2, orders=(1, 2, 3, 4), precision="bf16x3") as p:
        st = torch.cuda.current_stream(dev)
        for n_samp in (big.shape[1], N * m * 11 + 7):          # the second call is smaller
            x = big[:, :n_samp]
            say("static scratch", n_samp)
            want = _arrays(p.execute(x))
            out = p.allocate_outputs(dev)
            for t in (out.s1, out.s1_err, out.s2, out.s2_err, out.s3, out.s3_err, out.s4, out.s4_err):
                t.fill_(-1.0)
            rec = p.record(x)
            o = out.c_struct()
            rc = lib.ps_execute_static(p._handle, C.byref(rec), 1, C.byref(o), C.c_void_p(st.cuda_stream))
            L.check(rc, "ps_execute_static")
            torch.cuda.synchronize()
            got = _arrays(out)
            for k in want:
                assert np.array_equal(got[k], want[k], equal_nan=True), (n_samp, k)
        # more workspace than the static array holds: refused, nothing enqueued
        need = p.workspace_bytes([big])
        assert need < L.PS_STATIC_SCRATCH_BYTES
    with Plan(frame_len=8192, n_freq=2048, m=10) as q:
        n_big = 8192 * 10 * 400
        xb = torch.zeros(n_big, dtype=torch.float32, device=dev)
        assert q.workspace_bytes([xb]) > L.PS_STATIC_SCRATCH_BYTES
        out = q.allocate_outputs(dev)
        rec = q.record(xb)
        o = out.c_struct()
        rc = lib.ps_execute_static(q._handle, C.byref(rec), 1, C.byref(o), C.c_void_p(st.cuda_stream))
        assert rc == L.PS_E_WORKSPACE, rc
        torch.cuda.synchronize()
