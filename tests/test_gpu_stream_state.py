"""Running accumulation over a record delivered in pieces, with checkpoint
and resume (ps_stream_*), and the per-point comparison of two estimates
(ps_spectra_zscore).  Section 4.2: the chunk average and its error bar
depend on the chunks only through the sums of x, (Re x)^2, (Im x)^2 and
their count, which are the exported state; resuming from it is exact.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_2505_01231_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch.device("cuda:0")


def _host(sp, keys=("s1", "s2", "s3", "s4")):
    out = {}
    for k in keys:
        t = getattr(sp, k)
        if t is None:
            continue
        out[k] = t.cpu().numpy()
        out[k + "_err"] = getattr(sp, k + "_err").cpu().numpy()
    return out


def _complex(a):
    return a[..., 0] + 1j * a[..., 1]


def _rel(a, b):
    s = np.nanmax(np.abs(b))
    return float(np.nanmax(np.abs(a - b)) / s)


def _pieces(total, seed, lo, hi):
    rng = np.random.default_rng(seed)
    cuts, at = [], 0
    while at < total:
        n = int(min(total - at, rng.integers(lo, hi)))
        cuts.append((at, at + n))
        at += n
    return cuts


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_stream_pieces_match_oracle_and_execute(dev, precision):
    """Two int16 channels pushed in pieces of irregular length (shorter and
    longer than a chunk): the accumulated S1..S4 equal the oracle on the whole
    record, and ps_execute on the whole record up to the order of FP64
    additions."""
    from paper_2505_01231_amd import Accumulator, Plan
    N, Nf, m = 512, 96, 6
    z, _ = synth.mixed_channels(N * m * 23 + 333, seed=7)
    z = z[:2].copy()
    x = torch.from_numpy(z).to(dev)
    say("stream pieces", precision)
    with Plan(frame_len=N, n_freq=Nf, m=m, n_channels=2, orders=(1, 2, 3, 4), precision=precision) as p:
        acc = Accumulator(p, max_push_samples=N * m * 5, dtype=torch.int16)
        for a, b in _pieces(z.shape[1], 3, 100, N * m * 5):
            acc.push(x[:, a:b])
        got = _host(acc.end())
        cnt = acc.counts()
        whole = _host(p.execute(x))
        torch.cuda.synchronize()
        acc.close()
        assert cnt == {"chunks": 23, "samples": z.shape[1], "carry": 333}
        for k in whole:
            assert _rel(got[k], whole[k]) <= 1e-12, k
        ref = O.polyspectra(z, N, Nf, m, orders=(1, 2, 3, 4), combos2=p.combos2, combos3=p.combos3,
                            combos4=p.combos4)
    for k in ("s2", "s3", "s4"):
        assert _rel(_complex(got[k]), ref[k]) <= TOL, k
        assert _rel(got[k + "_err"], ref[k + "_err"]) <= TOL, k + "_err"
    assert _rel(_complex(got["s1"]), ref["s1"]) <= TOL


def test_stream_four_channels_every_orbit(dev):
    """Four int16 channels with every combination orbit (10 + 40 + 76
    spectra, the largest finalize tables an accumulator builds), pushed in
    pieces, with an intermediate end: the accumulated spectra equal ps_execute
    on the whole record up to the order of FP64 additions."""
    from paper_2505_01231_amd import Accumulator, Plan
    N, Nf, m = 256, 40, 4
    z, _ = synth.mixed_channels(N * m * 9 + 77, seed=19)
    x = torch.from_numpy(z).to(dev)
    say("stream four channels")
    with Plan(frame_len=N, n_freq=Nf, m=m, n_channels=4, orders=(1, 2, 3, 4), precision="bf16x3") as p:
        assert (len(p.combos2), len(p.combos3), len(p.combos4)) == (10, 40, 76)
        acc = Accumulator(p, max_push_samples=N * m * 4, dtype=torch.int16)
        for i, (a, b) in enumerate(_pieces(z.shape[1], 11, 500, N * m * 4)):
            acc.push(x[:, a:b])
            if i == 1:
                acc.end()
        got = _host(acc.end())
        whole = _host(p.execute(x))
        torch.cuda.synchronize()
        assert acc.counts() == {"chunks": 9, "samples": z.shape[1], "carry": 77}
        acc.close()
    for k in whole:
        assert _rel(got[k], whole[k]) <= 1e-12, k


def test_stream_resume_is_bit_exact(dev):
    """Export after some pushes, tear everything down, import into a new
    accumulator of a new plan and push the rest: the outputs equal the
    uninterrupted accumulation bit for bit.  An ps_stream_end in the middle
    does not disturb the state."""
    from paper_2505_01231_amd import Accumulator, Plan
    N, Nf, m = 1024, 200, 10
    z = synth.ar2_chi2(N * m * 17 + 4321, seed=12)
    x = torch.from_numpy(z).to(dev)
    cuts = _pieces(len(z), 5, 1000, N * m * 3)
    kw = dict(frame_len=N, n_freq=Nf, m=m, orders=(1, 2, 3, 4), precision="bf16x3")
    say("stream resume", len(cuts), "pieces")
    with Plan(**kw) as p:
        acc = Accumulator(p, N * m * 3)
        for i, (a, b) in enumerate(cuts):
            acc.push(x[a:b])
            if i == len(cuts) // 3:
                acc.end()                       # an intermediate look
        full = _host(acc.end())
        torch.cuda.synchronize()
        full_state = acc.export_state()
        acc.close()
    split = len(cuts) // 2
    with Plan(**kw) as p:
        acc = Accumulator(p, N * m * 3)
        for a, b in cuts[:split]:
            acc.push(x[a:b])
        state = acc.export_state()
        acc.close()
    with Plan(**kw) as p2:
        acc2 = Accumulator(p2, N * m * 3)
        acc2.import_state(state)
        for a, b in cuts[split:]:
            acc2.push(x[a:b])
        res = _host(acc2.end())
        torch.cuda.synchronize()
        res_state = acc2.export_state()
        acc2.close()
    for k in full:
        assert np.array_equal(full[k], res[k], equal_nan=True), k
    # the resumed accumulator ends in the uninterrupted one's state, byte for byte
    assert bytes(res_state) == bytes(full_state)


def test_stream_import_rejects_other_configurations(dev):
    from paper_2505_01231_amd import Accumulator, Plan
    from paper_2505_01231_amd._lib import PolyspecError
    N, Nf, m = 512, 64, 8
    z = synth.ar2_chi2(N * m * 3 + 100, seed=2)
    x = torch.from_numpy(z).to(dev)
    with Plan(frame_len=N, n_freq=Nf, m=m) as p:
        acc = Accumulator(p, len(z))
        acc.push(x)
        state = acc.export_state()
        acc.close()
    for kw, dtype in ((dict(m=m + 1), torch.float32), (dict(m=m, precision="bf16x3"), torch.float32),
                      (dict(m=m, n_freq=Nf + 1), torch.float32), (dict(m=m), torch.float64),
                      (dict(m=m, window="hann"), torch.float32)):
        kw = {"frame_len": N, "n_freq": Nf, **kw}
        with Plan(**kw) as q:
            acc = Accumulator(q, len(z), dtype=dtype)
            with pytest.raises(PolyspecError):
                acc.import_state(state)
            acc.close()
    with Plan(frame_len=N, n_freq=Nf, m=m) as q:
        acc = Accumulator(q, len(z))
        with pytest.raises(PolyspecError):
            acc.import_state(state[:-8])        # truncated
        acc.import_state(state)                 # the right one is accepted
        assert acc.counts() == {"chunks": 3, "samples": len(z), "carry": 100}
        acc.close()


def test_stream_without_a_chunk_gives_nan(dev):
    from paper_2505_01231_amd import Accumulator, Plan
    N, Nf, m = 256, 32, 4
    z = synth.ar2_chi2(N * m - 1, seed=3)
    with Plan(frame_len=N, n_freq=Nf, m=m) as p:
        acc = Accumulator(p, N * m)
        acc.push(torch.from_numpy(z).to(dev))
        out = _host(acc.end())
        torch.cuda.synchronize()
        assert acc.counts() == {"chunks": 0, "samples": N * m - 1, "carry": N * m - 1}
        acc.close()
    for k, v in out.items():
        assert np.all(np.isnan(v)), k


def test_c_client_stream_resume(dev, tmp_path):
    """Through the C ABI alone: the C client pushes a record in pieces, once
    straight through and once with a checkpoint to a file, a torn-down plan
    and accumulator, and a resume; both output files are identical and match
    the oracle."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = os.path.join(root, "paper_2505_01231_amd", "ps_c_client")
    assert os.path.exists(exe), "ps_c_client is missing: python -m paper_2505_01231_amd.build"
    N, Nf, m = 512, 100, 10
    z = synth.ar2_chi2(N * m * 9 + 777, seed=43, dtype=np.float32)
    inp = tmp_path / "z.f32"
    z.tofile(inp)
    outs = []
    for split in (0, 4):
        out = tmp_path / f"s{split}.f64"
        say("C client stream, split", split)
        r = subprocess.run([exe, "stream", str(inp), str(out), str(N), str(Nf), str(m), "1", "3001", str(split),
                            str(tmp_path / "state.bin")], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stderr
        outs.append(np.fromfile(out, dtype=np.float64))
    assert np.array_equal(outs[0], outs[1], equal_nan=True)
    ref = O.polyspectra(z, N, Nf, m, window_kind="acg")
    d = outs[0]
    assert int(d[0]) == ref["n_chunks"] == 9
    sizes = [2 * Nf, 2 * Nf, 2 * Nf * Nf, 2 * Nf * Nf, 2 * Nf * Nf, 2 * Nf * Nf]
    parts = np.split(d[1:], np.cumsum(sizes)[:-1])
    for i, k in enumerate(("s2", "s3", "s4")):
        got = parts[2 * i].reshape(-1, 2)
        assert _rel(got[:, 0] + 1j * got[:, 1], ref[k].ravel()) <= TOL, k
        assert _rel(parts[2 * i + 1].reshape(-1, 2), ref[k + "_err"].reshape(-1, 2)) <= TOL, k


def test_zscore_of_two_estimates(dev):
    """ps_spectra_zscore: |a - b| / sqrt(sa^2 + sb^2) per real component,
    against the same formula in numpy on the host."""
    from paper_2505_01231_amd import Plan, m_dependence
    N, Nf = 512, 64
    z = synth.ar2_chi2(N * 40 * 7, seed=21)
    x = torch.from_numpy(z).to(dev)
    outs = {}
    for m in (10, 40):
        with Plan(frame_len=N, n_freq=Nf, m=m) as p:
            outs[m] = p.execute(x)
    torch.cuda.synchronize()
    for key in ("s2", "s3", "s4"):
        got = m_dependence(outs[10], outs[40], key).cpu().numpy()
        a, ae = getattr(outs[10], key).cpu().numpy(), getattr(outs[10], key + "_err").cpu().numpy()
        b, be = getattr(outs[40], key).cpu().numpy(), getattr(outs[40], key + "_err").cpu().numpy()
        with np.errstate(invalid="ignore", divide="ignore"):
            want = np.abs(a - b) / np.sqrt(ae * ae + be * be)
        assert np.allclose(got, want, rtol=1e-14, atol=0, equal_nan=True), key
