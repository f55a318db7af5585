"""Records of several frame lengths in ONE execute (the batching form with
uneven records at frame lengths 1024 / 2048 / 4096 in the paper-derived
configuration; here at smaller sizes the oracle finishes in seconds): each
stage is one launch over every record, frame length and combination, and
every record's spectra equal the oracle's at its own N and N_f (Sections 3,
4, 4.2 and 7)."""
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


def _rel(a, b):
    """Max |a - b| / max |b| over the finite entries; NaN where, and only
    where, the other side is NaN (0 when both are all NaN)."""
    a, b = np.asarray(a), np.asarray(b)
    assert np.array_equal(np.isnan(a), np.isnan(b))
    ok = ~np.isnan(b)
    if not ok.any():
        return 0.0
    s = np.max(np.abs(b[ok]))
    d = np.max(np.abs(a[ok] - b[ok]))
    return float(d / s) if s > 0 else float(d)


def _host(sp):
    out = {}
    for k in ("s1", "s2", "s3", "s4"):
        t = getattr(sp, k)
        if t is not None:
            out[k] = t.cpu().numpy()
            out[k + "_err"] = getattr(sp, k + "_err").cpu().numpy()
    return out


def _check(got, ref, label, keys=("s2", "s3", "s4")):
    errs = {}
    for k in keys:
        errs[k] = _rel(got[k][..., 0] + 1j * got[k][..., 1], ref[k])
        errs[k + "_err"] = _rel(got[k + "_err"], ref[k + "_err"])
    say(label, {k: f"{v:.1e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= TOL, (label, k, v)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_mixed_frame_lengths_four_int16_channels(dev, precision):
    """Four int16 channels (two AR(2)/chi-square sources mixed with noise),
    records at N = 256, 512 and 1024 in one execute with N_f = N / 4 and every
    combination orbit (10 / 40 / 76); each record equals the oracle at its own
    frame length, and the same records through single-length plans up to the
    order of FP64 additions."""
    from paper_2505_01231_amd import Plan
    m = 6
    spec = [(512, 3), (256, 4), (1024, 2), (256, 1), (512, 5), (1024, 3), (256, 0)]
    zs, fls = [], []
    for i, (N, nch) in enumerate(spec):
        z, clipped = synth.mixed_channels(N * m * nch + 37 * i, seed=200 + i)
        assert clipped == 0
        zs.append(z)
        fls.append(N)
    xs = [torch.from_numpy(np.ascontiguousarray(z)).to(dev) for z in zs]
    say("mixed frame lengths, 4 int16 channels", precision)
    with Plan(frame_len=256, n_freq=64, m=m, n_channels=4, precision=precision, frame_lens=(512, 1024)) as p:
        assert [p.frame_info(n)["n_freq"] for n in (256, 512, 1024)] == [64, 128, 256]
        outs = p.execute(xs, frame_lens=fls)
        torch.cuda.synchronize()
        got = [_host(o) for o in outs]
        combos = dict(combos2=p.combos2, combos3=p.combos3, combos4=p.combos4)
        assert [len(c) for c in combos.values()] == [10, 40, 76]
    for i, (z, N) in enumerate(zip(zs, fls)):
        Np = outs[i].n_chunks
        assert Np == (z.shape[1] // N) // m
        if Np == 0:
            assert all(np.all(np.isnan(v)) for v in got[i].values())
            continue
        ref = O.polyspectra(z, N, N // 4, m, window_kind="acg", **combos)
        _check(got[i], ref, f"N={N} rec {i}")
    # the same records through plans of one frame length each
    for N in (256, 512, 1024):
        idx = [i for i, n in enumerate(fls) if n == N]
        with Plan(frame_len=N, n_freq=N // 4, m=m, n_channels=4, precision=precision) as q:
            single = q.execute([xs[i] for i in idx])
            torch.cuda.synchronize()
            for j, i in enumerate(idx):
                h = _host(single[j])
                for k in h:
                    assert _rel(got[i][k], h[k]) <= 1e-12, (N, i, k)


def test_mixed_frame_lengths_options(dev):
    """One channel, frame lengths 512 and 2048 in one execute, with S1,
    interlaced windows, c3^(opt) for S3 and the natural estimator, and through
    the per-chunk schedule and a captured graph: each against the oracle at its
    own frame length."""
    from paper_2505_01231_amd import Plan
    m = 5
    zs = [synth.ar2_chi2(2048 * m * 3 + 900, seed=301, dtype=np.float32),
          synth.ar2_chi2(512 * m * 7 + 300, seed=302, dtype=np.float32),
          synth.ar2_chi2(2048 * m * 2 + 100, seed=303, dtype=np.float32)]
    fls = [2048, 512, 2048]
    xs = [torch.from_numpy(z).to(dev) for z in zs]
    cases = [dict(), dict(interlaced=True), dict(estimator="c3opt"), dict(estimator="natural"),
             dict(schedule="per_chunk")]
    for kw in cases:
        say("mixed frame lengths", kw)
        with Plan(frame_len=512, n_freq=40, m=m, orders=(1, 2, 3, 4), precision="bf16x3", frame_lens=(2048,),
                  **kw) as p:
            outs = [_host(o) for o in p.execute(xs, frame_lens=fls)]
            torch.cuda.synchronize()
        for i, (z, N) in enumerate(zip(zs, fls)):
            nf = 40 * N // 512
            okw = dict(window_kind="acg", orders=(1, 2, 3, 4))
            if kw.get("estimator"):
                okw["estimator"] = kw["estimator"]
            ref = (O.polyspectra_interlaced if kw.get("interlaced") else O.polyspectra)(z, N, nf, m, **okw)
            _check(outs[i], ref, f"{kw} N={N}")
            assert _rel(outs[i]["s1"][:, 0], ref["s1"].real) <= TOL
    # graph replay equals the eager run bit for bit, with new data in between
    with Plan(frame_len=512, n_freq=40, m=m, precision="bf16x3", frame_lens=(2048,)) as p:
        eager = [_host(o) for o in p.execute(xs, frame_lens=fls)]
        g = p.graph(xs, frame_lens=fls)
        for rep in range(3):
            outs = g.launch()
            torch.cuda.synchronize()
            for i in range(len(xs)):
                h = _host(outs[i])
                for k in h:
                    assert np.array_equal(h[k], eager[i][k], equal_nan=True), (rep, i, k)
        g.close()


def test_mixed_frame_lengths_refusals(dev):
    from paper_2505_01231_amd import Plan
    from paper_2505_01231_amd._lib import PolyspecError
    x = torch.zeros(4096 * 10, device=dev)
    with Plan(frame_len=1024, n_freq=64, m=10, frame_lens=(4096,)) as p:
        with pytest.raises(PolyspecError):
            p.execute(x, frame_lens=2048)       # not among the plan's frame lengths
    with pytest.raises(PolyspecError):
        Plan(frame_len=1024, n_freq=65, m=10, frame_lens=(256,))   # 65 * 256 / 1024 is not an integer
    with pytest.raises(PolyspecError):
        Plan(frame_len=1024, n_freq=64, m=10, frame_lens=(512,), complex_signal=True)
