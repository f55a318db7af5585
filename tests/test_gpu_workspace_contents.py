"""The outputs depend on the inputs alone: the same records run once into a
workspace filled with 0xFF bytes (NaN in every float view) and outputs
prefilled with NaN, and once into a zeroed workspace and outputs prefilled
with 7.0, give the same bits, and every output of a record with two or more
chunks is written (no prefill value survives).  A kernel that read a
workspace region no earlier stage wrote, or left part of an output
unwritten, would fail here.  Configurations: the three precisions on a grid
that is not a multiple of the tile edge with S1..S4, two channels with every
orbit (matrix-core and vector cross-channel S4), interlaced windows, c3^opt,
the natural estimator, a frame length that is not a power of two, two frame
lengths in one call, complex records, and sequential spectra; each call of
the averaging entry point carries a record of one chunk (NaN error bars)
beside the longer ones."""
import numpy as np
import pytest

from paper_2505_01231_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("s1", "s1_err", "s2", "s2_err", "s3", "s3_err", "s4", "s4_err")


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch.device("cuda:0")


def _fill(sp, value):
    for k in KEYS:
        t = getattr(sp, k)
        if t is not None:
            t.fill_(value)


def _host(sp):
    return {k: getattr(sp, k).cpu().numpy().copy() for k in KEYS if getattr(sp, k) is not None}


def _two_runs(plan, xs, dev, frame_lens=None):
    fls = frame_lens or [0] * len(xs)
    need = plan.workspace_bytes(xs, frame_lens)
    runs = []
    for ws_byte, out_val in ((0xFF, float("nan")), (0x00, 7.0)):
        ws = torch.full((need,), ws_byte, dtype=torch.uint8, device=dev)
        outs = [plan.allocate_outputs(dev, fl) for fl in fls]
        for o in outs:
            _fill(o, out_val)
        got = plan.execute(xs, workspace=ws, outputs=outs, frame_lens=frame_lens)
        torch.cuda.synchronize()
        runs.append(([_host(o) for o in got], [o.n_chunks for o in got]))
    return runs


def _check(runs, label, finite=True):
    (a, na), (b, nb) = runs
    assert na == nb
    for i, (ra, rb) in enumerate(zip(a, b)):
        for k in ra:
            assert np.array_equal(ra[k], rb[k], equal_nan=True), (label, i, k)
            if finite and na[i] >= 2:
                assert np.isfinite(ra[k]).all(), (label, i, k, "an output element was not written")
            if finite and na[i] == 1 and not k.endswith("_err"):
                assert np.isfinite(ra[k]).all(), (label, i, k, "an output element was not written")


def _real(n, seed):
    return synth.ar2_chi2(n, seed=seed, dtype=np.float32)


CASES = [
    ("fp32 ragged grid", dict(frame_len=512, n_freq=100, m=10, orders=(1, 2, 3, 4), precision="fp32"), 1),
    ("bf16x3 ragged grid", dict(frame_len=512, n_freq=100, m=10, orders=(1, 2, 3, 4), precision="bf16x3"), 1),
    ("fp16x2s ragged grid", dict(frame_len=512, n_freq=100, m=10, orders=(1, 2, 3, 4), precision="fp16x2s"), 1),
    ("fp16x2s S2+S4 only", dict(frame_len=512, n_freq=90, m=10, orders=(2, 4), precision="fp16x2s"), 1),
    ("two channels bf16x3", dict(frame_len=256, n_freq=40, m=6, n_channels=2, precision="bf16x3"), 2),
    ("two channels fp32", dict(frame_len=256, n_freq=40, m=6, n_channels=2, precision="fp32"), 2),
    ("interlaced fp16x2s", dict(frame_len=512, n_freq=64, m=8, interlaced=True, precision="fp16x2s"), 1),
    ("c3opt two channels", dict(frame_len=256, n_freq=48, m=10, n_channels=2, estimator="c3opt",
                                precision="bf16x3"), 2),
    ("natural estimator", dict(frame_len=256, n_freq=48, m=6, estimator="natural", precision="fp16x2s"), 1),
    ("direct transform N=768", dict(frame_len=768, n_freq=150, m=10, precision="fp16x2s"), 1),
]


@pytest.mark.parametrize("label,kw,channels", CASES, ids=[c[0] for c in CASES])
def test_outputs_independent_of_workspace_contents(dev, label, kw, channels):
    from paper_2505_01231_amd import Plan
    say("workspace contents:", label)
    N, m = kw["frame_len"], kw["m"]
    if channels == 1:
        z = _real(N * m * 7 + 123, seed=61)
        xs = [torch.from_numpy(z).to(dev), torch.from_numpy(z[: N * m + 9].copy()).to(dev)]
    else:
        z, _ = synth.mixed_channels(N * m * 7 + 123, seed=62)
        z = np.ascontiguousarray(z[:channels])
        xs = [torch.from_numpy(z).to(dev), torch.from_numpy(np.ascontiguousarray(z[:, : N * m + 9])).to(dev)]
    with Plan(**kw) as p:
        runs = _two_runs(p, xs, dev)
    _check(runs, label)


def test_two_frame_lengths_independent_of_workspace_contents(dev):
    from paper_2505_01231_amd import Plan
    say("workspace contents: two frame lengths in one call")
    z = _real(1024 * 8 * 5 + 77, seed=63)
    xs = [torch.from_numpy(z).to(dev), torch.from_numpy(z[: 512 * 8 * 3 + 5].copy()).to(dev),
          torch.from_numpy(z[: 1024 * 8 + 1].copy()).to(dev)]
    with Plan(frame_len=512, n_freq=64, m=8, frame_lens=(512, 1024), precision="bf16x3") as p:
        runs = _two_runs(p, xs, dev, frame_lens=[1024, 512, 1024])
    _check(runs, "two frame lengths")


def test_complex_records_independent_of_workspace_contents(dev):
    from paper_2505_01231_amd import Plan
    say("workspace contents: complex records")
    N, Nf, m = 256, 30, 6
    rng = np.random.default_rng(64)
    z = (rng.standard_normal(N * m * 6 + 31) + 1j * rng.standard_normal(N * m * 6 + 31)).astype(np.complex64)
    xs = [torch.from_numpy(z).to(dev), torch.from_numpy(z[: N * m + 3].copy()).to(dev)]
    with Plan(frame_len=N, n_freq=Nf, m=m, complex_signal=True, precision="bf16x3") as p:
        runs = _two_runs(p, xs, dev)
    _check(runs, "complex", finite=False)


def test_sequential_spectra_independent_of_workspace_contents(dev):
    from paper_2505_01231_amd import Plan
    say("workspace contents: sequential spectra")
    N, Nf, m = 512, 72, 8
    z = _real(N * m * 6 + 40, seed=65)
    x = torch.from_numpy(z).to(dev)
    got = []
    with Plan(frame_len=N, n_freq=Nf, m=m, orders=(1, 2, 3, 4), precision="fp16x2s") as p:
        first = p.sequential(x, 1, 4)
        torch.cuda.synchronize()
        need = p._last_workspace.numel()                       # the size the binding allocated
        for ws_byte in (0xFF, 0x00):
            ws = torch.full((need,), ws_byte, dtype=torch.uint8, device=dev)
            sp = p.sequential(x, 1, 4, workspace=ws)
            torch.cuda.synchronize()
            got.append(_host(sp))
    ref = _host(first)
    for k in ("s1", "s2", "s3", "s4"):
        assert np.isfinite(got[0][k]).all(), k
        for g in got:
            assert np.array_equal(g[k], ref[k], equal_nan=True), k
