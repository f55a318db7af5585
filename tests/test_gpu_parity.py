"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Error metric, per spectrum s (and per error-bar array):
    err_s = max_grid |S_gpu - S_oracle| / max_grid |S_oracle|      (complex modulus)
Tolerance 1e-5 for every spectrum and error bar (the accuracy bar the
mixed-precision path must meet); bit-exact checks where the result is
integer-like (NaN flags, determinism, schedule equivalence up to FP64 order).
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2505_01231_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch.device("cuda:0")


def run_gpu(z, dev, **plan_kw):
    from paper_2505_01231_amd import Plan
    x = torch.from_numpy(np.ascontiguousarray(z)).to(dev)
    with Plan(**plan_kw) as p:
        out = p.execute(x)
        torch.cuda.synchronize()
        res = {"n_chunks": out.n_chunks, "flags": out.flags}
        for key in ("s2", "s3", "s4"):
            t = getattr(out, key)
            if t is not None:
                res[key] = torch.view_as_complex(t).cpu().numpy()
                res[key + "_err"] = getattr(out, key + "_err").cpu().numpy()
        res["plan"] = dict(n_freq=p.n_freq, combos2=p.combos2, combos3=p.combos3, combos4=p.combos4)
    return res


def rel_err(a, b):
    scale = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / scale) if scale > 0 else float(np.max(np.abs(a - b)))


def compare(gpu, ref, keys=("s2", "s3", "s4"), tol=TOL, label=""):
    report = {}
    for k in keys:
        if k not in gpu:
            continue
        e = rel_err(gpu[k], ref[k])
        ee = rel_err(gpu[k + "_err"], ref[k + "_err"])
        report[k] = (e, ee)
    say(label, {k: f"{v[0]:.2e}/{v[1]:.2e}" for k, v in report.items()})
    for k, (e, ee) in report.items():
        assert e <= tol, (label, k, e)
        assert ee <= tol, (label, k + "_err", ee)
    return report


WIN = {"hann": "hann", "acg": "acg", "hann_periodic": "hann_periodic"}


def both(z, dev, N, Nf, m, dt=1.0, window="acg", orders=(2, 3, 4), combos2=None, combos3=None,
         combos4=None, n_channels=1, **kw):
    gpu = run_gpu(z, dev, frame_len=N, n_freq=Nf, m=m, dt=dt, window=window, orders=orders,
                  n_channels=n_channels, combos2=combos2, combos3=combos3, combos4=combos4, **kw)
    ref = O.polyspectra(z, N, Nf, m, dt=dt, window_kind=window, orders=orders,
                        combos2=gpu["plan"]["combos2"], combos3=gpu["plan"]["combos3"],
                        combos4=gpu["plan"]["combos4"])
    return gpu, ref


# ---------------------------------------------------------------- stage a1
@pytest.mark.parametrize("N,dtype", [(256, np.float64), (1024, np.float32), (8192, np.float32),
                                     (2048, np.int16), (512, np.float64)])
def test_coefficients_match_oracle(dev, N, dtype):
    from paper_2505_01231_amd import Plan
    say("coefficients", N, dtype.__name__)
    m = 4
    Nf = N // 4
    if dtype == np.int16:
        z = np.clip(np.rint(synth.ar2_chi2(N * m * 3 + 17, seed=7) * 300), -32768, 32767).astype(np.int16)
    else:
        z = synth.ar2_chi2(N * m * 3 + 17, seed=7, dtype=dtype)
    with Plan(frame_len=N, n_freq=Nf, m=m, window="acg") as p:
        a = p.coefficients(torch.from_numpy(z).to(dev))
        torch.cuda.synchronize()
        a = a.cpu().numpy()[0]
        K = p.n_coef
    g = O.window("acg", N)
    fr = O.chunk_frames(z, N, m).reshape(-1, N)
    ref = O.coefficients(fr, g, 1.0, K)
    e = rel_err(a, ref)
    say("  coef rel err", e)
    assert a.shape == ref.shape
    assert e < 2e-6


@pytest.mark.parametrize("dtype", [np.float32, np.float64, np.int16])
def test_coefficients_unaligned_frames(dev, dtype):
    """Frames that start at an odd sample address (a view from sample 1 and an
    odd channel stride) take the scalar sample loads of the transform."""
    from paper_2505_01231_amd import Plan
    say("coefficients unaligned", dtype.__name__)
    N, m, C = 1024, 4, 2
    L_ = N * m * 2 + 4                  # channel stride L_ + 3 is odd
    raw = synth.ar2_chi2(C * (L_ + 3) + 1, seed=11)
    if dtype == np.int16:
        raw = np.clip(np.rint(raw * 300), -32768, 32767)
    base = torch.from_numpy(raw.astype(dtype)).to(dev)
    # channel c = base[1 + c (L_ + 3) : ... + L_]: channel 0 starts at an odd
    # address, channel 1 (odd stride) at an even one
    x = base[1:1 + C * (L_ + 3)].view(C, L_ + 3)[:, :L_]
    assert x.stride(0) % 2 == 1 and x.data_ptr() % (2 * x.element_size()) != 0
    with Plan(frame_len=N, n_freq=N // 4, m=m, n_channels=C, window="acg") as p:
        a = p.coefficients(x)
        torch.cuda.synchronize()
        a = a.cpu().numpy()
        K = p.n_coef
    g = O.window("acg", N)
    xc = x.cpu().numpy()
    for c in range(C):
        fr = O.chunk_frames(xc[c], N, m).reshape(-1, N)
        ref = O.coefficients(fr, g, 1.0, K)
        e = rel_err(a[c], ref)
        say("  channel", c, "coef rel err", e)
        assert e < 2e-6


# ---------------------------------------------------------------- configurations
PRECISIONS = ["fp32", "bf16x3", "fp16x2s"]


@pytest.mark.parametrize("precision", PRECISIONS)
def test_white_noise_config(dev, precision):
    """51,200 float64 white Gaussian samples, N = 256, Hann, N_f = 64, m = 10."""
    say("white-noise config", precision)
    z = synth.white_gaussian(51_200, seed=1)
    gpu, ref = both(z, dev, 256, 64, 10, window="hann", precision=precision)
    assert gpu["n_chunks"] == 20
    compare(gpu, ref, label="white")
    # physics on the GPU result: flat S2 = sigma^2 dt = 1, S3 and S4 consistent with zero
    s2 = gpu["s2"][0]
    assert abs(np.mean(s2.real) - 1) < 0.05
    for k in ("s3", "s4"):
        z_re = gpu[k][0].real / gpu[k + "_err"][0][..., 0]
        assert np.mean(np.abs(z_re) > 3.5) < 0.02


@pytest.mark.parametrize("precision", PRECISIONS)
def test_ar2_subset(dev, precision):
    """The AR(2)/chi-square signal (r = 0.95, theta = 0.3 pi) on its 2^20-sample
    subset: N = 4096, acG window, N_f = 512, m = 10 (25 chunks, 8 tile rows)."""
    say("ar2 subset N=4096 Nf=512", precision)
    z = synth.ar2_chi2(1 << 20, seed=2)
    gpu, ref = both(z, dev, 4096, 512, 10, window="acg", precision=precision)
    assert gpu["n_chunks"] == 25
    compare(gpu, ref, label=f"ar2-4096-{precision}")


@pytest.mark.parametrize("precision", PRECISIONS)
def test_ar2_n8192_subset(dev, precision):
    """The same signal at N = 8192, N_f = 2048 (32 tile rows) on 2^21 samples
    (25 chunks)."""
    say("ar2 subset N=8192 Nf=2048", precision)
    z = synth.ar2_chi2(1 << 21, seed=3)
    gpu, ref = both(z, dev, 8192, 2048, 10, window="acg", precision=precision, orders=(2, 4))
    compare(gpu, ref, keys=("s2", "s4"), label=f"ar2-8192-{precision}")


@pytest.mark.parametrize("precision", PRECISIONS)
def test_ragged_grid_and_tail(dev, precision):
    """N_f not a multiple of the tile, leftover samples, odd m, dt != 1."""
    say("ragged N=1024 Nf=200 m=7", precision)
    z = synth.ar2_chi2(1024 * 7 * 9 + 1000, seed=12, r=0.9, dtype=np.float32)
    gpu, ref = both(z, dev, 1024, 200, 7, dt=0.37, window="hann_periodic", precision=precision)
    assert gpu["n_chunks"] == 9
    compare(gpu, ref, label="ragged")


@pytest.mark.parametrize("orders,Nf", [((2,), 129), ((3,), 65), ((4,), 100), ((2, 4), 128)])
def test_order_subsets(dev, orders, Nf):
    say("orders", orders, Nf)
    z = synth.ar2_chi2(256 * 6 * 5, seed=13, dtype=np.float64)
    gpu, ref = both(z, dev, 256, Nf, 6, window="acg", orders=orders)
    compare(gpu, ref, keys=tuple(f"s{o}" for o in orders), label=f"orders{orders}")


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("Nf", [1, 2, 3])
def test_tiny_grids(dev, precision, Nf):
    """N_f of 1-3: one tile, almost all of it outside the grid."""
    say("tiny grid", Nf, precision)
    z = synth.ar2_chi2(256 * 5 * 6 + 11, seed=21 + Nf, dtype=np.float32)
    gpu, ref = both(z, dev, 256, Nf, 5, window="hann", precision=precision)
    compare(gpu, ref, label=f"tiny-{Nf}-{precision}")


@pytest.mark.parametrize("precision", PRECISIONS)
def test_largest_grid_for_s3(dev, precision):
    """N_f = N/4 + 1, the largest grid with S3: the third factor a_(k+l) reaches
    the Nyquist coefficient k + l = N/2, and the grid is one point past four
    whole tiles."""
    say("N_f = N/4 + 1", precision)
    N = 1024
    Nf = N // 4 + 1
    z = synth.ar2_chi2(N * 10 * 4 + 3, seed=33, dtype=np.float32)
    gpu, ref = both(z, dev, N, Nf, 10, window="acg", precision=precision)
    compare(gpu, ref, label=f"largest-{precision}")


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_large_m_uses_several_frame_batches(dev, precision):
    say("m=37", precision)
    z = synth.ar2_chi2(512 * 37 * 4, seed=14, dtype=np.float32)
    gpu, ref = both(z, dev, 512, 96, 37, window="acg", precision=precision)
    compare(gpu, ref, label="m37")


@pytest.mark.parametrize("m", [4, 10])
@pytest.mark.parametrize("n_chunks", [1, 2, 3, 4, 5, 7])
def test_fp16_records_every_piece_length(dev, m, n_chunks):
    """Scaled FP16x2 S4 from the centring pass's records for records of 1-7
    chunks: pieces of every length relative to the kernel's three staging
    buffers (copies two chunks ahead, the ones past a piece's end repeated),
    and chunks with fewer frames than the records hold."""
    say("fp16 records", m, n_chunks)
    z = synth.ar2_chi2(256 * m * n_chunks + 17, seed=40 + n_chunks, dtype=np.float32)
    gpu, ref = both(z, dev, 256, 100, m, window="acg", precision="fp16x2s", orders=(2, 4))
    assert gpu["n_chunks"] == n_chunks
    if n_chunks == 1:       # one chunk: the spectra are defined, the error bars are not
        for k in ("s2", "s4"):
            assert rel_err(gpu[k], ref[k]) <= TOL, k
            assert np.isnan(gpu[k + "_err"]).all()
    else:
        compare(gpu, ref, keys=("s2", "s4"), label=f"fp16-records-m{m}-c{n_chunks}")


def test_fp16_split_needs_one_batch_per_chunk(dev):
    from paper_2505_01231_amd import Plan
    from paper_2505_01231_amd._lib import PS_E_UNSUPPORTED, PolyspecError
    with pytest.raises(PolyspecError) as e:
        Plan(frame_len=512, n_freq=96, m=11, precision="fp16x2s")
    assert e.value.status == PS_E_UNSUPPORTED
    Plan(frame_len=512, n_freq=96, m=11, precision="fp16x2s", orders=(2, 3)).close()


def test_cross_channel_s2_s3(dev):
    """Two channels, explicit combinations (Section 7)."""
    say("cross channels")
    rng = np.random.default_rng(15)
    s = synth.ar2_chi2(256 * 8 * 12 + 3, seed=15, r=0.9, dtype=np.float64)
    z = np.stack([s[:-3] + 0.3 * rng.standard_normal(len(s) - 3), s[3:] ** 2 - 1.0])
    gpu, ref = both(z, dev, 256, 40, 8, window="hann", n_channels=2, orders=(2, 3),
                    combos2=[(0, 1), (1, 0), (1, 1)], combos3=[(0, 1, 1), (1, 0, 0), (0, 0, 1), (1, 1, 0)])
    compare(gpu, ref, keys=("s2", "s3"), label="cross")


@pytest.mark.parametrize("m", [12, 13, 15])
def test_exact_size_s3_batches(dev, m):
    """The default S3 batch (exactly 12 or 13 frames for such chunks, else
    several batches of 10): the spectra equal the oracle's and, bit for bit,
    those of the 16-frame batch (the frames are added in the same order)."""
    from paper_2505_01231_amd import Plan
    say("exact-size S3 batch", m)
    N, Nf = 512, 100
    z = synth.ar2_chi2(N * m * 6 + 21, seed=190 + m, dtype=np.float32)
    x = torch.from_numpy(z).to(dev)
    with Plan(frame_len=N, n_freq=Nf, m=m, orders=(3,), window="hann") as p:
        a = torch.view_as_complex(p.execute(x).s3).cpu().numpy()
        p.set_tuning(8, 16)
        b = torch.view_as_complex(p.execute(x).s3).cpu().numpy()
        torch.cuda.synchronize()
    assert np.array_equal(a, b)
    ref = O.polyspectra(z, N, Nf, m, orders=(3,), window_kind="hann")
    assert rel_err(a[0], ref["s3"][0]) <= TOL


# ---------------------------------------------------------------- schedule, determinism, edges
@pytest.mark.parametrize("precision", PRECISIONS)
def test_per_chunk_schedule_matches_batched(dev, precision):
    say("per-chunk vs batched", precision)
    z = synth.ar2_chi2(1024 * 10 * 13, seed=16, dtype=np.float32)
    kw = dict(frame_len=1024, n_freq=256, m=10, window="acg", precision=precision)
    a = run_gpu(z, dev, schedule="batched", **kw)
    b = run_gpu(z, dev, schedule="per_chunk", **kw)
    for k in ("s2", "s3", "s4"):
        assert rel_err(a[k], b[k]) < 1e-12, k
        assert rel_err(a[k + "_err"], b[k + "_err"]) < 1e-9, k


@pytest.mark.parametrize("precision", PRECISIONS)
def test_deterministic(dev, precision):
    say("determinism", precision)
    z = synth.ar2_chi2(2048 * 10 * 6, seed=17, dtype=np.float32)
    kw = dict(frame_len=2048, n_freq=512, m=10, window="acg", precision=precision)
    a = run_gpu(z, dev, **kw)
    b = run_gpu(z, dev, **kw)
    for k in ("s2", "s3", "s4", "s2_err", "s3_err", "s4_err"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k


@pytest.mark.parametrize("precision", PRECISIONS)
def test_identical_chunks_have_zero_error_bars(dev, precision):
    """A record made of one chunk repeated six times: every chunk's estimate is
    the same, so the averages equal that one chunk's estimate and the error
    bars (Section 4.2) vanish up to the FP64 rounding of the sums."""
    N, Nf, m = 512, 80, 10
    one = synth.ar2_chi2(N * m, seed=23, dtype=np.float32)
    say("identical chunks", precision)
    kw = dict(frame_len=N, n_freq=Nf, m=m, window="acg", precision=precision, orders=(1, 2, 3, 4))
    rep = run_gpu(np.tile(one, 6), dev, **kw)
    single = run_gpu(one, dev, **kw)
    assert rep["n_chunks"] == 6 and single["n_chunks"] == 1
    for k in ("s2", "s3", "s4"):
        scale = np.max(np.abs(single[k]))
        assert np.max(np.abs(rep[k] - single[k])) <= 1e-12 * scale, k
        assert np.all(np.isfinite(rep[k + "_err"])), k
        assert np.max(rep[k + "_err"]) <= 1e-7 * scale, k


@pytest.mark.parametrize("precision,q,orders", [("fp32", 8, (2, 3, 4)), ("bf16x3", 8, (2, 3, 4)),
                                                ("fp16x2s", 8, (2, 3, 4)), ("fp16x2s", -24, (2, 3, 4)),
                                                ("fp16x2s", 40, (2, 4))])
def test_power_of_two_scaling_is_exact(dev, precision, q, orders):
    """z -> 2^q z scales S_n by 2^(nq) (a cumulant of order n is homogeneous
    of degree n): with a power of two every product, split and scale in the
    path is exact, so the outputs scale bit for bit.  q = 40 puts the
    coefficients near 10^16, beyond the FP32 fourth powers' range, which the
    scaled FP16 x 2 S4 reaches through its per-column scales."""
    N, Nf, m = 512, 64, 10
    z = synth.ar2_chi2(N * m * 5, seed=24, dtype=np.float32)
    say("power-of-two scaling", precision, q, orders)
    kw = dict(frame_len=N, n_freq=Nf, m=m, window="acg", precision=precision, orders=orders)
    base = run_gpu(z, dev, **kw)
    scaled = run_gpu(np.ldexp(z, q).astype(np.float32), dev, **kw)
    for n in orders:
        k = f"s{n}"
        for key in (k, k + "_err"):
            assert np.all(np.isfinite(scaled[key])), key
            assert np.array_equal(scaled[key], base[key] * 2.0 ** (n * q)), key    # exact: a power of two


@pytest.mark.parametrize("precision", PRECISIONS)
def test_time_reversal_conjugates(dev, precision):
    """Appendix C: for a symmetric window, reversing a record of whole chunks
    conjugates S3 and leaves S2 and S4 (and every error bar) unchanged: each
    reversed frame's coefficients are e^(-2 pi j k/N) conj(a_k), whose phase
    factors cancel in a_k a_l a*_(k+l), and the chunks are the same set."""
    N, Nf, m = 512, 100, 10
    z = synth.ar2_chi2(N * m * 8, seed=25, dtype=np.float32)
    say("time reversal", precision)
    for window in ("hann", "acg"):
        kw = dict(frame_len=N, n_freq=Nf, m=m, window=window, precision=precision)
        fwd = run_gpu(z, dev, **kw)
        rev = run_gpu(z[::-1].copy(), dev, **kw)
        for k in ("s2", "s3", "s4"):
            want = np.conj(fwd[k]) if k == "s3" else fwd[k]
            assert rel_err(rev[k], want) <= TOL, (window, k, rel_err(rev[k], want))
            assert rel_err(rev[k + "_err"], fwd[k + "_err"]) <= TOL, (window, k)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_duplicated_channel_reduces_to_single(dev, precision):
    """Two copies of one signal as two channels: every combination's S2, S3,
    S4 and error bars equal the single-channel spectra (the cross-channel
    kernels against the single-channel ones)."""
    N, Nf, m = 256, 48, 8
    z = synth.ar2_chi2(N * m * 9, seed=26, dtype=np.float32)
    say("duplicated channel", precision)
    one = run_gpu(z, dev, frame_len=N, n_freq=Nf, m=m, precision=precision)
    two = run_gpu(np.stack([z, z]), dev, frame_len=N, n_freq=Nf, m=m, n_channels=2, precision=precision)
    for k in ("s2", "s3", "s4"):
        assert two[k].shape[0] > 1
        for i in range(two[k].shape[0]):
            assert rel_err(two[k][i], one[k][0]) <= TOL, (k, i, rel_err(two[k][i], one[k][0]))
            assert rel_err(two[k + "_err"][i], one[k + "_err"][0]) <= TOL, (k, i)


def test_sampling_interval_scaling_is_exact(dev):
    """dt -> dt / 4 scales S_n by 4^-(n-1) (the prefactor dt^(n-1) of the
    normalisation): a power of two, so bit for bit, error bars included."""
    N, Nf, m = 512, 64, 10
    z = synth.ar2_chi2(N * m * 4, seed=27, dtype=np.float32)
    say("dt scaling")
    kw = dict(frame_len=N, n_freq=Nf, m=m, window="acg", precision="fp16x2s")
    base = run_gpu(z, dev, dt=1.0, **kw)
    fine = run_gpu(z, dev, dt=0.25, **kw)
    for n in (2, 3, 4):
        for key in (f"s{n}", f"s{n}_err"):
            assert np.array_equal(fine[key], base[key] * 0.25 ** (n - 1)), key


def test_record_beyond_2p31_samples(dev):
    """A record longer than 2^31 samples (int16, 4.3 GB, 1.68 million chunks):
    one 1280-sample chunk repeated, a period that does not divide 2^31, so a
    sample offset wrapped at 32 bits would read a shifted chunk.  Every chunk
    is then the same: the averages equal that chunk's estimate and the error
    bars vanish up to the FP64 rounding of 1.68 million equal terms."""
    from paper_2505_01231_amd import Plan
    N, Nf, m = 256, 8, 5
    reps = (1 << 31) // (N * m) + 3
    z, _ = synth.mixed_channels(N * m, seed=28)
    pattern = torch.from_numpy(np.ascontiguousarray(z[0])).to(dev)
    say("record beyond 2^31 samples", reps * N * m)
    with Plan(frame_len=N, n_freq=Nf, m=m, precision="bf16x3") as p:
        one = p.execute(pattern)
        torch.cuda.synchronize()
        ref = {k: getattr(one, k).cpu().numpy() for k in ("s2", "s3", "s4")}
        x = pattern.repeat(reps)
        assert x.numel() > (1 << 31)
        out = p.execute(x)
        torch.cuda.synchronize()
        assert out.n_chunks == reps
        got = {k: getattr(out, k).cpu().numpy() for k in ("s2", "s3", "s4")}
        err = {k: getattr(out, k + "_err").cpu().numpy() for k in ("s2", "s3", "s4")}
        del x
    for k in ("s2", "s3", "s4"):
        scale = np.max(np.abs(ref[k]))
        assert np.max(np.abs(got[k] - ref[k])) <= 1e-9 * scale, k
        assert np.max(err[k]) <= 1e-6 * scale, k


def test_edge_records(dev):
    """Several records in one call: no complete chunk (NaN), one chunk (NaN error
    bars), and a normal record."""
    from paper_2505_01231_amd import Plan
    say("edge records")
    N, m, Nf = 256, 4, 32
    z = synth.ar2_chi2(N * m * 5, seed=18, dtype=np.float32)
    xs = [torch.from_numpy(z[: N * m - 1]).to(dev), torch.from_numpy(z[: N * m + 5]).to(dev),
          torch.from_numpy(z).to(dev)]
    with Plan(frame_len=N, n_freq=Nf, m=m, window="hann") as p:
        outs = p.execute(xs)
        torch.cuda.synchronize()
        assert [o.n_chunks for o in outs] == [0, 1, 5]
        assert outs[0].flags == 1 and outs[1].flags == 2 and outs[2].flags == 0
        for key in ("s2", "s3", "s4"):
            assert torch.isnan(getattr(outs[0], key)).all()
            assert torch.isnan(getattr(outs[0], key + "_err")).all()
            assert torch.isfinite(getattr(outs[1], key)).all()
            assert torch.isnan(getattr(outs[1], key + "_err")).all()
        ref = O.polyspectra(z, N, Nf, m, window_kind="hann")
        for key in ("s2", "s3", "s4"):
            assert rel_err(torch.view_as_complex(getattr(outs[2], key)).cpu().numpy(), ref[key]) < TOL
        one = O.polyspectra(z[: N * m + 5], N, Nf, m, window_kind="hann")
        assert rel_err(torch.view_as_complex(outs[1].s4).cpu().numpy(), one["s4"]) < TOL


def test_errors_are_reported_not_faulted(dev):
    from paper_2505_01231_amd import Plan
    from paper_2505_01231_amd._lib import PolyspecError
    say("error paths")
    z = torch.zeros(256 * 40, device=dev)
    with Plan(frame_len=256, n_freq=32, m=4) as p:
        small = torch.empty(16, dtype=torch.uint8, device=dev)
        import ctypes as C
        from paper_2505_01231_amd import _lib as L
        rec = (L.ps_record * 1)(p.record(z))
        outs = (L.ps_output * 1)()
        st = L.load().ps_execute(p._handle, rec, 1, small.data_ptr(), small.numel(), outs, None)
        assert st == L.PS_E_WORKSPACE
        with pytest.raises(ValueError):
            p.execute(torch.zeros((2, 256 * 40), device=dev))   # two channels for a one-channel plan
        x = torch.zeros(256 * 40, device=dev)
        rec = (L.ps_record * 1)(p.record(x))
        rec[0].dtype = 9
        assert L.load().ps_execute(p._handle, rec, 1, small.data_ptr(), small.numel(), outs, None) \
            == L.PS_E_INVALID_ARG
        # a record of more chunks than the per-record counters hold is refused
        # before anything reads it
        rec = (L.ps_record * 1)(p.record(x))
        rec[0].n_samples = (1 << 31) * 256 * 4
        assert L.load().ps_execute(p._handle, rec, 1, small.data_ptr(), small.numel(), outs, None) \
            == L.PS_E_UNSUPPORTED
        nbytes = C.c_size_t(0)
        assert L.load().ps_workspace_size(p._handle, rec, 1, C.byref(nbytes)) == L.PS_E_UNSUPPORTED
        with pytest.raises(PolyspecError):
            L.check(L.PS_E_INVALID_ARG, "x")


# ---------------------------------------------------------------- full size, sampled
@pytest.mark.parametrize("precision", ["bf16x3", "fp16x2s"])
def test_full_size_sampled_points(dev, precision):
    """The benchmark workload itself (2^28 float32 AR(2)/chi-square samples,
    N = 8192, N_f = 2048, m = 10, 3276 chunks) in the benchmark's launch
    configuration; the oracle evaluates S2, S3 and S4 point by point on a sample
    of grid points that includes the GPU's largest |S3| and |S4|."""
    from paper_2505_01231_amd import Plan
    say("full size 2^28, N=8192, Nf=2048", precision)
    N, Nf, m = 8192, 2048, 10
    z = synth.ar2_chi2(1 << 28, seed=3)
    x = torch.from_numpy(z).to(dev)
    with Plan(frame_len=N, n_freq=Nf, m=m, window="acg", precision=precision) as p:
        out = p.execute(x)
        torch.cuda.synchronize()
        s2 = torch.view_as_complex(out.s2[0]).cpu().numpy()
        s3 = torch.view_as_complex(out.s3[0]).cpu().numpy()
        s4 = torch.view_as_complex(out.s4[0]).cpu().numpy()
        e4 = out.s4_err[0].cpu().numpy()
    del x
    assert out.n_chunks == 3276
    rng = np.random.default_rng(7)
    pts = [tuple(int(v) for v in np.unravel_index(np.argmax(np.abs(s3)), s3.shape)),
           tuple(int(v) for v in np.unravel_index(np.argmax(np.abs(s4)), s4.shape)),
           (0, 0), (0, Nf - 1), (Nf - 1, Nf - 1), (Nf - 1, 0), (63, 64), (64, 63)]
    pts += [tuple(int(v) for v in rng.integers(0, Nf, 2)) for _ in range(16)]
    bins2 = [pts[0][0], pts[1][0], 0, 1, Nf - 1] + [int(v) for v in rng.integers(0, Nf, 8)]
    say("  oracle on", len(pts), "points")
    ref = O.polyspectra_at(z, N, m, window_kind="acg", points2=bins2, points3=pts, points4=pts)
    got2 = s2[bins2]
    got3 = np.array([s3[k, l] for k, l in pts])
    got4 = np.array([s4[k, l] for k, l in pts])
    got4e = np.array([e4[k, l, 0] for k, l in pts])
    errs = {"s2": rel_err(got2, ref["s2"]), "s3": rel_err(got3, ref["s3"]),
            "s4": rel_err(got4, ref["s4"]), "s4_err": rel_err(got4e, ref["s4_err"][:, 0])}
    say("  sampled rel err", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= TOL, (k, v)


def test_full_size_c3opt_sampled_points(dev):
    """c3^(opt) at the benchmark size (3276 chunks of 11 S3 rows, 2.5 GB of
    workspace): sampled grid points, including the GPU's largest |S3| and the
    bin-0 lines, equal the oracle's point-by-point evaluation."""
    from paper_2505_01231_amd import Plan
    say("full size 2^28 c3opt")
    N, Nf, m = 8192, 2048, 10
    z = synth.ar2_chi2(1 << 28, seed=3)
    x = torch.from_numpy(z).to(dev)
    with Plan(frame_len=N, n_freq=Nf, m=m, window="acg", orders=(2, 3), estimator="c3opt") as p:
        out = p.execute(x)
        torch.cuda.synchronize()
        s3 = torch.view_as_complex(out.s3[0]).cpu().numpy()
        e3 = out.s3_err[0].cpu().numpy()
    del x
    rng = np.random.default_rng(8)
    pts = [tuple(int(v) for v in np.unravel_index(np.argmax(np.abs(s3)), s3.shape)),
           (0, 0), (0, 700), (900, 0), (Nf - 1, Nf - 1), (63, 64)]
    pts += [tuple(int(v) for v in rng.integers(0, Nf, 2)) for _ in range(12)]
    ref = O.polyspectra_at(z, N, m, window_kind="acg", points3=pts, estimator="c3opt")
    got3 = np.array([s3[k, l] for k, l in pts])
    got3e = np.array([e3[k, l] for k, l in pts])
    errs = {"s3": rel_err(got3, ref["s3"]), "s3_err": rel_err(got3e, ref["s3_err"])}
    say("  sampled rel err", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= TOL, (k, v)


def test_more_chunks_than_a_grid_dimension(dev):
    """A record with more chunks than the 65536 limit of the y/z grid
    dimensions (2^28 samples at N = 256, m = 10: 104857 chunks): its means
    equal the chunk-weighted means of a batched run over chunk-aligned slices
    of it (the same chunk sums, added in another order), and a sample of grid
    points matches the oracle."""
    from paper_2505_01231_amd import Plan
    say("104857 chunks, N=256")
    N, Nf, m = 256, 64, 10
    L = 1 << 28
    g = torch.Generator(device=dev)
    g.manual_seed(11)
    x = torch.randn(L, device=dev, generator=g)
    x = x * x - 1.0                               # chi-square(1), centred: non-zero S3 and S4
    chunk = N * m
    with Plan(frame_len=N, n_freq=Nf, m=m, window="acg", precision="bf16x3") as p:
        full = p.execute(x)
        torch.cuda.synchronize()
        assert full.n_chunks == (L // N) // m == 104857
        per = 30000
        parts = [x[i * per * chunk:min(L, (i + 1) * per * chunk)] for i in range(4)]
        outs = p.execute(parts)
        torch.cuda.synchronize()
        n = np.array([o.n_chunks for o in outs], dtype=np.float64)
        assert n.sum() == full.n_chunks
        for key in ("s2", "s3", "s4"):
            f = getattr(full, key).cpu().numpy()
            comb = sum(ni * getattr(o, key).cpu().numpy() for ni, o in zip(n, outs)) / n.sum()
            assert rel_err(comb, f) <= 1e-12, (key, rel_err(comb, f))
        s3 = torch.view_as_complex(full.s3[0]).cpu().numpy()
        s4 = torch.view_as_complex(full.s4[0]).cpu().numpy()
    z = x.cpu().numpy().astype(np.float64)
    del x, parts
    pts = [(0, 0), (5, 17), (63, 63), (31, 2), (10, 40)]
    ref = O.polyspectra_at(z, N, m, window_kind="acg", points3=pts, points4=pts)
    e3 = rel_err(np.array([s3[k, l] for k, l in pts]), ref["s3"])
    e4 = rel_err(np.array([s4[k, l] for k, l in pts]), ref["s4"])
    say("  sampled rel err s3", f"{e3:.2e}", "s4", f"{e4:.2e}")
    assert e3 <= TOL and e4 <= TOL


# ---------------------------------------------------------------- channel combinations
@pytest.mark.parametrize("precision", PRECISIONS)
def test_all_orbits_two_channels(dev, precision):
    """Every S2/S3/S4 combination orbit of two channels (Section 7), including the
    cross-channel S4 forms C4(a_k, b*_k, c_l, d*_l)."""
    say("all orbits, 2 channels", precision)
    rng = np.random.default_rng(21)
    s = synth.ar2_chi2(256 * 8 * 9 + 5, seed=21, r=0.9, dtype=np.float64)
    z = np.stack([s[:-5] + 0.5 * rng.standard_normal(len(s) - 5), s[5:] ** 2 - 1.0 + s[:-5]])
    gpu, ref = both(z, dev, 256, 40, 8, window="acg", n_channels=2, precision=precision)
    assert len(gpu["plan"]["combos4"]) == 7     # (16 + 4 + 4 + 4) / 4 orbits
    compare(gpu, ref, label=f"orbits2-{precision}")


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_all_orbits_four_channels_int16(dev, precision):
    """Four int16 channels mixed from two AR(2)/chi-square sources plus noise:
    all 10 / 40 / 76 combination orbits (the cross-channel S4 on the vector
    ALUs and on the matrix cores)."""
    say("all orbits, 4 int16 channels", precision)
    z, clipped = synth.mixed_channels(512 * 10 * 5 + 77, seed=4)
    assert clipped == 0
    gpu, ref = both(z, dev, 512, 64, 10, window="acg", n_channels=4, precision=precision)
    assert [len(gpu["plan"][f"combos{o}"]) for o in (2, 3, 4)] == [10, 40, 76]
    compare(gpu, ref, label=f"orbits4-int16-{precision}")


# ---------------------------------------------------------------- batching form
@pytest.mark.parametrize("precision", PRECISIONS)
def test_batched_uneven_records(dev, precision):
    """Many records of uneven length (including one without a complete chunk and
    one with a single chunk) and every combination orbit of 2 channels in ONE
    ps_execute: each stage is one launch over all records and combinations.
    Each record must equal the oracle and its own single-record execution."""
    from paper_2505_01231_amd import Plan
    say("batched uneven records", precision)
    N, Nf, m = 512, 100, 6
    rng = np.random.default_rng(31)
    lengths = [N * m * 3 + 17, N * m - 1, N * m + 100, N * m * 7, int(N * m * 4.5), N * m * 2]
    recs = []
    for i, L in enumerate(lengths):
        s = synth.ar2_chi2(L + 3, seed=40 + i, r=0.9, dtype=np.float32)
        recs.append(np.stack([s[:-3], (s[3:] ** 2 - 1).astype(np.float32)]))
    xs = [torch.from_numpy(np.ascontiguousarray(z)).to(dev) for z in recs]
    with Plan(frame_len=N, n_freq=Nf, m=m, window="hann", n_channels=2, precision=precision) as p:
        outs = p.execute(xs)
        torch.cuda.synchronize()
        singles = [p.execute(x) for x in xs]
        torch.cuda.synchronize()
        combos = dict(combos2=p.combos2, combos3=p.combos3, combos4=p.combos4)
        for i, z in enumerate(recs):
            o, s1 = outs[i], singles[i]
            assert o.n_chunks == (lengths[i] // N) // m
            if o.n_chunks == 0:
                assert torch.isnan(o.s3).all()
                continue
            ref = O.polyspectra(z, N, Nf, m, window_kind="hann", **combos)
            for key in ("s2", "s3", "s4"):
                g = torch.view_as_complex(getattr(o, key)).cpu().numpy()
                g1 = torch.view_as_complex(getattr(s1, key)).cpu().numpy()
                assert rel_err(g, ref[key]) <= TOL, (i, key, rel_err(g, ref[key]))
                assert rel_err(g, g1) <= 1e-12, (i, key)
                if o.n_chunks > 1:
                    e = getattr(o, key + "_err").cpu().numpy()
                    assert rel_err(e, ref[key + "_err"]) <= TOL, (i, key + "_err")


@pytest.mark.parametrize("precision", PRECISIONS)
def test_graph_replays_match_eager(dev, precision):
    """ps_graph_create / ps_graph_launch: the captured launch sequence replayed
    several times, with eager work and synchronisations in between and with the
    input contents changed between replays; every replay equals the eager run."""
    from paper_2505_01231_amd import Plan
    say("graph replays", precision)
    N, Nf, m = 1024, 160, 10
    zs = [synth.ar2_chi2(N * m * n + 33, seed=60 + n, dtype=np.float32) for n in (3, 1, 5)]
    xs = [torch.from_numpy(z).to(dev) for z in zs]
    with Plan(frame_len=N, n_freq=Nf, m=m, window="acg", precision=precision) as p:
        g = p.graph(xs)
        for rep in range(4):
            if rep == 2:      # new data in the same buffers
                for x, z in zip(xs, zs):
                    x.copy_(torch.from_numpy((1.5 * z[::-1]).copy()))
            outs = g.launch()
            torch.cuda.synchronize()
            eager = p.execute(xs)          # eager work between replays
            junk = torch.randn(1 << 20, device=dev).sum()
            torch.cuda.synchronize()
            for o, e in zip(outs, eager):
                for key in ("s2", "s3", "s4", "s2_err", "s3_err", "s4_err"):
                    a, b = getattr(o, key).cpu().numpy(), getattr(e, key).cpu().numpy()
                    assert np.array_equal(a, b, equal_nan=True), (rep, key)
            del junk
        g.close()


# ---------------------------------------------------------------- interlaced windows (Section 3)
def both_interlaced(z, dev, N, Nf, m, window="acg", n_channels=1, **kw):
    gpu = run_gpu(z, dev, frame_len=N, n_freq=Nf, m=m, window=window, n_channels=n_channels,
                  interlaced=True, **kw)
    ref = O.polyspectra_interlaced(z, N, Nf, m, window_kind=window, combos2=gpu["plan"]["combos2"],
                                   combos3=gpu["plan"]["combos3"], combos4=gpu["plan"]["combos4"])
    return gpu, ref


def _close_or_both_nan(a, b, tol):
    nan_a, nan_b = np.isnan(a), np.isnan(b)
    assert np.array_equal(nan_a, nan_b)
    if nan_a.all():
        return 0.0
    e = rel_err(np.where(nan_a, 0, a), np.where(nan_b, 0, b))
    assert e <= tol, e
    return e


@pytest.mark.parametrize("precision", PRECISIONS)
def test_interlaced_matches_oracle(dev, precision):
    """Interlaced windows: the spectra of the frames from sample 0 and of the
    frames from sample N/2, averaged (error bars averaged likewise)."""
    say("interlaced", precision)
    N, Nf, m = 256, 60, 8
    z = synth.ar2_chi2(N * m * 6 + 300, seed=71, dtype=np.float32)
    gpu, ref = both_interlaced(z, dev, N, Nf, m, precision=precision)
    assert gpu["n_chunks"] == ref["n_chunks"] == 6 and ref["n_chunks_shifted"] == 6
    compare(gpu, ref, label=f"interlaced-{precision}")


@pytest.mark.parametrize("dtype", [np.float64, np.int16])
def test_interlaced_channels_and_dtypes(dev, dtype):
    """Every combination orbit of two channels with interlaced windows; the
    shifted frame set starts N/2 elements of the record's own type later."""
    say("interlaced, 2 channels", np.dtype(dtype).name)
    N, Nf, m = 512, 64, 10
    if dtype == np.int16:
        z, clipped = synth.mixed_channels(N * m * 4 + 700, seed=72, n_channels=2)
        assert clipped == 0 and z.dtype == np.int16
    else:
        s = synth.ar2_chi2(N * m * 4 + 703, seed=72, r=0.9, dtype=np.float64)
        z = np.stack([s[:-3], s[3:] ** 2 - 1.0])
    gpu, ref = both_interlaced(z, dev, N, Nf, m, n_channels=2, precision="bf16x3")
    compare(gpu, ref, label=f"interlaced-2ch-{np.dtype(dtype).name}")


def test_interlaced_uneven_records(dev):
    """Several records in one execute with interlaced windows: a record without
    a complete chunk (NaN), one whose shifted set has no complete chunk (the
    first set alone, NaN error bars as Np = 1), one with a single chunk in each
    set, and longer ones; each equals the oracle and its own single execution."""
    from paper_2505_01231_amd import Plan
    say("interlaced uneven records")
    N, Nf, m = 256, 50, 6
    lengths = [N * m * 3 + 17, N * m - 1, N * m + N // 4, N * m + N // 2, N * m * 5 + 200]
    zs = [synth.ar2_chi2(L, seed=80 + i, r=0.9, dtype=np.float32) for i, L in enumerate(lengths)]
    xs = [torch.from_numpy(z).to(dev) for z in zs]
    with Plan(frame_len=N, n_freq=Nf, m=m, window="hann", precision="bf16x3", interlaced=True) as p:
        outs = p.execute(xs)
        torch.cuda.synchronize()
        singles = [p.execute(x) for x in xs]
        torch.cuda.synchronize()
        combos = dict(combos2=p.combos2, combos3=p.combos3, combos4=p.combos4)
        for i, z in enumerate(zs):
            o, s1 = outs[i], singles[i]
            ref = O.polyspectra_interlaced(z, N, Nf, m, window_kind="hann", **combos)
            assert o.n_chunks == ref["n_chunks"], i
            if o.n_chunks == 0:
                assert torch.isnan(o.s3).all() and torch.isnan(o.s4_err).all()
                continue
            for key in ("s2", "s3", "s4"):
                g = torch.view_as_complex(getattr(o, key)).cpu().numpy()
                g1 = torch.view_as_complex(getattr(s1, key)).cpu().numpy()
                assert rel_err(g, ref[key]) <= TOL, (i, key, rel_err(g, ref[key]))
                assert rel_err(g, g1) <= 1e-12, (i, key)
                _close_or_both_nan(getattr(o, key + "_err").cpu().numpy(), ref[key + "_err"], TOL)


def test_interlaced_graph_replays_match_eager(dev):
    """A captured interlaced execute replays bit-identically to the eager one."""
    from paper_2505_01231_amd import Plan
    say("interlaced graph")
    N, Nf, m = 1024, 160, 10
    zs = [synth.ar2_chi2(N * m * n + N // 2 + 9, seed=90 + n, dtype=np.float32) for n in (2, 4)]
    xs = [torch.from_numpy(z).to(dev) for z in zs]
    with Plan(frame_len=N, n_freq=Nf, m=m, window="acg", precision="bf16x3", interlaced=True) as p:
        g = p.graph(xs)
        for rep in range(3):
            outs = g.launch()
            torch.cuda.synchronize()
            eager = p.execute(xs)
            torch.cuda.synchronize()
            for o, e in zip(outs, eager):
                for key in ("s2", "s3", "s4", "s2_err", "s3_err", "s4_err"):
                    a, b = getattr(o, key).cpu().numpy(), getattr(e, key).cpu().numpy()
                    assert np.array_equal(a, b, equal_nan=True), (rep, key)
        g.close()


# ---------------------------------------------------------------- sequential spectra, quasi-spectra (Section 8)
@pytest.mark.parametrize("precision", PRECISIONS)
def test_sequential_spectra_match_oracle_chunks(dev, precision):
    """ps_execute_sequential: the short-time estimate of each chunk of a range,
    not averaged, equals the oracle's per-chunk spectra; error bars are NaN."""
    from paper_2505_01231_amd import Plan
    say("sequential", precision)
    N, Nf, m = 256, 40, 6
    z = synth.ar2_chi2(N * m * 7 + 50, seed=101, dtype=np.float32)
    ref = O.polyspectra(z, N, Nf, m, return_chunks=True)
    with Plan(frame_len=N, n_freq=Nf, m=m, precision=precision) as p:
        seq = p.sequential(torch.from_numpy(z).to(dev), chunk_lo=2, n_chunks=4)
        torch.cuda.synchronize()
        assert seq.n_chunks == 4
        for i in range(4):
            for o in (2, 3, 4):
                g = torch.view_as_complex(getattr(seq, f"s{o}")[i]).cpu().numpy()
                e = rel_err(g, ref[f"chunks{o}"][2 + i])
                assert e <= TOL, (precision, i, o, e)
                assert torch.isnan(getattr(seq, f"s{o}_err")[i]).all()


def test_sequential_spectra_channels_and_errors(dev):
    """Sequential spectra of every combination orbit of two channels (whole
    record), and the range checks of ps_execute_sequential."""
    import ctypes
    from paper_2505_01231_amd import Plan
    from paper_2505_01231_amd import _lib as L
    say("sequential, 2 channels")
    N, Nf, m = 256, 32, 5
    s = synth.ar2_chi2(N * m * 3 + 9, seed=102, r=0.9, dtype=np.float64)
    z = np.stack([s[:-3], s[3:] ** 2 - 1.0])
    x = torch.from_numpy(z).to(dev)
    with Plan(frame_len=N, n_freq=Nf, m=m, n_channels=2, precision="bf16x3") as p:
        seq = p.sequential(x)
        torch.cuda.synchronize()
        ref = O.polyspectra(z, N, Nf, m, return_chunks=True, combos2=p.combos2, combos3=p.combos3,
                            combos4=p.combos4)
        assert seq.n_chunks == ref["n_chunks"] == 3
        for c in range(3):
            for o in (2, 3, 4):
                g = torch.view_as_complex(getattr(seq, f"s{o}")[c]).cpu().numpy()
                assert rel_err(g, ref[f"chunks{o}"][c]) <= TOL, (c, o)
        rec = p.record(x)
        n = ctypes.c_size_t()
        for lo, cnt in ((2, 2), (-1, 1), (0, 4)):
            st = p._lib.ps_sequential_workspace_size(p._handle, ctypes.byref(rec), lo, cnt, ctypes.byref(n))
            assert st == L.PS_E_INVALID_ARG, (lo, cnt)
        empty = p.sequential(x, chunk_lo=3, n_chunks=0)
        assert empty.n_chunks == 0 and empty.s4.shape[0] == 0


def test_quasi_spectra_sweep(dev):
    """The m sweep of quasi-spectra on an oscillator whose frequency drifts:
    every m matches the oracle, and the diagonal of S4 / S2^2 grows with m
    (Section 8's quasi-correlations)."""
    from paper_2505_01231_amd import quasi_spectra
    say("quasi-spectra sweep")
    N, Nf = 256, 64
    z = synth.drifting_ar2(N * 1200, seed=103, theta0=0.1 * np.pi, theta1=0.7 * np.pi, dtype=np.float32)
    res = quasi_spectra(torch.from_numpy(z).to(dev), [10, 300], frame_len=N, n_freq=Nf, orders=(2, 4),
                        precision="bf16x3")
    q = {}
    for m, out in res.items():
        ref = O.polyspectra(z, N, Nf, m, orders=(2, 4))
        for key in ("s2", "s4"):
            g = torch.view_as_complex(getattr(out, key)).cpu().numpy()
            assert rel_err(g, ref[key]) <= TOL, (m, key)
        s2, s4 = out.s2[0, :, 0].cpu().numpy(), out.s4[0, :, :, 0].cpu().numpy()
        band = s2 > 0.2 * s2.max()
        q[m] = float((np.diag(s4)[band] / s2[band] ** 2).mean())
    say("  diagonal S4/S2^2 by m", q)
    assert q[300] > 3 * max(q[10], 1.0), q


# ---------------------------------------------------------------- first-order spectrum S1 (Section 3)
def _s1(out):
    return out.s1[:, 0].cpu().numpy(), out.s1_err.cpu().numpy()


@pytest.mark.parametrize("schedule", ["batched", "per_chunk"])
def test_s1_matches_oracle(dev, schedule):
    """S1 per channel (the windowed mean, with its error bar) next to S2..S4, on
    two channels with different offsets, in both schedules; a record without a
    chunk gives NaN."""
    from paper_2505_01231_amd import Plan
    say("S1", schedule)
    N, Nf, m = 512, 60, 6
    s = synth.ar2_chi2(N * m * 9 + 40, seed=111, r=0.9, dtype=np.float64)
    z = np.stack([s[:-3] + 1.5, 0.5 * (s[3:] ** 2 - 1.0) - 0.25]).astype(np.float32)
    with Plan(frame_len=N, n_freq=Nf, m=m, n_channels=2, orders=(1, 2, 3, 4), precision="bf16x3",
              schedule=schedule) as p:
        outs = p.execute([torch.from_numpy(z).to(dev), torch.from_numpy(z[:, :N * m - 1].copy()).to(dev)])
        torch.cuda.synchronize()
        ref = O.polyspectra(z, N, Nf, m, orders=(1, 2, 3, 4), combos2=p.combos2, combos3=p.combos3,
                            combos4=p.combos4)
        s1, e1 = _s1(outs[0])
        assert rel_err(s1, ref["s1"].real) <= TOL, (s1, ref["s1"])
        assert rel_err(e1, ref["s1_err"]) <= TOL
        assert np.all(outs[0].s1[:, 1].cpu().numpy() == 0)
        for key in ("s2", "s3", "s4"):
            g = torch.view_as_complex(getattr(outs[0], key)).cpu().numpy()
            assert rel_err(g, ref[key]) <= TOL, key
        assert torch.isnan(outs[1].s1).all() and torch.isnan(outs[1].s1_err).all()


def test_s1_alone_constant_interlaced_and_sequential(dev):
    """An S1-only plan at m = 1 on a constant record gives the constant with a
    zero error bar; S1 of interlaced windows and of sequential spectra follow
    the oracle."""
    from paper_2505_01231_amd import Plan
    say("S1 alone / interlaced / sequential")
    N = 256
    c = torch.full((N * 7 + 5,), -3.25, device=dev)
    with Plan(frame_len=N, n_freq=8, m=1, orders=(1,)) as p:
        o = p.execute(c)
        torch.cuda.synchronize()
        assert o.n_chunks == 7 and o.s2 is None
        assert abs(o.s1[0, 0].item() + 3.25) <= 1e-6 * 3.25 and abs(o.s1_err[0, 0].item()) <= 1e-6
    Nf, m = 40, 5
    z = synth.ar2_chi2(N * m * 6 + 200, seed=112, dtype=np.float32) + np.float32(0.75)
    x = torch.from_numpy(z).to(dev)
    with Plan(frame_len=N, n_freq=Nf, m=m, orders=(1, 2), interlaced=True) as p:
        o = p.execute(x)
        torch.cuda.synchronize()
        ref = O.polyspectra_interlaced(z, N, Nf, m, orders=(1, 2))
        s1, e1 = _s1(o)
        assert rel_err(s1, ref["s1"].real) <= TOL and rel_err(e1, ref["s1_err"]) <= TOL
    with Plan(frame_len=N, n_freq=Nf, m=m, orders=(1, 2)) as p:
        seq = p.sequential(x)
        torch.cuda.synchronize()
        ref = O.polyspectra(z, N, Nf, m, orders=(1, 2), return_chunks=True)
        g = seq.s1[:, :, 0].cpu().numpy()            # [chunks, channels]
        assert rel_err(g, ref["chunks1"].real) <= TOL


# ---------------------------------------------------------------- natural (plug-in) estimator (Section 6)
@pytest.mark.parametrize("precision", PRECISIONS)
def test_natural_estimator_matches_oracle(dev, precision):
    """estimator="natural": the plug-in cumulant estimates (biased at small m)
    equal the oracle's natural estimator and differ from the k-statistics."""
    say("natural estimator", precision)
    N, Nf, m = 256, 50, 5
    z = synth.ar2_chi2(N * m * 12 + 70, seed=121, dtype=np.float32)
    gpu = run_gpu(z, dev, frame_len=N, n_freq=Nf, m=m, precision=precision, estimator="natural")
    ref = O.polyspectra(z, N, Nf, m, estimator="natural")
    compare(gpu, ref, label=f"natural-{precision}")
    kst = O.polyspectra(z, N, Nf, m)
    assert rel_err(gpu["s4"], kst["s4"]) > 0.05      # m = 5: the two estimators differ


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_natural_estimator_cross_channels(dev, precision):
    """The natural estimator for every combination orbit of two channels (the
    cross-channel S4 kernels on the vector ALUs and on the matrix cores)."""
    say("natural estimator, 2 channels", precision)
    N, Nf, m = 256, 32, 6
    s = synth.ar2_chi2(N * m * 8 + 9, seed=122, r=0.9, dtype=np.float64)
    z = np.stack([s[:-3], s[3:] ** 2 - 1.0])
    gpu = run_gpu(z, dev, frame_len=N, n_freq=Nf, m=m, n_channels=2, precision=precision, estimator="natural")
    ref = O.polyspectra(z, N, Nf, m, estimator="natural", combos2=gpu["plan"]["combos2"],
                        combos3=gpu["plan"]["combos3"], combos4=gpu["plan"]["combos4"])
    compare(gpu, ref, label=f"natural-2ch-{precision}")


# ---------------------------------------------------------------- c3^(opt) (Section 4.1)
@pytest.mark.parametrize("precision", PRECISIONS)
def test_c3opt_matches_oracle(dev, precision):
    """estimator="c3opt": S3 by c3^(opt) (the S3 kernel over m shifted frames
    and one mean row per chunk) equals the oracle's direct formula; S2 and S4
    are still the k-statistics."""
    say("c3opt", precision)
    N, Nf, m = 256, 50, 10
    z = synth.ar2_chi2(N * m * 12 + 70, seed=181, dtype=np.float32)
    gpu = run_gpu(z, dev, frame_len=N, n_freq=Nf, m=m, precision=precision, estimator="c3opt")
    ref = O.polyspectra(z, N, Nf, m, estimator="c3opt")
    compare(gpu, ref, label=f"c3opt-{precision}")
    kst = O.polyspectra(z, N, Nf, m, orders=(3,))
    assert rel_err(gpu["s3"], kst["s3"]) > 1e-3


@pytest.mark.parametrize("m,schedule", [(2, "batched"), (2, "per_chunk"), (17, "batched"), (17, "per_chunk")])
def test_c3opt_channels_small_and_large_m(dev, m, schedule):
    """Two f64 channels with a mean offset (every S3 orbit, bias at bin 0 kept
    as the formula gives it), m = 2 (below the k-statistic's minimum) and
    m = 17 (the centring pass's loop form), in both schedules."""
    say("c3opt, 2 channels", m, schedule)
    N, Nf = 256, 24
    s = synth.ar2_chi2(N * m * 9 + 33, seed=182, r=0.9, dtype=np.float64)
    z = np.stack([s[:-5] + 0.4, s[5:] ** 2 - 0.5])
    gpu = run_gpu(z, dev, frame_len=N, n_freq=Nf, m=m, n_channels=2, orders=(2, 3), estimator="c3opt",
                  schedule=schedule, window="hann")
    ref = O.polyspectra(z, N, Nf, m, orders=(2, 3), window_kind="hann", estimator="c3opt",
                        combos2=gpu["plan"]["combos2"], combos3=gpu["plan"]["combos3"])
    compare(gpu, ref, keys=("s2", "s3"), label=f"c3opt-2ch-m{m}-{schedule}")


def test_c3opt_complex_interlaced_sequential(dev):
    """c3^(opt) on the complex path (signed grid), with interlaced windows, and
    per chunk (sequential spectra) against the oracle."""
    from paper_2505_01231_amd import Plan
    say("c3opt complex / interlaced / sequential")
    N, Nf, m = 256, 30, 8
    zc = _complex_signal(N * m * 6 + 20, seed=183, N=N).astype(np.complex64)
    gpu = run_gpu(zc, dev, frame_len=N, n_freq=Nf, m=m, complex_signal=True, orders=(2, 3), estimator="c3opt")
    ref = O.polyspectra_complex(zc, N, Nf, m, orders=(2, 3), estimator="c3opt")
    compare(gpu, ref, keys=("s2", "s3"), label="c3opt-complex")
    z = synth.ar2_chi2(N * m * 7 + 90, seed=184, dtype=np.float32)
    with Plan(frame_len=N, n_freq=Nf, m=m, precision="bf16x3", interlaced=True, estimator="c3opt") as p:
        out = p.execute(torch.from_numpy(z).to(dev))
        torch.cuda.synchronize()
        ref = O.polyspectra_interlaced(z, N, Nf, m, estimator="c3opt")
        for key in ("s2", "s3", "s4"):
            g = torch.view_as_complex(getattr(out, key)).cpu().numpy()
            assert rel_err(g, ref[key]) <= TOL, (key, rel_err(g, ref[key]))
            assert rel_err(getattr(out, key + "_err").cpu().numpy(), ref[key + "_err"]) <= TOL, key
    ref = O.polyspectra(z, N, Nf, m, orders=(3,), estimator="c3opt", return_chunks=True)
    with Plan(frame_len=N, n_freq=Nf, m=m, orders=(3,), estimator="c3opt") as p:
        seq = p.sequential(torch.from_numpy(z).to(dev), chunk_lo=1, n_chunks=3)
        torch.cuda.synchronize()
        for i in range(3):
            g = torch.view_as_complex(seq.s3[i]).cpu().numpy()
            assert rel_err(g, ref["chunks3"][1 + i]) <= TOL, i


def test_c3opt_graph_and_streamer(dev):
    """c3^(opt) through a captured graph (three replays, each bit-identical to
    the eager execute) and through the streamer's multi-window pushes (each
    window's spectra equal a single execute of that window)."""
    from paper_2505_01231_amd import Plan, Streamer
    say("c3opt graph / streamer")
    N, Nf, m = 512, 64, 10
    zs = [synth.ar2_chi2(N * m * n + 77, seed=185 + n, dtype=np.float32) for n in (2, 3)]
    xs = [torch.from_numpy(z).to(dev) for z in zs]
    with Plan(frame_len=N, n_freq=Nf, m=m, precision="bf16x3", estimator="c3opt") as p:
        g = p.graph(xs)
        for rep in range(3):
            outs = g.launch()
            torch.cuda.synchronize()
            eager = p.execute(xs)
            torch.cuda.synchronize()
            for o, e in zip(outs, eager):
                for key in ("s2", "s3", "s4", "s2_err", "s3_err", "s4_err"):
                    a, b = getattr(o, key).cpu().numpy(), getattr(e, key).cpu().numpy()
                    assert np.array_equal(a, b, equal_nan=True), (rep, key)
        g.close()
        ref = O.polyspectra(zs[1], N, Nf, m, estimator="c3opt")
        got = torch.view_as_complex(eager[1].s3).cpu().numpy()
        assert rel_err(got, ref["s3"]) <= TOL
        W = N * m * 3
        z = synth.modulated_ar2(4 * W, seed=186, total=4 * W, r=0.9)
        st = Streamer(p, W, dtype=torch.float32, depth=2, windows_per_push=2)
        for w0 in (0, 2):
            host = torch.from_numpy(z[w0 * W:(w0 + 2) * W].copy()).pin_memory()
            outs = [p.allocate_outputs(dev) for _ in range(2)]
            st.wait(st.push(host, outs))
            ref = p.execute([torch.from_numpy(z[(w0 + i) * W:(w0 + i + 1) * W].copy()).to(dev) for i in range(2)])
            torch.cuda.synchronize()
            for i in range(2):
                for k in ("s2", "s3", "s4", "s3_err"):
                    assert np.array_equal(getattr(outs[i], k).cpu().numpy(), getattr(ref[i], k).cpu().numpy()), (w0, i, k)
        st.close()


# ---------------------------------------------------------------- full frequency plane (Section 9)
def test_full_plane_matches_direct_evaluation(dev):
    """ps_full_plane gathers one combination's S2 / S3 / S4 on the signed grid
    (-N_f, N_f) from the positive quadrants of every orbit; the oracle evaluates
    the same points directly (a_{-k} = a_{N-k}), with no symmetry used."""
    import ctypes
    from paper_2505_01231_amd import Plan
    from paper_2505_01231_amd import _lib as L
    say("full plane, 3 channels")
    N, Nf, m = 256, 12, 8
    rng = np.random.default_rng(131)
    s = synth.ar2_chi2(N * m * 12 + 9, seed=131, r=0.8, dtype=np.float64)
    z = np.stack([s[:-6], s[3:-3] ** 2 - 1 + 0.3 * rng.standard_normal(len(s) - 6), s[6:] * s[:-6]])
    pts = [(k, l) for k in range(-Nf + 1, Nf) for l in range(-Nf + 1, Nf)]
    with Plan(frame_len=N, n_freq=Nf, m=m, n_channels=3, precision="bf16x3") as p:
        out = p.execute(torch.from_numpy(z).to(dev))
        for order, combo in ((2, (1, 0)), (3, (0, 1, 2)), (3, (2, 0, 1)), (3, (1, 1, 0)),
                             (4, (0, 1, 2, 0)), (4, (2, 1, 0, 1)), (4, (1, 1, 2, 2))):
            val, err = p.full_plane(out, order, combo)
            torch.cuda.synchronize()
            g = torch.view_as_complex(val).cpu().numpy()
            ge = err.cpu().numpy()
            if order == 2:
                ref = O.polyspectra_at(z, N, m, points2=list(range(-Nf + 1, Nf)), combo2=combo)
                rv, re_ = ref["s2"], ref["s2_err"]
            else:
                ref = O.polyspectra_at(z, N, m, **{f"points{order}": pts, f"combo{order}": combo})
                rv = ref[f"s{order}"].reshape(2 * Nf - 1, 2 * Nf - 1)
                re_ = ref[f"s{order}_err"].reshape(2 * Nf - 1, 2 * Nf - 1, 2)
            e, ee = rel_err(g, rv), rel_err(ge, re_)
            say("  order", order, combo, f"{e:.2e}/{ee:.2e}")
            assert e <= TOL and ee <= TOL, (order, combo, e, ee)
        # the positive quadrant is the execute's own output
        val, _ = p.full_plane(out, 3, (0, 1, 2))
        i = p.combos3.index((0, 1, 2))
        assert torch.equal(val[Nf - 1:, Nf - 1:], out.s3[i])
    # a plan without the needed orbits cannot build the plane
    with Plan(frame_len=N, n_freq=Nf, m=m, n_channels=3, combos3=[(0, 1, 2)], orders=(3,)) as p:
        out = p.execute(torch.from_numpy(z).to(dev))
        cb = (ctypes.c_int8 * 3)(0, 1, 2)
        st = p._lib.ps_full_plane(p._handle, 3, cb, ctypes.byref(out.c_struct()), None, None, None)
        assert st == L.PS_E_UNSUPPORTED
        torch.cuda.synchronize()


def test_section9_equivalences_on_full_planes(dev):
    """The equivalences of Section 9 between spectra of permuted channels, on
    the planes ps_full_plane gathers: S3_yyx(w) = S3_xyy(M w) with
    M = [[-1, -1], [1, 0]], S4_yxyy(k, l) = S4_xyyy(-k, l) and
    S4_xyyx(k, l) = S4_xyxy(k, -l), at every grid point whose image lies in
    the grid, and the mapped points against the oracle's direct evaluation."""
    from paper_2505_01231_amd import Plan
    say("Section 9 equivalences")
    N, Nf, m = 256, 10, 8
    s = synth.ar2_chi2(N * m * 10 + 7, seed=141, r=0.85, dtype=np.float64)
    z = np.stack([s[:-7], s[7:] ** 2 - 1.0 + 0.5 * s[:-7]])
    x, y = 0, 1
    E = 2 * Nf - 1
    at = lambda k: k + Nf - 1         # noqa: E731  (grid index of signed bin k)
    with Plan(frame_len=N, n_freq=Nf, m=m, n_channels=2, precision="bf16x3") as p:
        out = p.execute(torch.from_numpy(z).to(dev))
        planes = {}
        for order, combo in ((3, (x, y, y)), (3, (y, y, x)), (4, (x, y, y, y)), (4, (y, x, y, y)),
                             (4, (x, y, x, y)), (4, (x, y, y, x))):
            val, _ = p.full_plane(out, order, combo)
            planes[combo] = torch.view_as_complex(val).cpu().numpy()
        torch.cuda.synchronize()
    pairs = []          # (combo, point, image combo, image point)
    for k in range(-Nf + 1, Nf):
        for l in range(-Nf + 1, Nf):
            if abs(k + l) < Nf:
                pairs.append(((y, y, x), (k, l), (x, y, y), (-k - l, k)))
            pairs.append(((y, x, y, y), (k, l), (x, y, y, y), (-k, l)))
            pairs.append(((x, y, y, x), (k, l), (x, y, x, y), (k, -l)))
    # Away from zero frequencies both sides are gathered from the same stored
    # value; where a frequency is zero two stored quadrants hold the same
    # cumulant, computed separately, so they agree to the parity tolerance.
    scale = {c: np.abs(v).max() for c, v in planes.items()}
    for cb, (k, l), cb2, (k2, l2) in pairs:
        a, b = planes[cb][at(k), at(l)], planes[cb2][at(k2), at(l2)]
        tol = TOL if 0 in ((k, l, k + l) if len(cb) == 3 else (k, l)) else 1e-12
        assert abs(a - b) <= tol * scale[cb], (cb, k, l, cb2, k2, l2, a, b)
    # the mapped S3 points against the oracle's direct evaluation
    pts = [(k2, l2) for cb, _, cb2, (k2, l2) in pairs if len(cb2) == 3]
    ref = O.polyspectra_at(z, N, m, window_kind="acg", points3=pts, combo3=(x, y, y))
    got = np.array([planes[(x, y, y)][at(k2), at(l2)] for k2, l2 in pts])
    e = rel_err(got, ref["s3"])
    say("  S3_yyx via M vs oracle", f"{e:.2e}", len(pts), "points")
    assert e <= TOL


# ---------------------------------------------------------------- complex-valued signals
def _complex_signal(n, seed, q=3, N=256, channels=1):
    rng = np.random.default_rng(seed)
    out = []
    for c in range(channels):
        x = synth.ar2_chi2(n, seed=seed + c, r=0.9, dtype=np.float64)
        z = x * np.exp(2j * np.pi * (q + c) * np.arange(n) / N) + 0.3 * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
        out.append(z)
    return np.stack(out) if channels > 1 else out[0]


@pytest.mark.parametrize("precision", PRECISIONS)
def test_complex_signal_matches_oracle(dev, precision):
    """A complex record (a shifted AR(2)/chi-square process plus complex noise):
    S1..S4 on the signed grid (-N_f, N_f) equal the oracle's."""
    say("complex signal", precision)
    N, Nf, m = 256, 40, 8
    z = _complex_signal(N * m * 7 + 30, seed=151, N=N).astype(np.complex64)
    gpu = run_gpu(z, dev, frame_len=N, n_freq=Nf, m=m, precision=precision, complex_signal=True,
                  orders=(1, 2, 3, 4))
    ref = O.polyspectra_complex(z, N, Nf, m, orders=(1, 2, 3, 4))
    assert gpu["s3"].shape == (1, 2 * Nf - 1, 2 * Nf - 1)
    compare(gpu, ref, label=f"complex-{precision}")


def test_complex_path_on_real_data_equals_full_plane(dev):
    """Two real channels given as complex64: the complex plan's grids equal the
    real plan's outputs gathered onto the full plane (two GPU paths)."""
    from paper_2505_01231_amd import Plan
    say("complex path on real data")
    N, Nf, m = 256, 24, 8
    s = synth.ar2_chi2(N * m * 6 + 9, seed=152, r=0.9, dtype=np.float32)
    z = np.stack([s[:-3], s[3:] ** 2 - 1]).astype(np.float32)
    kw = dict(frame_len=N, n_freq=Nf, m=m, n_channels=2, precision="bf16x3")
    with Plan(complex_signal=True, **kw) as pc, Plan(**kw) as pr:
        oc = pc.execute(torch.from_numpy(z.astype(np.complex64)).to(dev))
        orl = pr.execute(torch.from_numpy(z).to(dev))
        assert pc.combos3 == pr.combos3 and pc.grid == 2 * Nf - 1
        for order in (2, 3, 4):
            combos = getattr(pc, f"combos{order}")
            for i, cb in enumerate(combos):
                val, err = pr.full_plane(orl, order, cb)
                torch.cuda.synchronize()
                g = torch.view_as_complex(getattr(oc, f"s{order}")[i]).cpu().numpy()
                ge = getattr(oc, f"s{order}_err")[i].cpu().numpy()
                r = torch.view_as_complex(val).cpu().numpy()
                assert rel_err(g, r) <= TOL, (order, cb, rel_err(g, r))
                assert rel_err(ge, err.cpu().numpy()) <= TOL, (order, cb)


def test_complex_channels_interlaced_and_errors(dev):
    """Two complex128 channels, every orbit, interlaced windows, vs the oracle;
    a real record on a complex plan and the full plane of a complex plan are
    refused."""
    import ctypes
    from paper_2505_01231_amd import Plan
    from paper_2505_01231_amd import _lib as L
    say("complex, 2 channels, interlaced")
    N, Nf, m = 256, 20, 6
    z = _complex_signal(N * m * 5 + 200, seed=153, N=N, channels=2)
    with Plan(frame_len=N, n_freq=Nf, m=m, n_channels=2, precision="bf16x3", complex_signal=True,
              interlaced=True, orders=(1, 2, 3, 4)) as p:
        out = p.execute(torch.from_numpy(z).to(dev))
        torch.cuda.synchronize()
        ref = O.polyspectra_interlaced(z, N, Nf, m, orders=(1, 2, 3, 4), combos2=p.combos2, combos3=p.combos3,
                                       combos4=p.combos4)
        for key in ("s1", "s2", "s3", "s4"):
            g = torch.view_as_complex(getattr(out, key)).cpu().numpy()
            assert rel_err(g, ref[key]) <= TOL, (key, rel_err(g, ref[key]))
            assert rel_err(getattr(out, key + "_err").cpu().numpy(), ref[key + "_err"]) <= TOL, key
        with pytest.raises(RuntimeError):
            p.execute(torch.from_numpy(z.real.copy()).to(dev))
        cb = (ctypes.c_int8 * 3)(0, 1, 0)
        st = p._lib.ps_full_plane(p._handle, 3, cb, ctypes.byref(out.c_struct()), None, None, None)
        assert st == L.PS_E_UNSUPPORTED


@pytest.mark.parametrize("precision", PRECISIONS)
def test_s4_plane_matches_oracle(dev, precision):
    """S4 on the plane parallel to the cut shifted by q = 3 bins, a real record
    given as complex: C4(a_{k+q}, a*_{k-q}, a_{l-q}, a*_{l+q}) on the signed grid
    (the cross-channel kernels, full grids) equals the oracle's."""
    say("S4 plane", precision)
    N, Nf, m = 256, 30, 8
    z = synth.ar2_chi2(N * m * 6 + 40, seed=171, dtype=np.float32).astype(np.complex64)
    gpu = run_gpu(z, dev, frame_len=N, n_freq=Nf, m=m, precision=precision, complex_signal=True, s4_shift=3,
                  orders=(2, 4))
    ref = O.polyspectra_complex(z, N, Nf, m, orders=(2, 4), s4_shift=3, combos4=gpu["plan"]["combos4"])
    compare(gpu, ref, keys=("s2", "s4"), label=f"plane-{precision}")


@pytest.mark.parametrize("estimator", ["kstat", "c3opt"])
def test_s4_plane_wide_shift_with_s3(dev, estimator):
    """Two complex channels, q = -N_f (a wider stored bin range, so S3's third
    factor sits at an offset column), S2, S3 and every S4 combination; with
    c3^(opt) the S3 rows carry the same offset."""
    say("S4 plane, wide shift, 2 channels", estimator)
    N, Nf, m = 256, 20, 6
    z = _complex_signal(N * m * 5 + 11, seed=172, N=N, channels=2).astype(np.complex64)
    gpu = run_gpu(z, dev, frame_len=N, n_freq=Nf, m=m, n_channels=2, precision="bf16x3", complex_signal=True,
                  s4_shift=-Nf, estimator=estimator)
    assert len(gpu["plan"]["combos4"]) == 16
    ref = O.polyspectra_complex(z, N, Nf, m, s4_shift=-Nf, combos2=gpu["plan"]["combos2"],
                                combos3=gpu["plan"]["combos3"], combos4=gpu["plan"]["combos4"], estimator=estimator)
    compare(gpu, ref, label=f"plane-wide-2ch-{estimator}")


# ---------------------------------------------------------------- frame lengths that are not a power of two
@pytest.mark.parametrize("N,dtype", [(768, np.float32), (1280, np.float64), (1536, np.int16), (1000, np.float32),
                                     (2560, np.float32), (3072, np.int16), (5120, np.float32), (6144, np.float64),
                                     (999, np.int16), (1021, np.float32), (2042, np.int16), (8190, np.float32)])
def test_direct_transform_frame_lengths_coefficients(dev, N, dtype):
    """Frame lengths that are not a power of two take the direct transform
    (FP64 accumulation; in two stages for N = N1 N2 with 8 <= N1 <= sqrt(N),
    8190 = 90 * 91 the largest LDS use, in one for the prime 1021 and for
    2042 = 2 * 1021): it equals the oracle's
    FFT of the frames for all K = N // 2 + 1 coefficients."""
    from paper_2505_01231_amd import Plan
    say("direct transform coefficients", N, dtype.__name__)
    m = 4
    Nf = N // 4 + 1
    if dtype == np.int16:
        z = np.clip(np.rint(synth.ar2_chi2(N * m * 3 + 17, seed=8) * 300), -32768, 32767).astype(np.int16)
    else:
        z = synth.ar2_chi2(N * m * 3 + 17, seed=8, dtype=dtype)
    with Plan(frame_len=N, n_freq=Nf, m=m, window="acg") as p:
        a = p.coefficients(torch.from_numpy(z).to(dev))
        torch.cuda.synchronize()
        a = a.cpu().numpy()[0]
        K = p.n_coef
    assert K == 2 * Nf - 1 <= N // 2 + 1
    g = O.window("acg", N)
    ref = O.coefficients(O.chunk_frames(z, N, m).reshape(-1, N), g, 1.0, K)
    e = rel_err(a, ref)
    say("  coef rel err", e)
    assert a.shape == ref.shape and e < 2e-6


@pytest.mark.parametrize("precision", PRECISIONS)
def test_direct_transform_frame_length_spectra(dev, precision):
    """S1..S4 at N = 1536 (2 * 3 * 256) vs the oracle."""
    say("direct transform spectra", precision)
    N, Nf, m = 1536, 120, 8
    z = synth.ar2_chi2(N * m * 6 + 5, seed=181, dtype=np.float32)
    gpu = run_gpu(z, dev, frame_len=N, n_freq=Nf, m=m, precision=precision, orders=(1, 2, 3, 4))
    ref = O.polyspectra(z, N, Nf, m, orders=(1, 2, 3, 4))
    compare(gpu, ref, label=f"dft-1536-{precision}")


def test_direct_transform_odd_length_channels_interlaced(dev):
    """An odd frame length (N = 1001) with two int16 channels, every orbit and
    interlaced windows (the second frame set N // 2 samples in) vs the oracle."""
    say("direct transform odd length, two channels, interlaced")
    N, Nf, m = 1001, 150, 5
    z, clipped = synth.mixed_channels(N * m * 5 + N // 2 + 9, seed=23, n_channels=2)
    assert clipped == 0 and z.dtype == np.int16
    gpu, ref = both_interlaced(z, dev, N, Nf, m, n_channels=2, precision="bf16x3")
    compare(gpu, ref, label="dft-1001-2ch-interlaced")


def test_direct_transform_through_every_entry_point(dev):
    """An odd frame length (N = 1000, the direct transform) through the other
    entry points: graph replays equal the eager run; a running accumulation
    pushed in pieces equals one execute; sequential spectra equal the oracle's
    per-chunk estimates; c3^(opt) and the natural estimator equal the oracle."""
    from paper_2505_01231_amd import Accumulator, Plan
    say("direct transform, every entry point")
    N, Nf, m = 1000, 120, 6
    z = synth.ar2_chi2(N * m * 7 + 321, seed=141, dtype=np.float32)
    x = torch.from_numpy(z).to(dev)
    with Plan(frame_len=N, n_freq=Nf, m=m, window="acg", precision="fp16x2s", orders=(1, 2, 3, 4)) as p:
        eager = p.execute(x)
        g = p.graph([x])
        for rep in range(3):
            outs = g.launch()
            torch.cuda.synchronize()
            for key in ("s2", "s3", "s4", "s2_err", "s3_err", "s4_err"):
                a, b = getattr(outs[0], key).cpu().numpy(), getattr(eager, key).cpu().numpy()
                assert np.array_equal(a, b, equal_nan=True), (rep, key)
        g.close()
        acc = Accumulator(p, max_push_samples=N * m * 2)
        cuts = [0, N * m * 2, N * m * 2 + 777, N * m * 3 + 782]
        cuts += list(range(cuts[-1] + N * m * 2, len(z), N * m * 2)) + [len(z)]
        for a, b in zip(cuts[:-1], cuts[1:]):
            acc.push(x[a:b])
        got = acc.end()
        torch.cuda.synchronize()
        acc.close()
        for key in ("s2", "s3", "s4", "s2_err", "s3_err", "s4_err"):
            e = rel_err(getattr(got, key).cpu().numpy(), getattr(eager, key).cpu().numpy())
            assert e <= 1e-12, key
        seq = p.sequential(x, chunk_lo=1, n_chunks=3)
        torch.cuda.synchronize()
        ref = O.polyspectra(z, N, Nf, m, orders=(1, 2, 3, 4), return_chunks=True)
        for i in range(3):
            for o in (2, 3, 4):
                gs = torch.view_as_complex(getattr(seq, f"s{o}")[i]).cpu().numpy()
                assert rel_err(gs, ref[f"chunks{o}"][1 + i]) <= TOL, (i, o)
        ev = {k: torch.view_as_complex(getattr(eager, k)).cpu().numpy() for k in ("s2", "s3", "s4")}
    for k in ("s2", "s3", "s4"):
        assert rel_err(ev[k], ref[k]) <= TOL, k
    for est in ("c3opt", "natural"):
        gpu = run_gpu(z, dev, frame_len=N, n_freq=Nf, m=m, window="acg", precision="bf16x3", estimator=est)
        refe = O.polyspectra(z, N, Nf, m, estimator=est)
        compare(gpu, refe, label=f"dft-1000-{est}")


# ---------------------------------------------------------------- launch configuration (autotuner)
def _tuning_case(dev):
    """Two channels (every S3/S4 orbit, so all four tile tables are used), a
    ragged grid (N_f = 200: 4 tiles of 64, 7 of 32) and m = 12, where the S3
    frame batch is a real choice."""
    s = synth.ar2_chi2(1024 * 12 * 4 + 9, seed=77, r=0.9, dtype=np.float32)
    z = np.stack([s[:-9], (s[9:] ** 2 - 1.0 + 0.3 * s[:-9]).astype(np.float32)])
    return z, torch.from_numpy(np.ascontiguousarray(z)).to(dev)


def _spectra(out):
    return {k: getattr(out, k).cpu().numpy() for k in ("s2", "s3", "s4", "s2_err", "s3_err", "s4_err")}


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_tuning_configurations_agree(dev, precision):
    """Every tile order and S3 frame batch computes the same spectra up to the
    order of FP64 additions; the default configuration equals the oracle."""
    from paper_2505_01231_amd import Plan
    say("tuning configurations", precision)
    z, x = _tuning_case(dev)
    with Plan(frame_len=1024, n_freq=200, m=12, window="acg", n_channels=2, precision=precision) as p:
        assert p.tuning == {"tile_group": 8, "s3_frame_batch": 0}
        base = _spectra(p.execute(x))
        torch.cuda.synchronize()
        ref = O.polyspectra(z, 1024, 200, 12, window_kind="acg", combos2=p.combos2, combos3=p.combos3,
                            combos4=p.combos4)
        for key in ("s2", "s3", "s4"):
            got = base[key][..., 0] + 1j * base[key][..., 1]
            assert rel_err(got, ref[key]) <= TOL, key
        for g in (1, 2, 4, 16):
            for fb in (10, 11, 16):
                p.set_tuning(g, fb)
                assert p.tuning == {"tile_group": g, "s3_frame_batch": fb}
                out = _spectra(p.execute(x))
                torch.cuda.synchronize()
                for key, b in base.items():
                    assert rel_err(out[key], b) <= 1e-12, (g, fb, key, rel_err(out[key], b))
        p.set_tuning(8, 0)


def test_autotune_keeps_the_fastest(dev):
    """ps_plan_autotune times all candidates, keeps the fastest in the plan and
    leaves the results unchanged up to FP64 addition order; bad values are
    rejected without changing the configuration."""
    from paper_2505_01231_amd import Plan
    from paper_2505_01231_amd._lib import PolyspecError
    say("autotune")
    z, x = _tuning_case(dev)
    with Plan(frame_len=1024, n_freq=200, m=12, window="acg", n_channels=2, precision="bf16x3") as p:
        base = _spectra(p.execute(x))
        rep = p.autotune(x, reps=2)
        torch.cuda.synchronize()
        cands = rep["candidates"]
        say("  candidates", [(c["tile_group"], c["s3_frame_batch"], round(ms, 3)) for c, ms in cands])
        assert len(cands) == 12                     # 4 tile orders x 3 S3 frame batches (m > 10)
        assert {(c["tile_group"], c["s3_frame_batch"]) for c, _ in cands} == \
            {(g, fb) for g in (1, 4, 8, 16) for fb in (0, 10, 16)}
        assert all(ms > 0 for _, ms in cands)
        fastest = min(cands, key=lambda c: c[1])[0]
        assert rep["best"] == fastest == p.tuning
        out = _spectra(p.execute(x))
        torch.cuda.synchronize()
        for key, b in base.items():
            assert rel_err(out[key], b) <= 1e-12, key
        kept = p.tuning
        for bad in ((3, 0), (8, 12), (0, 10)):
            with pytest.raises(PolyspecError):
                p.set_tuning(*bad)
            assert p.tuning == kept
        # a failing autotune (workspace too small: rejected on the host before
        # any launch) leaves the configuration as it was
        import ctypes as C
        from paper_2505_01231_amd import _lib as L
        p.set_tuning(1, 16)
        recs = (L.ps_record * 1)(p.record(x))
        small = torch.empty(256, dtype=torch.uint8, device=dev)
        o = p.allocate_outputs(dev)
        outs = (L.ps_output * 1)(L.ps_output(*[t.data_ptr() for t in (o.s2, o.s2_err, o.s3, o.s3_err, o.s4, o.s4_err)]))
        st = torch.cuda.current_stream(dev)
        rc = p._lib.ps_plan_autotune(p._handle, recs, 1, small.data_ptr(), small.numel(), outs, 1,
                                     C.c_void_p(st.cuda_stream), None)
        assert rc != 0
        assert p.tuning == {"tile_group": 1, "s3_frame_batch": 16}


def test_graph_follows_tuning_changes(dev):
    """A graph captured before ps_plan_set_tuning replays with the new tile order
    (the tables are rewritten in place; the captured S3 frame batch, which does
    not change the sums, stays) and matches an eager execute at that
    configuration bitwise."""
    from paper_2505_01231_amd import Plan
    say("graph after set_tuning")
    z, x = _tuning_case(dev)
    with Plan(frame_len=1024, n_freq=200, m=12, window="acg", n_channels=2, precision="bf16x3") as p:
        g = p.graph(x)
        for tg, fb in ((1, 10), (16, 16), (8, 0)):
            p.set_tuning(tg, fb)
            got = _spectra(g.launch())
            torch.cuda.synchronize()
            want = _spectra(p.execute(x))
            torch.cuda.synchronize()
            for key in got:
                assert np.array_equal(got[key], want[key], equal_nan=True), (tg, fb, key)
        g.close()


def test_plain_c_client(dev, tmp_path):
    """The ABI from C alone: paper_2505_01231_amd/ps_c_client (C99, gcc, device
    memory and stream from the HIP runtime, no PyTorch in its process) writes
    S2, S3, S4 and their error bars, which equal the oracle's."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = os.path.join(root, "paper_2505_01231_amd", "ps_c_client")
    assert os.path.exists(exe), "ps_c_client is missing: python -m paper_2505_01231_amd.build"
    N, Nf, m = 512, 100, 10
    z = synth.ar2_chi2(N * m * 5 + 17, seed=41, dtype=np.float32)
    inp, out = tmp_path / "z.f32", tmp_path / "s.f64"
    z.tofile(inp)
    ref = O.polyspectra(z, N, Nf, m, window_kind="acg")
    for precision in (0, 1):
        say("C client, precision", precision)
        r = subprocess.run([exe, str(inp), str(out), str(N), str(Nf), str(m), str(precision)],
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stderr
        d = np.fromfile(out, dtype=np.float64)
        assert int(d[0]) == ref["n_chunks"] == 5
        sizes = [2 * Nf, 2 * Nf, 2 * Nf * Nf, 2 * Nf * Nf, 2 * Nf * Nf, 2 * Nf * Nf]
        parts = np.split(d[1:], np.cumsum(sizes)[:-1])
        assert len(d) == 1 + sum(sizes)
        got = {"s2": parts[0].reshape(1, Nf, 2), "s2_err": parts[1].reshape(1, Nf, 2),
               "s3": parts[2].reshape(1, Nf, Nf, 2), "s3_err": parts[3].reshape(1, Nf, Nf, 2),
               "s4": parts[4].reshape(1, Nf, Nf, 2), "s4_err": parts[5].reshape(1, Nf, Nf, 2)}
        for key in ("s2", "s3", "s4"):
            got[key] = got[key][..., 0] + 1j * got[key][..., 1]
        compare(got, ref, label=f"c-client-{precision}")


# ---------------------------------------------------------------- streaming (quasi-polyspectra)
def test_streamer_time_resolved_windows(dev):
    """Consecutive windows of a host stream whose chi-square drive amplitude
    ramps from 0.5 to 2.0 (a non-stationary signal, Section 8), pushed from
    pinned memory through ps_streamer (copies overlap computation).  Every
    window equals ps_execute on the same samples bit for bit, two windows
    match the oracle, and the time-resolved spectra follow S_n ~ s^n."""
    from paper_2505_01231_amd import Plan, Streamer
    say("streamer windows")
    N, Nf, m, W, nwin = 2048, 128, 10, 1 << 19, 8
    total = W * nwin
    z = synth.modulated_ar2(total, seed=5, total=total, r=0.9)
    s_of_t = 0.5 + 1.5 * np.arange(total) / (total - 1)
    with Plan(frame_len=N, n_freq=Nf, m=m, window="acg", precision="bf16x3") as p:
        st = Streamer(p, W, dtype=torch.float32, depth=3)
        sets = [p.allocate_outputs(dev) for _ in range(3)]
        host = [torch.empty(W, dtype=torch.float32, pin_memory=True) for _ in range(3)]
        results = []
        slots = []
        for w in range(nwin):
            k = w % 3
            if w >= 3:
                st.wait(slots[w - 3])            # slot, host buffer and output set free again
                results[w - 3] = {key: getattr(sets[k], key).cpu().numpy() for key in ("s2", "s3", "s4")}
            host[k].copy_(torch.from_numpy(z[w * W:(w + 1) * W]))
            slots.append(st.push(host[k], sets[k]))
            results.append(None)
        for w in range(max(0, nwin - 3), nwin):
            st.wait(slots[w])
            results[w] = {key: getattr(sets[w % 3], key).cpu().numpy() for key in ("s2", "s3", "s4")}
        st.close()
        for w in range(nwin):
            ref = p.execute(torch.from_numpy(z[w * W:(w + 1) * W].copy()).to(dev))
            torch.cuda.synchronize()
            for key in ("s2", "s3", "s4"):
                assert np.array_equal(results[w][key], getattr(ref, key).cpu().numpy()), (w, key)
    for w in (0, nwin - 1):
        ref = O.polyspectra(z[w * W:(w + 1) * W], N, Nf, m, window_kind="acg")
        for key in ("s2", "s3", "s4"):
            got = results[w][key][..., 0] + 1j * results[w][key][..., 1]
            assert rel_err(got, ref[key]) <= TOL, (w, key)
    # time-resolved scaling with the window's drive amplitude
    s_w = np.array([s_of_t[w * W:(w + 1) * W].mean() for w in range(nwin)])
    for n, key, tol in ((2, "s2", 0.15), (3, "s3", 0.4), (4, "s4", 0.6)):
        amp = np.array([np.max(np.abs(results[w][key][0, ..., 0])) for w in range(nwin)])
        slope = np.polyfit(np.log(s_w), np.log(amp), 1)[0]
        say(f"  log-slope {key}: {slope:.2f} (expected {n})")
        assert abs(slope - n) < tol, (key, slope)


@pytest.mark.gpu
def test_streamer_multi_window_pushes(dev):
    """Several consecutive windows per push (ps_streamer_push_multi): groups of
    3, 2 and 3 windows through two staging slots.  Every window equals
    ps_execute over the same group of records bit for bit, and one window
    matches the oracle."""
    from paper_2505_01231_amd import Plan, Streamer
    say("streamer multi-window pushes")
    N, Nf, m, W = 2048, 128, 10, 1 << 18
    groups = [3, 2, 3]
    total = W * sum(groups)
    z = synth.modulated_ar2(total, seed=7, total=total, r=0.9)
    with Plan(frame_len=N, n_freq=Nf, m=m, window="acg", precision="bf16x3") as p:
        st = Streamer(p, W, dtype=torch.float32, depth=2, windows_per_push=3)
        with pytest.raises(ValueError):
            st.push(torch.empty(4 * W, dtype=torch.float32, pin_memory=True),
                    [p.allocate_outputs(dev) for _ in range(4)])
        results, w0 = [], 0
        for n in groups:
            host = torch.from_numpy(z[w0 * W:(w0 + n) * W].copy()).pin_memory()
            outs = [p.allocate_outputs(dev) for _ in range(n)]
            st.wait(st.push(host, outs))
            results.append([{k: getattr(o, k).cpu().numpy() for k in ("s2", "s3", "s4", "s4_err")} for o in outs])
            ref = p.execute([torch.from_numpy(z[(w0 + i) * W:(w0 + i + 1) * W].copy()).to(dev) for i in range(n)])
            torch.cuda.synchronize()
            for i in range(n):
                for k in ("s2", "s3", "s4", "s4_err"):
                    assert np.array_equal(results[-1][i][k], getattr(ref[i], k).cpu().numpy()), (w0 + i, k)
            w0 += n
        st.close()
    w = 6                                      # second window of the third group
    ref = O.polyspectra(z[w * W:(w + 1) * W], N, Nf, m, window_kind="acg")
    got = results[2][1]
    for key in ("s2", "s3", "s4"):
        g = got[key][..., 0] + 1j * got[key][..., 1]
        assert rel_err(g, ref[key]) <= TOL, key
