"""The direct transform kernels (frame lengths that are not a power of two,
k_window_dft and its two-stage form k_window_dft2) compiled from its own source for the CPU and run under
AddressSanitizer and UndefinedBehaviorSanitizer, with the launch shape and the
argument fields the library uses (test infrastructure; no GPU).

The code of ps_fft.hip up to the direct transform's launcher is taken verbatim
from the source file; a small header (tests/cpu_emulation/hip_shim.h) stands
in for the HIP runtime: each GPU thread of a block is a std::thread, LDS arrays
are arrays shared by the block's threads, the workgroup barrier is a
std::barrier.  Every buffer is allocated to its exact size, so any access
outside a buffer or an LDS array is reported.  The outputs are checked against
the windowed transform (Section 3, eq. a_k, +j sign) computed here with numpy."""
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2505_01231_amd", "csrc")
EMU = os.path.join(HERE, "cpu_emulation")

# (N, frames, dtype, misaligned, N1): frame counts and coefficient counts that
# leave partial frame and bin blocks, every input type, odd frame lengths; N1
# the library's factor for the two-stage form (0: one stage, as for a prime N)
INSTANCES = [(768, 12, 0, 0, 0), (1000, 5, 0, 1, 0), (1280, 33, 1, 0, 0), (1536, 12, 2, 0, 0), (1536, 12, 2, 1, 0),
             (999, 3, 1, 1, 0), (1536, 12, 2, 0, 32), (1536, 3, 2, 1, 32), (1000, 5, 0, 1, 25), (999, 3, 1, 0, 27),
             (8190, 2, 0, 0, 90), (6144, 2, 1, 0, 64), (1021, 2, 0, 0, 0)]


def library_factor(N):
    """The two-stage factor the library picks: the largest divisor of N not
    above its square root, if at least 8 (else 0, one stage)."""
    d = max(d for d in range(1, int(N ** 0.5) + 1) if N % d == 0)
    return d if d >= 8 else 0


def test_instances_use_the_library_factor():
    for N, _, _, _, n1 in INSTANCES:
        if n1:
            assert library_factor(N) == n1, N


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("dftemu")
    src = open(os.path.join(CSRC, "ps_fft.hip")).read()
    cut = re.search(r"\nhipError_t launch_dft\(", src)
    assert cut, "launcher marker not found in ps_fft.hip"
    body = src[:cut.start()] + "\n}  // namespace\n}  // namespace ps\n"
    (d / "ps_fft_extract.inc").write_text(body)
    exe = d / "dft_driver"
    cmd = ["g++", "-std=c++20", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-Wno-unknown-pragmas", "-Wno-unused-function", "-pthread",
           "-I", EMU, "-I", str(d), "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           os.path.join(EMU, "dft_driver.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def _reference(samples, g, N, K):
    frames = samples.reshape(-1, N) * g
    full = N * np.fft.ifft(frames, axis=-1)         # sum_i w_i exp(+2 pi j i k / N)
    return full[:, :K]


@pytest.mark.parametrize("N,frames,dtype,mis,n1", INSTANCES)
def test_direct_transform_kernel_in_bounds_and_correct(driver, tmp_path, N, frames, dtype, mis, n1):
    K = N // 2 + 1                      # the largest coefficient count (N_f = N/4 + 1 with S3)
    out = tmp_path / "out.f32"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(driver), str(N), str(frames), str(K), str(dtype), str(mis), str(n1), str(out)],
                       capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.returncode, r.stderr[-6000:])
    got = np.fromfile(out, dtype=np.float32).reshape(frames, K, 2)
    got = got[..., 0] + 1j * got[..., 1]
    raw = np.fromfile(str(out) + ".in", dtype=np.uint8)
    samples = raw[: frames * N * 8].view(np.float64)
    g = raw[frames * N * 8:].view(np.float32).astype(np.float64)
    ref = _reference(samples, g, N, K)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    assert err < 2e-7, err
