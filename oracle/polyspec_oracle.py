"""Plain FP64 CPU oracle of the unbiased polyspectrum estimator
(Sifft, Ghorbanietemad, Wagner, Haegele: "Correct Estimation of Higher-Order
Spectra", arXiv 2505.01231).

TEST INFRASTRUCTURE ONLY.  This package is the independent checker of the GPU
library: only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import it.  It shares no code, constants or tables with the GPU path
and never imports it; the GPU path never imports this package.

Everything here is deliberately slow and literal: numpy float64 /
complex128, the estimators written exactly as the paper prints them, no
blocking beyond splitting a loop over rows to bound memory.

Paper anchors (section / equation of the paper):

* Fourier coefficients: Section 3, eq. (a_k):
  a_k = (T/N) sum_{i=0}^{N-1} g_i z_i exp(+2 pi j i k / N), t0 = 0, T/N = dt.
  The +j sign follows the Fourier convention of Appendix A.
* Window: symmetric Hann, periodic Hann, or the approximate confined Gaussian
  window of Appendix B (sigma_t = 0.14 by default, Section 3).
* Spectra: S1 and S2 (end of Section 3), S3 and the two-dimensional S4 cut
  (Section 4), multichannel forms (Section 7):
    S1_a        = C1(a_0)                    / (dt sum g)     (C1 = mean)
    S2_ab(k)    = C2(a_k, b*_k)              / (dt sum g^2)
    S3_abc(k,l) = C3(a_k, b_l, c*_{k+l})     / (dt sum g^3)
    S4_abcd(k,l)= C4(a_k, b*_k, c_l, d*_l)   / (dt sum g^4)
  (N C / (T sum g^n) with T = N dt; g is real so g^2 g* = g^3 etc.)
* Cumulant estimators: the multivariate k-statistics of Section 4.1
  (eq. c2_estimator, c3_estimator, c4_estimator), evaluated over the m frames
  of one chunk; the factorized c4 of Appendix H as a cross-check.
* Averaging and error bars: Section 4.2.  The spectrum is the mean of the
  per-chunk estimates; Var = Np/(Np-1) (mean(x^2) - mean(x)^2) separately for
  the real and imaginary parts, sigma = sqrt(Var/Np).
* Alternative S3 estimator: c3^(opt) of the closing remark of Section 4.1
  (its reading is stated at c3opt3).
* Negative controls: the natural (plug-in) estimator of Section 6 (all
  m-dependent prefactors set to one) and the incomplete fourth cumulant of
  Section 4.3 (eq. C4pyHOSA).

Readings where the paper is silent or ambiguous (listed with reasons in the
design notes of the repository):
* i runs over 0..N-1 (the range printed just before the window definition has
  a typo).
* Frames are contiguous and non-overlapping; a chunk ("part" of the error
  estimate) is m consecutive frames; leftover frames and samples are dropped.
* The output grid is k, l in [0, N_f) (positive quadrant); S3 needs
  coefficients up to index 2 N_f - 2.
"""
from __future__ import annotations

import numpy as np

# --------------------------------------------------------------------------
# Window (Section 3 and Appendix B)
# --------------------------------------------------------------------------


def window(kind: str, N: int, param: float = 0.14, x=None) -> np.ndarray:
    """Window g_i, i = 0..N-1, in float64 (or the same formula at real
    positions ``x`` when given).

    'hann'          symmetric Hann sin^2(pi i / (N-1)), centred at (N-1)/2
    'hann_periodic' periodic Hann  sin^2(pi i / N)
    'acg'           approximate confined Gaussian, Appendix B:
                    g_k ~ G(k) - G(-1/2) [G(k+N) + G(k-N)] / [G(-1/2+N) + G(-1/2-N)]
                    with G(x) = exp(-(x - (N-1)/2)^2 / (4 N^2 sigma_t^2)).
    The overall scale of g does not matter: every S_n is invariant to g -> c g.
    """
    i = np.arange(N, dtype=np.float64) if x is None else np.asarray(x, dtype=np.float64)
    if kind == "hann":
        return np.sin(np.pi * i / (N - 1)) ** 2
    if kind == "hann_periodic":
        return np.sin(np.pi * i / N) ** 2
    if kind == "acg":
        s = float(param)

        def G(x):
            return np.exp(-((x - (N - 1) / 2.0) ** 2) / (4.0 * N * N * s * s))

        return G(i) - G(-0.5) * (G(i + N) + G(i - N)) / (G(-0.5 + N) + G(-0.5 - N))
    raise ValueError(f"unknown window {kind!r}")


# --------------------------------------------------------------------------
# Frames and Fourier coefficients (Section 3, eq. a_k)
# --------------------------------------------------------------------------


def chunk_count(n_samples: int, N: int, m: int) -> int:
    """Number of complete chunks (parts) Np = floor(floor(L / N) / m)."""
    return (int(n_samples) // N) // m


def chunk_frames(z: np.ndarray, N: int, m: int) -> np.ndarray:
    """Contiguous frames grouped into chunks: [..., Np, m, N] float64 (complex128
    for a complex signal)."""
    z = np.asarray(z)
    L = z.shape[-1]
    Np = chunk_count(L, N, m)
    x = z[..., : Np * m * N].astype(np.complex128 if np.iscomplexobj(z) else np.float64)
    return x.reshape(z.shape[:-1] + (Np, m, N))


def coefficients(frames: np.ndarray, g: np.ndarray, dt: float, K: int, method: str = "fft") -> np.ndarray:
    """a_k = dt * sum_i g_i x_i exp(+2 pi j i k / N) for k = 0..K-1 (eq. a_k).

    method 'dft': the sum written out as a matrix product (small N only).
    method 'fft': numpy's inverse FFT carries the +j sign and a 1/N factor,
                  so the sum equals N * ifft(g x).
    Indices k >= N wrap around (the DFT is N-periodic).
    """
    N = g.shape[0]
    k = np.arange(K)
    if method == "dft":
        i = np.arange(N)
        E = np.exp(2j * np.pi * np.outer(i, k % N) / N)
        return dt * ((frames * g) @ E)
    full = N * dt * np.fft.ifft(frames * g, axis=-1)
    return full[..., k % N]


def coefficients_at(frames: np.ndarray, g: np.ndarray, dt: float, bins) -> np.ndarray:
    """a_k for an arbitrary list of integer bins (negative allowed, taken mod N),
    by the direct sum of eq. a_k written as a matrix product."""
    N = g.shape[0]
    bins = np.asarray(bins, dtype=np.int64) % N
    i = np.arange(N)
    E = np.exp(2j * np.pi * np.outer(i, bins) / N)
    return dt * ((frames * g) @ E)


# --------------------------------------------------------------------------
# Cumulant estimators (Section 4.1); samples along the last axis
# --------------------------------------------------------------------------


def _mean(v):
    return v.mean(axis=-1)


def kstat2(x, y):
    """eq. c2_estimator: m/(m-1) (mean(xy) - mean(x) mean(y))."""
    m = x.shape[-1]
    return m / (m - 1) * (_mean(x * y) - _mean(x) * _mean(y))


def kstat3(x, y, z):
    """eq. c3_estimator."""
    m = x.shape[-1]
    mx, my, mz = _mean(x), _mean(y), _mean(z)
    body = (_mean(x * y * z) - _mean(x * y) * mz - _mean(x * z) * my
            - _mean(y * z) * mx + 2.0 * mx * my * mz)
    return m * m / ((m - 1) * (m - 2)) * body


def kstat4(x, y, z, w):
    """eq. c4_estimator, raw-moment form as printed."""
    m = x.shape[-1]
    mx, my, mz, mw = _mean(x), _mean(y), _mean(z), _mean(w)
    mxy, mxz, mxw = _mean(x * y), _mean(x * z), _mean(x * w)
    myz, myw, mzw = _mean(y * z), _mean(y * w), _mean(z * w)
    body = ((m + 1) * _mean(x * y * z * w)
            - (m + 1) * (_mean(x * y * z) * mw + _mean(x * y * w) * mz
                         + _mean(x * z * w) * my + _mean(y * z * w) * mx)
            - (m - 1) * (mxy * mzw + mxz * myw + mxw * myz)
            + 2 * m * (mxy * mz * mw + mxz * my * mw + mxw * my * mz
                       + myz * mx * mw + myw * mx * mz + mzw * mx * my)
            - 6 * m * mx * my * mz * mw)
    return m * m / ((m - 1) * (m - 2) * (m - 3)) * body


def kstat4_factorized(x, y, z, w):
    """Appendix H, eq. factorizedC4: the same estimator in centred variables."""
    m = x.shape[-1]
    xc = x - _mean(x)[..., None]
    yc = y - _mean(y)[..., None]
    zc = z - _mean(z)[..., None]
    wc = w - _mean(w)[..., None]
    body = ((m + 1) * _mean(xc * yc * zc * wc)
            - (m - 1) * (_mean(xc * yc) * _mean(zc * wc) + _mean(xc * zc) * _mean(yc * wc)
                         + _mean(xc * wc) * _mean(yc * zc)))
    return m * m / ((m - 1) * (m - 2) * (m - 3)) * body


# Negative controls -------------------------------------------------------


def natural2(x, y):
    """Natural (plug-in) estimator of Section 6: c2 with its prefactor set to one."""
    return _mean(x * y) - _mean(x) * _mean(y)


def natural3(x, y, z):
    """Natural estimator: c3 with its prefactor set to one."""
    mx, my, mz = _mean(x), _mean(y), _mean(z)
    return (_mean(x * y * z) - _mean(x * y) * mz - _mean(x * z) * my
            - _mean(y * z) * mx + 2.0 * mx * my * mz)


def natural4(x, y, z, w):
    """Natural estimator: every m-dependent factor of c4 set to one, i.e. the
    moment expression of eq. C4 with sample means in place of expectations."""
    mx, my, mz, mw = _mean(x), _mean(y), _mean(z), _mean(w)
    mxy, mxz, mxw = _mean(x * y), _mean(x * z), _mean(x * w)
    myz, myw, mzw = _mean(y * z), _mean(y * w), _mean(z * w)
    return (_mean(x * y * z * w)
            - (_mean(x * y * z) * mw + _mean(x * y * w) * mz
               + _mean(x * z * w) * my + _mean(y * z * w) * mx)
            - (mxy * mzw + mxz * myw + mxw * myz)
            + 2 * (mxy * mz * mw + mxz * my * mw + mxw * my * mz
                   + myz * mx * mw + myw * mx * mz + mzw * mx * my)
            - 6 * mx * my * mz * mw)


def incomplete4(x, y, z, w):
    """Section 4.3, eq. C4pyHOSA: mean of the product of centred variables only."""
    xc = x - _mean(x)[..., None]
    yc = y - _mean(y)[..., None]
    zc = z - _mean(z)[..., None]
    wc = w - _mean(w)[..., None]
    return _mean(xc * yc * zc * wc)


# Alternative third-order estimator ------------------------------------------


def c3opt3(x, y, z):
    """Section 4.1, closing remark on estimators other than the k-statistics:
    c3^(opt), an estimator of C3 for variables of zero mean (Fourier
    coefficients away from frequency zero), written multilinearly.

    The univariate form given there is mean(x^3) - 3 (m-1)/(m+1) (x^2 x).
    Reading: (x^2 x) is the average of x_i^2 x_j over distinct samples
    i != j, the unbiased estimate of <x^2><x>, whose expectation is zero for
    zero-mean x.  The estimator is then unbiased for zero-mean data, and
    3 (m-1)/(m+1) is exactly the coefficient of minimum variance for Gaussian
    data among all mean(x^3) - beta (x^2 x).  For three variables each
    product term becomes its symmetrised form:
        c3opt = mean(xyz) - (m-1)/(m+1) [U(xy, z) + U(xz, y) + U(yz, x)],
        U(p, r) = average of p_i r_j over i != j.
    Unlike the k-statistic it is biased where a mean is not zero."""
    m = x.shape[-1]

    def U(p, r):
        return (np.sum(p, axis=-1) * np.sum(r, axis=-1) - np.sum(p * r, axis=-1)) / (m * (m - 1))

    return _mean(x * y * z) - (m - 1) / (m + 1) * (U(x * y, z) + U(x * z, y) + U(y * z, x))


ESTIMATORS = {
    "kstat": (kstat2, kstat3, kstat4),
    "factorized": (kstat2, kstat3, kstat4_factorized),
    "natural": (natural2, natural3, natural4),
    "incomplete": (natural2, natural3, incomplete4),
    # S3 by c3^(opt); S2 and S4 by the k-statistics
    "c3opt": (kstat2, c3opt3, kstat4),
}


# --------------------------------------------------------------------------
# Chunk average and error estimate (Section 4.2)
# --------------------------------------------------------------------------


def average_with_error(per_chunk: np.ndarray):
    """per_chunk: [Np, ...] complex.  Returns (mean, err[..., 2]) where
    err = (sigma_Re, sigma_Im), sigma = sqrt(Var / Np) and
    Var = Np/(Np-1) (mean(x^2) - mean(x)^2).  Np == 1 gives sigma = NaN,
    Np == 0 gives NaN everywhere."""
    Np = per_chunk.shape[0]
    shape = per_chunk.shape[1:]
    if Np == 0:
        nan = np.full(shape, np.nan)
        return nan + 1j * nan, np.full(shape + (2,), np.nan)
    mean = per_chunk.mean(axis=0)
    err = np.empty(shape + (2,))
    for j, part in enumerate((per_chunk.real, per_chunk.imag)):
        if Np == 1:
            err[..., j] = np.nan
            continue
        mu = part.mean(axis=0)
        var = Np / (Np - 1) * ((part ** 2).mean(axis=0) - mu ** 2)
        err[..., j] = np.sqrt(np.maximum(var, 0.0) / Np)
    return mean, err


# --------------------------------------------------------------------------
# Spectra on the positive-quadrant grid
# --------------------------------------------------------------------------


def _norm(g, dt, n):
    return dt * np.sum(g ** n)


def chunk_spectra(A: np.ndarray, Nf: int, combos2=(), combos3=(), combos4=(),
                  estimator: str = "kstat", row_block: int = 64):
    """Un-normalised cumulant estimates for ONE chunk.

    A: coefficients [C, K, m] (frames along the last axis), K >= 2 Nf - 1 when
    S3 is requested.  Returns lists (per combo) of
      c2[k]   = est2(a_k, b*_k)
      c3[k,l] = est3(a_k, b_l, c*_{k+l})
      c4[k,l] = est4(a_k, b*_k, c_l, d*_l)
    """
    e2, e3, e4 = ESTIMATORS[estimator]
    out2 = [e2(A[a, :Nf], np.conj(A[b, :Nf])) for (a, b) in combos2]
    out3, out4 = [], []
    ls = np.arange(Nf)
    for (a, b, c) in combos3:
        res = np.empty((Nf, Nf), dtype=np.complex128)
        for k0 in range(0, Nf, row_block):
            ks = np.arange(k0, min(Nf, k0 + row_block))
            x = A[a, ks][:, None, :]
            y = A[b, :Nf][None, :, :]
            z = np.conj(A[c][ks[:, None] + ls[None, :]])
            res[ks] = e3(x, y, z)
        out3.append(res)
    for (a, b, c, d) in combos4:
        res = np.empty((Nf, Nf), dtype=np.complex128)
        for k0 in range(0, Nf, row_block):
            ks = np.arange(k0, min(Nf, k0 + row_block))
            x = A[a, ks][:, None, :]
            y = np.conj(A[b, ks])[:, None, :]
            z = A[c, :Nf][None, :, :]
            w = np.conj(A[d, :Nf])[None, :, :]
            res[ks] = e4(x, y, z, w)
        out4.append(res)
    return out2, out3, out4


def polyspectra(z, N: int, Nf: int, m: int, dt: float = 1.0, window_kind: str = "acg",
                window_param: float = 0.14, orders=(2, 3, 4), combos2=None, combos3=None,
                combos4=None, estimator: str = "kstat", method: str = "fft",
                return_chunks: bool = False, g=None):
    """S1, S2, S3, S4 of a real record (single channel [L] or channels [C, L]).

    Default combos for one channel: (0,0), (0,0,0), (0,0,0,0).  S1 (order 1,
    one value per channel) is included when 1 is in `orders`.
    Returns a dict with 's1' [C] complex and 's1_err' [C, 2] (order 1 only),
    's2' [n2, Nf] complex, 's2_err' [n2, Nf, 2],
    's3'/'s4' [n, Nf, Nf] complex and their errors, 'n_chunks', and (if asked)
    the per-chunk normalised spectra under 'chunks2/3/4'.
    """
    z = np.asarray(z)
    if z.ndim == 1:
        z = z[None, :]
    C = z.shape[0]
    combos2 = [(0, 0)] if combos2 is None else [tuple(c) for c in combos2]
    combos3 = [(0, 0, 0)] if combos3 is None else [tuple(c) for c in combos3]
    combos4 = [(0, 0, 0, 0)] if combos4 is None else [tuple(c) for c in combos4]
    if 2 not in orders:
        combos2 = []
    if 3 not in orders:
        combos3 = []
    if 4 not in orders:
        combos4 = []
    for cb in combos2 + combos3 + combos4:
        if max(cb) >= C:
            raise ValueError("combo refers to a missing channel")
    g = window(window_kind, N, window_param) if g is None else np.asarray(g, dtype=np.float64)
    K = 2 * Nf - 1 if combos3 else Nf
    frames = chunk_frames(z, N, m)            # [C, Np, m, N]
    Np = frames.shape[1]
    n2, n3, n4 = _norm(g, dt, 2), _norm(g, dt, 3), _norm(g, dt, 4)
    per2 = np.empty((Np, len(combos2), Nf), dtype=np.complex128)
    per3 = np.empty((Np, len(combos3), Nf, Nf), dtype=np.complex128)
    per4 = np.empty((Np, len(combos4), Nf, Nf), dtype=np.complex128)
    per1 = np.empty((Np, C), dtype=np.complex128)
    n1 = _norm(g, dt, 1)
    for p in range(Np):
        A = coefficients(frames[:, p], g, dt, K, method)      # [C, m, K]
        # first-order k-statistic: the mean of a_0 over the chunk's frames
        per1[p] = A[:, :, 0].mean(axis=1) / n1
        A = np.swapaxes(A, -1, -2)                            # [C, K, m]
        c2, c3, c4 = chunk_spectra(A, Nf, combos2, combos3, combos4, estimator)
        for i, v in enumerate(c2):
            per2[p, i] = v / n2
        for i, v in enumerate(c3):
            per3[p, i] = v / n3
        for i, v in enumerate(c4):
            per4[p, i] = v / n4
    out = {"n_chunks": Np, "combos2": combos2, "combos3": combos3, "combos4": combos4}
    if 1 in orders:
        out["s1"], out["s1_err"] = average_with_error(per1)
    out["s2"], out["s2_err"] = average_with_error(per2)
    out["s3"], out["s3_err"] = average_with_error(per3)
    out["s4"], out["s4_err"] = average_with_error(per4)
    if return_chunks:
        out["chunks2"], out["chunks3"], out["chunks4"] = per2, per3, per4
        if 1 in orders:
            out["chunks1"] = per1
    return out


def polyspectra_complex(z, N: int, Nf: int, m: int, dt: float = 1.0, window_kind: str = "acg",
                        window_param: float = 0.14, orders=(2, 3, 4), combos2=None, combos3=None,
                        combos4=None, estimator: str = "kstat", return_chunks: bool = False,
                        s4_shift: int = 0):
    """Spectra of a complex-valued record on the signed grid k, l in
    (-N_f, N_f): without a_{-k} = conj(a_k) the negative frequencies carry their
    own information, so the same definitions (Sections 3, 4 and 7) are
    evaluated at every signed index.  Coefficients are eq. a_k at signed bins
    (numpy's inverse FFT, index taken mod N).  Returns the keys of polyspectra
    with grids of 2 N_f - 1 points per axis, index k + N_f - 1; 's1' (order 1)
    is complex.  The conjugated arguments are those of the real-signal
    formulas (a_k, b*_k; a_k, b_l, c*_{k+l}; a_k, b*_k, c_l, d*_l).

    s4_shift = q selects a plane of the three-dimensional fourth-order spectrum
    parallel to the cut (Appendix on the full S4: shifting the channels in
    frequency by q bins): S4[k, l] = C4(a_{k+q}, b*_{k-q}, c_{l-q}, d*_{l+q}).
    """
    z = np.asarray(z)
    if z.ndim == 1:
        z = z[None, :]
    C = z.shape[0]
    combos2 = [(0, 0)] if combos2 is None else [tuple(c) for c in combos2]
    combos3 = [(0, 0, 0)] if combos3 is None else [tuple(c) for c in combos3]
    combos4 = [(0, 0, 0, 0)] if combos4 is None else [tuple(c) for c in combos4]
    combos2 = combos2 if 2 in orders else []
    combos3 = combos3 if 3 in orders else []
    combos4 = combos4 if 4 in orders else []
    e2, e3, e4 = ESTIMATORS[estimator]
    g = window(window_kind, N, window_param)
    jmax = max(2 * (Nf - 1) if combos3 else Nf - 1, (Nf - 1 + abs(s4_shift)) if combos4 else 0)
    bins = np.arange(-jmax, jmax + 1)               # coefficient column c holds bin c - jmax
    frames = chunk_frames(z.astype(np.complex128), N, m)     # [C, Np, m, N]
    Np = frames.shape[1]
    E = 2 * Nf - 1
    ks = np.arange(E) - (Nf - 1)                    # signed grid
    per1 = np.empty((Np, C), dtype=np.complex128)
    per2 = np.empty((Np, len(combos2), E), dtype=np.complex128)
    per3 = np.empty((Np, len(combos3), E, E), dtype=np.complex128)
    per4 = np.empty((Np, len(combos4), E, E), dtype=np.complex128)
    col = ks + jmax                                 # column of bin k
    for p in range(Np):
        full = N * dt * np.fft.ifft(frames[:, p] * g, axis=-1)   # [C, m, N]
        A = np.swapaxes(full[..., bins % N], -1, -2)             # [C, columns, m]
        per1[p] = A[:, jmax, :].mean(axis=-1) / _norm(g, dt, 1)
        for i, (a, b) in enumerate(combos2):
            per2[p, i] = e2(A[a, col], np.conj(A[b, col])) / _norm(g, dt, 2)
        for i, (a, b, c) in enumerate(combos3):
            x = A[a, col][:, None, :]
            y = A[b, col][None, :, :]
            w = np.conj(A[c][col[:, None] + ks[None, :]])         # bin k + l
            per3[p, i] = e3(x, y, w) / _norm(g, dt, 3)
        q = s4_shift
        for i, (a, b, c, d) in enumerate(combos4):
            x = A[a, col + q][:, None, :]
            y = np.conj(A[b, col - q])[:, None, :]
            u = A[c, col - q][None, :, :]
            w = np.conj(A[d, col + q])[None, :, :]
            per4[p, i] = e4(x, y, u, w) / _norm(g, dt, 4)
    out = {"n_chunks": Np, "combos2": combos2, "combos3": combos3, "combos4": combos4}
    if 1 in orders:
        out["s1"], out["s1_err"] = average_with_error(per1)
    out["s2"], out["s2_err"] = average_with_error(per2)
    out["s3"], out["s3_err"] = average_with_error(per3)
    out["s4"], out["s4_err"] = average_with_error(per4)
    if return_chunks:
        out["chunks1"], out["chunks2"], out["chunks3"], out["chunks4"] = per1, per2, per3, per4
    return out


def trispectrum_at(z, N: int, m: int, points, dt: float = 1.0, window_kind: str = "acg",
                   window_param: float = 0.14, combo=(0, 0, 0, 0), estimator: str = "kstat"):
    """The full fourth-order spectrum at listed frequency triples (w1, w2, w3),
    as the general definition has it: C4(a_w1, a_w2, a_w3, a_w4) with
    w4 = -(w1 + w2 + w3), every component unconjugated, negative bins taken
    mod N (the Fourier components of the record at negative frequencies).
    Normalised by dt sum g^4 like the cut.  Returns (values [n], errors [n, 2]).
    """
    z = np.asarray(z)
    if z.ndim == 1:
        z = z[None, :]
    g = window(window_kind, N, window_param)
    e4 = ESTIMATORS[estimator][2]
    pts = [(int(a), int(b), int(c)) for a, b, c in points]
    bins = sorted({w for p in pts for w in p} | {-(a + b + c) for a, b, c in pts})
    colx = {b: i for i, b in enumerate(bins)}
    frames = chunk_frames(z, N, m)                          # [C, Np, m, N]
    C, Np = frames.shape[0], frames.shape[1]
    coef = np.stack([coefficients_at(frames[ch].reshape(Np * m, N), g, dt, bins) for ch in range(C)])
    coef = np.moveaxis(coef.reshape(C, Np, m, len(bins)), 2, -1)     # [C, Np, bins, m]
    ca, cb, cc, cd = combo
    per = np.stack([e4(coef[ca, :, colx[a]], coef[cb, :, colx[b]], coef[cc, :, colx[c]],
                       coef[cd, :, colx[-(a + b + c)]]) for a, b, c in pts], axis=1) / _norm(g, dt, 4)
    return average_with_error(per)


def polyspectra_interlaced(z, N: int, Nf: int, m: int, **kw):
    """Interlaced windows (Section 3): the window weighs the middle of each
    frame more than its edges, and frames shifted by half a window (T/2, i.e.
    N/2 samples) weigh the other parts; the interlaced result is the average of
    the spectra of both frame sets.

    Each set is estimated on its own: the frames of record z, and the frames of
    z without its first N/2 samples, each cut into its own chunks.  The paper
    gives no error estimate for the average; the reading adopted is the average
    of the two sets' error bars (the sets overlap, their estimates are
    positively correlated, and sd(X + Y) <= sd(X) + sd(Y) makes this never an
    underestimate).  If the shifted set has no complete chunk the first set's
    result is returned alone.  Keyword arguments are those of polyspectra
    (of polyspectra_complex for a complex record).
    Adds 'n_chunks_shifted' to the result.
    """
    z = np.asarray(z)
    spectra = polyspectra_complex if np.iscomplexobj(z) else polyspectra
    first = spectra(z, N, Nf, m, **kw)
    shifted_z = z[..., N // 2:]
    if chunk_count(shifted_z.shape[-1], N, m) == 0:
        out = dict(first)
        out["n_chunks_shifted"] = 0
        return out
    second = spectra(shifted_z, N, Nf, m, **kw)
    out = dict(first)
    for key in ("s1", "s2", "s3", "s4", "s1_err", "s2_err", "s3_err", "s4_err"):
        if key in first:
            out[key] = 0.5 * (first[key] + second[key])
    out["n_chunks_shifted"] = second["n_chunks"]
    return out


def polyspectra_at(z, N: int, m: int, dt: float = 1.0, window_kind: str = "acg",
                   window_param: float = 0.14, points2=(), points3=(), points4=(),
                   combo2=(0, 0), combo3=(0, 0, 0), combo4=(0, 0, 0, 0),
                   estimator: str = "kstat", frame_block: int = 4096):
    """The same spectra evaluated at listed integer frequency indices only
    (negative indices allowed: a_{-k} is taken as a_{N-k}, the N-periodic DFT).
    Used for sampled checks at full record sizes and for full-plane symmetry
    checks.  Coefficients come from the direct sum of eq. a_k, restricted to the
    needed bins.  Returns dict with 's2' [n], 's3' [n], 's4' [n] complex and
    their errors [n, 2], plus 'n_chunks'.
    """
    z = np.asarray(z)
    if z.ndim == 1:
        z = z[None, :]
    g = window(window_kind, N, window_param)
    e2, e3, e4 = ESTIMATORS[estimator]
    points2 = [int(k) for k in points2]
    points3 = [(int(k), int(l)) for (k, l) in points3]
    points4 = [(int(k), int(l)) for (k, l) in points4]
    bins = sorted(set(points2) | {k for k, _ in points3} | {l for _, l in points3}
                  | {k + l for k, l in points3} | {k for k, _ in points4} | {l for _, l in points4})
    col = {b: i for i, b in enumerate(bins)}
    C = z.shape[0]
    Np = chunk_count(z.shape[-1], N, m)
    n_frames = Np * m
    coef = np.empty((C, n_frames, len(bins)), dtype=np.complex128)
    for c in range(C):
        for f0 in range(0, n_frames, frame_block):
            f1 = min(n_frames, f0 + frame_block)
            fr = z[c, f0 * N: f1 * N].astype(np.float64).reshape(f1 - f0, N)
            coef[c, f0:f1] = coefficients_at(fr, g, dt, bins)
    coef = coef.reshape(C, Np, m, len(bins))
    coef = np.moveaxis(coef, 2, -1)                          # [C, Np, bins, m]

    def a(ch, k):
        return coef[ch, :, col[k], :]

    def ac(ch, k):
        return np.conj(coef[ch, :, col[k], :])

    out = {"n_chunks": Np}
    ca, cb = combo2
    per2 = np.stack([e2(a(ca, k), ac(cb, k)) for k in points2], axis=1) / _norm(g, dt, 2) \
        if points2 else np.empty((Np, 0), complex)
    ca, cb, cc = combo3
    per3 = np.stack([e3(a(ca, k), a(cb, l), ac(cc, k + l)) for k, l in points3], axis=1) / _norm(g, dt, 3) \
        if points3 else np.empty((Np, 0), complex)
    ca, cb, cc, cd = combo4
    per4 = np.stack([e4(a(ca, k), ac(cb, k), a(cc, l), ac(cd, l)) for k, l in points4], axis=1) / _norm(g, dt, 4) \
        if points4 else np.empty((Np, 0), complex)
    out["s2"], out["s2_err"] = average_with_error(per2)
    out["s3"], out["s3_err"] = average_with_error(per3)
    out["s4"], out["s4_err"] = average_with_error(per4)
    return out
