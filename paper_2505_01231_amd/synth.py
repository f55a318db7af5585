"""Seeded synthetic input signals.

This module draws the test and benchmark signals and nothing else: it holds
none of the estimator's arithmetic, so the CPU oracle and the GPU path can both
be fed from it without sharing any part of the method.

Signals (all real valued, numpy PCG64 via ``default_rng(seed)``):

* ``white_gaussian``  -- i.i.d. N(0, sigma^2).
* ``ar2_chi2``        -- x_n = 2 r cos(theta) x_{n-1} - r^2 x_{n-2} + e_n with
  e_n = w_n^2 - 1, w ~ N(0,1) (a centred chi-square(1) drive, so the drive
  cumulants are kappa2 = 2, kappa3 = 8, kappa4 = 48).  It is the discrete
  analogue of the paper's damped, stochastically driven oscillator (Section 5),
  and the chi-square drive makes the bispectrum and trispectrum non-zero.
* ``mixed_channels``  -- several channels formed by a random mixing matrix of
  two latent AR(2)/chi-square sources plus independent Gaussian noise, then
  quantised to int16 (the multichannel setting of Section 7).
* ``modulated_ar2``   -- an AR(2)/chi-square process whose drive amplitude
  ramps linearly in time: a non-stationary signal for quasi-polyspectra
  (Section 8).
* ``drifting_ar2``    -- a Gaussian-driven AR(2) whose resonance angle moves
  linearly from theta0 to theta1 over the record (Section 8's oscillator with a
  drifting frequency); theta0 == theta1 gives the stationary process.
"""
from __future__ import annotations

import numpy as np
from scipy.signal import lfilter

# Drive cumulants of e = w^2 - 1 with w ~ N(0,1).
CHI2_KAPPA = {2: 2.0, 3: 8.0, 4: 48.0}


def white_gaussian(n: int, seed: int, sigma: float = 1.0, dtype=np.float64) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (sigma * rng.standard_normal(n)).astype(dtype)


def chi2_drive(n: int, rng: np.random.Generator) -> np.ndarray:
    w = rng.standard_normal(n)
    w *= w
    w -= 1.0
    return w


def ar2_coeffs(r: float, theta: float):
    """Denominator of the AR(2) recursion (numerator is 1)."""
    return np.array([1.0, -2.0 * r * np.cos(theta), r * r])


def ar2_chi2(n: int, seed: int, r: float = 0.95, theta: float = 0.3 * np.pi,
             burn: int = 10_000, dtype=np.float32) -> np.ndarray:
    """AR(2) with poles r e^{+-j theta}, driven by centred chi-square(1) noise.

    Generated in float64 with ``burn`` discarded start-up samples, then cast.
    """
    rng = np.random.default_rng(seed)
    e = chi2_drive(n + burn, rng)
    x = lfilter([1.0], ar2_coeffs(r, theta), e)
    return x[burn:].astype(dtype)


def mixed_channels(n: int, seed: int, n_channels: int = 4, thetas=(0.3 * np.pi, 0.12 * np.pi),
                   r: float = 0.95, lsb_std: float = 1024.0, burn: int = 10_000):
    """Channels = M @ [s1, s2] + noise at 0 dB SNR, scaled to ``lsb_std`` LSB and
    rounded/clipped to int16.  Returns (int16 array [C, n], number of clipped samples).
    """
    rng = np.random.default_rng(seed)
    src = []
    for th in thetas:
        e = chi2_drive(n + burn, rng)
        src.append(lfilter([1.0], ar2_coeffs(r, th), e)[burn:])
    src = np.stack(src)                                   # [2, n]
    mix = rng.standard_normal((n_channels, len(thetas)))  # [C, 2]
    sig = mix @ src                                       # [C, n]
    out = np.empty((n_channels, n), dtype=np.int16)
    clipped = 0
    for c in range(n_channels):
        p = np.sqrt(np.mean(sig[c] ** 2))
        ch = sig[c] + p * rng.standard_normal(n)          # equal noise power: 0 dB
        ch *= lsb_std / np.std(ch)
        ch = np.rint(ch)
        clipped += int(np.count_nonzero((ch > 32767) | (ch < -32768)))
        out[c] = np.clip(ch, -32768, 32767).astype(np.int16)
    return out, clipped


def uneven_record_lengths(n_records: int, seed: int, lo_log2: float = 16.0, hi_log2: float = 22.0):
    """Record lengths floor(2^(lo + (hi - lo) u)) with u ~ U(0, 1)."""
    rng = np.random.default_rng(seed)
    u = rng.random(n_records)
    return np.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)


def modulated_ar2(n: int, seed: int, start: int = 0, total: int | None = None,
                  s0: float = 0.5, s1: float = 2.0, r: float = 0.95,
                  theta: float = 0.3 * np.pi, burn: int = 10_000, dtype=np.float32) -> np.ndarray:
    """AR(2)/chi-square whose drive scale ramps linearly from s0 to s1 over
    ``total`` samples; returns samples [start, start + n) of that stream.
    (The drive of the block is drawn from ``seed`` and ``start`` so blocks are
    reproducible on their own; the filter is restarted with a burn-in.)"""
    total = n if total is None else total
    rng = np.random.default_rng([seed, start])
    e = chi2_drive(n + burn, rng)
    t = (np.arange(start - burn, start + n, dtype=np.float64)).clip(0, None)
    e *= s0 + (s1 - s0) * t / max(total - 1, 1)
    x = lfilter([1.0], ar2_coeffs(r, theta), e)
    return x[burn:].astype(dtype)


def drifting_ar2(n: int, seed: int, theta0: float, theta1: float, r: float = 0.98,
                 burn: int = 2000, dtype=np.float64) -> np.ndarray:
    """x_n = 2 r cos(theta_n) x_{n-1} - r^2 x_{n-2} + w_n, w ~ N(0, 1), with
    theta_n moving linearly from theta0 (at the first kept sample) to theta1
    (at the last); ``burn`` start-up samples at theta0 are discarded."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(n + burn)
    theta = np.concatenate([np.full(burn, theta0), np.linspace(theta0, theta1, n)])
    c1, c2 = 2.0 * r * np.cos(theta), r * r
    x = np.zeros(n + burn)
    for i in range(2, n + burn):
        x[i] = c1[i] * x[i - 1] - c2 * x[i - 2] + w[i]
    return x[burn:].astype(dtype)
