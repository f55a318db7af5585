"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: exact
expectations by enumeration, an independent library routine, exact
finite-sample identities (Parseval), closed-form expectations of linear
processes, and the symmetry / invariance statements of the paper.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.signal
import scipy.stats

import oracle as O
from paper_2505_01231_amd import synth

# --------------------------------------------------------------------------
# 1. k-statistics: exact unbiasedness by enumeration (Section 4.1)
# --------------------------------------------------------------------------


def _set_partitions(items):
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for p in _set_partitions(rest):
        yield [[first]] + p
        for i in range(len(p)):
            yield p[:i] + [[first] + p[i]] + p[i + 1:]


def _joint_cumulant(values, probs, idx):
    """Joint cumulant from moments by the set-partition (Moebius) formula,
    independent of the moment expressions printed in the paper."""
    total = 0
    for part in _set_partitions(list(range(len(idx)))):
        b = len(part)
        term = (-1) ** (b - 1) * math.factorial(b - 1)
        for block in part:
            mom = 0
            for v, p in zip(values, probs):
                prod = 1
                for i in block:
                    prod *= v[idx[i]]
                mom += p * prod
            term *= mom
        total += term
    return total


def _expected_estimator(est, values, probs, idx, m):
    """E[est] over all m-tuples of i.i.d. draws of a discrete distribution."""
    n_out = len(values)
    tuples = np.array(list(itertools.product(range(n_out), repeat=m)))       # [T, m]
    p = np.prod(np.array([float(q) for q in probs])[tuples], axis=1)          # [T]
    vals = np.array(values, dtype=complex)                                    # [n_out, 4]
    args = [vals[tuples, j] for j in idx]                                     # each [T, m]
    return np.sum(p * est(*args))


REAL_VALUES = [(1, -2, 0, 3), (-1, 1, 2, -1), (2, 0, -3, 1)]
REAL_PROBS = [Fraction(1, 2), Fraction(1, 3), Fraction(1, 6)]
CPLX_VALUES = [(1 + 2j, -1j, 2, 1 - 1j), (-2 + 1j, 1 + 1j, -1j, 3), (1, 2 - 1j, 1 + 1j, -1 + 2j)]
CPLX_PROBS = [0.25, 0.45, 0.30]


@pytest.mark.parametrize("values,probs", [(REAL_VALUES, REAL_PROBS), (CPLX_VALUES, CPLX_PROBS)])
@pytest.mark.parametrize("order,idx,m", [
    (2, (0, 1), 2), (2, (0, 1), 3), (2, (2, 2), 4),
    (3, (0, 1, 2), 3), (3, (0, 1, 2), 4), (3, (1, 1, 3), 5),
    (4, (0, 1, 2, 3), 4), (4, (0, 1, 2, 3), 5), (4, (0, 0, 1, 1), 5), (4, (3, 2, 3, 0), 6),
])
def test_kstat_unbiased_by_enumeration(values, probs, order, idx, m):
    est = {2: O.kstat2, 3: O.kstat3, 4: O.kstat4}[order]
    got = _expected_estimator(est, values, probs, idx, m)
    want = complex(_joint_cumulant(values, probs, idx))
    assert abs(got - want) <= 1e-11 * max(1.0, abs(want)), (got, want)
    # the factorized form (Appendix H) has the same expectation
    if order == 4:
        got_f = _expected_estimator(O.kstat4_factorized, values, probs, idx, m)
        assert abs(got_f - want) <= 1e-11 * max(1.0, abs(want))


def test_natural_estimator_is_biased():
    # the plug-in estimator misses the cumulant at finite m (Section 6)
    idx, m = (0, 1, 2, 3), 5
    want = complex(_joint_cumulant(REAL_VALUES, REAL_PROBS, idx))
    got = _expected_estimator(O.natural4, REAL_VALUES, REAL_PROBS, idx, m)
    assert abs(got - want) > 1e-2 * abs(want)
    got = _expected_estimator(O.incomplete4, REAL_VALUES, REAL_PROBS, idx, m)
    assert abs(got - want) > 1e-2 * abs(want)


def _empirical_cumulant(samples, idx):
    """Joint cumulant of the empirical distribution of m samples (each drawn
    with probability 1/m), by the set-partition formula: the plug-in value that
    the natural estimator of Section 6 is by construction."""
    m = len(samples)
    return _joint_cumulant(samples, [Fraction(1, m)] * m, idx)


@pytest.mark.parametrize("m", [4, 5, 9])
def test_natural_estimators_are_empirical_cumulants(m):
    """natural2/3/4 equal the joint cumulants of the sample's empirical
    distribution (computed without the paper's moment expressions), and
    incomplete4 its joint central fourth moment (computed by explicit loops)."""
    rng = np.random.default_rng(100 + m)
    xs = [tuple(int(v) for v in rng.integers(-4, 5, size=4)) for _ in range(m)]
    cols = [np.array([float(s[j]) for s in xs]) for j in range(4)]
    for est, idx in ((O.natural2, (0, 1)), (O.natural3, (0, 1, 2)), (O.natural3, (2, 2, 3)),
                     (O.natural4, (0, 1, 2, 3)), (O.natural4, (1, 1, 3, 3)), (O.natural4, (2, 2, 2, 2))):
        want = float(_empirical_cumulant(xs, idx))
        got = float(est(*[cols[j] for j in idx]))
        assert abs(got - want) <= 1e-12 * max(1.0, abs(want)), (est.__name__, idx, got, want)
    # incomplete fourth cumulant: the mean of the product of centred values
    means = [Fraction(sum(s[j] for s in xs), m) for j in range(4)]
    want = sum((s[0] - means[0]) * (s[1] - means[1]) * (s[2] - means[2]) * (s[3] - means[3]) for s in xs) / m
    got = float(O.incomplete4(*cols))
    assert abs(got - float(want)) <= 1e-12 * max(1.0, abs(float(want)))


@pytest.mark.parametrize("m", [5, 10, 37])
def test_univariate_natural_matches_scipy_moments(m):
    """Univariate plug-in cumulants from scipy's central moments m_n:
    natural2 = m_2, natural3 = m_3, natural4 = m_4 - 3 m_2^2, incomplete4 = m_4."""
    rng = np.random.default_rng(7 * m)
    x = rng.standard_normal(m) ** 3 + 0.4
    m2, m3, m4 = (scipy.stats.moment(x, n) for n in (2, 3, 4))
    assert np.isclose(O.natural2(x, x), m2, rtol=1e-12)
    assert np.isclose(O.natural3(x, x, x), m3, rtol=1e-11, atol=1e-13)
    assert np.isclose(O.natural4(x, x, x, x), m4 - 3 * m2 * m2, rtol=1e-11, atol=1e-13)
    assert np.isclose(O.incomplete4(x, x, x, x), m4, rtol=1e-12)


@pytest.mark.parametrize("m", [4, 5, 6])
def test_natural_and_incomplete_expectations_by_enumeration(m):
    """Exact expectations over all m-tuples against the textbook closed forms
    for i.i.d. samples (kappa: joint cumulants, mu: joint central moments):
      E natural2 = (m-1)/m kappa_xy,
      E natural3 = (m-1)(m-2)/m^2 kappa_xyz,
      E natural4 = (m-1)/m^3 [(m^2-6m+6) kappa_xyzw - 2m (kappa_xy kappa_zw + kappa_xz kappa_yw + kappa_xw kappa_yz)],
      E incomplete4 = (m-1)/m^3 [(m^2-3m+3) mu_xyzw + (2m-3)(mu_xy mu_zw + mu_xz mu_yw + mu_xw mu_yz)]."""
    vals, probs = REAL_VALUES, REAL_PROBS

    def kap(*idx):
        return float(_joint_cumulant(vals, probs, idx))

    def mu(*idx):
        mean = [sum(p * v[j] for v, p in zip(vals, probs)) for j in range(4)]
        tot = 0
        for v, p in zip(vals, probs):
            prod = p
            for j in idx:
                prod *= v[j] - mean[j]
            tot += prod
        return float(tot)

    x, y, z, w = 0, 1, 2, 3
    got = _expected_estimator(O.natural2, vals, probs, (x, y), m)
    assert np.isclose(got, (m - 1) / m * kap(x, y), rtol=1e-12)
    got = _expected_estimator(O.natural3, vals, probs, (x, y, z), m)
    assert np.isclose(got, (m - 1) * (m - 2) / m ** 2 * kap(x, y, z), rtol=1e-12)
    pairs_k = kap(x, y) * kap(z, w) + kap(x, z) * kap(y, w) + kap(x, w) * kap(y, z)
    want = (m - 1) / m ** 3 * ((m * m - 6 * m + 6) * kap(x, y, z, w) - 2 * m * pairs_k)
    got = _expected_estimator(O.natural4, vals, probs, (x, y, z, w), m)
    assert np.isclose(got, want, rtol=1e-12), (got, want)
    pairs_m = mu(x, y) * mu(z, w) + mu(x, z) * mu(y, w) + mu(x, w) * mu(y, z)
    want = (m - 1) / m ** 3 * ((m * m - 3 * m + 3) * mu(x, y, z, w) + (2 * m - 3) * pairs_m)
    got = _expected_estimator(O.incomplete4, vals, probs, (x, y, z, w), m)
    assert np.isclose(got, want, rtol=1e-12), (got, want)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_univariate_matches_scipy_kstat(n):
    rng = np.random.default_rng(11)
    for m in (5, 10, 37):
        x = rng.standard_normal(m) ** 3 + 0.3
        est = {2: O.kstat2, 3: O.kstat3, 4: O.kstat4}[n]
        got = est(*([x] * n))
        assert np.isclose(got, scipy.stats.kstat(x, n), rtol=1e-11, atol=1e-12)


def test_factorized_equals_raw_form():
    rng = np.random.default_rng(3)
    shape = (7, 5, 10)
    args = [rng.standard_normal(shape) + 1j * rng.standard_normal(shape) + 0.7 for _ in range(4)]
    a = O.kstat4(*args)
    b = O.kstat4_factorized(*args)
    assert np.max(np.abs(a - b)) <= 1e-10 * np.max(np.abs(a))


# --------------------------------------------------------------------------
# 2. Window and coefficients (Section 3, Appendix B)
# --------------------------------------------------------------------------


@pytest.mark.parametrize("N", [16, 255, 256, 4096])
def test_hann_windows_match_scipy(N):
    assert np.allclose(O.window("hann", N), scipy.signal.windows.hann(N, sym=True), atol=1e-15)
    assert np.allclose(O.window("hann_periodic", N), scipy.signal.windows.hann(N, sym=False), atol=1e-15)


@pytest.mark.parametrize("N", [64, 256, 8192])
def test_acg_window_confinement(N):
    g = O.window("acg", N, 0.14)
    # symmetric about (N-1)/2 and peaked in the middle
    assert np.allclose(g, g[::-1], rtol=1e-13, atol=1e-15)
    assert np.argmax(g) in ((N - 1) // 2, N // 2)
    # the approximate confined Gaussian vanishes half a sample outside both
    # edges (the defining property of the construction in Appendix B)
    edge = O.window("acg", N, 0.14, x=[-0.5, N - 0.5])
    assert np.all(np.abs(edge) <= 1e-14 * g.max())
    # a wider sigma_t gives a wider window
    assert O.window("acg", N, 0.3)[N // 8] / O.window("acg", N, 0.3).max() > g[N // 8] / g.max()


@pytest.mark.parametrize("N", [256, 4096])
def test_acg_rms_width_is_sigma_t(N):
    """sigma_t is the window's RMS temporal width in units of T = N (the RMS
    time-bandwidth measure the paper cites for the choice sigma_t = 0.14,
    Section 3): the energy-weighted spread of g about (N-1)/2,
    sqrt(sum (i - c)^2 g_i^2 / sum g_i^2).  Where the confinement terms of
    Appendix B are negligible (small sigma_t) it equals sigma_t N; at 0.14
    they narrow the window slightly.  A wrong width constant in G (2 N^2 or
    8 N^2 in place of 4 N^2) moves the ratio by a factor sqrt(2)."""
    i = np.arange(N)
    c = (N - 1) / 2

    def rms(s):
        g2 = O.window("acg", N, s) ** 2
        return np.sqrt(np.sum(g2 * (i - c) ** 2) / np.sum(g2))

    for s in (0.03, 0.05, 0.08):
        assert abs(rms(s) / (N * s) - 1) < 1e-5, s
    assert 0.97 < rms(0.14) / (N * 0.14) < 1.0


@pytest.mark.parametrize("N", [64, 96, 75, 77, 101])
def test_fft_and_direct_sum_agree(N):
    """eq. a_k by numpy's FFT equals the sum written out, at powers of two and
    at the frame lengths that are not (composite, odd, prime)."""
    rng = np.random.default_rng(5)
    K = N
    fr = rng.standard_normal((3, N))
    g = O.window("acg", N)
    a = O.coefficients(fr, g, 0.25, K, "fft")
    b = O.coefficients(fr, g, 0.25, K, "dft")
    assert np.allclose(a, b, rtol=0, atol=1e-12 * np.abs(b).max())
    # +j sign (Appendix A): sum_i sin(2 pi k0 i/N) exp(+2 pi j i k0/N) = +j N/2,
    # while the e^{-j} convention would give -j N/2
    i = np.arange(N)
    k0 = 5
    s = np.sin(2 * np.pi * k0 * i / N)
    a = O.coefficients(s[None], np.ones(N), 1.0, N, "dft")[0]
    assert np.isclose(a[k0], 1j * N / 2, atol=1e-9)
    assert np.isclose(a[N - k0], -1j * N / 2, atol=1e-9)


# --------------------------------------------------------------------------
# 3. Exact finite-sample identity: Parseval + the variance sum rule (Section 3)
# --------------------------------------------------------------------------


@pytest.mark.parametrize("window_kind,dt,m", [("hann", 1.0, 10), ("acg", 0.37, 4), ("hann_periodic", 2.0, 7)])
def test_s2_variance_sum_rule_per_chunk(window_kind, dt, m):
    """sum_{k=0}^{N-1} S2_k * 2 pi/(N dt) = 2 pi * (sum_i g_i^2 s_i^2)/(sum g^2),
    with s_i^2 the unbiased sample variance over the m frames at position i.
    This is exact per chunk (Parseval) and checks the dt power, the window
    normalisation and the m/(m-1) factor of c2; in expectation it is the
    variance sum rule int S2 dw = 2 pi sigma^2 of Section 3."""
    rng = np.random.default_rng(17)
    N = 32
    z = rng.standard_normal(N * m * 6) * 1.7 + 0.4
    out = O.polyspectra(z, N, N, m, dt=dt, window_kind=window_kind, orders=(2,), return_chunks=True)
    g = O.window(window_kind, N)
    fr = O.chunk_frames(z, N, m)
    for p in range(out["n_chunks"]):
        lhs = np.sum(out["chunks2"][p, 0]) * 2 * np.pi / (N * dt)
        s2 = np.var(fr[p], axis=0, ddof=1)
        rhs = 2 * np.pi * np.sum(g ** 2 * s2) / np.sum(g ** 2)
        assert np.isclose(lhs.real, rhs, rtol=1e-12)
        assert abs(lhs.imag) < 1e-12 * rhs


# --------------------------------------------------------------------------
# 4. Closed-form expectations for white noise (frames exactly i.i.d.)
# --------------------------------------------------------------------------


def _zscores(est, err, want, imag=True):
    """(estimate - expected) / sigma for the real parts and, when the spectrum
    is not real by construction (``imag``), the imaginary parts."""
    out = [(est.real - np.real(want)) / err[..., 0]]
    if imag:
        # points that are real by construction (e.g. S3 at k = l = 0, where a_0
        # is real) have a zero imaginary spread; leave them out
        e = err[..., 1]
        live = e > 1e-9 * err[..., 0]
        out.append(((est.imag - np.imag(want)) / np.where(live, e, 1.0))[live])
    return np.concatenate([o.ravel() for o in out])


def test_white_chi2_flat_spectra():
    """i.i.d. noise with cumulants kappa_n: E S_n = kappa_n dt^(n-1) at every grid
    point (the window normalisation makes this exact for any window)."""
    dt = 0.5
    N, Nf, m = 32, 8, 10
    rng = np.random.default_rng(21)
    w = rng.standard_normal(N * m * 2500)
    z = w * w - 1.0                                 # kappa2=2, kappa3=8, kappa4=48
    out = O.polyspectra(z, N, Nf, m, dt=dt, window_kind="acg")
    for n, key in ((2, "s2"), (3, "s3"), (4, "s4")):
        want = synth.CHI2_KAPPA[n] * dt ** (n - 1)
        zs = _zscores(out[key][0], out[key + "_err"][0], want, imag=(n == 3))
        assert np.mean(np.abs(zs) > 3.5) < 0.01, (key, np.sort(np.abs(zs))[-5:])
        assert abs(np.mean(zs)) < 0.5, (key, np.mean(zs))
        # the grid mean is close to the closed form
        assert abs(np.mean(out[key][0].real) / want - 1) < 0.05


@pytest.mark.parametrize("gen", ["white", "ar2"])
def test_gaussian_gives_zero_higher_orders(gen):
    """Gaussian input: S3 and S4 vanish within their error bars (Sections 4.3, 5)."""
    N, Nf, m = 64, 16, 10
    n = N * m * 400
    if gen == "white":
        z = synth.white_gaussian(n, seed=31)
    else:
        rng = np.random.default_rng(32)
        z = scipy.signal.lfilter([1.0], synth.ar2_coeffs(0.8, 0.3 * np.pi), rng.standard_normal(n))
    out = O.polyspectra(z, N, Nf, m, window_kind="hann")
    for key in ("s3", "s4"):
        zs = _zscores(out[key][0], out[key + "_err"][0], 0.0, imag=(key == "s3"))
        assert np.mean(np.abs(zs) > 3) < 0.02, (key, np.mean(np.abs(zs) > 3))
        assert abs(np.mean(zs)) < 0.35
    # the incomplete cumulant (Section 4.3) and the natural estimator (Section 6)
    # show a spurious trispectrum for the same Gaussian data
    for est in ("incomplete", "natural"):
        bad = O.polyspectra(z, N, Nf, m, window_kind="hann", orders=(4,), estimator=est)
        zs = _zscores(bad["s4"][0], bad["s4_err"][0], 0.0, imag=False)
        assert np.mean(np.abs(zs) > 3) > 0.3, est


def test_unbiased_at_small_m():
    """Exact unbiasedness at the smallest m (Section 4.1): over many i.i.d.
    chunks the mean estimate matches the closed form, while the natural and
    incomplete estimators miss it by many standard errors."""
    dt = 1.0
    N, Nf, m = 16, 4, 4
    rng = np.random.default_rng(41)
    w = rng.standard_normal(N * m * 40000)
    z = w * w - 1.0
    for est, ok in (("kstat", True), ("factorized", True), ("natural", False), ("incomplete", False)):
        out = O.polyspectra(z, N, Nf, m, dt=dt, window_kind="hann_periodic", orders=(4,), estimator=est)
        zs = _zscores(out["s4"][0], out["s4_err"][0], 48.0, imag=False)
        if ok:
            assert np.max(np.abs(zs)) < 4.5, (est, np.max(np.abs(zs)))
        else:
            assert np.max(np.abs(zs)) > 8, (est, np.max(np.abs(zs)))


# --------------------------------------------------------------------------
# 4b. c3^(opt), the alternative third-order estimator (closing remark of
#     Section 4.1)
# --------------------------------------------------------------------------


def test_c3opt_pair_averages_by_brute_force():
    """The closed form of the averages over distinct samples i != j against
    explicit loops, three complex variables and one real variable."""
    rng = np.random.default_rng(51)
    m = 5
    x, y, z = (rng.standard_normal(m) + 1j * rng.standard_normal(m) for _ in range(3))
    pairs = [(i, j) for i in range(m) for j in range(m) if i != j]
    u = sum(x[i] * y[i] * z[j] + x[i] * z[i] * y[j] + y[i] * z[i] * x[j] for i, j in pairs) / len(pairs)
    want = sum(x[i] * y[i] * z[i] for i in range(m)) / m - (m - 1) / (m + 1) * u
    assert abs(O.c3opt3(x, y, z) - want) < 1e-13 * abs(want)
    r = rng.standard_normal(m)
    u1 = sum(r[i] ** 2 * r[j] for i, j in pairs) / len(pairs)
    want1 = sum(v ** 3 for v in r) / m - 3 * (m - 1) / (m + 1) * u1
    assert abs(O.c3opt3(r, r, r) - want1) < 1e-13 * max(1.0, abs(want1))


def _zero_mean(values, probs):
    vals = np.array(values, dtype=complex)
    w = np.array([float(q) for q in probs])
    return [tuple(v) for v in vals - (w[:, None] * vals).sum(axis=0)]


@pytest.mark.parametrize("values,probs", [(REAL_VALUES, REAL_PROBS), (CPLX_VALUES, CPLX_PROBS)])
@pytest.mark.parametrize("idx,m", [((0, 1, 2), 2), ((0, 1, 2), 3), ((1, 1, 3), 4), ((2, 2, 2), 5)])
def test_c3opt_unbiased_for_zero_mean(values, probs, idx, m):
    """Exact expectation over every m-tuple: c3^(opt) equals C3 when every
    variable has mean zero, already at m = 2, and misses it when the means are
    left in (the k-statistic does not)."""
    zero = _zero_mean(values, probs)
    got = _expected_estimator(O.c3opt3, zero, probs, idx, m)
    want = complex(_joint_cumulant(zero, probs, idx))
    assert abs(got - want) <= 1e-11 * max(1.0, abs(want)), (got, want)
    biased = _expected_estimator(O.c3opt3, values, probs, idx, m)
    want_b = complex(_joint_cumulant(values, probs, idx))
    assert abs(biased - want_b) > 1e-3 * max(1.0, abs(want_b))


@pytest.mark.parametrize("m", [3, 5, 6])
def test_c3opt_coefficient_minimises_gaussian_variance(m):
    """Among the unbiased estimators mean(x^3) - beta (x^2 x) of a zero-mean
    variable, beta = 3(m-1)/(m+1) has the least variance for Gaussian x.
    Gaussian expectations are exact from the 4-node Gauss-Hermite rule (exact
    to degree 7 in each sample; these statistics reach degree 6)."""
    nodes, weights = np.polynomial.hermite_e.hermegauss(4)
    weights = weights / weights.sum()
    tup = np.array(list(itertools.product(range(4), repeat=m)))
    x = nodes[tup]                                            # [T, m]
    p = np.prod(weights[tup], axis=1)
    t1 = np.mean(x ** 3, axis=1)
    pairs = [(i, j) for i in range(m) for j in range(m) if i != j]
    u = sum(x[:, i] ** 2 * x[:, j] for i, j in pairs) / len(pairs)
    # Var(t1 - beta u) = a - 2 b beta + c beta^2 (t1 and u have mean zero)
    a, b, c = np.sum(p * t1 * t1), np.sum(p * t1 * u), np.sum(p * u * u)
    beta = b / c
    assert abs(beta - 3 * (m - 1) / (m + 1)) < 1e-12
    est = O.c3opt3(x, x, x)
    assert np.max(np.abs(est - (t1 - beta * u))) < 1e-12
    var_opt = np.sum(p * est ** 2)
    var_k3 = np.sum(p * O.kstat3(x, x, x) ** 2)
    # textbook normal-sample variances: Var k3 = 6m/((m-1)(m-2)), Var mean(x^3) = 15/m;
    # the minimum a - b^2/c works out to 6(m+4)/(m(m+1))
    assert abs(var_k3 - 6 * m / ((m - 1) * (m - 2))) < 1e-10
    assert abs(a - 15 / m) < 1e-10
    assert abs(var_opt - 6 * (m + 4) / (m * (m + 1))) < 1e-10
    assert var_opt < min(var_k3, a)
    if m >= 5:
        # the k-statistic beats the plain third moment for Gaussian data
        assert var_k3 < a


@pytest.mark.parametrize("m", [2, 3, 10])
def test_c3opt_spectrum_unbiased_for_white_chi2(m):
    """White chi-square(1) noise minus its mean: S3 = kappa_3 = 8 at every
    point (dt = 1), and every Fourier coefficient has mean zero, so c3^(opt)
    is unbiased on the whole grid, down to m = 2.  S2 and S4 stay the
    k-statistics (identical to the default estimator)."""
    N, Nf = 16, 4
    rng = np.random.default_rng(61 + m)
    w = rng.standard_normal(N * 24000)
    z = w * w - 1.0
    out = O.polyspectra(z, N, Nf, m, window_kind="hann_periodic", orders=(2, 3), estimator="c3opt")
    zs = _zscores(out["s3"][0], out["s3_err"][0], 8.0, imag=True)
    assert np.max(np.abs(zs)) < 4.5, np.max(np.abs(zs))
    if m >= 3:
        ref = O.polyspectra(z, N, Nf, m, window_kind="hann_periodic", orders=(2, 3))
        assert np.array_equal(out["s2"], ref["s2"])
        assert not np.allclose(out["s3"], ref["s3"])


def test_c3opt_biased_by_a_nonzero_mean():
    """With the noise's mean left in, a_0 and a_1 (window leakage of the
    periodic Hann window) have nonzero means: c3^(opt) is far off at (0, 0),
    still unbiased where k, l, k + l avoid bins 0 and 1, and the k-statistic
    is unbiased everywhere."""
    N, Nf, m = 16, 4, 10
    rng = np.random.default_rng(71)
    w = rng.standard_normal(N * 24000)
    z = w * w
    out = O.polyspectra(z, N, Nf, m, window_kind="hann_periodic", orders=(3,), estimator="c3opt")
    ref = O.polyspectra(z, N, Nf, m, window_kind="hann_periodic", orders=(3,))
    s, e = out["s3"][0], out["s3_err"][0]
    assert abs(s[0, 0].real - 8.0) / e[0, 0, 0] > 8
    far = np.ix_([2, 3], [2, 3])
    assert np.max(np.abs(_zscores(s[far], e[far], 8.0))) < 4.5
    assert np.max(np.abs(_zscores(ref["s3"][0], ref["s3_err"][0], 8.0))) < 4.5


# --------------------------------------------------------------------------
# 5. Linear process: exact finite-window expectations (multilinearity)
# --------------------------------------------------------------------------


def _beta(g, h, K):
    """beta_k(t) = sum_i g_i h_{i-t} exp(+2 pi j i k/N) for all drive times t
    that reach the frame (t from -(len(h)-1)... to N-1 relative to the frame)."""
    N = len(g)
    P = len(h)
    ts = np.arange(-(P - 1), N)
    i = np.arange(N)
    lag = i[None, :] - ts[:, None]                        # [T, N]
    H = np.where((lag >= 0) & (lag < P), h[np.clip(lag, 0, P - 1)], 0.0)
    E = np.exp(2j * np.pi * np.outer(i, np.arange(K)) / N)
    return (H * g[None, :]) @ E                            # [T, K]


@pytest.mark.slow
def test_ar2_chi2_matches_linear_process_expectations():
    """x = h * e with i.i.d. drive e: C_n of the coefficients follows from
    multilinearity, e.g. C3(a_k, a_l, a*_{k+l}) = kappa3 dt^3 sum_t b_k b_l b*_{k+l}.
    Frames of this short-memory process are nearly independent, so the
    unbiased estimates agree with these values within their error bars."""
    r, th = 0.8, 0.3 * np.pi
    N, Nf, m, dt = 128, 24, 10, 1.0          # grid reaches past the resonance at k ~ 19
    n = N * m * 4000
    rng = np.random.default_rng(51)
    e = rng.standard_normal(n + 2000) ** 2 - 1.0
    z = scipy.signal.lfilter([1.0], synth.ar2_coeffs(r, th), e)[2000:]
    out = O.polyspectra(z, N, Nf, m, dt=dt, window_kind="hann")
    g = O.window("hann", N)
    h = scipy.signal.lfilter([1.0], synth.ar2_coeffs(r, th), np.r_[1.0, np.zeros(299)])
    B = _beta(g, h, 2 * Nf - 1)
    k = np.arange(Nf)
    kap = synth.CHI2_KAPPA
    want2 = kap[2] * dt * np.sum(np.abs(B[:, :Nf]) ** 2, axis=0) / np.sum(g ** 2)
    want3 = kap[3] * dt ** 2 * np.einsum("tk,tl,tkl->kl", B[:, :Nf], B[:, :Nf],
                                         np.conj(B[:, k[:, None] + k[None, :]])) / np.sum(g ** 3)
    P = np.abs(B[:, :Nf]) ** 2
    want4 = kap[4] * dt ** 3 * (P.T @ P) / np.sum(g ** 4)
    for key, want in (("s2", want2), ("s3", want3), ("s4", want4)):
        zs = _zscores(out[key][0], out[key + "_err"][0], want, imag=(key == "s3"))
        assert np.max(np.abs(zs)) < 5.0, (key, np.max(np.abs(zs)))
        assert np.mean(np.abs(zs) > 3) < 0.02
        # and the estimate resolves the structure: strongly non-zero where expected
        assert np.max(np.abs(want) / out[key + "_err"][0][..., 0]) > 10


# --------------------------------------------------------------------------
# 6. Cross spectra: FT sign and time order (Section 7.1)
# --------------------------------------------------------------------------


def test_time_shifted_copy_cross_spectrum_phase():
    """z2(t) = z1(t + s dt) with white z1: S2_{z1 z2}(w_k) = sigma^2 dt
    exp(+j w_k s dt) (sum_i g_i g_{i+s}/sum g^2), the e^{+j w dt} of Section 7.1
    including the window-overlap factor of a finite frame."""
    N, Nf, m, s, dt = 64, 32, 10, 3, 0.5
    z1 = synth.white_gaussian(N * m * 800 + s, seed=61)
    z = np.stack([z1[:-s], z1[s:]])
    out = O.polyspectra(z, N, Nf, m, dt=dt, window_kind="hann", orders=(2,), combos2=[(0, 1)])
    g = O.window("hann", N)
    k = np.arange(Nf)
    want = dt * np.exp(2j * np.pi * k * s / N) * np.sum(g[:-s] * g[s:]) / np.sum(g ** 2)
    zs = _zscores(out["s2"][0], out["s2_err"][0], want)
    assert np.max(np.abs(zs)) < 4.5, np.max(np.abs(zs))
    # and the opposite sign is firmly rejected
    zs_wrong = _zscores(out["s2"][0], out["s2_err"][0], np.conj(want))
    assert np.max(np.abs(zs_wrong)) > 20


def test_derivative_cross_spectrum_sign():
    """v = dx/dt (central difference): S_vx = -j sin(w dt)/dt S_xx, so Im S_vx < 0
    at positive frequencies and Re S_vx ~ 0 (Section 7.1)."""
    N, Nf, m, dt = 128, 48, 10, 1.0
    rng = np.random.default_rng(71)
    x = scipy.signal.lfilter([1.0], synth.ar2_coeffs(0.9, 0.2 * np.pi), rng.standard_normal(N * m * 300 + 2002))[2000:]
    v = (x[2:] - x[:-2]) / (2 * dt)
    z = np.stack([v, x[1:-1]])
    out = O.polyspectra(z, N, Nf, m, dt=dt, window_kind="acg", orders=(2,), combos2=[(0, 1), (1, 1)])
    s_vx, s_xx = out["s2"][0], out["s2"][1].real
    w = 2 * np.pi * np.arange(Nf) / (N * dt)
    want = -1j * np.sin(w * dt) / dt * s_xx
    peak = np.argmax(s_xx)
    band = slice(max(1, peak - 3), peak + 4)
    assert np.all(s_vx[band].imag < 0)
    assert np.allclose(s_vx[band], want[band], rtol=0.1, atol=0.1 * np.abs(want[band]).max())


# --------------------------------------------------------------------------
# 7. Symmetries and isomorphisms (Section 9) -- exact identities of the estimator
# --------------------------------------------------------------------------


def _three_channels(n, seed):
    rng = np.random.default_rng(seed)
    e = rng.standard_normal((2, n + 500)) ** 2 - 1
    s1 = scipy.signal.lfilter([1.0], synth.ar2_coeffs(0.8, 0.3 * np.pi), e[0])[500:]
    s2 = scipy.signal.lfilter([1.0], synth.ar2_coeffs(0.7, 0.1 * np.pi), e[1])[500:]
    return np.stack([s1 + 0.5 * s2, s2 * s1 * 0.3 + rng.standard_normal(n), s2 - 0.2 * s1 ** 2])


def test_symmetries_and_channel_isomorphisms():
    N, Nf, m = 32, 8, 10
    z = _three_channels(N * m * 12, 81)
    kw = dict(window_kind="acg")
    c2 = [(0, 1), (1, 0), (2, 2)]
    c3 = [(0, 1, 2), (1, 0, 2), (2, 2, 2)]
    c4 = [(0, 1, 2, 0), (2, 0, 0, 1), (1, 0, 0, 2), (1, 1, 1, 1)]
    out = O.polyspectra(z, N, Nf, m, combos2=c2, combos3=c3, combos4=c4, **kw)
    tol = 1e-12
    s2, s3, s4 = out["s2"], out["s3"], out["s4"]
    # S2_xy = conj S2_yx; S2_zz real and non-negative (Section 9, second order)
    assert np.allclose(s2[0], np.conj(s2[1]), atol=tol * np.abs(s2[0]).max())
    assert np.all(np.abs(s2[2].imag) <= tol * np.abs(s2[2]).max()) and np.all(s2[2].real >= 0)
    # S3_xyz(k,l) = S3_yxz(l,k); single channel S3 symmetric
    assert np.allclose(s3[0], s3[1].T, atol=tol * np.abs(s3[0]).max())
    assert np.allclose(s3[2], s3[2].T, atol=tol * np.abs(s3[2]).max())
    # S4_abcd(k,l) = S4_cdab(l,k); S4_badc = conj S4_abcd; single channel real, symmetric
    assert np.allclose(s4[0], s4[1].T, atol=tol * np.abs(s4[0]).max())
    assert np.allclose(s4[2], np.conj(s4[0]), atol=tol * np.abs(s4[0]).max())
    assert np.all(np.abs(s4[3].imag) <= tol * np.abs(s4[3]).max())
    assert np.allclose(s4[3], s4[3].T, atol=tol * np.abs(s4[3]).max())
    # errors transform the same way
    assert np.allclose(out["s4_err"][0], out["s4_err"][1].transpose(1, 0, 2), rtol=1e-9)


def test_s3_isomorphism_with_negative_frequencies():
    """S3_yyx(w) = S3_xyy(M w), M = [[-1,-1],[1,0]] (Section 9)."""
    N, m = 32, 10
    z = _three_channels(N * m * 8, 82)[:2]
    pts = [(k, l) for k in range(0, 7) for l in range(0, 7)]
    mpts = [(-k - l, k) for (k, l) in pts]
    yyx = O.polyspectra_at(z, N, m, points3=pts, combo3=(1, 1, 0))
    xyy = O.polyspectra_at(z, N, m, points3=mpts, combo3=(0, 1, 1))
    assert np.allclose(yyx["s3"], xyy["s3"], rtol=0, atol=1e-12 * np.abs(yyx["s3"]).max())
    # the point evaluator agrees with the grid evaluator on the positive quadrant
    grid = O.polyspectra(z, N, 8, m, combos3=[(1, 1, 0)], orders=(3,))
    ks = np.array(pts)
    assert np.allclose(yyx["s3"], grid["s3"][0][ks[:, 0], ks[:, 1]], atol=1e-12 * np.abs(yyx["s3"]).max())


def test_duplicated_channels_reduce_to_single_channel():
    """a = b = c = d gives the single-channel spectra exactly (Section 7)."""
    N, Nf, m = 32, 8, 10
    x = synth.ar2_chi2(N * m * 6, seed=83, r=0.8, dtype=np.float64)
    single = O.polyspectra(x, N, Nf, m)
    dup = O.polyspectra(np.stack([x, x]), N, Nf, m, combos2=[(0, 1)], combos3=[(1, 0, 1)], combos4=[(0, 1, 1, 0)])
    for key in ("s2", "s3", "s4", "s2_err", "s3_err", "s4_err"):
        assert np.array_equal(single[key], dup[key]), key


# --------------------------------------------------------------------------
# 8. Invariances (Appendix C and the normalisation)
# --------------------------------------------------------------------------


def test_invariances():
    N, Nf, m, dt = 32, 8, 5, 1.0
    x = synth.ar2_chi2(N * m * 6, seed=91, r=0.8, dtype=np.float64)
    base = O.polyspectra(x, N, Nf, m, dt=dt, window_kind="hann")

    def close(a, b, scale=1.0):
        return np.allclose(a, b * scale, rtol=1e-9, atol=1e-11 * np.abs(b * scale).max())

    # time reversal of the whole record conjugates every spectrum (Appendix C,
    # symmetric window); error bars are unchanged
    rev = O.polyspectra(x[::-1].copy(), N, Nf, m, dt=dt, window_kind="hann")
    for key in ("s2", "s3", "s4"):
        assert close(rev[key], np.conj(base[key])), key
        assert np.allclose(rev[key + "_err"], base[key + "_err"], rtol=1e-8,
                           atol=1e-9 * np.max(base[key + "_err"])), key
    # a constant offset leaves all orders >= 2 unchanged (per-chunk centring)
    off = O.polyspectra(x + 3.25, N, Nf, m, dt=dt, window_kind="hann")
    for key in ("s2", "s3", "s4"):
        assert np.allclose(off[key], base[key], rtol=1e-8, atol=1e-9 * np.abs(base[key]).max()), key
    # z -> alpha z scales S_n by alpha^n; dt -> lam dt by lam^(n-1); g -> c g changes nothing
    alpha, lam = -1.7, 0.3
    sc = O.polyspectra(alpha * x, N, Nf, m, dt=dt, window_kind="hann")
    dd = O.polyspectra(x, N, Nf, m, dt=lam * dt, window_kind="hann")
    gg = O.polyspectra(x, N, Nf, m, dt=dt, g=2.5 * O.window("hann", N))
    for n, key in ((2, "s2"), (3, "s3"), (4, "s4")):
        assert close(sc[key], base[key], alpha ** n), key
        assert close(dd[key], base[key], lam ** (n - 1)), key
        assert close(gg[key], base[key]), key


# --------------------------------------------------------------------------
# 9. Error bars (Section 4.2)
# --------------------------------------------------------------------------


def test_error_bar_edge_cases():
    N, Nf, m = 16, 4, 4
    rng = np.random.default_rng(95)
    one = rng.standard_normal(N * m)
    rep = np.tile(one, 7)                      # 7 identical chunks -> sigma = 0
    out = O.polyspectra(rep, N, Nf, m)
    for key in ("s2", "s3", "s4"):
        assert np.all(out[key + "_err"] <= 1e-6 * np.abs(out[key]).max() + 1e-300)
    single = O.polyspectra(one, N, Nf, m)      # Np = 1 -> sigma is NaN, the mean is defined
    assert np.all(np.isnan(single["s4_err"])) and np.all(np.isfinite(single["s4"]))
    empty = O.polyspectra(one[:-1], N, Nf, m)  # no complete chunk -> NaN
    assert empty["n_chunks"] == 0 and np.all(np.isnan(empty["s2"]))


@pytest.mark.slow
def test_error_bar_matches_spread_over_independent_records():
    """sigma^2 = Var/Np is an unbiased estimate of the variance of the chunk
    average, so its mean over independent records matches the spread of the
    averages across those records (Section 4.2)."""
    N, Nf, m, Np = 32, 8, 10, 4         # small Np: the Np/(Np-1) factor is 4/3
    res = {k: ([], []) for k in ("s2", "s3", "s4")}
    for seed in range(800):
        w = np.random.default_rng(1000 + seed).standard_normal(N * m * Np)
        out = O.polyspectra(w, N, Nf, m)
        for k, (means, errs) in res.items():
            means.append(out[k][0].real)
            errs.append(out[k + "_err"][0][..., 0])
    for k, (means, errs) in res.items():
        spread2 = np.var(np.array(means), axis=0, ddof=1)
        ratio = np.mean(np.array(errs) ** 2, axis=0) / spread2
        assert 0.9 < np.median(ratio) < 1.1, (k, np.median(ratio))


# --------------------------------------------------------------------------
# Interlaced windows (Section 3)
# --------------------------------------------------------------------------


def test_interlaced_weights_the_shifted_half_window():
    """White noise present only in the first quarter of every N-sample period.
    The frames from sample 0 see it under the first quarter of the window, the
    frames shifted by N/2 under its third quarter.  Frames are independent, so
    E S2_k = kappa2 dt (sum of g^2 over the occupied samples) / sum g^2 at every
    k, and the interlaced average is kappa2 dt (A + B) / (2 sum g^2), A and B
    the sums of g^2 over the first and third quarters of a symmetric Hann
    window (taken from scipy).  A is small: a missing shift gives A, a shift by
    N/4 sees the fourth quarter (= A by symmetry), a sum instead of an average
    doubles the result."""
    N, Nf, m, Np, dt = 64, 17, 10, 150, 0.5
    L = N * m * Np + N                  # both frame sets hold Np chunks
    w = np.random.default_rng(97).standard_normal(L)
    z = np.where((np.arange(L) % N) < N // 4, w, 0.0)
    out = O.polyspectra_interlaced(z, N, Nf, m, dt=dt, window_kind="hann", orders=(2,))
    assert out["n_chunks"] == Np and out["n_chunks_shifted"] == Np
    g2 = scipy.signal.windows.hann(N, sym=True) ** 2
    A, B = g2[:N // 4].sum(), g2[N // 2:3 * N // 4].sum()
    expect = dt * (A + B) / (2 * g2.sum())
    got = out["s2"][0].real
    assert abs(got.mean() / expect - 1) < 0.05, (got.mean(), expect)
    # every bin within 5 of its own error bars
    assert np.all(np.abs(got - expect) < 5 * out["s2_err"][0][:, 0])
    assert A / (A + B) < 0.1            # the alternatives above are far away


def test_interlaced_without_shifted_chunk_is_the_first_set():
    """A record whose shifted frame set has no complete chunk: the first set's
    spectra alone (the shifted set starts N/2 samples later and so holds one
    frame fewer here)."""
    N, Nf, m = 32, 8, 5
    z = np.random.default_rng(98).standard_normal(N * m + N // 4)
    out = O.polyspectra_interlaced(z, N, Nf, m)
    ref = O.polyspectra(z, N, Nf, m)
    assert out["n_chunks"] == 1 and out["n_chunks_shifted"] == 0
    for key in ("s2", "s3", "s4"):
        assert np.array_equal(out[key], ref[key])


@pytest.mark.slow
def test_interlaced_error_bar_is_conservative():
    """The interlaced error bar (the mean of the two sets' sigmas) against the
    spread of the interlaced spectrum over independent white-noise records:
    the two sets overlap by half a window, so their estimates are positively
    correlated and the variance of their average lies between sigma^2 / 2
    (independent) and sigma^2 (identical).  The reported sigma^2 must not fall
    below the spread (ratio >= 0.9) and exceeds it by at most the factor 2 of
    independent sets (ratio <= 2.5 with sampling noise)."""
    N, Nf, m, Np = 32, 8, 6, 5
    res = {k: ([], []) for k in ("s2", "s3", "s4")}
    for seed in range(300):
        w = np.random.default_rng(3000 + seed).standard_normal(N * m * Np + N)
        out = O.polyspectra_interlaced(w, N, Nf, m, window_kind="hann")
        for k, (means, errs) in res.items():
            means.append(out[k][0].real)
            errs.append(out[k + "_err"][0][..., 0])
    for k, (means, errs) in res.items():
        spread2 = np.var(np.array(means), axis=0, ddof=1)
        ratio = np.median(np.mean(np.array(errs) ** 2, axis=0) / spread2)
        assert 0.9 < ratio < 2.5, (k, ratio)


# --------------------------------------------------------------------------
# Quasi-polyspectra (Section 8): dependence on m flags non-stationarity
# --------------------------------------------------------------------------


def _diag_kurtosis(out):
    """Mean over the band (S2 above a fifth of its peak) of S4(k, k) / S2(k)^2."""
    s2, s4 = out["s2"][0].real, out["s4"][0].real
    band = s2 > 0.2 * s2.max()
    return float((np.diag(s4)[band] / s2[band] ** 2).mean())


@pytest.mark.slow
def test_quasi_spectra_depend_on_m_only_when_nonstationary():
    """A Gaussian oscillator has zero trispectrum, for any m, when stationary.
    When its frequency drifts, a chunk of many frames sees the power of each
    bin rise and fall as the resonance passes, so the short-time estimates
    acquire positive fourth cumulants on the diagonal (the quasi-correlations
    of Section 8) that grow with m.  Measured by S4(k, k) / S2(k)^2 over the
    band: near 0 for the stationary record at m = 40 and 400, large for the
    drifting record at m = 400 and much smaller at m = 40."""
    N, Nf, L = 64, 25, 64 * 4000
    still = synth.drifting_ar2(L, seed=5, theta0=0.3 * np.pi, theta1=0.3 * np.pi)
    drift = synth.drifting_ar2(L, seed=5, theta0=0.1 * np.pi, theta1=0.7 * np.pi)
    q = {(name, m): _diag_kurtosis(O.polyspectra(z, N, Nf, m, orders=(2, 4)))
         for name, z in (("still", still), ("drift", drift)) for m in (40, 400)}
    assert abs(q["still", 40]) < 3 and abs(q["still", 400]) < 3, q
    assert q["drift", 400] > 30, q
    assert q["drift", 400] - q["drift", 40] > 25, q


# --------------------------------------------------------------------------
# First-order spectrum S1 (Section 3): the windowed mean
# --------------------------------------------------------------------------


@pytest.mark.parametrize("window_kind", ["hann", "acg"])
def test_s1_of_a_constant_is_the_constant(window_kind):
    """z = c gives a_0 = dt c sum g in every frame, so S1 = c exactly and its
    error bar is 0 (a wrong bin, normalisation or dt factor breaks this)."""
    N, Nf, m, c, dt = 32, 4, 5, -2.75, 0.5
    z = np.full(N * m * 4, c)
    out = O.polyspectra(z, N, Nf, m, dt=dt, window_kind=window_kind, orders=(1,))
    assert np.allclose(out["s1"], c, rtol=1e-13, atol=0)
    assert np.all(np.abs(out["s1_err"]) < 1e-12)


def test_s1_shift_and_scale():
    """S1 is linear: S1(alpha z + c) = alpha S1(z) + c per channel, while S2
    does not see the offset (per-chunk centring)."""
    N, Nf, m = 32, 6, 4
    rng = np.random.default_rng(99)
    z = rng.standard_normal((2, N * m * 6))
    a = O.polyspectra(z, N, Nf, m, orders=(1, 2))
    b = O.polyspectra(3.0 * z + np.array([[1.5], [-4.0]]), N, Nf, m, orders=(1, 2))
    assert np.allclose(b["s1"], 3.0 * a["s1"] + np.array([1.5, -4.0]), rtol=0, atol=1e-12)
    assert np.allclose(b["s1_err"], 3.0 * a["s1_err"], rtol=1e-10)
    assert np.allclose(b["s2"], 9.0 * a["s2"], rtol=1e-10)


def test_s1_of_white_noise_is_its_mean():
    """E S1 = mu for i.i.d. samples of mean mu (any window), within the
    estimator's own error bar."""
    N, Nf, m = 64, 4, 10
    z = 0.7 + np.random.default_rng(100).standard_normal(N * m * 200)
    out = O.polyspectra(z, N, Nf, m, orders=(1,))
    s1, e = out["s1"][0].real, out["s1_err"][0][0]
    assert abs(s1 - 0.7) < 4 * e and 0 < e < 0.01


# --------------------------------------------------------------------------
# Complex-valued signals: spectra on the signed grid
# --------------------------------------------------------------------------


def test_complex_path_on_a_real_signal_is_the_full_plane():
    """A real record given as complex: the signed-grid spectra equal the
    point evaluator's values at negative frequencies (which uses no grid)."""
    N, Nf, m = 32, 5, 6
    z = synth.ar2_chi2(N * m * 12, seed=141, r=0.8, dtype=np.float64)
    out = O.polyspectra_complex(z.astype(np.complex128), N, Nf, m, orders=(1, 2, 3, 4))
    ks = list(range(-Nf + 1, Nf))
    pts = [(k, l) for k in ks for l in ks]
    ref = O.polyspectra_at(z, N, m, points2=ks, points3=pts, points4=pts)
    for key in ("s2", "s3", "s4"):
        got = out[key][0].ravel()
        assert np.allclose(got, ref[key], rtol=0, atol=1e-12 * np.abs(ref[key]).max()), key
    assert np.allclose(out["s1"][0], O.polyspectra(z, N, Nf, m, orders=(1,))["s1"][0], atol=1e-12)


def test_complex_frequency_shift():
    """z = x exp(+2 pi j q n / N) shifts every coefficient, a_k(z) = a_{k+q}(x),
    so S2_z(k) = S2_x(k + q) and S4_z(k, l) = S4_x(k + q, l + q) exactly."""
    N, Nf, m, q = 32, 5, 6, 3
    x = synth.ar2_chi2(N * m * 10, seed=142, r=0.8, dtype=np.float64)
    z = x * np.exp(2j * np.pi * q * np.arange(len(x)) / N)
    out = O.polyspectra_complex(z, N, Nf, m, orders=(2, 4))
    ks = list(range(-Nf + 1, Nf))
    pts = [(k + q, l + q) for k in ks for l in ks]
    ref = O.polyspectra_at(x, N, m, points2=[k + q for k in ks], points4=pts)
    assert np.allclose(out["s2"][0], ref["s2"], rtol=0, atol=1e-12 * np.abs(ref["s2"]).max())
    assert np.allclose(out["s4"][0].ravel(), ref["s4"], rtol=0, atol=1e-12 * np.abs(ref["s4"]).max())


def test_complex_white_noise():
    """Circular complex Gaussian white noise, E|z|^2 = 2: S2 = 2 dt at every
    signed frequency (not symmetric by construction, flat by statistics);
    S3 and S4 consistent with zero."""
    N, Nf, m, dt = 32, 6, 8, 0.5
    rng = np.random.default_rng(143)
    z = rng.standard_normal(N * m * 300) + 1j * rng.standard_normal(N * m * 300)
    out = O.polyspectra_complex(z, N, Nf, m, dt=dt, window_kind="hann")
    s2, e2 = out["s2"][0], out["s2_err"][0]
    assert np.all(np.abs(s2.real - 2 * dt) < 5 * e2[:, 0])
    for key in ("s3", "s4"):
        t = np.abs(out[key][0].real) / out[key + "_err"][0][..., 0]
        assert np.mean(t > 3) < 0.02, (key, np.mean(t > 3))


def test_s4_planes_by_frequency_shifted_signals():
    """The Appendix's own construction of a plane parallel to the cut: the
    signals x = z1 e^{+j dw t}, y = z2 e^{-j dw t}, z = z3 e^{-j dw t},
    w = z4 e^{+j dw t} (dw = 2 pi q / T, i.e. e^{2 pi j q n / N} at sample n)
    put through the q = 0 cut of the complex-signal estimator give the plane
    of the original channels shifted by q bins."""
    N, Nf, m = 32, 5, 6
    s = synth.ar2_chi2(N * m * 9 + 5, seed=171, r=0.85, dtype=np.float64)
    z = np.stack([s[:-5], s[5:] ** 2 - 1.0, s[2:-3] * s[:-5]])
    n = np.arange(z.shape[1])
    for q, (a, b, c, d) in ((2, (0, 0, 0, 0)), (-3, (0, 1, 2, 0)), (4, (2, 1, 1, 0)), (1, (1, 2, 0, 2))):
        up = np.exp(2j * np.pi * q * n / N)
        shifted = np.stack([z[a] * up, z[b] / up, z[c] / up, z[d] * up])
        cut = O.polyspectra_complex(shifted, N, Nf, m, orders=(4,), combos4=[(0, 1, 2, 3)], s4_shift=0)
        plane = O.polyspectra_complex(z.astype(np.complex128), N, Nf, m, orders=(4,), combos4=[(a, b, c, d)],
                                      s4_shift=q)
        scale = np.abs(plane["s4"][0]).max()
        assert np.allclose(cut["s4"][0], plane["s4"][0], rtol=0, atol=1e-11 * scale), (q, (a, b, c, d))
        assert np.allclose(cut["s4_err"][0], plane["s4_err"][0], rtol=0,
                           atol=1e-11 * plane["s4_err"][0].max()), (q, (a, b, c, d))


def test_s4_planes_are_planes_of_the_three_dimensional_spectrum():
    """The plane shifted by q bins equals the full fourth-order spectrum at
    (k + q, -k + q, l - q) (Appendix on the full S4), evaluated directly with
    unconjugated components at negative frequencies; q = 0 is the cut."""
    N, Nf, m = 32, 5, 6
    s = synth.ar2_chi2(N * m * 10 + 3, seed=161, r=0.8, dtype=np.float64)
    z = np.stack([s[:-3], s[3:] ** 2 - 1.0])
    ks = range(-Nf + 1, Nf)
    for q, combo in ((2, (0, 0, 0, 0)), (-3, (0, 1, 1, 0)), (0, (1, 0, 0, 1))):
        out = O.polyspectra_complex(z.astype(np.complex128), N, Nf, m, orders=(4,), combos4=[combo], s4_shift=q)
        pts = [(k + q, -k + q, l - q) for k in ks for l in ks]
        ref, ref_err = O.trispectrum_at(z, N, m, pts, combo=combo)
        got = out["s4"][0].ravel()
        assert np.allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max()), (q, combo)
        assert np.allclose(out["s4_err"][0].reshape(-1, 2), ref_err, rtol=0, atol=1e-12 * ref_err.max()), (q, combo)
