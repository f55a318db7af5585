// Stage a1: windowed real FFT of every frame (Section 3, eq. a_k), and the
// per-chunk centring a' = a - mean_f a that the k-statistics of Section 4.1
// need in their centred form (Appendix H).
//
//   a_k = sum_{i<N} g_i z_i exp(+2 pi j i k / N),  k < K        (dt folded into the output scale)
//
// The N real samples of a frame are packed as M = N/2 complex points
// x_n = w_{2n} + j w_{2n+1} (w = g z), transformed by a Stockham FFT with the
// +j sign, and unpacked: with X the M-point transform,
//   E_k = (X_k + conj X_{M-k}) / 2,  O_k = (X_k - conj X_{M-k}) / (2j),
//   a_k = E_k + exp(+2 pi j k / N) O_k   (indices of X taken mod M).
// T = M/16 threads per frame each hold 16 points in registers; the passes are
// radix 16 (one radix-2/4/8 pass when log2 M is not a multiple of 4), so a
// 4096-point transform takes three passes through LDS.  The first pass reads
// the windowed samples from global memory straight into registers.  LDS holds
// X with one padding entry per 16 (index i at i + i/16), which keeps the
// first pass's 16-strided writes free of bank conflicts.  A 256-thread block
// transforms 256/T frames.  Twiddles come from tables computed in FP64 on the
// host: exp(+2 pi j t / N) for the unpack, and one table per later pass laid
// out [r][k], so that the twiddles of consecutive threads are consecutive
// entries (a gather from the plain table touches up to one cache line per
// lane).  The stage streams N samples in and K complex values out per frame.
// A complex-valued signal (complex float32 / float64 samples) needs no packing:
// its frames of M samples are windowed and transformed as they are (the same
// passes, instantiated for twice the frame length), and column c of the output
// holds X at bin c - jmax, taken mod M.
#include "ps_internal.h"

namespace ps {
namespace {

constexpr int kFftThreads = 256;
constexpr int kFftLds = kFftThreads * 17;      // float2 entries: 4096 points + padding per block

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 mulj(float2 a) { return make_float2(-a.y, a.x); }   // j a
__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

// 4-point DFT with the +j sign on v[o], v[o+S], v[o+2S], v[o+3S], in place, natural order.
template <int S>
__device__ __forceinline__ void dft4(float2* v, int o) {
    const float2 a = v[o], b = v[o + S], c = v[o + 2 * S], d = v[o + 3 * S];
    const float2 s02 = cadd(a, c), d02 = csub(a, c), s13 = cadd(b, d), d13 = csub(b, d);
    v[o] = cadd(s02, s13);
    v[o + S] = cadd(d02, mulj(d13));
    v[o + 2 * S] = csub(s02, s13);
    v[o + 3 * S] = csub(d02, mulj(d13));
}
template <int S>
__device__ __forceinline__ void dft2(float2* v, int o) {
    const float2 a = v[o], b = v[o + S];
    v[o] = cadd(a, b);
    v[o + S] = csub(a, b);
}

// exp(+2 pi j q s / 16) for q, s < 4
__device__ __forceinline__ float2 w16(int qs) {
    constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508978f, h = 0.70710678118654752f;
    switch (qs) {
        case 1: return make_float2(c1, s1);
        case 2: return make_float2(h, h);
        case 3: return make_float2(s1, c1);
        case 4: return make_float2(0.f, 1.f);
        case 6: return make_float2(-h, h);
        case 9: return make_float2(-c1, -s1);
        default: return make_float2(1.f, 0.f);
    }
}

// R-point DFT (+j sign) of v[o .. o+R); output k is left at v[o + opos<R>(k)].
template <int R>
__device__ __forceinline__ void dft(float2* v, int o) {
    if constexpr (R == 16) {
        // n = q + 4 r, k = s + 4 t: DFT4 over r, twiddle exp(2 pi j q s / 16), DFT4 over q
#pragma unroll
        for (int q = 0; q < 4; ++q) dft4<4>(v, o + q);
#pragma unroll
        for (int q = 1; q < 4; ++q)
#pragma unroll
            for (int s2 = 1; s2 < 4; ++s2) v[o + q + 4 * s2] = cmul(v[o + q + 4 * s2], w16(q * s2));
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) dft4<1>(v, o + 4 * s2);
    } else if constexpr (R == 8) {
        // n = q + 2 r, k = s + 4 t: DFT4 over r, twiddle exp(2 pi j q s / 8), DFT2 over q
        dft4<2>(v, o);
        dft4<2>(v, o + 1);
        constexpr float h = 0.70710678118654752f;
        v[o + 3] = cmul(v[o + 3], make_float2(h, h));
        v[o + 5] = mulj(v[o + 5]);
        v[o + 7] = cmul(v[o + 7], make_float2(-h, h));
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) dft2<1>(v, o + 2 * s2);
    } else if constexpr (R == 4) {
        dft4<1>(v, o);
    } else {
        dft2<1>(v, o);
    }
}
template <int R>
__device__ __forceinline__ constexpr int opos(int k) {
    return R == 16 ? 4 * (k & 3) + (k >> 2) : R == 8 ? 2 * (k & 3) + (k >> 2) : k;
}

// Pair of consecutive samples (2n, 2n+1) as float2: one vector load when the
// frame is aligned for it, two scalar loads otherwise.
template <typename T>
__device__ __forceinline__ float2 sample_pair(const T* __restrict__ xf, int n, bool vec);
template <>
__device__ __forceinline__ float2 sample_pair<float>(const float* __restrict__ xf, int n, bool vec) {
    if (vec) return reinterpret_cast<const float2*>(xf)[n];
    return make_float2(xf[2 * n], xf[2 * n + 1]);
}
template <>
__device__ __forceinline__ float2 sample_pair<double>(const double* __restrict__ xf, int n, bool vec) {
    if (vec) {
        const double2 d = reinterpret_cast<const double2*>(xf)[n];
        return make_float2((float)d.x, (float)d.y);
    }
    return make_float2((float)xf[2 * n], (float)xf[2 * n + 1]);
}
template <>
__device__ __forceinline__ float2 sample_pair<int16_t>(const int16_t* __restrict__ xf, int n, bool vec) {
    if (vec) {
        const short2 d = reinterpret_cast<const short2*>(xf)[n];
        return make_float2((float)d.x, (float)d.y);
    }
    return make_float2((float)xf[2 * n], (float)xf[2 * n + 1]);
}

template <typename T>
__device__ __forceinline__ void load_first(float2 (&v)[16], const T* __restrict__ xf, const float* __restrict__ g,
                                           int t, int Tn, bool live) {
    if (!live) {
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = make_float2(0.f, 0.f);
        return;
    }
    // One branch per frame (the alignment is the frame's), not one per load.
    float2 x[16];
    if ((reinterpret_cast<uintptr_t>(xf) % (2 * sizeof(T))) == 0) {
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = sample_pair(xf, t + r * Tn, true);
    } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = sample_pair(xf, t + r * Tn, false);
    }
    const float2* __restrict__ g2 = reinterpret_cast<const float2*>(g);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const float2 w = g2[t + r * Tn];
        v[r] = make_float2(w.x * x[r].x, w.y * x[r].y);
    }
}

// Complex samples (n = t + r Tn) times the real window g_n.
template <typename T2>
__device__ __forceinline__ void load_first_cplx(float2 (&v)[16], const T2* __restrict__ xf,
                                                const float* __restrict__ g, int t, int Tn, bool live) {
    if (!live) {
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = make_float2(0.f, 0.f);
        return;
    }
    T2 x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = xf[t + r * Tn];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const float w = g[t + r * Tn];
        v[r] = make_float2(w * (float)x[r].x, w * (float)x[r].y);
    }
}

// Twiddles of a Stockham pass of radix R and span Ns (see fft_pass) for the
// butterflies of thread t: w[b R + r] = exp(+2 pi j r k / (R Ns)), k = j mod Ns,
// from the pass's table tbl[r Ns + k] (consecutive threads read consecutive k).
template <int LOG2M, int R>
__device__ __forceinline__ void pass_twiddles(float2 (&w)[16], int t, int Ns, const float2* __restrict__ tbl) {
    constexpr int M = 1 << LOG2M, Tn = M / 16, B = 16 / R;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int k = (t + b * Tn) & (Ns - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) w[b * R + r] = tbl[r * Ns + k];
    }
}

// Stockham pass of radix R and span Ns over the M points of one frame held in
// LDS at s: butterfly j reads x[j + r M/R], twiddles by exp(+2 pi j r k / (R Ns))
// with k = j mod Ns (w, from pass_twiddles), and writes y[(j - k) R + k + r Ns].
// Thread t owns the 16/R butterflies j = t + b T.  FROM_REGS: the inputs are
// already in v (first pass, Ns = 1, natural order).
template <int LOG2M, int R, bool FROM_REGS>
__device__ __forceinline__ void fft_pass(float2 (&v)[16], const float2 (&w)[16], float2* s, int t, int Ns) {
    constexpr int M = 1 << LOG2M, Tn = M / 16, B = 16 / R;
    if (!FROM_REGS) {
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int r = 0; r < R; ++r) v[b * R + r] = s[pad(t + b * Tn + r * (M / R))];
        lds_barrier();
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int r = 1; r < R; ++r) v[b * R + r] = cmul(v[b * R + r], w[b * R + r]);
    }
#pragma unroll
    for (int b = 0; b < B; ++b) dft<R>(v, b * R);
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = t + b * Tn, k = j & (Ns - 1);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) s[pad(base + r * Ns)] = v[b * R + opos<R>(r)];
    }
    lds_barrier();
}

// One block's frames of one class: block `blk` of the class transforms its
// frames g_lo + blk F + (0..F-1) of channel `c`.
template <int LOG2N, bool CPLX>
__device__ __forceinline__ void window_rfft_block(const FftClass& a, int64_t blk, int c, float2* lds) {
    constexpr int N = 1 << LOG2N;
    constexpr int LOG2M = LOG2N - 1;
    constexpr int M = N / 2, Tn = M / 16, F = kFftThreads / Tn;
    constexpr int P16 = LOG2M / 4, REM = LOG2M % 4;
    // radices of the passes after the first (0: none)
    constexpr int R2 = fft_radix2(LOG2N), R3 = fft_radix3(LOG2N);
    static_assert(P16 <= 3 && !(P16 == 3 && REM), "frame length up to 8192");

    const int fl = threadIdx.x / Tn, t = threadIdx.x % Tn;
    float2* s = lds + fl * (M + M / 16);
    const int64_t gf = a.g_lo + blk * F + fl;     // frame of the class
    const bool live = gf < a.g_hi;
    RecDesc rec = a.single;
    if (a.recs && live) {
        int lo = 0, hi = a.n_recs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.recs[mid].frame0 <= gf) lo = mid;
            else hi = mid - 1;
        }
        rec = a.recs[lo];
    }
    const int64_t off = c * rec.chan_stride + (gf - rec.frame0) * (CPLX ? M : N);
    const float* __restrict__ g = a.g;
    const float2* __restrict__ tw = a.tw;

    // The second pass's twiddles are requested before the samples, the third
    // pass's just before its LDS reads (one pass ahead they spill registers).
    float2 v[16], w2[16], w3[16];
    if constexpr (R2 > 0) pass_twiddles<LOG2M, R2>(w2, t, 16, tw + N);
    if constexpr (CPLX) {
        if (rec.dtype == 3) load_first_cplx(v, static_cast<const float2*>(rec.data) + off, g, t, Tn, live);
        else load_first_cplx(v, static_cast<const double2*>(rec.data) + off, g, t, Tn, live);
    } else {
        if (rec.dtype == 0) load_first(v, static_cast<const float*>(rec.data) + off, g, t, Tn, live);
        else if (rec.dtype == 1) load_first(v, static_cast<const double*>(rec.data) + off, g, t, Tn, live);
        else load_first(v, static_cast<const int16_t*>(rec.data) + off, g, t, Tn, live);
    }

    fft_pass<LOG2M, 16, true>(v, w2, s, t, 1);
    if constexpr (R2 > 0) fft_pass<LOG2M, R2, false>(v, w2, s, t, 16);
    if constexpr (R3 > 0) pass_twiddles<LOG2M, R3>(w3, t, 16 * R2, tw + N + 16 * R2);
    if constexpr (R3 > 0) fft_pass<LOG2M, R3, false>(v, w3, s, t, 16 * R2);

    if (!live) return;
    // K <= M + 1: at most KMAX outputs per thread, unrolled so that their
    // twiddle loads are issued together.
    constexpr int KMAX = (M + 1 + Tn - 1) / Tn;
    const int K = a.K;
    float2* o = a.out + c * a.out_chan_stride + (gf - a.out_g0) * K;
    if constexpr (CPLX) {
#pragma unroll
        for (int i = 0; i < KMAX; ++i) {
            const int col = t + i * Tn;
            if (col >= K) break;
            o[col] = s[pad((col - a.jmax) & (M - 1))];
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        const int k = t + i * Tn;
        if (k >= K) break;
        const float2 xk = s[pad(k & (M - 1))];
        const float2 xm = s[pad((M - k) & (M - 1))];
        const float er = 0.5f * (xk.x + xm.x);
        const float ei = 0.5f * (xk.y - xm.y);
        const float orr = 0.5f * (xk.y + xm.y);   // (X_k - conj X_{M-k}) * (-j/2)
        const float oi = -0.5f * (xk.x - xm.x);
        const float2 w = tw[k];
        o[k] = make_float2(er + w.x * orr - w.y * oi, ei + w.x * oi + w.y * orr);
    }
}

template <int LOG2N, bool CPLX>
__global__ __launch_bounds__(kFftThreads, 4) void k_window_rfft(FftArgs a) {
    __shared__ float2 lds[kFftLds];
    window_rfft_block<LOG2N, CPLX>(a.cls[0], blockIdx.x, blockIdx.y, lds);
}

// Several frame lengths in one launch (real signals): a block finds its class
// from its index and runs that frame length's transform.
template <int LOG2N>
__device__ __forceinline__ void rfft_class(const FftClass& k, int64_t blk, int c, float2* lds) {
    window_rfft_block<LOG2N, false>(k, blk, c, lds);
}

__global__ __launch_bounds__(kFftThreads, 4) void k_window_rfft_multi(FftArgs a) {
    __shared__ float2 lds[kFftLds];
    int ci = 0;
    for (int i = 1; i < a.n_cls; ++i)
        if ((int64_t)blockIdx.x >= a.cls[i].block0) ci = i;
    const FftClass& k = a.cls[ci];
    const int64_t blk = (int64_t)blockIdx.x - k.block0;
    switch (k.log2n) {
        case 8: rfft_class<8>(k, blk, blockIdx.y, lds); break;
        case 9: rfft_class<9>(k, blk, blockIdx.y, lds); break;
        case 10: rfft_class<10>(k, blk, blockIdx.y, lds); break;
        case 11: rfft_class<11>(k, blk, blockIdx.y, lds); break;
        case 12: rfft_class<12>(k, blk, blockIdx.y, lds); break;
        default: rfft_class<13>(k, blk, blockIdx.y, lds); break;
    }
}

// Frame lengths that are not a power of two: the windowed transform by its
// definition (Section 3, eq. a_k),
//   a_k = sum_{i<N} g_i z_i exp(+2 pi j i k / N),  k < K,
// as the product of the windowed frames [frames x N] with the exponentials
// [N x K], accumulated in FP64; exp(+2 pi j t / N) for t = i k mod N comes from
// an FP64 table of N entries (tw64).  N^2/2 complex products per frame where
// the FFT takes ~N log2 N: the path of the lengths that neither the FFT nor
// the two-stage form below takes (primes, and lengths without a divisor
// between 8 and sqrt(N)).
// A 256-thread block computes kDftFrames frames x kDftBins bins of one
// channel: thread (tf, tb) = (tid / 16, tid % 16) accumulates the frames
// f0 + tf + 16 u (u < 2) at the bins k0 + tb + 16 v (v < 4).  The samples pass
// in steps of kDftStep: each thread stages 4 windowed samples of one frame
// (FP64) and 8 exponentials of the step, then every thread adds the step's
// products.  Grid: x = frame blocks, y = channels, z = bin blocks.
constexpr int kDftFrames = 32, kDftBins = 64, kDftStep = 32;

__device__ __forceinline__ double dft_sample(const RecDesc& rec, int64_t idx) {
    if (rec.dtype == 0) return (double)static_cast<const float*>(rec.data)[idx];
    if (rec.dtype == 1) return static_cast<const double*>(rec.data)[idx];
    return (double)static_cast<const int16_t*>(rec.data)[idx];
}

__global__ __launch_bounds__(256) void k_window_dft(FftArgs args) {
    const FftClass& a = args.cls[0];
    __shared__ double sw[kDftFrames][kDftStep + 1];     // windowed samples of the step
    __shared__ double2 st[kDftStep][kDftBins];          // exponentials of the step

    const int N = a.dft_n, K = a.K;
    const int tid = threadIdx.x;
    const int tf = tid >> 4, tb = tid & 15;
    const int64_t f0 = a.g_lo + (int64_t)blockIdx.x * kDftFrames;
    const int k0 = (int)blockIdx.z * kDftBins;
    const int c = blockIdx.y;

    // staging role: frame lf of the block, samples ls .. ls + 3 of each step
    const int lf = tid >> 3, ls = 4 * (tid & 7);
    const int64_t gf = f0 + lf;
    const bool live = gf < a.g_hi;
    RecDesc rec = a.single;
    if (a.recs && live) {
        int lo = 0, hi = a.n_recs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.recs[mid].frame0 <= gf) lo = mid;
            else hi = mid - 1;
        }
        rec = a.recs[lo];
    }
    const int64_t off = c * rec.chan_stride + (gf - rec.frame0) * N;

    double acc[2][4][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v][0] = acc[u][v][1] = 0.0;

    for (int i0 = 0; i0 < N; i0 += kDftStep) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + ls + q;
            sw[lf][ls + q] = (live && i < N) ? (double)a.g[i] * dft_sample(rec, off + i) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + 256 * q;                     // < kDftStep * kDftBins
            const int s = e / kDftBins, b = e % kDftBins;
            const int i = i0 + s, k = k0 + b;
            st[s][b] = (i < N && k < K) ? a.tw64[(int)(((int64_t)i * k) % N)] : make_double2(0.0, 0.0);
        }
        lds_barrier();
#pragma unroll 4
        for (int s = 0; s < kDftStep; ++s) {
            const double w0 = sw[tf][s], w1 = sw[tf + 16][s];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double2 t = st[s][tb + 16 * v];
                acc[0][v][0] = fma(w0, t.x, acc[0][v][0]);
                acc[0][v][1] = fma(w0, t.y, acc[0][v][1]);
                acc[1][v][0] = fma(w1, t.x, acc[1][v][0]);
                acc[1][v][1] = fma(w1, t.y, acc[1][v][1]);
            }
        }
        lds_barrier();
    }

#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int64_t g = f0 + tf + 16 * u;
        if (g >= a.g_hi) continue;
        float2* o = a.out + c * a.out_chan_stride + (g - a.out_g0) * K;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int k = k0 + tb + 16 * v;
            if (k < K) o[k] = make_float2((float)acc[u][v][0], (float)acc[u][v][1]);
        }
    }
}

// The same transform in two stages when N = N1 N2 factors well (N1 <= N2,
// both from dft_n1): with n = N2 n1 + n2 and k = k1 + N1 k2 (Cooley-Tukey),
//   Y[k1][n2] = exp(+2 pi j n2 k1 / N) sum_{n1 < N1} w[N2 n1 + n2] exp(+2 pi j n1 k1 / N1),
//   a_{k1 + N1 k2} = sum_{n2 < N2} Y[k1][n2] exp(+2 pi j n2 k2 / N2),
// N (N1 + N2) products instead of N K.  One block per frame and channel: the
// windowed frame (FP32), the two stages' exponentials and Y (FP32, rows
// padded by one) sit in LDS, every sum is accumulated in FP64, every
// exponential comes from the FP64 table of exp(+2 pi j t / N)
// (exp(+2 pi j t / N1) = entry t N2, exp(+2 pi j t / N2) = entry t N1).
// LDS (dynamic): the N samples (FP32), the exponentials of the two stages
// exp(+2 pi j t / N1), t < N1, and exp(+2 pi j t / N2), t < N2 (FP64), then Y.
__host__ __device__ constexpr size_t dft2_sx_bytes(int N) { return ((size_t)N * 4 + 15) / 16 * 16; }
__host__ __device__ constexpr size_t dft2_lds_bytes(int N, int N1) {
    return dft2_sx_bytes(N) + (size_t)(N1 + N / N1) * 16 + (size_t)N1 * (N / N1 + 1) * 8;
}

__global__ __launch_bounds__(256) void k_window_dft2(FftArgs args) {
    const FftClass& a = args.cls[0];
    HIP_DYNAMIC_SHARED(double2, dyn)
    const int N = a.dft_n, N1 = a.dft_n1, N2 = N / N1, K = a.K;
    float* sx = reinterpret_cast<float*>(dyn);                        // windowed samples of the frame
    double2* sw1 = dyn + dft2_sx_bytes(N) / 16;                       // exp(+2 pi j t / N1)
    double2* sw2 = sw1 + N1;                                          // exp(+2 pi j t / N2)
    float2* sy = reinterpret_cast<float2*>(sw2 + N2);                 // Y, N1 rows of N2 + 1

    const int tid = threadIdx.x;
    const int64_t gf = a.g_lo + (int64_t)blockIdx.x;
    const int c = blockIdx.y;
    if (gf >= a.g_hi) return;                            // (block-uniform)
    RecDesc rec = a.single;
    if (a.recs) {
        int lo = 0, hi = a.n_recs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.recs[mid].frame0 <= gf) lo = mid;
            else hi = mid - 1;
        }
        rec = a.recs[lo];
    }
    const int64_t off = c * rec.chan_stride + (gf - rec.frame0) * N;
    for (int i = tid; i < N; i += 256) sx[i] = (float)((double)a.g[i] * dft_sample(rec, off + i));
    for (int t = tid; t < N1; t += 256) sw1[t] = a.tw64[t * N2];
    for (int t = tid; t < N2; t += 256) sw2[t] = a.tw64[t * N1];
    lds_barrier();

    // stage 1: (k1, n2) = (e / N2, e % N2), e < N
    for (int e = tid; e < N; e += 256) {
        const int k1 = e / N2, n2 = e - k1 * N2;
        double yr = 0.0, yi = 0.0;
        int t = 0;                                       // n1 k1 mod N1
        for (int n1 = 0; n1 < N1; ++n1) {
            const double x = sx[N2 * n1 + n2];
            const double2 w = sw1[t];
            yr = fma(x, w.x, yr);
            yi = fma(x, w.y, yi);
            t += k1;
            if (t >= N1) t -= N1;
        }
        const double2 w = a.tw64[n2 * k1];               // n2 k1 < N
        sy[k1 * (N2 + 1) + n2] = make_float2((float)(yr * w.x - yi * w.y), (float)(yr * w.y + yi * w.x));
    }
    lds_barrier();

    // stage 2: coefficient k = k1 + N1 k2 < K
    float2* o = a.out + c * a.out_chan_stride + (gf - a.out_g0) * K;
    for (int k = tid; k < K; k += 256) {
        const int k2 = k / N1, k1 = k - k2 * N1;
        const float2* y = sy + k1 * (N2 + 1);
        const int step = k2 % N2;
        double xr = 0.0, xi = 0.0;
        int t = 0;                                       // n2 k2 mod N2
        for (int n2 = 0; n2 < N2; ++n2) {
            const float2 v = y[n2];
            const double2 w = sw2[t];
            xr = fma((double)v.x, w.x, fma(-(double)v.y, w.y, xr));
            xi = fma((double)v.x, w.y, fma((double)v.y, w.x, xi));
            t += step;
            if (t >= N2) t -= N2;
        }
        o[k] = make_float2((float)xr, (float)xi);
    }
}

hipError_t launch_dft(const FftArgs& a, hipStream_t st) {
    const FftClass& c = a.cls[0];
    const int64_t n = c.g_hi - c.g_lo;
    if (c.dft_n < 2 || !c.tw64 || c.K < 1) return hipErrorInvalidValue;
    if (c.dft_n1 > 0) {                 // two stages, N = N1 N2
        const int n2 = c.dft_n / c.dft_n1;
        if (n2 * c.dft_n1 != c.dft_n || c.dft_n1 > n2) return hipErrorInvalidValue;
        const size_t lds = dft2_lds_bytes(c.dft_n, c.dft_n1);
        if (lds > 160 * 1024) return hipErrorInvalidValue;
        if (n > 0x7fffffff) return hipErrorInvalidConfiguration;
        k_window_dft2<<<dim3((unsigned)n, a.n_channels), 256, lds, st>>>(a);
        return hipGetLastError();
    }
    const int64_t bx = (n + kDftFrames - 1) / kDftFrames, bz = (c.K + kDftBins - 1) / kDftBins;
    if (bx > 0x7fffffff) return hipErrorInvalidConfiguration;
    k_window_dft<<<dim3((unsigned)bx, a.n_channels, (unsigned)bz), 256, 0, st>>>(a);
    return hipGetLastError();
}

template <int LOG2N>
hipError_t launch_n(const FftArgs& a, hipStream_t st) {
    constexpr int M = (1 << LOG2N) / 2, F = kFftThreads / (M / 16);
    const int64_t n = a.cls[0].g_hi - a.cls[0].g_lo;
    dim3 grid((unsigned)((n + F - 1) / F), a.n_channels);
    if (a.cplx) {
        if constexpr (LOG2N >= 9) k_window_rfft<LOG2N, true><<<grid, kFftThreads, 0, st>>>(a);
        else return hipErrorInvalidValue;
    } else {
        k_window_rfft<LOG2N, false><<<grid, kFftThreads, 0, st>>>(a);
    }
    return hipGetLastError();
}

// a_k(f) -= (1/m) sum_{f' in chunk} a_k(f'), in place, one thread per (chunk, k).
// Chunks of up to kCentreRegs frames stay in registers between the mean and
// the subtraction, so each coefficient is read from HBM once.
//
// For the c3^(opt) estimator of S3 (Section 4.1) the same pass also writes the
// rows S3 multiplies: with x_f, y_f, z_f the chunk's three factors, x' = x - mean
// and P = sum over the three pairs of (1/m) sum_f x'_f y'_f times the third
// factor's mean, R = the product of the three means,
//   c3opt = ((m+4) M3' + 4 P + (4 - 2m) R) / (m + 1),  M3' = (1/m) sum x'y'z'.
// Since sum_f x'_f = 0, the rows x'_f + alpha mean with alpha = 4/(m+4) give
//   (1/m) sum_f (x' + alpha xm)(y' + alpha ym)(z' + alpha zm) = M3' + alpha P + alpha^3 R,
// and one more row mu mean per chunk, mu^3 = m ((4 - 2m)/(m+4) - alpha^3), adds
// the rest of R: the plain S3 sum over the m + 1 rows, times (m+4)/((m+1) m),
// is c3opt.
constexpr int kCentreRegs = 16;

// float16 word pair (lo, hi), each rounded to nearest even.
typedef _Float16 f16x2_v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t f16_pair(float lo, float hi) {
    const f16x2_v v = {(_Float16)lo, (_Float16)hi};
    return __builtin_bit_cast(uint32_t, v);
}

// The operand records of the matrix-core S4 kernel for one column of one
// chunk (see kOpWords): piece i of value v (Re, Im, P) of column k at the
// 16-byte unit (3 v + i) op4_cols + k of the chunk's block, and the pair
// (p = sum_f P, s^2) at p4[chunk][k].  v holds the chunk's m <= kOpFrames
// uncentred values; a column without coefficients (k >= K, padding up to
// op4_cols) gets zero records, p = 0 and s = 1.
__device__ __forceinline__ void write_op_records(const CentreClass& cl, int64_t chunk, int k, int m,
                                                 const float2 (&v)[kCentreRegs], float mr, float mi, bool live) {
    const int64_t ngp = cl.op4_cols;
    uint4* rec = reinterpret_cast<uint4*>(cl.op4 + blockIdx.y * cl.op4_cs + chunk * (3 * kOpWords) * ngp) + k;
    float re[kOpFrames], im[kOpFrames], amax = 0.f;
#pragma unroll
    for (int f = 0; f < kOpFrames; ++f) {
        const bool on = live && f < m;
        re[f] = on ? v[f].x - mr : 0.f;                     // the centred values written to coef
        im[f] = on ? v[f].y - mi : 0.f;
        amax = fmaxf(amax, fmaxf(fabsf(re[f]), fabsf(im[f])));
    }
    const float s = pow2_above(amax);
    const float inv_s = 1.0f / s, inv_s2 = inv_s * inv_s;    // exact: powers of two
    float psum = 0.f;
#pragma unroll
    for (int val = 0; val < 3; ++val) {
        uint32_t w[10];
#pragma unroll
        for (int f = 0; f < kOpFrames; f += 2) {
            float x[2], l[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const float P = fmaf(re[f + u], re[f + u], im[f + u] * im[f + u]);
                if (val == 2) psum += P;
                x[u] = val == 0 ? re[f + u] * inv_s : val == 1 ? im[f + u] * inv_s : P * inv_s2;
                l[u] = x[u] - (float)(_Float16)x[u];
            }
            w[f >> 1] = f16_pair(x[0], x[1]);
            w[5 + (f >> 1)] = f16_pair(l[0], l[1]);
        }
        uint4* dst = rec + val * kOpPieces * ngp;
        dst[0] = make_uint4(w[0], w[1], w[2], w[3]);                // H: h words 0..3
        dst[ngp] = make_uint4(w[5], w[6], w[7], w[8]);              // L: l words 0..3
        dst[2 * ngp] = make_uint4(w[4], w[9], 0u, 0u);              // T: h word 4, l word 4
    }
    double2* pp = reinterpret_cast<double2*>(cl.p4 + blockIdx.y * cl.p4_cs + chunk * 2 * ngp) + k;
    *pp = make_double2((double)psum, (double)(s * s));
}

// Grid: x = the classes' (chunk, 256-wide k block) pairs, chunk-major within
// each class; y = channel (the chunk count can exceed the 65536 limit of the y
// and z grid dimensions).
__global__ __launch_bounds__(256) void k_centre(CentreArgs a) {
    int ci = 0;
    for (int i = 1; i < a.n_cls; ++i)
        if ((int64_t)blockIdx.x >= a.cls[i].block0) ci = i;
    const CentreClass& cl = a.cls[ci];
    const int K = cl.K, m = a.m;
    const int kblocks = (K + 255) / 256;
    const int64_t local = (int64_t)blockIdx.x - cl.block0;
    const int64_t chunk = local / kblocks;
    const int k = (int)(local - chunk * kblocks) * 256 + threadIdx.x;
    if (k >= K) {
        if (cl.op4 && k < cl.op4_cols) {            // padding columns of the S4 operand records
            float2 z[kCentreRegs];
#pragma unroll
            for (int f = 0; f < kCentreRegs; ++f) z[f] = make_float2(0.f, 0.f);
            write_op_records(cl, chunk, k, m, z, 0.f, 0.f, false);
        }
        return;
    }
    float2* p = cl.coef + blockIdx.y * cl.coef_chan_stride + chunk * m * K + k;
    // c3^(opt): the chunk's rows for S3, frames shifted by alpha mean, then mu mean
    float2* q = cl.out3 ? cl.out3 + blockIdx.y * cl.out3_cs + chunk * (m + 1) * K + k : nullptr;
    const float inv = 1.0f / (float)m;
    const float alpha = a.alpha, mu = a.mu;
    // S1: the chunk's mean of a_0 (real for a real signal)
    auto keep_mean = [&](float mr, float mi) {
        if (a.s1 && k == a.s1_col) a.s1[blockIdx.y * a.s1_cs + cl.s1_chunk0 + chunk] = make_float2(mr, mi);
        if (q) q[(int64_t)m * K] = make_float2(mu * mr, mu * mi);
    };
    auto put = [&](int f, float2 v, float mr, float mi) {
        const float2 c = make_float2(v.x - mr, v.y - mi);
        p[(int64_t)f * K] = c;
        if (q) q[(int64_t)f * K] = make_float2(fmaf(alpha, mr, c.x), fmaf(alpha, mi, c.y));
    };
    if (m <= kCentreRegs) {
        float2 v[kCentreRegs];
        float sr = 0.f, si = 0.f;
#pragma unroll
        for (int f = 0; f < kCentreRegs; ++f) {
            if (f < m) {
                v[f] = p[(int64_t)f * K];
                sr += v[f].x;
                si += v[f].y;
            }
        }
        const float mr = sr * inv, mi = si * inv;
        keep_mean(mr, mi);
#pragma unroll
        for (int f = 0; f < kCentreRegs; ++f)
            if (f < m) put(f, v[f], mr, mi);
        if (cl.op4 && k < cl.op4_cols) write_op_records(cl, chunk, k, m, v, mr, mi, true);
        return;
    }
    float sr = 0.f, si = 0.f;
    for (int f = 0; f < m; ++f) {
        const float2 v = p[(int64_t)f * K];
        sr += v.x;
        si += v.y;
    }
    const float mr = sr * inv, mi = si * inv;
    keep_mean(mr, mi);
    for (int f = 0; f < m; ++f) put(f, p[(int64_t)f * K], mr, mi);
}

}  // namespace

hipError_t launch_window_rfft(const FftArgs& a, hipStream_t s) {
    if (a.n_cls <= 0 || a.n_channels <= 0) return hipSuccess;
    if (a.n_cls > 1) {          // several frame lengths: one launch, a class per block range
        if (a.cplx || a.n_cls > kMaxClasses) return hipErrorInvalidValue;
        for (int i = 0; i < a.n_cls; ++i)
            if (a.cls[i].dft_n) return hipErrorInvalidValue;
        int64_t blocks = 0;
        for (int i = 0; i < a.n_cls; ++i) {
            const FftClass& c = a.cls[i];
            const int F = kFftThreads / ((1 << c.log2n) / 32);
            if (c.block0 != blocks || c.g_hi < c.g_lo || c.log2n < 8 || c.log2n > 13) return hipErrorInvalidValue;
            blocks += (c.g_hi - c.g_lo + F - 1) / F;
        }
        if (blocks <= 0) return hipSuccess;
        if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
        k_window_rfft_multi<<<dim3((unsigned)blocks, a.n_channels), kFftThreads, 0, s>>>(a);
        return hipGetLastError();
    }
    const FftClass& c0 = a.cls[0];
    if (c0.g_hi <= c0.g_lo || c0.n_recs <= 0) return hipSuccess;
    if (c0.dft_n) {            // N not a power of two: the direct transform
        if (a.cplx) return hipErrorInvalidValue;
        return launch_dft(a, s);
    }
    switch (c0.log2n) {
        case 8: return launch_n<8>(a, s);
        case 9: return launch_n<9>(a, s);
        case 10: return launch_n<10>(a, s);
        case 11: return launch_n<11>(a, s);
        case 12: return launch_n<12>(a, s);
        case 13: return launch_n<13>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_centre(const CentreArgs& a, hipStream_t s) {
    if (a.n_cls <= 0 || a.n_cls > kMaxClasses) return a.n_cls <= 0 ? hipSuccess : hipErrorInvalidValue;
    int64_t nx = 0;
    for (int i = 0; i < a.n_cls; ++i) {
        const CentreClass& c = a.cls[i];
        if (c.block0 != nx || c.n_chunks < 0) return hipErrorInvalidValue;
        nx += (int64_t)((c.K + 255) / 256) * c.n_chunks;
    }
    if (nx <= 0) return hipSuccess;
    if (nx > 0x7fffffff) return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)nx, a.n_channels);
    k_centre<<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace ps
