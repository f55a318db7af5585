// Stage a1: windowed real FFT of every frame (Section 3, eq. a_k), and the
// per-chunk centring a' = a - mean_f a that the k-statistics of Section 4.1
// need in their centred form (Appendix H).
//
//   a_k = sum_{i<N} g_i z_i exp(+2 pi j i k / N),  k < K        (dt folded into the output scale)
//
// One 256-thread block transforms one frame; the frames of every record of a
// batch form one launch (the block finds its record by binary search over the
// records' first global frame).  The N real samples are packed as
// M = N/2 complex points x_n = w_{2n} + j w_{2n+1} (w = g z), transformed by a
// radix-4 (plus one radix-2) Stockham FFT in LDS with the +j sign, and
// unpacked: with X the M-point transform,
//   E_k = (X_k + conj X_{M-k}) / 2,  O_k = (X_k - conj X_{M-k}) / (2j),
//   a_k = E_k + exp(+2 pi j k / N) O_k   (indices of X taken mod M).
// Twiddles come from a table exp(+2 pi j t / N) computed in FP64 on the host.
// The stage streams N samples in and K complex values out per frame: it is
// bound by HBM bandwidth, not arithmetic.
#include "ps_internal.h"

namespace ps {
namespace {

constexpr int kFftThreads = 256;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <typename T>
__device__ __forceinline__ void load_windowed(float2* s, const T* __restrict__ xf, const float* __restrict__ g,
                                              int M, int tid) {
    for (int n = tid; n < M; n += kFftThreads) {
        const float w0 = g[2 * n] * static_cast<float>(xf[2 * n]);
        const float w1 = g[2 * n + 1] * static_cast<float>(xf[2 * n + 1]);
        s[n] = make_float2(w0, w1);
    }
}

template <int LOG2N>
__global__ __launch_bounds__(kFftThreads) void k_window_rfft(FftArgs a) {
    constexpr int N = 1 << LOG2N;
    constexpr int M = N / 2;
    constexpr int LOG2M = LOG2N - 1;
    __shared__ float2 s[M];

    const int64_t gf = a.g_lo + blockIdx.x;     // global frame
    const int c = blockIdx.y;
    RecDesc r = a.single;
    if (a.recs) {
        int lo = 0, hi = a.n_recs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.recs[mid].frame0 <= gf) lo = mid;
            else hi = mid - 1;
        }
        r = a.recs[lo];
    }
    const int64_t off = c * r.chan_stride + (gf - r.frame0) * N;
    const int tid = threadIdx.x;
    const float* __restrict__ g = a.g;
    const float2* __restrict__ tw = a.tw;
    if (r.dtype == 0) load_windowed(s, static_cast<const float*>(r.data) + off, g, M, tid);
    else if (r.dtype == 1) load_windowed(s, static_cast<const double*>(r.data) + off, g, M, tid);
    else load_windowed(s, static_cast<const int16_t*>(r.data) + off, g, M, tid);
    __syncthreads();

    // Radix-4 Stockham passes: span Ns = 1, 4, 16, ...; butterfly j reads
    // x[j + r M/4], twiddles by exp(+2 pi j r k / (4 Ns)) with k = j mod Ns,
    // applies the 4-point DFT (+j) and writes to (j - k) * 4 + k + r Ns.
    constexpr int B4 = M / 4;
    constexpr int P4 = (B4 + kFftThreads - 1) / kFftThreads;
    int Ns = 1;
#pragma unroll 1
    for (int pass = 0; pass < LOG2M / 2; ++pass) {
        float2 v[P4][4];
#pragma unroll
        for (int q = 0; q < P4; ++q) {
            const int j = tid + q * kFftThreads;
            if (j < B4) {
#pragma unroll
                for (int r = 0; r < 4; ++r) v[q][r] = s[j + r * B4];
            }
        }
        __syncthreads();
        const int step = N / (Ns * 4);
#pragma unroll
        for (int q = 0; q < P4; ++q) {
            const int j = tid + q * kFftThreads;
            if (j < B4) {
                const int k = j & (Ns - 1);
                const float2 v0 = v[q][0];
                const float2 v1 = cmul(v[q][1], tw[k * step]);
                const float2 v2 = cmul(v[q][2], tw[2 * k * step]);
                const float2 v3 = cmul(v[q][3], tw[3 * k * step]);
                const float2 s02 = make_float2(v0.x + v2.x, v0.y + v2.y);
                const float2 d02 = make_float2(v0.x - v2.x, v0.y - v2.y);
                const float2 s13 = make_float2(v1.x + v3.x, v1.y + v3.y);
                const float2 d13 = make_float2(v1.x - v3.x, v1.y - v3.y);
                // y1 = d02 + j d13, y3 = d02 - j d13 (the +j 4-point kernel)
                const int base = (j - k) * 4 + k;
                s[base] = make_float2(s02.x + s13.x, s02.y + s13.y);
                s[base + Ns] = make_float2(d02.x - d13.y, d02.y + d13.x);
                s[base + 2 * Ns] = make_float2(s02.x - s13.x, s02.y - s13.y);
                s[base + 3 * Ns] = make_float2(d02.x + d13.y, d02.y - d13.x);
            }
        }
        __syncthreads();
        Ns *= 4;
    }
    if constexpr (LOG2M & 1) {
        constexpr int B2 = M / 2;
        constexpr int P2 = (B2 + kFftThreads - 1) / kFftThreads;
        float2 v[P2][2];
#pragma unroll
        for (int q = 0; q < P2; ++q) {
            const int j = tid + q * kFftThreads;
            if (j < B2) {
                v[q][0] = s[j];
                v[q][1] = s[j + B2];
            }
        }
        __syncthreads();
        const int step = N / (Ns * 2);
#pragma unroll
        for (int q = 0; q < P2; ++q) {
            const int j = tid + q * kFftThreads;
            if (j < B2) {
                const int k = j & (Ns - 1);
                const float2 v0 = v[q][0];
                const float2 v1 = cmul(v[q][1], tw[k * step]);
                const int base = (j - k) * 2 + k;
                s[base] = make_float2(v0.x + v1.x, v0.y + v1.y);
                s[base + Ns] = make_float2(v0.x - v1.x, v0.y - v1.y);
            }
        }
        __syncthreads();
    }

    const int K = a.K;
    float2* o = a.out + c * a.out_chan_stride + (gf - a.out_g0) * K;
    for (int k = tid; k < K; k += kFftThreads) {
        const float2 xk = s[k & (M - 1)];
        const float2 xm = s[(M - k) & (M - 1)];
        const float er = 0.5f * (xk.x + xm.x);
        const float ei = 0.5f * (xk.y - xm.y);
        const float orr = 0.5f * (xk.y + xm.y);   // (X_k - conj X_{M-k}) * (-j/2)
        const float oi = -0.5f * (xk.x - xm.x);
        const float2 w = tw[k];
        o[k] = make_float2(er + w.x * orr - w.y * oi, ei + w.x * oi + w.y * orr);
    }
}

template <int LOG2N>
hipError_t launch_n(const FftArgs& a, hipStream_t st) {
    const int64_t n = a.g_hi - a.g_lo;
    dim3 grid((unsigned)n, a.n_channels);
    k_window_rfft<LOG2N><<<grid, kFftThreads, 0, st>>>(a);
    return hipGetLastError();
}

// a_k(f) -= (1/m) sum_{f' in chunk} a_k(f'), in place, one thread per (chunk, k).
// Chunks of up to kCentreRegs frames stay in registers between the mean and
// the subtraction, so each coefficient is read from HBM once.
constexpr int kCentreRegs = 16;

__global__ __launch_bounds__(256) void k_centre(float2* __restrict__ coef, int64_t coef_cs, int K, int m) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= K) return;
    float2* p = coef + blockIdx.z * coef_cs + (int64_t)blockIdx.y * m * K + k;
    const float inv = 1.0f / (float)m;
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
#pragma unroll
        for (int f = 0; f < kCentreRegs; ++f)
            if (f < m) p[(int64_t)f * K] = make_float2(v[f].x - mr, v[f].y - mi);
        return;
    }
    float sr = 0.f, si = 0.f;
    for (int f = 0; f < m; ++f) {
        const float2 v = p[(int64_t)f * K];
        sr += v.x;
        si += v.y;
    }
    const float mr = sr * inv, mi = si * inv;
    for (int f = 0; f < m; ++f) {
        const float2 v = p[(int64_t)f * K];
        p[(int64_t)f * K] = make_float2(v.x - mr, v.y - mi);
    }
}

}  // namespace

hipError_t launch_window_rfft(const FftArgs& a, hipStream_t s) {
    if (a.g_hi <= a.g_lo || a.n_channels <= 0 || a.n_recs <= 0) return hipSuccess;
    switch (a.log2n) {
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
    if (a.n_chunks <= 0) return hipSuccess;
    dim3 grid((a.K + 255) / 256, (unsigned)a.n_chunks, a.n_channels);
    k_centre<<<grid, 256, 0, s>>>(a.coef, a.coef_chan_stride, a.K, a.m);
    return hipGetLastError();
}

}  // namespace ps
