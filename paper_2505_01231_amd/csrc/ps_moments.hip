// Per-chunk moment sums, k-statistic combination and FP64 chunk accumulation
// (Sections 3, 4, 4.1, 4.2 and 7; the centred form of Appendix H).
//
// Inputs are the coefficients a_k(f) of stage a1 and their per-chunk means;
// every kernel works with the chunk-centred values a' = a - mean_f a.  For a
// chunk of m frames (sums over f):
//
//   S2:  s2_k   = sum a'_k b'*_k                           c2 = s2 / (m-1)
//   S3:  T3_kl  = sum a'_k b'_l c'*_{k+l}                  c3 = m T3 / ((m-1)(m-2))
//   S4 (one channel, real):
//        X = sum Re_k Re_l, Y = sum Im_k Im_l, U = sum Re_k Im_l, V = sum Im_k Re_l,
//        M4 = sum P_k P_l, p_k = sum P_k with P = |a'|^2, and since
//        |sum a'_k a'_l|^2 + |sum a'_k a'*_l|^2 = 2 (X^2 + Y^2 + U^2 + V^2),
//        c4 = [m(m+1) M4 - (m-1)(p_k p_l + 2(X^2+Y^2+U^2+V^2))] / ((m-1)(m-2)(m-3)).
//
// Each kernel accumulates, per grid point, the FP64 sums over its chunks of the
// estimate (without its constant prefactor) and of its squared real and
// imaginary parts; the finalize kernels turn those into the mean and the
// Section 4.2 error bar.  The prefactors, the window sums and dt are applied
// there.
//
// Work split: a launch covers the chunk range [chunk0, chunk1) split into
// n_split contiguous parts; each block owns one 64x64 output tile and one part
// and writes its own partial sums (no atomics: the reduction order is fixed).
// Consecutive block ids are spread over the 8 XCDs by the hardware; the ids are
// remapped so that the blocks resident on one XCD work on the same chunk part
// at the same time and share its coefficients in that XCD's L2.
#include "ps_internal.h"

namespace ps {
namespace {

__device__ __forceinline__ float2 ld_centred(const float2* __restrict__ p, float2 mu) {
    const float2 v = *p;
    return make_float2(v.x - mu.x, v.y - mu.y);
}

// Remap blockIdx.x onto (split, tile) so that each XCD sees a contiguous,
// split-major range of work items.
__device__ __forceinline__ bool xcd_work_item(int n_tiles, int n_split, int& split, int& tile) {
    const int total = n_tiles * n_split;
    const int per_xcd = (total + 7) >> 3;
    const int b = blockIdx.x;
    const int v = (b & 7) * per_xcd + (b >> 3);
    if (v >= total) return false;
    split = v / n_tiles;
    tile = v - split * n_tiles;
    return true;
}

__device__ __forceinline__ void split_range(int chunk0, int chunk1, int n_split, int split, int& c0,
                                            int& c1) {
    const int64_t n = chunk1 - chunk0;
    c0 = chunk0 + (int)((n * split) / n_split);
    c1 = chunk0 + (int)((n * (split + 1)) / n_split);
}

// ------------------------------------------------------------------ S2
__global__ __launch_bounds__(256) void k_s2(S2Args p) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    const int split = blockIdx.y;
    if (k >= p.Nf) return;
    int c0, c1;
    split_range(p.chunk0, p.chunk1, p.n_split, split, c0, c1);
    const CoefView& v = p.v;
    const float2* A = v.coef + p.a * v.coef_chan_stride;
    const float2* B = v.coef + p.b * v.coef_chan_stride;
    const float2* MA = v.mean + p.a * v.mean_chan_stride;
    const float2* MB = v.mean + p.b * v.mean_chan_stride;
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int c = c0; c < c1; ++c) {
        const float2 ma = MA[(int64_t)(c - v.mean_chunk0) * v.K + k];
        const float2 mb = MB[(int64_t)(c - v.mean_chunk0) * v.K + k];
        const int64_t base = (int64_t)(c - v.coef_chunk0) * v.m * v.K + k;
        float re = 0.f, im = 0.f;
        for (int f = 0; f < v.m; ++f) {
            const float2 x = ld_centred(A + base + (int64_t)f * v.K, ma);
            const float2 y = ld_centred(B + base + (int64_t)f * v.K, mb);
            re += x.x * y.x + x.y * y.y;   // x * conj(y)
            im += x.y * y.x - x.x * y.y;
        }
        s0 += re;
        s1 += im;
        s2 += (double)re * re;
        s3 += (double)im * im;
    }
    double* o = p.part + (int64_t)split * 4 * p.Nf + k;
    if (p.accumulate) {
        s0 += o[0];
        s1 += o[p.Nf];
        s2 += o[2 * p.Nf];
        s3 += o[3 * p.Nf];
    }
    o[0] = s0;
    o[p.Nf] = s1;
    o[2 * p.Nf] = s2;
    o[3 * p.Nf] = s3;
}

// ------------------------------------------------------------------ S3
// Thread (ti, tj) = (tid / 16, tid % 16) owns the grid points
// (k0 + ti + 16u, l0 + tj + 16v), u, v < 4, whose third factor sits at
// k + l = k0 + l0 + ti + tj + 16(u + v).  Per frame it reads 4 + 4 + 7 values
// from LDS and does 16 complex triple products (8 FMA-class ops each).
constexpr int kS3Threads = 256;

__global__ __launch_bounds__(kS3Threads, 2) void k_s3(GridArgs p) {
    __shared__ float2 sA[kFrameBatch][kTile];
    __shared__ float2 sB[kFrameBatch][kTile];
    __shared__ float2 sC[kFrameBatch][2 * kTile];

    int split, tile;
    if (!xcd_work_item(p.n_tiles, p.n_split, split, tile)) return;
    int c0, c1;
    split_range(p.chunk0, p.chunk1, p.n_split, split, c0, c1);
    const int2 t = p.tiles[tile];
    const int k0 = t.x * kTile, l0 = t.y * kTile;
    const CoefView& v = p.v;
    const float2* A = v.coef + p.ch[0] * v.coef_chan_stride;
    const float2* B = v.coef + p.ch[1] * v.coef_chan_stride;
    const float2* C = v.coef + p.ch[2] * v.coef_chan_stride;
    const float2* MA = v.mean + p.ch[0] * v.mean_chan_stride;
    const float2* MB = v.mean + p.ch[1] * v.mean_chan_stride;
    const float2* MC = v.mean + p.ch[2] * v.mean_chan_stride;

    const int tid = threadIdx.x;
    const int ti = tid >> 4, tj = tid & 15;
    double acc[16][4];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q][0] = acc[q][1] = acc[q][2] = acc[q][3] = 0.0;

    // Column handled by this thread in the cooperative loads: 0..63 -> a_k,
    // 64..127 -> b_l, 128..254 -> c_{k+l}; 255 idle.
    const int col = tid;
    const float2* src = nullptr;
    const float2* msrc = nullptr;
    bool live = false;
    if (col < kTile) {
        live = k0 + col < p.Nf;
        src = A + k0 + col;
        msrc = MA + k0 + col;
    } else if (col < 2 * kTile) {
        live = l0 + col - kTile < p.Nf;
        src = B + l0 + col - kTile;
        msrc = MB + l0 + col - kTile;
    } else if (col < 4 * kTile - 1) {
        live = k0 + l0 + col - 2 * kTile < v.K;
        src = C + k0 + l0 + col - 2 * kTile;
        msrc = MC + k0 + l0 + col - 2 * kTile;
    }

#pragma unroll 1
    for (int c = c0; c < c1; ++c) {
        const float2 m_here = live ? msrc[(int64_t)(c - v.mean_chunk0) * v.K] : make_float2(0.f, 0.f);
        const int64_t fbase = (int64_t)(c - v.coef_chunk0) * v.m * v.K;
        float tr[16], tim[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) tr[q] = tim[q] = 0.f;

#pragma unroll 1
        for (int fb = 0; fb < v.m; fb += kFrameBatch) {
            const int nf = min(kFrameBatch, v.m - fb);
            __syncthreads();
            for (int f = 0; f < nf; ++f) {
                float2 x = live ? ld_centred(src + fbase + (int64_t)(fb + f) * v.K, m_here)
                                : make_float2(0.f, 0.f);
                if (col < kTile) {
                    sA[f][col] = x;
                } else if (col < 2 * kTile) {
                    sB[f][col - kTile] = x;
                } else if (col < 4 * kTile - 1) {
                    sC[f][col - 2 * kTile] = make_float2(x.x, -x.y);   // conjugate
                }
            }
            __syncthreads();
#pragma unroll 1
            for (int f = 0; f < nf; ++f) {
                float2 a[4], b[4], cc[7];
#pragma unroll
                for (int u = 0; u < 4; ++u) a[u] = sA[f][ti + 16 * u];
#pragma unroll
                for (int u = 0; u < 4; ++u) b[u] = sB[f][tj + 16 * u];
#pragma unroll
                for (int w = 0; w < 7; ++w) cc[w] = sC[f][ti + tj + 16 * w];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        const float pr = a[u].x * b[w].x - a[u].y * b[w].y;
                        const float pi = a[u].x * b[w].y + a[u].y * b[w].x;
                        const float2 z = cc[u + w];
                        tr[u * 4 + w] += pr * z.x - pi * z.y;
                        tim[u * 4 + w] += pr * z.y + pi * z.x;
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const double re = tr[q], im = tim[q];
            acc[q][0] += re;
            acc[q][1] += im;
            acc[q][2] += re * re;
            acc[q][3] += im * im;
        }
    }

    double* o = p.part + ((int64_t)split * p.n_tiles + tile) * 4 * (kTile * kTile);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int idx = (ti + 16 * u) * kTile + tj + 16 * w;
#pragma unroll
            for (int comp = 0; comp < 4; ++comp) {
                double val = acc[u * 4 + w][comp];
                if (p.accumulate) val += o[comp * kTile * kTile + idx];
                o[comp * kTile * kTile + idx] = val;
            }
        }
    }
}

// ------------------------------------------------------------------ S4, one channel
// Plain FP32 vector arithmetic for the frame sums; FP64 for the combination
// and the chunk sums.  Partials hold (sum v, sum v^2) with
// v = M4 - gamma (p_k p_l + 2(X^2+Y^2+U^2+V^2)), gamma = (m-1)/(m(m+1)).
constexpr int kS4Threads = 256;

__global__ __launch_bounds__(kS4Threads, 2) void k_s4_single(GridArgs p) {
    __shared__ float2 sA[kFrameBatch][kTile];
    __shared__ float2 sB[kFrameBatch][kTile];

    int split, tile;
    if (!xcd_work_item(p.n_tiles, p.n_split, split, tile)) return;
    int c0, c1;
    split_range(p.chunk0, p.chunk1, p.n_split, split, c0, c1);
    const int2 t = p.tiles[tile];
    const int k0 = t.x * kTile, l0 = t.y * kTile;
    const CoefView& v = p.v;
    const float2* A = v.coef + p.ch[0] * v.coef_chan_stride;
    const float2* MA = v.mean + p.ch[0] * v.mean_chan_stride;

    const int tid = threadIdx.x;
    const int ti = tid >> 4, tj = tid & 15;
    double acc[16][2];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q][0] = acc[q][1] = 0.0;

    const int col = tid;
    bool live = false;
    const float2* src = nullptr;
    const float2* msrc = nullptr;
    if (col < kTile) {
        live = k0 + col < p.Nf;
        src = A + k0 + col;
        msrc = MA + k0 + col;
    } else if (col < 2 * kTile) {
        live = l0 + col - kTile < p.Nf;
        src = A + l0 + col - kTile;
        msrc = MA + l0 + col - kTile;
    }
    const double gamma = p.gamma;

#pragma unroll 1
    for (int c = c0; c < c1; ++c) {
        const float2 m_here = live ? msrc[(int64_t)(c - v.mean_chunk0) * v.K] : make_float2(0.f, 0.f);
        const int64_t fbase = (int64_t)(c - v.coef_chunk0) * v.m * v.K;
        float X[16], Y[16], U[16], V[16], M4[16], pk[4], pl[4];
#pragma unroll
        for (int q = 0; q < 16; ++q) X[q] = Y[q] = U[q] = V[q] = M4[q] = 0.f;
#pragma unroll
        for (int u = 0; u < 4; ++u) pk[u] = pl[u] = 0.f;

#pragma unroll 1
        for (int fb = 0; fb < v.m; fb += kFrameBatch) {
            const int nf = min(kFrameBatch, v.m - fb);
            __syncthreads();
            if (col < 2 * kTile) {
                for (int f = 0; f < nf; ++f) {
                    float2 x = live ? ld_centred(src + fbase + (int64_t)(fb + f) * v.K, m_here)
                                    : make_float2(0.f, 0.f);
                    if (col < kTile) sA[f][col] = x;
                    else sB[f][col - kTile] = x;
                }
            }
            __syncthreads();
#pragma unroll 1
            for (int f = 0; f < nf; ++f) {
                float2 a[4], b[4];
                float Pa[4], Pb[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a[u] = sA[f][ti + 16 * u];
                    b[u] = sB[f][tj + 16 * u];
                    Pa[u] = a[u].x * a[u].x + a[u].y * a[u].y;
                    Pb[u] = b[u].x * b[u].x + b[u].y * b[u].y;
                    pk[u] += Pa[u];
                    pl[u] += Pb[u];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        const int q = u * 4 + w;
                        X[q] += a[u].x * b[w].x;
                        Y[q] += a[u].y * b[w].y;
                        U[q] += a[u].x * b[w].y;
                        V[q] += a[u].y * b[w].x;
                        M4[q] += Pa[u] * Pb[w];
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int q = u * 4 + w;
                const double x = X[q], y = Y[q], uu = U[q], vv = V[q];
                const double sq = x * x + y * y + uu * uu + vv * vv;
                const double val = (double)M4[q] - gamma * ((double)pk[u] * (double)pl[w] + 2.0 * sq);
                acc[q][0] += val;
                acc[q][1] += val * val;
            }
        }
    }

    double* o = p.part + ((int64_t)split * p.n_tiles + tile) * 2 * (kTile * kTile);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int idx = (ti + 16 * u) * kTile + tj + 16 * w;
#pragma unroll
            for (int comp = 0; comp < 2; ++comp) {
                double val = acc[u * 4 + w][comp];
                if (p.accumulate) val += o[comp * kTile * kTile + idx];
                o[comp * kTile * kTile + idx] = val;
            }
        }
    }
}

int blocks_per_cu(const void* fn, int threads) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, threads, 0) != hipSuccess || n < 1) n = 1;
    return n;
}

}  // namespace

hipError_t launch_s2(const S2Args& a, hipStream_t s) {
    if (a.chunk1 <= a.chunk0) return hipSuccess;
    dim3 grid((a.Nf + 255) / 256, a.n_split);
    k_s2<<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_s3(const GridArgs& a, hipStream_t s) {
    if (a.chunk1 <= a.chunk0) return hipSuccess;
    const int total = a.n_tiles * a.n_split;
    dim3 grid(((total + 7) / 8) * 8);
    k_s3<<<grid, kS3Threads, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_s4_single(const GridArgs& a, hipStream_t s) {
    if (a.chunk1 <= a.chunk0) return hipSuccess;
    const int total = a.n_tiles * a.n_split;
    dim3 grid(((total + 7) / 8) * 8);
    k_s4_single<<<grid, kS4Threads, 0, s>>>(a);
    return hipGetLastError();
}

int s3_blocks_per_cu() { return blocks_per_cu(reinterpret_cast<const void*>(&k_s3), kS3Threads); }
int s4_blocks_per_cu() { return blocks_per_cu(reinterpret_cast<const void*>(&k_s4_single), kS4Threads); }

}  // namespace ps
