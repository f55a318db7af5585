// Per-chunk moment sums, k-statistic combination and FP64 chunk accumulation
// (Sections 3, 4, 4.1, 4.2 and 7; the centred form of Appendix H).
//
// Inputs are the chunk-centred coefficients a' = a - mean_f a of stage a1
// (centred in place by launch_centre).  For a chunk of m frames (sums over f):
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
// Work: each stage is one launch over every segment (record x combination);
// a block takes its share of the segment's (tile, chunk) units as described at
// Sched (whole tiles in rounds, plus one stream-K run over the remaining
// tiles) and writes one partial-sum slot per piece (no atomics: the reduction
// order is fixed).  Consecutive block ids are dealt round-robin over the 8 XCDs
// by the hardware; the ids are remapped so that each XCD sees a contiguous
// range of blocks: the tiles of one round on one XCD then walk the same chunks
// at the same time and share their coefficients in that XCD's L2.
#include <type_traits>

#include "ps_internal.h"

namespace ps {
namespace {

// A block's share of its segment.
struct Block {
    const Seg* s;
    Sched sc;
    int64_t j;              // block index within the segment
    int64_t v, v1;          // remaining units of the block's stream-K run
    int64_t round;          // next whole-tile round
    int cbase;              // record chunk of the segment's chunk 0 in this launch
};

// One piece of work: a tile and a range of its chunks.
struct Item {
    int tile, c0, c1;       // c0, c1: record chunk indices
    int k0, l0;
    int ch[4];
    double* part;           // partial-sum slot of the piece
};

// Coefficients of the item's record: chunk c, frame f, column k of channel ch
// is at coef[ch * cs + off + (c m + f) K + k].
// `coef` points at the coefficient of grid index 0 of the first factors:
// column col0 of the region (0 for real signals; for complex signals grid
// index k' is bin k' - (N_f - 1), stored at column k' + col0).  S3's third
// factor, bin k + l, sits at column k' + l' + col3 (col3 = 0 unless an S4
// plane widened the stored bin range).
struct View {
    const float2* coef;
    int64_t cs, off;
    int K, m, Nf, col0, col3;
};

__device__ __forceinline__ bool resolve_block(const BatchArgs& b, Block& bk, View& v) {
    const int64_t per_xcd = (b.n_items + 7) >> 3;
    const int64_t x = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (x >= b.n_items) return false;
    const Seg& s = b.segs[find_seg(b.segs, b.n_segs, x)];
    bk.s = &s;
    bk.j = x - s.item0;
    int64_t cb = 0, ce = s.n_chunks;
    if (b.per_chunk) {
        cb = max(cb, (int64_t)b.win_lo);
        ce = min(ce, (int64_t)b.win_hi);
    }
    if (ce <= cb) return false;
    bk.cbase = (int)cb;
    bk.sc = Sched{s.n_tiles, ce - cb, s.blocks};
    bk.v = bk.sc.run_begin(bk.j);
    bk.v1 = bk.sc.run_begin(bk.j + 1);
    bk.round = 0;
    v.coef = b.coef + b.col0;
    v.col0 = b.col0;
    v.col3 = b.col3;
    v.cs = s.cs;
    // (per-chunk schedule: the segment's block holds chunk win_lo at row 0)
    v.off = s.coef - (b.per_chunk ? (int64_t)b.win_lo * b.m * s.K : 0);
    v.K = s.K;
    v.m = b.m;
    v.Nf = s.Nf;
    return true;
}

// Next piece of the block: first its run, then its whole tiles.  Uniform over
// the block.  EDGE = tile edge (0: 256-wide k blocks of S2), NCOMP = partial
// components per grid point.
template <int EDGE, int NCOMP>
__device__ __forceinline__ bool next_item(const BatchArgs& b, Block& bk, Item& it) {
    const Seg& s = *bk.s;
    int64_t t, c0, c1, slot;
    if (bk.v < bk.v1) {
        const int64_t T1 = bk.sc.T1(), W = bk.sc.W;
        t = T1 + bk.v / W;
        c0 = bk.v % W;
        c1 = min(W, c0 + (bk.v1 - bk.v));
        slot = T1 + bk.j + (t - T1);
        bk.v += c1 - c0;
    } else if (bk.round < bk.sc.rounds()) {
        t = bk.round * bk.sc.B + bk.j;
        c0 = 0;
        c1 = bk.sc.W;
        slot = t;
        ++bk.round;
    } else {
        return false;
    }
    it.tile = (int)t;
    it.c0 = bk.cbase + (int)c0;
    it.c1 = bk.cbase + (int)c1;
    if (EDGE > 0) {
        const int2 tt = s.tile_tab[t];
        it.k0 = tt.x * EDGE;
        it.l0 = tt.y * EDGE;
        it.part = b.part + s.part + slot * NCOMP * EDGE * EDGE;
    } else {
        it.k0 = (int)t * 256;
        it.l0 = 0;
        it.part = b.part + s.part + slot * NCOMP * 256;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) it.ch[q] = s.ch[q];
    return true;
}

// ------------------------------------------------------------------ S2
// For one channel, chunks of up to kS2Regs frames are loaded whole before
// their products (one round trip to memory per chunk, not one per frame); a
// pair of channels keeps the per-frame loop (its two register arrays would
// cost occupancy for a kernel of a few microseconds).
constexpr int kS2Regs = 16;

__global__ __launch_bounds__(256) void k_s2(BatchArgs p) {
    Block bk;
    View v;
    if (!resolve_block(p, bk, v)) return;
    Item it;
    while (next_item<0, 4>(p, bk, it)) {
        // Lanes past the grid write zero sums: every lane's slots are read
        // when a running accumulation adds them to its state.
        const int k = it.k0 + threadIdx.x;
        const int c_end = k < v.Nf ? it.c1 : it.c0;
        const float2* A = v.coef + it.ch[0] * v.cs;
        const float2* B = v.coef + it.ch[1] * v.cs;
        const bool same = it.ch[0] == it.ch[1];      // S2 of one channel: one load per frame
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        for (int c = it.c0; c < c_end; ++c) {
            const int64_t base = v.off + (int64_t)c * v.m * v.K + k;
            float re = 0.f, im = 0.f;
            if (v.m <= kS2Regs && same) {
                // all loads of the chunk in flight at once; x conj(x) = |x|^2
                float2 x[kS2Regs];
#pragma unroll
                for (int f = 0; f < kS2Regs; ++f)
                    if (f < v.m) x[f] = A[base + (int64_t)f * v.K];
#pragma unroll
                for (int f = 0; f < kS2Regs; ++f)
                    if (f < v.m) re += x[f].x * x[f].x + x[f].y * x[f].y;
            } else {
                for (int f = 0; f < v.m; ++f) {
                    const float2 x = A[base + (int64_t)f * v.K];
                    const float2 y = B[base + (int64_t)f * v.K];
                    re += x.x * y.x + x.y * y.y;   // x * conj(y)
                    im += x.y * y.x - x.x * y.y;
                }
            }
            s0 += re;
            s1 += im;
            s2 += (double)re * re;
            s3 += (double)im * im;
        }
        double* o = it.part + threadIdx.x;
        if (p.accumulate) {
            s0 += o[0];
            s1 += o[256];
            s2 += o[512];
            s3 += o[768];
        }
        o[0] = s0;
        o[256] = s1;
        o[512] = s2;
        o[768] = s3;
    }
}

// ------------------------------------------------------------------ S3
// Thread (ti, tj) = (tid / 16, tid % 16) owns the grid points
// (k0 + ti + 16u, l0 + tj + 16v), u, v < 4, whose third factor sits at
// k + l = k0 + l0 + ti + tj + 16(u + v).  Per frame it reads 4 + 4 + 7 values
// from LDS and does 16 complex triple products as 2 multiplies + 6 FMAs each.
// Frames are staged through LDS in batches of FB; the next batch is fetched
// into registers while the current one is being multiplied.  On a diagonal
// tile of a symmetric spectrum (k0 == l0) the points with u > v lie below the
// diagonal (k > l), which the finalize never reads: that form skips them.
constexpr int kS3Threads = 256;

// One piece of work (a tile and a range of its chunks) of k_s3.
template <int FB, bool DIAG>
__device__ __forceinline__ void s3_item(const BatchArgs& p, const View& v, const Item& it, float2 (*sA)[kTile],
                                        float2 (*sB)[kTile], float2 (*sC)[2 * kTile]) {
    const int c0 = it.c0, c1 = it.c1;
    const int k0 = it.k0, l0 = it.l0;

    const int tid = threadIdx.x;
    const int ti = tid >> 4, tj = tid & 15;
    double acc[16][4];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q][0] = acc[q][1] = acc[q][2] = acc[q][3] = 0.0;

    // Loader role: column 0..63 -> a_k, 64..127 -> b_l, 128..254 -> c_{k+l}; 255 idle.
    const int col = tid;
    const float2* src = nullptr;
    bool live = false;
    if (col < kTile) {
        live = k0 + col < v.Nf;
        src = v.coef + it.ch[0] * v.cs + k0 + col;
    } else if (col < 2 * kTile) {
        live = l0 + col - kTile < v.Nf;
        src = v.coef + it.ch[1] * v.cs + l0 + col - kTile;
    } else if (col < 4 * kTile - 1) {
        live = k0 + l0 + col - 2 * kTile < 2 * v.Nf - 1;      // grid sums k' + l' <= 2 (Ng - 1)
        src = v.coef - v.col0 + v.col3 + it.ch[2] * v.cs + k0 + l0 + col - 2 * kTile;
    }

    const int per_chunk = (v.m + FB - 1) / FB;
    const int n_batches = (c1 - c0) * per_chunk;
    float2 pre[FB];
    auto fetch = [&](int b) {
        const int c = c0 + b / per_chunk;
        const int fb = (b % per_chunk) * FB;
        const int nf = min(FB, v.m - fb);
        const float2* q = src + v.off + ((int64_t)c * v.m + fb) * v.K;
#pragma unroll
        for (int f = 0; f < FB; ++f)
            pre[f] = (live && f < nf) ? q[(int64_t)f * v.K] : make_float2(0.f, 0.f);
    };
    if (n_batches > 0) fetch(0);

    float tr[16], tm[16];
#pragma unroll 1
    for (int b = 0; b < n_batches; ++b) {
        const int fbi = b % per_chunk;
        const int nf = min(FB, v.m - fbi * FB);
        if (fbi == 0) {
#pragma unroll
            for (int q = 0; q < 16; ++q) tr[q] = tm[q] = 0.f;
        }
        lds_barrier();
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            if (col < kTile) sA[f][col] = pre[f];
            else if (col < 2 * kTile) sB[f][col - kTile] = pre[f];
            else if (col < 4 * kTile - 1) sC[f][col - 2 * kTile] = pre[f];
        }
        lds_barrier();
        if (b + 1 < n_batches) fetch(b + 1);
#pragma unroll 2
        for (int f = 0; f < nf; ++f) {
            float2 a[4], bb[4], cc[7];
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = sA[f][ti + 16 * u];
#pragma unroll
            for (int u = 0; u < 4; ++u) bb[u] = sB[f][tj + 16 * u];
#pragma unroll
            for (int w = 0; w < 7; ++w) cc[w] = sC[f][ti + tj + 16 * w];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    if (DIAG && u > w) continue;
                    // p = a b;  T3 += p * conj(c)
                    const float pr = fmaf(a[u].x, bb[w].x, -(a[u].y * bb[w].y));
                    const float pi = fmaf(a[u].x, bb[w].y, a[u].y * bb[w].x);
                    const float2 z = cc[u + w];
                    float r = fmaf(pr, z.x, tr[u * 4 + w]);
                    tr[u * 4 + w] = fmaf(pi, z.y, r);
                    float m = fmaf(pi, z.x, tm[u * 4 + w]);
                    tm[u * 4 + w] = fmaf(-pr, z.y, m);
                }
            }
        }
        if (fbi == per_chunk - 1) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                if (DIAG && (q >> 2) > (q & 3)) continue;
                const double re = tr[q], im = tm[q];
                acc[q][0] += re;
                acc[q][1] += im;
                acc[q][2] = fma(re, re, acc[q][2]);
                acc[q][3] = fma(im, im, acc[q][3]);
            }
        }
    }

    double* o = it.part;
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

template <int FB>
__global__ __launch_bounds__(kS3Threads, 2) void k_s3(BatchArgs p) {
    __shared__ float2 sA[FB][kTile];
    __shared__ float2 sB[FB][kTile];
    __shared__ float2 sC[FB][2 * kTile];

    Block bk;
    View v;
    if (!resolve_block(p, bk, v)) return;
    Item it;
    while (next_item<kTile, 4>(p, bk, it)) {
        if (bk.s->tiles == kSym64 && it.k0 == it.l0) s3_item<FB, true>(p, v, it, sA, sB, sC);
        else s3_item<FB, false>(p, v, it, sA, sB, sC);
    }
}

// ------------------------------------------------------------------ S4, one channel
// Plain FP32 vector arithmetic for the frame sums; FP64 for the combination
// and the chunk sums.  Partials hold (sum v, sum v^2) with
// v = M4 - gamma (p_k p_l + 2(X^2+Y^2+U^2+V^2)), gamma = (m-1)/(m(m+1)) for the
// k-statistic (1/m for the natural estimator).
constexpr int kS4Threads = 256;

__global__ __launch_bounds__(kS4Threads, 2) void k_s4_single(BatchArgs p) {
    __shared__ float2 sA[kFrameBatch][kTile];
    __shared__ float2 sB[kFrameBatch][kTile];

    Block bk;
    View v;
    if (!resolve_block(p, bk, v)) return;
    Item it;
    while (next_item<kTile, 2>(p, bk, it)) {
    const int c0 = it.c0, c1 = it.c1;
    const int k0 = it.k0, l0 = it.l0;
    const float2* A = v.coef + it.ch[0] * v.cs;

    const int tid = threadIdx.x;
    const int ti = tid >> 4, tj = tid & 15;
    double acc[16][2];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q][0] = acc[q][1] = 0.0;

    const int col = tid;
    bool live = false;
    const float2* src = nullptr;
    if (col < kTile) {
        live = k0 + col < v.Nf;
        src = A + k0 + col;
    } else if (col < 2 * kTile) {
        live = l0 + col - kTile < v.Nf;
        src = A + l0 + col - kTile;
    }
    const double gamma = p.gamma;

#pragma unroll 1
    for (int c = c0; c < c1; ++c) {
        const int64_t fbase = v.off + (int64_t)c * v.m * v.K;
        float X[16], Y[16], U[16], V[16], M4[16], pk[4], pl[4];
#pragma unroll
        for (int q = 0; q < 16; ++q) X[q] = Y[q] = U[q] = V[q] = M4[q] = 0.f;
#pragma unroll
        for (int u = 0; u < 4; ++u) pk[u] = pl[u] = 0.f;

#pragma unroll 1
        for (int fb = 0; fb < v.m; fb += kFrameBatch) {
            const int nf = min(kFrameBatch, v.m - fb);
            lds_barrier();
            if (col < 2 * kTile) {
                for (int f = 0; f < nf; ++f) {
                    const float2 x = live ? src[fbase + (int64_t)(fb + f) * v.K] : make_float2(0.f, 0.f);
                    if (col < kTile) sA[f][col] = x;
                    else sB[f][col - kTile] = x;
                }
            }
            lds_barrier();
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

    double* o = it.part;
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
}

// ------------------------------------------------------------------ S4, one channel, matrix cores
// The same sums as k_s4_single, with the frame contractions on the matrix
// cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation).  Each FP32 operand x is
// split into three bfloat16 terms x = h + m + l, each rounded to nearest
// (h = bf16(x), m = bf16(x - h), l = bf16(x - h - m); both differences are
// exact), so |x - h - m - l| <= 2^-25 |x|.  The six products
// h.h + h.m + m.h + h.l + l.h + m.m lie side by side along the contraction
// dimension: per frame f the k-side operand row holds [h h m h l m] and the
// l-side row [h m h l h m] at positions 6f..6f+5, so one contraction over
// 6 x 10 frames (padded to 64) yields the frame sum to ~2^-23 relative (the
// dropped m.l + l.m + l.l are below 2^-23 |x y|).  One packed conversion per
// 32-bit word gives the words directly: k side bf16x2(x, x) = [h h],
// bf16x2(x - h, x) = [m h], bf16x2(x - h - m, x - h) = [l m]; l side
// [h m], [h l], [h m] likewise.
//
// LDS holds, per batch of 10 frames, the operand rows of both sides: rows
// 0..63 Re, 64..127 Im, 128..191 P = |a'|^2 of the tile's 64 columns, 144 B
// apart (the 32-row, 16-byte-per-lane reads of the 32x32x16 operands are free
// of bank conflicts at that stride).  Wave w owns the 32 x 32 quadrant
// (k0 + 32 (w / 2), l0 + 32 (w % 2)) of the tile with five accumulators X, U,
// V, Y, M4, so all five sums of a grid point sit in the same lane and register
// and the k-statistic combination runs there.  The frame sums leave the matrix
// cores as FP32; the cancellation-prone combination (Section 4.1, eq. c4 in
// the centred form of Appendix H) is formed from them in FP64,
//   v = M4 - gamma (p_k p_l + 2 (X^2 + Y^2 + U^2 + V^2)),  gamma = (m-1)/(m(m+1)),
// with the squares, the product p_k p_l and the subtraction in double (gamma
// rounded to double biases v by at most 2^-53 of the subtracted term), then
// added to the FP64 chunk sums.  p_k and p_l are the FP32 frame sums of P,
// kept per column in LDS as doubles (the k side pre-multiplied by -gamma).
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float floatx2_t __attribute__((ext_vector_type(2)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));
typedef float floatx16_t __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

constexpr int kMfmaFrames = 10;      // frames per operand batch: 6 x 10 = 60 <= 64 slots
constexpr int kOpDw = 36;            // 32-bit words per LDS operand row (144 B; 32 used)
constexpr int kS4MThreads = 256;

// bf16x2 word (lo, hi), each rounded to nearest even.
__device__ __forceinline__ uint32_t pk_bf16(float lo, float hi) {
    const floatx2_t v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}
__device__ __forceinline__ float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// The three words of x for one frame slot: k side [h h][m h][l m] (SIDE 0),
// l side [h m][h l][h m] (SIDE 1; the third word equals the first).
template <int SIDE>
__device__ __forceinline__ void split_words(float x, uint32_t& w0, uint32_t& w1, uint32_t& w2) {
    const uint32_t hh = pk_bf16(x, x);
    const float r = x - bf_lo(hh);                        // x - h, exact
    if (SIDE == 0) {
        w0 = hh;
        w1 = pk_bf16(r, x);                               // [m h]
        const float s = r - bf_lo(w1);                    // x - h - m, exact
        w2 = pk_bf16(s, r);                               // [l m]
    } else {
        w0 = pk_bf16(x, r);                               // [h m]
        const float s = r - bf_hi(w0);
        w1 = pk_bf16(x, s);                               // [h l]
        w2 = w0;
    }
}

__device__ __forceinline__ float xor1(float v) {        // value of the neighbouring lane (lane ^ 1)
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}

// Stage one batch of this thread's frame slots (frames half + 2j) of column
// `col` into the operand rows of its side; returns the sum of P over them.
template <int SIDE>
__device__ __forceinline__ float stage_rows(uint32_t (*op)[kOpDw], int col, int half, const float2 (&pre)[kMfmaFrames / 2]) {
    float pa = 0.f;
#pragma unroll
    for (int j = 0; j < kMfmaFrames / 2; ++j) {
        const int f = half + 2 * j;
        const float re = pre[j].x, im = pre[j].y;
        const float P = fmaf(re, re, im * im);
        pa += P;
        uint32_t a0, a1, a2, b0, b1, b2, e0, e1, e2;
        split_words<SIDE>(re, a0, a1, a2);
        split_words<SIDE>(im, b0, b1, b2);
        split_words<SIDE>(P, e0, e1, e2);
        uint32_t* wr = &op[col][3 * f];
        uint32_t* wi = &op[kTile + col][3 * f];
        uint32_t* wp = &op[2 * kTile + col][3 * f];
        wr[0] = a0; wr[1] = a1; wr[2] = a2;
        wi[0] = b0; wi[1] = b1; wi[2] = b2;
        wp[0] = e0; wp[1] = e1; wp[2] = e2;
    }
    return pa;
}

// ONE_BATCH: every chunk fits one frame batch (m <= 10, compile-time).
template <bool ONE_BATCH>
__global__ __launch_bounds__(kS4MThreads, 2) void k_s4_mfma_bf16(BatchArgs p) {
    __shared__ __attribute__((aligned(16))) uint32_t opK[3 * kTile][kOpDw];
    __shared__ __attribute__((aligned(16))) uint32_t opL[3 * kTile][kOpDw];
    __shared__ double psum[2][kTile];          // -gamma p_k (k side), p_l (l side)

    Block bk;
    View v;
    if (!resolve_block(p, bk, v)) return;

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int r32 = lane & 31, kh = lane >> 5;
    const int rowK = 32 * (w >> 1) + r32, rowL = 32 * (w & 1) + r32;

    // Loader role: thread -> (side, column, half of the frame slots).  The LDS
    // serves a wave's 32-bit writes in two lane groups, {0-15, 32-47} and
    // {16-31, 48-63}; at the 144-byte row stride columns c and c + 16 share a
    // bank, so lanes 32-47 take columns 8-15 and lanes 16-31 columns 16-23:
    // each group then writes 16 consecutive columns, in distinct banks.
    const int side = __builtin_amdgcn_readfirstlane(tid >> 7);    // uniform per wave
    const int col = 32 * (w & 1) + (((lane >> 1) & 7) | (((lane >> 5) & 1) << 3) | (((lane >> 4) & 1) << 4));
    const int half = tid & 1;
    uint32_t(*op)[kOpDw] = side ? opL : opK;

    // Zero the padding words 30..31 of every row once; they are never written again.
    for (int r = tid; r < 2 * 3 * kTile; r += kS4MThreads) {
        uint32_t* row = (r < 3 * kTile) ? opK[r] : opL[r - 3 * kTile];
        row[3 * kMfmaFrames] = 0u;
        row[3 * kMfmaFrames + 1] = 0u;
    }
    const double gamma = p.gamma;                       // (m-1)/(m(m+1)) (natural: 1/m)
    const double m2g = -2.0 * gamma;

    Item it;
    while (next_item<kTile, 2>(p, bk, it)) {
    const int c0 = it.c0, c1 = it.c1;
    const int k0 = it.k0, l0 = it.l0;
    const int gcol = (side ? l0 : k0) + col;
    const bool live = gcol < v.Nf;
    const float2* src = v.coef + it.ch[0] * v.cs + gcol;

    double acc[16][2];
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r][0] = acc[r][1] = 0.0;

    constexpr int kSlots = kMfmaFrames / 2;       // frame slots of this thread: half + 2j
    const int per_chunk = (v.m + kMfmaFrames - 1) / kMfmaFrames;
    const int n_batches = (c1 - c0) * per_chunk;
    float2 pre[kSlots];
    auto fetch = [&](int b) {
        const int c = c0 + b / per_chunk;
        const int fb = (b % per_chunk) * kMfmaFrames;
        const int nf = min(kMfmaFrames, v.m - fb);
        const float2* q = src + v.off + ((int64_t)c * v.m + fb) * v.K;
#pragma unroll
        for (int j = 0; j < kSlots; ++j) {
            const int f = half + 2 * j;
            pre[j] = (live && f < nf) ? q[(int64_t)f * v.K] : make_float2(0.f, 0.f);
        }
    };
    if (n_batches > 0) fetch(0);

    floatx16_t d[5];
    float pacc = 0.f;
#pragma unroll 1
    for (int b = 0; b < n_batches; ++b) {
        const int fbi = ONE_BATCH ? 0 : b % per_chunk;
        const bool first = ONE_BATCH || fbi == 0, last = ONE_BATCH || fbi == per_chunk - 1;
        if (first) pacc = 0.f;
        lds_barrier();
        pacc += side == 0 ? stage_rows<0>(op, col, half, pre) : stage_rows<1>(op, col, half, pre);
        if (last) {
            const float tot = pacc + xor1(pacc);          // p over the chunk's frames (FP32 sum)
            if (half == 0) psum[side][col] = side == 0 ? -gamma * (double)tot : (double)tot;
        }
        lds_barrier();
        // Four K steps of 16 slots (the scheduling barrier keeps each step's
        // operand reads next to its contractions: fewer live registers).  The
        // wave runs them at raised priority, so that the matrix pipe is fed
        // while the other wave of the SIMD uses the vector ALU.
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int wo = 8 * ks + 4 * kh;                // first word of this lane's 8 slots
            const bf16x8_t aR = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4_t*>(&opK[rowK][wo]));
            const bf16x8_t aI = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4_t*>(&opK[kTile + rowK][wo]));
            const bf16x8_t aP = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4_t*>(&opK[2 * kTile + rowK][wo]));
            const bf16x8_t bR = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4_t*>(&opL[rowL][wo]));
            const bf16x8_t bI = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4_t*>(&opL[kTile + rowL][wo]));
            const bf16x8_t bP = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4_t*>(&opL[2 * kTile + rowL][wo]));
            if (first && ks == 0) {
                const floatx16_t z = {};
                d[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aR, bR, z, 0, 0, 0);   // X
                d[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aR, bI, z, 0, 0, 0);   // U
                d[2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aI, bR, z, 0, 0, 0);   // V
                d[3] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aI, bI, z, 0, 0, 0);   // Y
                d[4] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aP, bP, z, 0, 0, 0);   // M4
            } else {
                d[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aR, bR, d[0], 0, 0, 0);
                d[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aR, bI, d[1], 0, 0, 0);
                d[2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aI, bR, d[2], 0, 0, 0);
                d[3] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aI, bI, d[3], 0, 0, 0);
                d[4] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aP, bP, d[4], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        __builtin_amdgcn_s_setprio(0);
        // Next batch's loads overlap the epilogue.
        if (b + 1 < n_batches) fetch(b + 1);
        if (!last) continue;

        // Register r of lane (kh, r32) is grid point
        // k = k0 + 32 (w / 2) + 8 (r / 4) + 4 kh + r % 4, l = l0 + 32 (w % 2) + r32.
        // The k-statistic combination in FP64.
        const double pl = psum[1][rowL];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const double X = d[0][r], U = d[1][r], V = d[2][r], Y = d[3][r];
            const double sq = fma(X, X, fma(Y, Y, fma(U, U, V * V)));
            const double npk = psum[0][32 * (w >> 1) + 8 * (r >> 2) + 4 * kh + (r & 3)];
            const double val = fma(m2g, sq, fma(npk, pl, (double)d[4][r]));
            acc[r][0] += val;
            acc[r][1] = fma(val, val, acc[r][1]);
        }
    }

    double* o = it.part;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int idx = (32 * (w >> 1) + 8 * (r >> 2) + 4 * kh + (r & 3)) * kTile + 32 * (w & 1) + r32;
#pragma unroll
        for (int comp = 0; comp < 2; ++comp) {
            double val = acc[r][comp];
            if (p.accumulate) val += o[comp * kTile * kTile + idx];
            o[comp * kTile * kTile + idx] = val;
        }
    }
    }
}

// ------------------------------------------------------------------ S4, one channel, FP16 x 2 scaled
// The same sums on the matrix cores with v_mfma_f32_16x16x32_f16.  Per chunk
// and column, the values are scaled by a power of two s = 2^e with
// max_f(|Re|, |Im|) < s (exact), P by s^2, and split in two float16 terms
// x = h + l (h = fp16(x), l = fp16(x - h)): with |x/s| < 1 the representation
// error is below 2^-22 s, i.e. relative to the column's largest value.  The
// three products h.h + h.l + l.h sit along the contraction dimension, per frame
// [h h l] on the k side and [h l h] on the l side (slots 3f..3f+2, 30 of 32
// used), so one MFMA contraction per chunk yields the FP32-accurate sums;
// l.l (below 2^-22) is dropped.  The epilogue undoes the scales exactly:
// X, Y, U, V and M4 carry (s_k s_l)^2 after squaring / by construction.
typedef _Float16 halfx8_t __attribute__((ext_vector_type(8)));

constexpr int kF16Stride = 40;       // halves per LDS operand row (80 B: 16-B aligned, conflict-free)
constexpr int kF16Frames = 10;       // frames per operand batch: 3 x 10 = 30 <= 32

__device__ __forceinline__ uint32_t pack_h(_Float16 lo, _Float16 hi) {
    return (uint32_t)__builtin_bit_cast(unsigned short, lo) | ((uint32_t)__builtin_bit_cast(unsigned short, hi) << 16);
}

// Write the split terms of two consecutive frames (x0 at frame f, x1 at f+1)
// into an operand row: slots 3f .. 3f+5 = 12 bytes.
template <int SIDE>
__device__ __forceinline__ void put_pair_f16(unsigned short* row, int f, float x0, float x1) {
    const _Float16 h0 = (_Float16)x0, h1 = (_Float16)x1;
    const _Float16 l0 = (_Float16)(x0 - (float)h0), l1 = (_Float16)(x1 - (float)h1);
    uint32_t* w = reinterpret_cast<uint32_t*>(row + 3 * f);
    if (SIDE == 0) {            // [h0 h0 l0 | h1 h1 l1]
        w[0] = pack_h(h0, h0);
        w[1] = pack_h(l0, h1);
        w[2] = pack_h(h1, l1);
    } else {                    // [h0 l0 h0 | h1 l1 h1]
        w[0] = pack_h(h0, l0);
        w[1] = pack_h(h0, h1);
        w[2] = pack_h(l1, h1);
    }
}

__global__ __launch_bounds__(kS4MThreads, 2) void k_s4_mfma_f16(BatchArgs p) {
    __shared__ __attribute__((aligned(16))) unsigned short opK[3 * kTile][kF16Stride];
    __shared__ __attribute__((aligned(16))) unsigned short opL[3 * kTile][kF16Stride];
    __shared__ float psum[2][2][kTile];
    __shared__ float sc2[2][kTile];              // s^2 per column of each side

    Block bk;
    View v;
    if (!resolve_block(p, bk, v)) return;

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;

    // Loader role: thread -> (side, column, half); half 0 owns the frame pairs
    // (0,1), (4,5), (8,9), half 1 owns (2,3), (6,7).
    const int side = tid >> 7;
    const int col = (tid >> 1) & (kTile - 1);
    const int half = tid & 1;
    unsigned short(*op)[kF16Stride] = side ? opL : opK;

    // Zero the padding slots 30..31 of every row once.
    for (int r = tid; r < 2 * 3 * kTile; r += kS4MThreads) {
        unsigned short* row = (r < 3 * kTile) ? opK[r] : opL[r - 3 * kTile];
        *reinterpret_cast<uint32_t*>(row + 3 * kF16Frames) = 0u;
    }

    Item it;
    while (next_item<kTile, 2>(p, bk, it)) {
    const int c0 = it.c0, c1 = it.c1;
    const int k0 = it.k0, l0 = it.l0;
    const int gcol = (side ? l0 : k0) + col;
    const bool live = gcol < v.Nf;
    const float2* src = v.coef + it.ch[0] * v.cs + gcol;

    double acc[4][4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[a][e][0] = acc[a][e][1] = 0.0;
    const double gamma_d = p.gamma;

    constexpr int kPairs = 3;                 // pair slots per thread (half 1 uses 2)
    const int per_chunk = (v.m + kF16Frames - 1) / kF16Frames;
    const int n_batches = (c1 - c0) * per_chunk;
    float2 pre[2 * kPairs];
    auto fetch = [&](int b) {
        const int c = c0 + b / per_chunk;
        const int fb = (b % per_chunk) * kF16Frames;
        const int nf = min(kF16Frames, v.m - fb);
        const float2* q = src + v.off + ((int64_t)c * v.m + fb) * v.K;
#pragma unroll
        for (int j = 0; j < kPairs; ++j) {
            const int f = 2 * (half + 2 * j);
#pragma unroll
            for (int u = 0; u < 2; ++u)
                pre[2 * j + u] = (live && f + u < nf && f < kF16Frames) ? q[(int64_t)(f + u) * v.K]
                                                                        : make_float2(0.f, 0.f);
        }
    };
    if (n_batches > 0) fetch(0);

    floatx4_t d[4][5];
    float pacc = 0.f;
    const floatx4_t zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int b = 0; b < n_batches; ++b) {
        const int fbi = b % per_chunk;
        // Column scale (shared by the chunk's frame batches: the first batch sets it).
        float amax = 0.f;
#pragma unroll
        for (int j = 0; j < 2 * kPairs; ++j) amax = fmaxf(amax, fmaxf(fabsf(pre[j].x), fabsf(pre[j].y)));
        amax = fmaxf(amax, __shfl_xor(amax, 1));
        if (fbi == 0) pacc = 0.f;
        lds_barrier();
        if (fbi == 0 && half == 0) sc2[side][col] = pow2_above(amax) * pow2_above(amax);
        lds_barrier();
        const float s2 = sc2[side][col];
        const float inv_s = 1.0f / sqrtf(s2);       // exact: s is a power of two
        const float inv_s2 = 1.0f / s2;
#pragma unroll
        for (int j = 0; j < kPairs; ++j) {
            const int f = 2 * (half + 2 * j);
            if (f >= kF16Frames) break;
            const float2 a0 = pre[2 * j], a1 = pre[2 * j + 1];
            const float P0 = a0.x * a0.x + a0.y * a0.y, P1 = a1.x * a1.x + a1.y * a1.y;
            pacc += P0 + P1;
            if (side == 0) {
                put_pair_f16<0>(op[col], f, a0.x * inv_s, a1.x * inv_s);
                put_pair_f16<0>(op[kTile + col], f, a0.y * inv_s, a1.y * inv_s);
                put_pair_f16<0>(op[2 * kTile + col], f, P0 * inv_s2, P1 * inv_s2);
            } else {
                put_pair_f16<1>(op[col], f, a0.x * inv_s, a1.x * inv_s);
                put_pair_f16<1>(op[kTile + col], f, a0.y * inv_s, a1.y * inv_s);
                put_pair_f16<1>(op[2 * kTile + col], f, P0 * inv_s2, P1 * inv_s2);
            }
        }
        lds_barrier();
        {
            const int koff = lg * 8;
            const int rk = w * 16 + li;
            const halfx8_t aR = *reinterpret_cast<const halfx8_t*>(&opK[rk][koff]);
            const halfx8_t aI = *reinterpret_cast<const halfx8_t*>(&opK[kTile + rk][koff]);
            const halfx8_t aP = *reinterpret_cast<const halfx8_t*>(&opK[2 * kTile + rk][koff]);
            const bool z = fbi == 0;
#pragma unroll
            for (int lb = 0; lb < 4; ++lb) {
                const int rl = lb * 16 + li;
                const halfx8_t bR = *reinterpret_cast<const halfx8_t*>(&opL[rl][koff]);
                const halfx8_t bI = *reinterpret_cast<const halfx8_t*>(&opL[kTile + rl][koff]);
                const halfx8_t bP = *reinterpret_cast<const halfx8_t*>(&opL[2 * kTile + rl][koff]);
                d[lb][0] = __builtin_amdgcn_mfma_f32_16x16x32_f16(aR, bR, z ? zero : d[lb][0], 0, 0, 0);  // X
                d[lb][1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(aR, bI, z ? zero : d[lb][1], 0, 0, 0);  // U
                d[lb][2] = __builtin_amdgcn_mfma_f32_16x16x32_f16(aI, bR, z ? zero : d[lb][2], 0, 0, 0);  // V
                d[lb][3] = __builtin_amdgcn_mfma_f32_16x16x32_f16(aI, bI, z ? zero : d[lb][3], 0, 0, 0);  // Y
                d[lb][4] = __builtin_amdgcn_mfma_f32_16x16x32_f16(aP, bP, z ? zero : d[lb][4], 0, 0, 0);  // M4
            }
        }
        if (b + 1 < n_batches) fetch(b + 1);
        if (fbi != per_chunk - 1) continue;

        psum[side][half][col] = pacc;
        lds_barrier();
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int kl = w * 16 + 4 * lg + e;
            const float pk = psum[0][0][kl] + psum[0][1][kl];
            const float s2k = sc2[0][kl];
#pragma unroll
            for (int lb = 0; lb < 4; ++lb) {
                const int ll = lb * 16 + li;
                const float pl = psum[1][0][ll] + psum[1][1][ll];
                const float sig = s2k * sc2[1][ll];           // (s_k s_l)^2, a power of two
                const double X = d[lb][0][e], U = d[lb][1][e], V = d[lb][2][e], Y = d[lb][3][e];
                const double sq = fma(X, X, fma(Y, Y, fma(U, U, V * V)));
                const double q = fma(2.0 * (double)sig, sq, (double)pk * (double)pl);
                const double val = fma(-gamma_d, q, (double)d[lb][4][e] * (double)sig);
                acc[lb][e][0] += val;
                acc[lb][e][1] = fma(val, val, acc[lb][e][1]);
            }
        }
    }

    double* o = it.part;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
#pragma unroll
        for (int lb = 0; lb < 4; ++lb) {
            const int idx = (w * 16 + 4 * lg + e) * kTile + lb * 16 + li;
#pragma unroll
            for (int comp = 0; comp < 2; ++comp) {
                double val = acc[lb][e][comp];
                if (p.accumulate) val += o[comp * kTile * kTile + idx];
                o[comp * kTile * kTile + idx] = val;
            }
        }
    }
    }
}

// ------------------------------------------------------------------ S4, one channel, matrix cores, scaled FP16 x 2, pre-split operands
// The sums of k_s4_mfma_f16 from the operand records the centring pass writes
// (see kOpWords): per chunk and column a power of two s, the values scaled by
// s (P by s^2) and split in two float16 terms x = h + l, stored as the pieces
// H = h words 0..3, L = l words 0..3, T = (h word 4, l word 4, 0, 0) (a word
// holds two frames).  Each frame sum h_k h_l + h_k l_l + l_k h_l is one
// contraction of two K steps of v_mfma_f32_32x32x16_f16; the lanes of the
// lower and upper K half (kh) of step ks pair the k-side and l-side words
//   ks 0:  kh 0: H_k . H_l      kh 1: H_k . L_l
//   ks 1:  kh 0: L_k . H_l      kh 1: (h4 l4 h4 0)_k . (h4 h4 l4 0)_l
// so every operand is a staged piece read as it is (the lane picks the piece
// by its kh), or for kh 1 of step 1 a piece with one or two words taken from
// another lane half's position (a select per word).  64 x 64 tiles, four
// waves of 32 x 32.
//
// The records and the (p, s^2) pairs of a chunk travel from memory into one
// of kS4Stages LDS staging buffers by asynchronous copies issued
// kS4Stages - 1 chunks ahead; one workgroup barrier per chunk both publishes
// the chunk's copies and frees the buffer the previous chunk was read from.
// Staging reads are LDS reads in inline assembly with their wait in the same
// statement (see read_lds_ops): the compiler's own wait for copies in
// flight cannot tell the buffers apart and would drain all of them.
//
// With the scale sigma = s_k^2 s_l^2 (exact) of the point, M4 and
// X^2 + Y^2 + U^2 + V^2 of the scaled values are both sigma times the
// unscaled ones, so the chunk's term is
//   v = sigma (M4' - 2 gamma (X'^2 + Y'^2 + U'^2 + V'^2)) - gamma p_k p_l,
// formed in FP64 (p = sum_f P unscaled, FP32 from the centring pass, stored
// as FP64 with s^2); the sum of the four squares, positive terms, in FP32.

// Asynchronous copy of 16 bytes per lane from global memory into LDS: lane i
// writes lds + 16 i (lds uniform over the wave); completion is counted like a
// global load, in issue order.
__device__ __forceinline__ void copy_to_lds16(const void* g, void* lds) {
    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)g,
                                     (void __attribute__((address_space(3)))*)lds, 16, 0, 0);
}

// Workgroup barrier with copies still in flight: the caller has waited for
// what it needs; the empty asm statements keep the compiler from moving
// memory accesses across (and from adding a wait for the copies, as the LDS
// fence of lds_barrier can).
__device__ __forceinline__ void lds_sync() {
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    __asm__ volatile("" ::: "memory");
}
// Workgroup barrier after which every memory access the waves issued,
// copies included, is complete.  s_waitcnt fields on this target: vmcnt bits
// 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8.
__device__ __forceinline__ void copies_barrier() {
    __builtin_amdgcn_s_waitcnt(0x0070);        // vmcnt(0) lgkmcnt(0)
    lds_barrier();
}

typedef unsigned u32x4_v __attribute__((ext_vector_type(4)));
// 16-byte LDS reads at base + OFF (base: byte address in LDS, 16-byte
// aligned; OFF an immediate), complete when the statement ends.  The twelve
// operand reads of one chunk: four bases, three value offsets each.
template <unsigned O0, unsigned O1, unsigned O2>
__device__ __forceinline__ void read_lds_ops(unsigned aK0, unsigned aL0, unsigned aK1, unsigned aL1,
                                             u32x4_v (&x)[12]) {
    __asm__ volatile(
        "ds_read_b128 %0, %12 offset:%16\n\t"
        "ds_read_b128 %1, %12 offset:%17\n\t"
        "ds_read_b128 %2, %12 offset:%18\n\t"
        "ds_read_b128 %3, %13 offset:%16\n\t"
        "ds_read_b128 %4, %13 offset:%17\n\t"
        "ds_read_b128 %5, %13 offset:%18\n\t"
        "ds_read_b128 %6, %14 offset:%16\n\t"
        "ds_read_b128 %7, %14 offset:%17\n\t"
        "ds_read_b128 %8, %14 offset:%18\n\t"
        "ds_read_b128 %9, %15 offset:%16\n\t"
        "ds_read_b128 %10, %15 offset:%17\n\t"
        "ds_read_b128 %11, %15 offset:%18\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(x[0]), "=&v"(x[1]), "=&v"(x[2]), "=&v"(x[3]), "=&v"(x[4]), "=&v"(x[5]),
          "=&v"(x[6]), "=&v"(x[7]), "=&v"(x[8]), "=&v"(x[9]), "=&v"(x[10]), "=&v"(x[11])
        : "v"(aK0), "v"(aL0), "v"(aK1), "v"(aL1), "i"(O0), "i"(O1), "i"(O2)
        : "memory");
}
// Two runs of four consecutive 16-byte values, at base + OFF and base + OFF
// + 128, and (second form) one more at base2 + OFF2.
template <unsigned OFF>
__device__ __forceinline__ void read_lds_x8(unsigned base, u32x4_v (&x)[8]) {
    __asm__ volatile(
        "ds_read_b128 %0, %8 offset:%9\n\t"
        "ds_read_b128 %1, %8 offset:%10\n\t"
        "ds_read_b128 %2, %8 offset:%11\n\t"
        "ds_read_b128 %3, %8 offset:%12\n\t"
        "ds_read_b128 %4, %8 offset:%13\n\t"
        "ds_read_b128 %5, %8 offset:%14\n\t"
        "ds_read_b128 %6, %8 offset:%15\n\t"
        "ds_read_b128 %7, %8 offset:%16\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(x[0]), "=&v"(x[1]), "=&v"(x[2]), "=&v"(x[3]), "=&v"(x[4]), "=&v"(x[5]), "=&v"(x[6]), "=&v"(x[7])
        : "v"(base), "i"(OFF), "i"(OFF + 16), "i"(OFF + 32), "i"(OFF + 48),
          "i"(OFF + 128), "i"(OFF + 144), "i"(OFF + 160), "i"(OFF + 176)
        : "memory");
}
template <unsigned OFF, unsigned OFF2>
__device__ __forceinline__ void read_lds_x8_1(unsigned base, unsigned base2, u32x4_v (&x)[8], u32x4_v& y) {
    __asm__ volatile(
        "ds_read_b128 %0, %9 offset:%11\n\t"
        "ds_read_b128 %1, %9 offset:%12\n\t"
        "ds_read_b128 %2, %9 offset:%13\n\t"
        "ds_read_b128 %3, %9 offset:%14\n\t"
        "ds_read_b128 %4, %9 offset:%15\n\t"
        "ds_read_b128 %5, %9 offset:%16\n\t"
        "ds_read_b128 %6, %9 offset:%17\n\t"
        "ds_read_b128 %7, %9 offset:%18\n\t"
        "ds_read_b128 %8, %10 offset:%19\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(x[0]), "=&v"(x[1]), "=&v"(x[2]), "=&v"(x[3]), "=&v"(x[4]), "=&v"(x[5]), "=&v"(x[6]), "=&v"(x[7]),
          "=&v"(y)
        : "v"(base), "v"(base2), "i"(OFF), "i"(OFF + 16), "i"(OFF + 32), "i"(OFF + 48),
          "i"(OFF + 128), "i"(OFF + 144), "i"(OFF + 160), "i"(OFF + 176), "i"(OFF2)
        : "memory");
}

// The wave's copy of a value the compiler cannot prove uniform (it is):
// uniform addresses let a copy take a scalar base and the lane's offset.
__device__ __forceinline__ const char* wave_uniform(const void* p) {
    const uint64_t u = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return reinterpret_cast<const char*>(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ unsigned lds_addr(const void* p) {
    return (unsigned)(size_t)(const __attribute__((address_space(3))) char*)p;
}

constexpr int kS4Stages = 3;            // staging buffers: copies kS4Stages - 1 chunks ahead
constexpr int kS4CopiesPerWave = 5;     // copies per wave and chunk (see copy_chunk)

// One chunk's staged operands of a 64 x 64 tile.
struct S4Stage {
    uint4 rec[2][3][kOpPieces][kTile];  // [side k, l][value Re, Im, P][piece H, L, T][column]
    double2 pw[2][kTile];               // [side][column]: (p, s^2)
};

__global__ __launch_bounds__(kS4MThreads, 2) void k_s4_mfma_f16_pre(BatchArgs p) {
    __shared__ __attribute__((aligned(16))) S4Stage stage[kS4Stages];

    Block bk;
    View v;
    if (!resolve_block(p, bk, v)) return;

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int r32 = lane & 31, kh = lane >> 5;
    const int rowK = 32 * (w >> 1) + r32, rowL = 32 * (w & 1) + r32;
    const int wv = __builtin_amdgcn_readfirstlane(w);
    const double gamma = p.gamma;
    const double m2g = -2.0 * gamma;
    // Records: 3 kOpWords ngp words per chunk; value v, piece i of column k
    // is the 16-byte unit (3 v + i) ngp + k of the chunk's block; the (p, s^2)
    // pairs: ngp per chunk.
    const int64_t ngp = (int64_t)(v.Nf + kTile - 1) / kTile * kTile;
    const int64_t cunits = 3 * kOpPieces * ngp;                    // 16-byte units per chunk
    const int64_t cbase = p.per_chunk ? -(int64_t)p.win_lo : 0;   // per-chunk schedule: chunk win_lo at 0
    const uint32_t lane16 = 16u * lane;

    // Lane addresses of its operands and pair values in stage 0 (stage b is
    // b sizeof(S4Stage) further, an immediate offset of the reads): step 0
    // reads piece H of its k-side column and piece H (kh 0) or L (kh 1) of
    // its l-side column, step 1 piece L or T of the k side and H or T of the
    // l side, each for Re, Im, P.
    const unsigned aK0 = lds_addr(&stage[0].rec[0][0][0][rowK]);
    const unsigned aK1 = lds_addr(&stage[0].rec[0][0][1 + kh][rowK]);
    const unsigned aL0 = lds_addr(&stage[0].rec[1][0][kh][rowL]);
    const unsigned aL1 = lds_addr(&stage[0].rec[1][0][2 * kh][rowL]);
    constexpr unsigned kValBytes = kOpPieces * kTile * sizeof(uint4);
    const unsigned aPk = lds_addr(&stage[0].pw[0][32 * (w >> 1) + 4 * kh]);
    const unsigned aPl = lds_addr(&stage[0].pw[1][rowL]);
    static_assert(sizeof(S4Stage) % 16 == 0, "stage alignment");
    static_assert((kS4Stages - 1) * sizeof(S4Stage) + 2 * kValBytes < 65536 &&
                  (kS4Stages - 1) * sizeof(S4Stage) + 24 * 16 + 176 < 65536,
                  "LDS read offsets are 16-bit immediates");

    Item it;
    while (next_item<kTile, 2>(p, bk, it)) {
    const Seg& sg = *bk.s;
    const int c0 = it.c0, c1 = it.c1;          // c1 > c0: pieces are never empty
    const int k0 = __builtin_amdgcn_readfirstlane(it.k0), l0 = __builtin_amdgcn_readfirstlane(it.l0);
    const char* base = wave_uniform(p.op4 + it.ch[0] * sg.op4_cs + sg.op4);
    const char* pbase = wave_uniform(p.p4 + it.ch[0] * sg.p4_cs + sg.p4);

    // Copy of chunk c into stage b: 18 record copies (side, value, piece) and
    // the two sides' (p, s^2) pairs, 64 columns of 16 bytes each; wave wv
    // issues records wv, wv + 4, wv + 8, wv + 12, then record 16 + wv (waves
    // 0, 1) or side wv - 2's pairs (waves 2, 3): kS4CopiesPerWave each.
    // Copies past the piece's last chunk repeat it (into a buffer no step
    // reads), so that every path issues the same copies.
    auto copy_chunk = [&](int b, int c) {
        c = min(c, c1 - 1);
        S4Stage& st = stage[b];
        const char* rc = base + (cbase + c) * cunits * (int64_t)sizeof(uint4);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int q = wv + 4 * j;
            const int side = q / (3 * kOpPieces), vp = q % (3 * kOpPieces);
            const char* g = rc + ((int64_t)vp * ngp + (side ? l0 : k0)) * (int64_t)sizeof(uint4);
            copy_to_lds16(g + lane16, &st.rec[side][0][0][0] + vp * kTile);
        }
        if (wv < 2) {
            const int vp = 7 + wv;                             // records 16, 17: l side, value 2, pieces 1, 2
            const char* g = rc + ((int64_t)vp * ngp + l0) * (int64_t)sizeof(uint4);
            copy_to_lds16(g + lane16, &st.rec[1][0][0][0] + vp * kTile);
        } else {
            const int side = wv - 2;
            const char* g = pbase + ((cbase + c) * ngp + (side ? l0 : k0)) * (int64_t)sizeof(double2);
            copy_to_lds16(g + lane16, &st.pw[side][0]);
        }
    };

    double acc[16][2];
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r][0] = acc[r][1] = 0.0;

    // Chunk c from stage B (a compile-time index, so that every LDS read
    // offset is an immediate).
    auto step = [&](auto B, int c) {
        constexpr int b = decltype(B)::value;
        constexpr unsigned so = b * sizeof(S4Stage);
        // Chunk c's copies have landed once at most the next kS4Stages - 2
        // chunks' copies are in flight (each wave waits for its own, the
        // barrier for the others'); the barrier also frees the stage chunk
        // c - 1 was read from, which takes chunk c + kS4Stages - 1.
        static_assert(kS4Stages == 3 && kS4CopiesPerWave == 5, "the vmcnt below counts 5 copies in flight");
        __builtin_amdgcn_s_waitcnt(0x0075);                            // vmcnt(5) lgkmcnt(0)
        lds_sync();
        copy_chunk(b == 0 ? kS4Stages - 1 : b - 1, c + kS4Stages - 1);

        u32x4_v op[12];
        read_lds_ops<so, so + kValBytes, so + 2 * kValBytes>(aK0, aL0, aK1, aL1, op);
        floatx16_t d[5];
        {
            const floatx16_t z = {};
            const halfx8_t aR = __builtin_bit_cast(halfx8_t, op[0]), aI = __builtin_bit_cast(halfx8_t, op[1]),
                           aP = __builtin_bit_cast(halfx8_t, op[2]);
            const halfx8_t bR = __builtin_bit_cast(halfx8_t, op[3]), bI = __builtin_bit_cast(halfx8_t, op[4]),
                           bP = __builtin_bit_cast(halfx8_t, op[5]);
            d[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(aR, bR, z, 0, 0, 0);     // X
            d[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(aR, bI, z, 0, 0, 0);     // U
            d[2] = __builtin_amdgcn_mfma_f32_32x32x16_f16(aI, bR, z, 0, 0, 0);     // V
            d[3] = __builtin_amdgcn_mfma_f32_32x32x16_f16(aI, bI, z, 0, 0, 0);     // Y
            d[4] = __builtin_amdgcn_mfma_f32_32x32x16_f16(aP, bP, z, 0, 0, 0);     // M4
        }
        {
            // step 1, kh 1: k side (h4 l4 h4 0) from T = (h4 l4 0 0), l side
            // (h4 h4 l4 0); kh 0 takes the pieces as read
            halfx8_t a1[3], b1[3];
#pragma unroll
            for (int val = 0; val < 3; ++val) {
                const u32x4_v q = op[6 + val], t = op[9 + val];
                const u32x4_v qa = {q.x, q.y, kh ? q.x : q.z, q.w};
                const u32x4_v tb = {t.x, kh ? t.x : t.y, kh ? t.y : t.z, t.w};
                a1[val] = __builtin_bit_cast(halfx8_t, qa);
                b1[val] = __builtin_bit_cast(halfx8_t, tb);
            }
            d[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1[0], b1[0], d[0], 0, 0, 0);
            d[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1[0], b1[1], d[1], 0, 0, 0);
            d[2] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1[1], b1[0], d[2], 0, 0, 0);
            d[3] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1[1], b1[1], d[3], 0, 0, 0);
            d[4] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1[2], b1[2], d[4], 0, 0, 0);
        }

        // Register r of lane (kh, r32) is grid point
        // k = k0 + 32 (w / 2) + 8 (r / 4) + 4 kh + r % 4, l = l0 + 32 (w % 2) + r32.
        // The k-statistic combination in FP64, the (p, s^2) pairs of the
        // k side read for two runs of four columns (r / 4 = j, j + 1) at a time.
        double pl = 0.0, sl2 = 0.0;
        auto combine = [&](int j, const u32x4_v* pk) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 4 * j + i;
                const double2 kp = __builtin_bit_cast(double2, pk[i]);    // (p_k, s_k^2)
                const float X = d[0][r], U = d[1][r], V = d[2][r], Y = d[3][r];
                const double sq = fmaf(X, X, fmaf(Y, Y, fmaf(U, U, V * V)));
                const double sig = kp.y * sl2;
                const double val = fma(sig, fma(m2g, sq, (double)d[4][r]), kp.x * pl);
                acc[r][0] += val;
                acc[r][1] = fma(val, val, acc[r][1]);
            }
        };
        {
            u32x4_v pk[8], lp;
            read_lds_x8_1<so, so>(aPk, aPl, pk, lp);
            const double2 l2 = __builtin_bit_cast(double2, lp);
            pl = -gamma * l2.x;
            sl2 = l2.y;
            combine(0, pk);
            combine(1, pk + 4);
        }
        {
            u32x4_v pk[8];
            read_lds_x8<so + 16 * 16>(aPk, pk);
            combine(2, pk);
            combine(3, pk + 4);
        }
    };

    // (every wave is done with the previous piece's stages and has no memory
    // access of its own in flight: the counts waited for below are the
    // copies' alone)
    copies_barrier();
#pragma unroll
    for (int j = 0; j < kS4Stages - 1; ++j) copy_chunk(j, c0 + j);
    static_assert(kS4Stages == 3, "the loop below cycles through three stages");
#pragma unroll 1
    for (int c = c0;;) {
        step(std::integral_constant<int, 0>{}, c);
        if (++c >= c1) break;
        step(std::integral_constant<int, 1>{}, c);
        if (++c >= c1) break;
        step(std::integral_constant<int, 2>{}, c);
        if (++c >= c1) break;
    }

    double* o = it.part;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int idx = (32 * (w >> 1) + 8 * (r >> 2) + 4 * kh + (r & 3)) * kTile + 32 * (w & 1) + r32;
#pragma unroll
        for (int comp = 0; comp < 2; ++comp) {
            double val = acc[r][comp];
            if (p.accumulate) val += o[comp * kTile * kTile + idx];
            o[comp * kTile * kTile + idx] = val;
        }
    }
    }
}

// ------------------------------------------------------------------ S4, channel combinations
// C4(a_k, b*_k, c_l, d*_l) for general channels (Section 7), in the centred
// form of Appendix H with x = a'_k, y = b'*_k, z = c'_l, w = d'*_l:
//   c4 = [m(m+1) sum xyzw - (m-1)(sum xy sum zw + sum xz sum yw + sum xw sum yz)]
//        / ((m-1)(m-2)(m-3)),
// where, with E_k = a'_k b'*_k and F_l = c'_l d'*_l,
//   sum xyzw = sum E_k F_l,  sum xy = e_k = sum E_k,  sum zw = f_l = sum F_l,
//   sum xz = G_ac = sum a'_k c'_l,   sum yw = conj(G_bd),
//   sum xw = H_ad = sum a'_k d'*_l,  sum yz = conj(H_bc).
// Five complex frame sums per grid point (FP32 vector arithmetic), the
// combination and the chunk sums in FP64.  Tiles are 32 x 32; each thread owns
// the grid points (k0 + ti + 16u, l0 + tj + 16v), u, v < 2.
constexpr int kS4XThreads = 256;

__device__ __forceinline__ void cmac(float2& acc, float2 x, float2 y) {        // acc += x y
    acc.x = fmaf(x.x, y.x, fmaf(-x.y, y.y, acc.x));
    acc.y = fmaf(x.x, y.y, fmaf(x.y, y.x, acc.y));
}
__device__ __forceinline__ void cmacc(float2& acc, float2 x, float2 y) {       // acc += x conj(y)
    acc.x = fmaf(x.x, y.x, fmaf(x.y, y.y, acc.x));
    acc.y = fmaf(x.y, y.x, fmaf(-x.x, y.y, acc.y));
}

__global__ __launch_bounds__(kS4XThreads, 2) void k_s4_cross(BatchArgs p) {
    __shared__ float2 sv[4][kFrameBatch][kTileX];   // a'_k, b'_k, c'_l, d'_l

    Block bk;
    View v;
    if (!resolve_block(p, bk, v)) return;
    Item it;
    while (next_item<kTileX, 4>(p, bk, it)) {
    const int c0 = it.c0, c1 = it.c1;
    const int k0 = it.k0, l0 = it.l0;

    const int tid = threadIdx.x;
    const int ti = tid >> 4, tj = tid & 15;
    // Loader role: (array, column, half of the frames).
    const int arr = (tid & 127) >> 5, col = tid & 31, half = tid >> 7;
    const int gcol = (arr < 2 ? k0 : l0) + col;
    const bool live = gcol < v.Nf;
    // S4 planes: factors a and d at column + q, b and c at column - q
    const float2* src = v.coef + it.ch[arr] * v.cs + gcol + ((arr == 0 || arr == 3) ? p.s4_shift : -p.s4_shift);

    double acc[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q][0] = acc[q][1] = acc[q][2] = acc[q][3] = 0.0;
    const double gamma = p.gamma;

#pragma unroll 1
    for (int c = c0; c < c1; ++c) {
        const int64_t fbase = v.off + (int64_t)c * v.m * v.K;
        float2 sef[4], gac[4], gbd[4], had[4], hbc[4], e[2], f[2];
#pragma unroll
        for (int q = 0; q < 4; ++q) sef[q] = gac[q] = gbd[q] = had[q] = hbc[q] = make_float2(0.f, 0.f);
        e[0] = e[1] = f[0] = f[1] = make_float2(0.f, 0.f);
#pragma unroll 1
        for (int fb = 0; fb < v.m; fb += kFrameBatch) {
            const int nf = min(kFrameBatch, v.m - fb);
            lds_barrier();
            for (int fr = half; fr < nf; fr += 2)
                sv[arr][fr][col] = live ? src[fbase + (int64_t)(fb + fr) * v.K] : make_float2(0.f, 0.f);
            lds_barrier();
#pragma unroll 1
            for (int fr = 0; fr < nf; ++fr) {
                float2 a[2], b[2], cc[2], d[2], E[2], F[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    a[u] = sv[0][fr][ti + 16 * u];
                    b[u] = sv[1][fr][ti + 16 * u];
                    cc[u] = sv[2][fr][tj + 16 * u];
                    d[u] = sv[3][fr][tj + 16 * u];
                    E[u] = make_float2(fmaf(a[u].x, b[u].x, a[u].y * b[u].y), fmaf(a[u].y, b[u].x, -(a[u].x * b[u].y)));
                    F[u] = make_float2(fmaf(cc[u].x, d[u].x, cc[u].y * d[u].y), fmaf(cc[u].y, d[u].x, -(cc[u].x * d[u].y)));
                    e[u].x += E[u].x;
                    e[u].y += E[u].y;
                    f[u].x += F[u].x;
                    f[u].y += F[u].y;
                }
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int w = 0; w < 2; ++w) {
                        const int q = u * 2 + w;
                        cmac(sef[q], E[u], F[w]);
                        cmac(gac[q], a[u], cc[w]);
                        cmac(gbd[q], b[u], d[w]);
                        cmacc(had[q], a[u], d[w]);
                        cmacc(hbc[q], b[u], cc[w]);
                    }
            }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int w = 0; w < 2; ++w) {
                const int q = u * 2 + w;
                // T = e f + G_ac conj(G_bd) + H_ad conj(H_bc), in FP64
                const double er = e[u].x, ei = e[u].y, fr_ = f[w].x, fi = f[w].y;
                double tr = er * fr_ - ei * fi, tim = er * fi + ei * fr_;
                const double g1r = gac[q].x, g1i = gac[q].y, g2r = gbd[q].x, g2i = gbd[q].y;
                tr += g1r * g2r + g1i * g2i;
                tim += g1i * g2r - g1r * g2i;
                const double h1r = had[q].x, h1i = had[q].y, h2r = hbc[q].x, h2i = hbc[q].y;
                tr += h1r * h2r + h1i * h2i;
                tim += h1i * h2r - h1r * h2i;
                const double vr = fma(-gamma, tr, (double)sef[q].x);
                const double vi = fma(-gamma, tim, (double)sef[q].y);
                acc[q][0] += vr;
                acc[q][1] += vi;
                acc[q][2] = fma(vr, vr, acc[q][2]);
                acc[q][3] = fma(vi, vi, acc[q][3]);
            }
    }

    constexpr int TT = kTileX * kTileX;
    double* o = it.part;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const int idx = (ti + 16 * u) * kTileX + tj + 16 * w;
#pragma unroll
            for (int comp = 0; comp < 4; ++comp) {
                double val = acc[u * 2 + w][comp];
                if (p.accumulate) val += o[comp * TT + idx];
                o[comp * TT + idx] = val;
            }
        }
    }
}

// ------------------------------------------------------------------ S4, channel combinations, matrix cores
// The sums of k_s4_cross on the matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation, the BF16 x 3 split and 6-slot frame layout of k_s4_mfma_bf16).
// Each complex frame sum is four real Gram contractions, e.g.
//   sum E_k F_l = (sum E_r F_r - sum E_i F_i) + j (sum E_r F_i + sum E_i F_r),
// so the five sums E F, a c, b c*, b d, a d* take 20 Grams between six k-side
// row types (Re, Im of E = a' b'*, a', b') and six l-side types (F = c' d'*,
// c', d').  Tiles are 32 x 32; wave w owns the 16 x 16 block
// (16 (w / 2), 16 (w % 2)) with 20 accumulators of 4 registers, lane (lg, li)
// holding grid points (4 lg + e, li).  LDS rows are 160 bytes apart, a stride
// at which the 16-row, 16-byte-per-lane operand reads of 16x16x32 are free of
// bank conflicts.  As in k_s4_mfma_bf16 the Grams leave the matrix cores as
// FP32 and everything after them is FP64: the complex frame sums are
// assembled from the real Grams, and the k-statistic combination
//   v = sum E F - gamma T,  T = e f + G_ac conj(G_bd) + H_ad conj(H_bc),
// gamma = (m-1)/(m(m+1)), is formed in double before the FP64 chunk sums.
constexpr int kOpDwX = 40;           // 32-bit words per LDS operand row (160 B; 32 used)
constexpr int kS4XMThreads = 256;
constexpr int kCrossSlots = 3;       // frame slots q, q + 4, q + 8 of a loader thread

// Stage this thread's frame slots of column `col`: P = x conj(y) and the split
// words of (Re P, Im P, Re x, Im x, Re y, Im y) into row types 0..5; returns
// the sum of P over the slots.
template <int SIDE>
__device__ __forceinline__ float2 stage_cross(uint32_t (*op)[kOpDwX], int col, int q, const float2 (&px)[kCrossSlots],
                                              const float2 (&py)[kCrossSlots]) {
    float2 pa = make_float2(0.f, 0.f);
#pragma unroll
    for (int j = 0; j < kCrossSlots; ++j) {
        const int f = q + 4 * j;
        if (f >= kMfmaFrames) break;
        const float2 x = px[j], y = py[j];
        const float2 P = make_float2(fmaf(x.x, y.x, x.y * y.y), fmaf(x.y, y.x, -(x.x * y.y)));
        pa.x += P.x;
        pa.y += P.y;
        const float val[6] = {P.x, P.y, x.x, x.y, y.x, y.y};
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            uint32_t w0, w1, w2;
            split_words<SIDE>(val[t], w0, w1, w2);
            uint32_t* wr = &op[t * kTileX + col][3 * f];
            wr[0] = w0;
            wr[1] = w1;
            wr[2] = w2;
        }
    }
    return pa;
}

// ONE_BATCH: every chunk fits one frame batch (m <= 10), so each batch starts
// and ends a chunk (compile-time).
template <bool ONE_BATCH>
__global__ __launch_bounds__(kS4XMThreads, 2) void k_s4_cross_mfma(BatchArgs p) {
    __shared__ __attribute__((aligned(16))) uint32_t opA[6 * kTileX][kOpDwX];
    __shared__ __attribute__((aligned(16))) uint32_t opB[6 * kTileX][kOpDwX];
    __shared__ float2 psum[2][kTileX];

    Block bk;
    View v;
    if (!resolve_block(p, bk, v)) return;

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int rowA = 16 * (w >> 1) + li, rowB = 16 * (w & 1) + li;

    // Loader role: (side, column, frame residue q): frames q, q + 4, q + 8.
    // Columns c and c + 8 share an LDS bank at the 160-byte row stride, so the
    // lanes of each 32-bit write group ({0-15, 32-47}, {16-31, 48-63}) take
    // eight consecutive columns (as in k_s4_mfma_bf16).
    const int side = __builtin_amdgcn_readfirstlane(tid >> 7);    // uniform per wave
    const int col = 16 * (w & 1) + (((lane >> 2) & 3) | (((lane >> 5) & 1) << 2) | (((lane >> 4) & 1) << 3));
    const int q = tid & 3;
    uint32_t(*op)[kOpDwX] = side ? opB : opA;

    for (int r = tid; r < 2 * 6 * kTileX; r += kS4XMThreads) {
        uint32_t* row = (r < 6 * kTileX) ? opA[r] : opB[r - 6 * kTileX];
        row[3 * kMfmaFrames] = 0u;
        row[3 * kMfmaFrames + 1] = 0u;
    }
    const double gamma = p.gamma;                       // (m-1)/(m(m+1)) (natural: 1/m)

    Item it;
    while (next_item<kTileX, 4>(p, bk, it)) {
    const int c0 = it.c0, c1 = it.c1;
    const int gcol = (side ? it.l0 : it.k0) + col;
    const bool live = gcol < v.Nf;
    // S4 planes: a (k side) and d (l side) at column + q, b and c at column - q
    const int shx = side ? -p.s4_shift : p.s4_shift;
    const float2* srcx = v.coef + it.ch[2 * side] * v.cs + gcol + shx;        // a (k side) or c (l side)
    const float2* srcy = v.coef + it.ch[2 * side + 1] * v.cs + gcol - shx;    // b or d

    double acc[4][4];
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[e][0] = acc[e][1] = acc[e][2] = acc[e][3] = 0.0;

    constexpr int kJ = kCrossSlots;
    const int per_chunk = (v.m + kMfmaFrames - 1) / kMfmaFrames;
    const int n_batches = (c1 - c0) * per_chunk;
    float2 px[kJ], py[kJ];
    auto fetch = [&](int b) {
        const int c = c0 + b / per_chunk;
        const int fb = (b % per_chunk) * kMfmaFrames;
        const int nf = min(kMfmaFrames, v.m - fb);
        const int64_t o = v.off + ((int64_t)c * v.m + fb) * v.K;
#pragma unroll
        for (int j = 0; j < kJ; ++j) {
            const int f = q + 4 * j;
            const bool ok = live && f < nf;
            px[j] = ok ? srcx[o + (int64_t)f * v.K] : make_float2(0.f, 0.f);
            py[j] = ok ? srcy[o + (int64_t)f * v.K] : make_float2(0.f, 0.f);
        }
    };
    if (n_batches > 0) fetch(0);

    floatx4_t d[20];
    float2 pacc = make_float2(0.f, 0.f);
#pragma unroll 1
    for (int b = 0; b < n_batches; ++b) {
        const int fbi = ONE_BATCH ? 0 : b % per_chunk;
        const bool first = ONE_BATCH || fbi == 0, last = ONE_BATCH || fbi == per_chunk - 1;
        if (first) pacc = make_float2(0.f, 0.f);
        lds_barrier();
        {   // E = x conj(y) (k side: a b*, l side: c d*)
            const float2 pa = side == 0 ? stage_cross<0>(op, col, q, px, py) : stage_cross<1>(op, col, q, px, py);
            pacc.x += pa.x;
            pacc.y += pa.y;
        }
        if (last) {
            float2 tot = pacc;
            tot.x += xor1(tot.x);
            tot.y += xor1(tot.y);
            tot.x += __shfl_xor(tot.x, 2);
            tot.y += __shfl_xor(tot.y, 2);
            if (q == 0) psum[side][col] = tot;
        }
        lds_barrier();
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int wo = 16 * ks + 4 * lg;
            bf16x8_t A[6], B[6];
#pragma unroll
            for (int t = 0; t < 6; ++t) {
                A[t] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4_t*>(&opA[t * kTileX + rowA][wo]));
                B[t] = __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const u32x4_t*>(&opB[t * kTileX + rowB][wo]));
            }
            // (A type, B type) of the 20 Grams: E.F, a.c, b.c, b.d, a.d, each rr, ii, ri, ir
            constexpr int ga[20] = {0, 1, 0, 1, 2, 3, 2, 3, 4, 5, 4, 5, 4, 5, 4, 5, 2, 3, 2, 3};
            constexpr int gb[20] = {0, 1, 1, 0, 2, 3, 3, 2, 2, 3, 3, 2, 4, 5, 5, 4, 4, 5, 5, 4};
            const floatx4_t z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int g = 0; g < 20; ++g)
                d[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ga[g]], B[gb[g]], (first && ks == 0) ? z : d[g], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
        __builtin_amdgcn_s_setprio(0);
        if (b + 1 < n_batches) fetch(b + 1);
        if (!last) continue;

        const float2 fl32 = psum[1][rowB];
        const double flr = fl32.x, fli = fl32.y;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float2 ek = psum[0][16 * (w >> 1) + 4 * lg + e];
            double g[20];
#pragma unroll
            for (int i = 0; i < 20; ++i) g[i] = d[i][e];
            // complex frame sums from the real Grams, in FP64
            const double sef_r = g[0] - g[1], sef_i = g[2] + g[3];
            const double gac_r = g[4] - g[5], gac_i = g[6] + g[7];
            const double hbc_r = g[8] + g[9], hbc_i = g[11] - g[10];
            const double gbd_r = g[12] - g[13], gbd_i = g[14] + g[15];
            const double had_r = g[16] + g[17], had_i = g[19] - g[18];
            // T = e f + G_ac conj(G_bd) + H_ad conj(H_bc)
            const double ekr = ek.x, eki = ek.y;
            double tr = fma(ekr, flr, -(eki * fli));
            double ti = fma(ekr, fli, eki * flr);
            tr = fma(gac_r, gbd_r, fma(gac_i, gbd_i, tr));
            ti = fma(gac_i, gbd_r, fma(-gac_r, gbd_i, ti));
            tr = fma(had_r, hbc_r, fma(had_i, hbc_i, tr));
            ti = fma(had_i, hbc_r, fma(-had_r, hbc_i, ti));
            const double vr = fma(-gamma, tr, sef_r);
            const double vi = fma(-gamma, ti, sef_i);
            acc[e][0] += vr;
            acc[e][1] += vi;
            acc[e][2] = fma(vr, vr, acc[e][2]);
            acc[e][3] = fma(vi, vi, acc[e][3]);
        }
    }

    constexpr int TT = kTileX * kTileX;
    double* o = it.part;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int idx = (16 * (w >> 1) + 4 * lg + e) * kTileX + rowB;
#pragma unroll
        for (int comp = 0; comp < 4; ++comp) {
            double val = acc[e][comp];
            if (p.accumulate) val += o[comp * TT + idx];
            o[comp * TT + idx] = val;
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

static dim3 item_grid(const BatchArgs& a) { return dim3((unsigned)(((a.n_items + 7) / 8) * 8)); }

hipError_t launch_s2(const BatchArgs& a, hipStream_t s) {
    if (a.n_items <= 0) return hipSuccess;
    k_s2<<<item_grid(a), 256, 0, s>>>(a);
    return hipGetLastError();
}

// Frame batch of the S3 kernel, by rows per chunk r (m, or m + 1 for
// c3^(opt)): exactly r for r = 11..13 (one batch), else 10 (the default
// m = 10 fits one batch; longer chunks take several).  Measured at 2^28
// samples, the 10-frame instance has the lowest cost per row; a single
// batch of 11 to 13 beats it by 1-4 %, one of 14 to 16 loses to it by 2-8 %
// and the 16-frame batch with a remainder by 12-20 %.
bool s3_small_batch(int m) { return m <= kFrameBatchSmall || m % kFrameBatchSmall == 0; }

hipError_t launch_s3(const BatchArgs& a, hipStream_t s) {
    if (a.n_items <= 0) return hipSuccess;
    const int fb = a.s3_fb ? a.s3_fb
                   : (!s3_small_batch(a.m) && a.m <= 13) ? a.m
                                                        : kFrameBatchSmall;
    const dim3 g = item_grid(a);
    switch (fb) {
        case kFrameBatchSmall: k_s3<kFrameBatchSmall><<<g, kS3Threads, 0, s>>>(a); break;
        case kFrameBatchRow: k_s3<kFrameBatchRow><<<g, kS3Threads, 0, s>>>(a); break;
        case 12: k_s3<12><<<g, kS3Threads, 0, s>>>(a); break;
        case 13: k_s3<13><<<g, kS3Threads, 0, s>>>(a); break;
        default: k_s3<kFrameBatch><<<g, kS3Threads, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

hipError_t launch_s4_single(const BatchArgs& a, hipStream_t s) {
    if (a.n_items <= 0) return hipSuccess;
    k_s4_single<<<item_grid(a), kS4Threads, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_s4_mfma(const BatchArgs& a, hipStream_t s) {
    if (a.n_items <= 0) return hipSuccess;
    if (a.m <= kMfmaFrames)
        k_s4_mfma_bf16<true><<<item_grid(a), kS4MThreads, 0, s>>>(a);
    else
        k_s4_mfma_bf16<false><<<item_grid(a), kS4MThreads, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_s4_cross_mfma(const BatchArgs& a, hipStream_t s) {
    if (a.n_items <= 0) return hipSuccess;
    if (a.m <= kMfmaFrames)
        k_s4_cross_mfma<true><<<item_grid(a), kS4XMThreads, 0, s>>>(a);
    else
        k_s4_cross_mfma<false><<<item_grid(a), kS4XMThreads, 0, s>>>(a);
    return hipGetLastError();
}

int s4_cross_mfma_blocks_per_cu() {
    return blocks_per_cu(reinterpret_cast<const void*>(&k_s4_cross_mfma<false>), kS4XMThreads);
}

hipError_t launch_s4_cross(const BatchArgs& a, hipStream_t s) {
    if (a.n_items <= 0) return hipSuccess;
    k_s4_cross<<<item_grid(a), kS4XThreads, 0, s>>>(a);
    return hipGetLastError();
}

int s4_cross_blocks_per_cu() {
    return blocks_per_cu(reinterpret_cast<const void*>(&k_s4_cross), kS4XThreads);
}

int s3_blocks_per_cu() {
    return blocks_per_cu(reinterpret_cast<const void*>(&k_s3<kFrameBatch>), kS3Threads);
}
int s4_blocks_per_cu() { return blocks_per_cu(reinterpret_cast<const void*>(&k_s4_single), kS4Threads); }
hipError_t launch_s4_mfma_f16(const BatchArgs& a, hipStream_t s) {
    if (a.n_items <= 0) return hipSuccess;
    if (a.op4) {
        if (a.m > kOpFrames) return hipErrorInvalidValue;
        k_s4_mfma_f16_pre<<<item_grid(a), kS4MThreads, 0, s>>>(a);
        return hipGetLastError();
    }
    k_s4_mfma_f16<<<item_grid(a), kS4MThreads, 0, s>>>(a);
    return hipGetLastError();
}

int s4_mfma_f16_blocks_per_cu() {
    return blocks_per_cu(reinterpret_cast<const void*>(&k_s4_mfma_f16), kS4MThreads);
}

int s4_mfma_pre_blocks_per_cu() {
    return blocks_per_cu(reinterpret_cast<const void*>(&k_s4_mfma_f16_pre), kS4MThreads);
}

int s4_mfma_blocks_per_cu() {
    return blocks_per_cu(reinterpret_cast<const void*>(&k_s4_mfma_bf16<false>), kS4MThreads);
}

}  // namespace ps
