// Chunk average and error bars (Section 4.2), in FP64.
//
// The moment kernels leave, per grid point and piece of work (a tile and a
// range of its chunks), the sums over chunks of the un-scaled estimate x (its
// real and imaginary parts) and of their squares.  Here a tile's pieces are
// added in slot order (fixed, see Sched) and
//   mean  = scale * sum x / Np
//   Var   = Np/(Np-1) (sum x^2 / Np - (sum x / Np)^2)          (per Re and Im)
//   sigma = |scale| * sqrt(Var / Np)
// where `scale` carries the k-statistic prefactor, dt^(n-1) and 1/sum g^n.
// Np == 0 gives NaN everywhere; Np == 1 gives NaN error bars.
// With interlaced windows a segment also carries the sums of the frame set
// shifted by N/2 (its own chunks, n_chunks2 > 0): the output is the average of
// the two sets' means and of their sigmas (Section 3 averages the interlaced
// spectra; the mean of the sigmas bounds the error of the average whatever
// the correlation between the overlapping sets).
#include "ps_internal.h"

namespace ps {
namespace {

__device__ __forceinline__ void mean_sigma(double s, double s2, double np, double scale, double& mean,
                                           double& sigma) {
    if (np < 1.0) {
        mean = __longlong_as_double(0x7ff8000000000000LL);
        sigma = mean;
        return;
    }
    const double mu = s / np;
    mean = scale * mu;
    if (np < 2.0) {
        sigma = __longlong_as_double(0x7ff8000000000000LL);
        return;
    }
    const double var = np / (np - 1.0) * (s2 / np - mu * mu);
    sigma = fabs(scale) * sqrt(fmax(var, 0.0) / np);
}

// The interlaced average of the two frame sets' results at one grid point.
__device__ __forceinline__ void combine_sets(double& mean, double& sigma, double mean2, double sigma2) {
    mean = 0.5 * (mean + mean2);
    sigma = 0.5 * (sigma + sigma2);
}

// S2: one block per (record, combination, 16-wide k group of a 256-wide k
// block).  Thread (g, kk) adds the slots s0 + g, s0 + g + 16, ... of point kk
// (of each frame set); the 16 group sums are then added in LDS in group order
// (a fixed order, so the result does not depend on timing).
constexpr int kVecGroups = 16;

__global__ __launch_bounds__(256) void k_finalize_vec(FinalizeArgs p) {
    __shared__ double red[kVecGroups][8][16];
    const int64_t x = blockIdx.x / kVecGroups;         // item: a 256-wide k block
    if (x >= p.n_items) return;
    const int sub = blockIdx.x % kVecGroups;
    const Seg& sg = p.segs[find_seg(p.segs, p.n_segs, x)];
    const int64_t t = x - sg.item0;
    const int kk = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int kl = 16 * sub + kk;                       // k within the item
    const int k = (int)t * 256 + kl;
    const bool two = sg.n_chunks2 > 0;
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int set = 0; set < (two ? 2 : 1); ++set) {
        const int64_t W = set ? sg.n_chunks2 : sg.n_chunks;
        int64_t s0 = 0, ns = 0;
        if (W > 0) slot_range(Sched{sg.n_tiles, W, set ? sg.blocks2 : sg.blocks}, t, s0, ns);
        const double* part = p.part + (set ? sg.part2 : sg.part) + kl;
        for (int64_t slot = s0 + g; slot < s0 + ns; slot += kVecGroups) {
            const double* q = part + slot * 4 * 256;
            for (int c = 0; c < 4; ++c) s[4 * set + c] += q[c * 256];
        }
    }
    const int nc = two ? 8 : 4;                         // uniform over the block
    for (int c = 0; c < nc; ++c) red[g][c][kk] = s[c];
    __syncthreads();
    if (g != 0 || k >= sg.Nf) return;
    for (int c = 0; c < nc; ++c) {
        s[c] = 0;
        for (int gg = 0; gg < kVecGroups; ++gg) s[c] += red[gg][c][kk];
    }
    double mr, sr, mi, si;
    mean_sigma(s[0], s[2], (double)sg.n_chunks, sg.scale, mr, sr);
    mean_sigma(s[1], s[3], (double)sg.n_chunks, sg.scale, mi, si);
    if (two) {
        double mr2, sr2, mi2, si2;
        mean_sigma(s[4], s[6], (double)sg.n_chunks2, sg.scale, mr2, sr2);
        mean_sigma(s[5], s[7], (double)sg.n_chunks2, sg.scale, mi2, si2);
        combine_sets(mr, sr, mr2, sr2);
        combine_sets(mi, si, mi2, si2);
    }
    if (sg.out) {
        sg.out[2 * k] = mr;
        sg.out[2 * k + 1] = mi;
    }
    if (sg.err) {
        sg.err[2 * k] = sr;
        sg.err[2 * k + 1] = si;
    }
}

// S3 / S4: one block per (record, combination, tile, 16 x 16 sub-block of the
// tile): adds the tile's slots in slot order and writes the sub-block's grid
// points (all of them, or only k <= l for symmetric spectra); a symmetric
// spectrum also gets its mirror (l, k) <- (k, l), k < l, written through an
// LDS transpose so that both writes are row-contiguous.
__global__ __launch_bounds__(256) void k_finalize_tiles(FinalizeArgs p) {
    __shared__ double2 sm[16][17], se[16][17];
    const int64_t x = blockIdx.x;
    if (x >= p.n_items) return;
    const Seg& sg = p.segs[find_seg(p.segs, p.n_segs, x)];
    const int E = sg.tiles >= kSym32 ? kTileX : kTile;
    const int TT = E * E;
    const int sub = E / 16, per_tile = sub * sub;
    const int64_t local = x - sg.item0;
    const int tile = (int)(local / per_tile);
    const int sb = (int)(local - (int64_t)tile * per_tile);
    const int2 t = sg.tile_tab[tile];
    const int kb = t.x * E + 16 * (sb / sub), lb = t.y * E + 16 * (sb % sub);   // sub-block origin
    const int i = threadIdx.x >> 4, j = threadIdx.x & 15;
    const int ncomp = sg.ncomp;
    const bool two = sg.n_chunks2 > 0;

    const int k = kb + i, l = lb + j;
    const bool valid = k < sg.Nf && l < sg.Nf && !(sg.sym && k > l);
    double mr = 0.0, sr = 0.0, mi = 0.0, si = 0.0;
    // The point's offset inside the tile does not depend on the tile table,
    // and every component of every slot is loaded before any is added (one
    // round trip to memory, not one per component).
    const int idx = (16 * (sb / sub) + i) * E + 16 * (sb % sub) + j;
    for (int set = 0; set < (two ? 2 : 1); ++set) {
        const int64_t W = set ? sg.n_chunks2 : sg.n_chunks;
        const double np = (double)W;
        int64_t s0 = 0, ns = 0;
        if (W > 0) slot_range(Sched{sg.n_tiles, W, set ? sg.blocks2 : sg.blocks}, tile, s0, ns);
        const double* base = p.part + (set ? sg.part2 : sg.part) + idx;
        double s[4] = {0, 0, 0, 0};
        for (int64_t slot = s0; slot < s0 + ns; ++slot) {
            const double* q = base + slot * ncomp * TT;
            double v[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] = c < ncomp ? q[c * TT] : 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) s[c] += v[c];
        }
        double r_m, r_s, i_m = 0.0, i_s = 0.0;
        if (ncomp == 4) {
            mean_sigma(s[0], s[2], np, sg.scale, r_m, r_s);
            mean_sigma(s[1], s[3], np, sg.scale, i_m, i_s);
        } else {
            mean_sigma(s[0], s[1], np, sg.scale, r_m, r_s);
            if (np < 1.0) i_m = r_m;    // NaN
            if (np < 2.0) i_s = r_s;    // NaN
        }
        if (set == 0) {
            mr = r_m, sr = r_s, mi = i_m, si = i_s;
        } else {
            combine_sets(mr, sr, r_m, r_s);
            combine_sets(mi, si, i_m, i_s);
        }
    }
    if (valid) {
        const int64_t o = ((int64_t)k * sg.Nf + l) * 2;
        if (sg.out) {
            sg.out[o] = mr;
            sg.out[o + 1] = mi;
        }
        if (sg.err) {
            sg.err[o] = sr;
            sg.err[o + 1] = si;
        }
    }
    if (!sg.sym) return;            // uniform over the block
    sm[i][j] = make_double2(mr, mi);
    se[i][j] = make_double2(sr, si);
    __syncthreads();
    // thread (i, j) now writes point (kb + j, lb + i) to (lb + i, kb + j)
    const int km = kb + j, lm = lb + i;
    if (km < lm && lm < sg.Nf) {
        const int64_t o = ((int64_t)lm * sg.Nf + km) * 2;
        if (sg.out) {
            const double2 v = sm[j][i];
            sg.out[o] = v.x;
            sg.out[o + 1] = v.y;
        }
        if (sg.err) {
            const double2 v = se[j][i];
            sg.err[o] = v.x;
            sg.err[o + 1] = v.y;
        }
    }
}

__global__ void k_fill_nan(double* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = __longlong_as_double(0x7ff8000000000000LL);
}

// S1: one block per (record, channel).  Thread t adds the per-chunk means of
// a_0 of chunks t, t + 256, ... in FP64 (of each frame set; real and imaginary
// parts and their squares); the partial sums are then added in a fixed tree
// order.  For a real signal a_0 is real, so Im and sigma_Im come out 0 (NaN
// where the mean or the error bar is undefined).
__global__ __launch_bounds__(256) void k_finalize_s1(FinalizeArgs p) {
    __shared__ double red[8][256];
    const int64_t x = blockIdx.x;
    if (x >= p.n_items) return;
    const Seg& sg = p.segs[find_seg(p.segs, p.n_segs, x)];
    const bool two = sg.n_chunks2 > 0;
    const float2* v = p.s1 + (int64_t)sg.ch[0] * p.s1_cs;
    const int tid = threadIdx.x;
    for (int set = 0; set < 2; ++set) {
        const int64_t c0 = set ? sg.part2 : sg.part, W = set ? (two ? sg.n_chunks2 : 0) : sg.n_chunks;
        double sr = 0.0, si = 0.0, sr2 = 0.0, si2 = 0.0;
        for (int64_t c = tid; c < W; c += 256) {
            const float2 d = v[c0 + c];
            sr += d.x;
            si += d.y;
            sr2 = fma((double)d.x, (double)d.x, sr2);
            si2 = fma((double)d.y, (double)d.y, si2);
        }
        red[4 * set][tid] = sr;
        red[4 * set + 1][tid] = si;
        red[4 * set + 2][tid] = sr2;
        red[4 * set + 3][tid] = si2;
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h)
            for (int q = 0; q < 8; ++q) red[q][tid] += red[q][tid + h];
        __syncthreads();
    }
    if (tid != 0) return;
    double mr, sr, mi, si;
    mean_sigma(red[0][0], red[2][0], (double)sg.n_chunks, sg.scale, mr, sr);
    mean_sigma(red[1][0], red[3][0], (double)sg.n_chunks, sg.scale, mi, si);
    if (two) {
        double mr2, sr2, mi2, si2;
        mean_sigma(red[4][0], red[6][0], (double)sg.n_chunks2, sg.scale, mr2, sr2);
        mean_sigma(red[5][0], red[7][0], (double)sg.n_chunks2, sg.scale, mi2, si2);
        combine_sets(mr, sr, mr2, sr2);
        combine_sets(mi, si, mi2, si2);
    }
    if (sg.out) {
        sg.out[0] = mr;
        sg.out[1] = mi;
    }
    if (sg.err) {
        sg.err[0] = sr;
        sg.err[1] = si;
    }
}

// Running accumulation (ps_stream_*): one block per (segment, tile, group of
// 256 points of the tile).  A segment names one combination and up to two
// pieces of the batch (the chunk completed from the carry buffer, set 0, and
// the chunks of the pushed samples, set 1); the block adds each point's slots
// of set 0, then of set 1, in slot order, and adds the result to the state
// slot of that tile (Seg.out), so the order of additions is fixed.
__global__ __launch_bounds__(256) void k_accumulate(AccumArgs p) {
    const int64_t x = blockIdx.x;
    if (x >= p.n_items) return;
    const Seg& sg = p.segs[find_seg(p.segs, p.n_segs, x)];
    const int P = sg.tiles < 0 ? 256 : (sg.tiles >= kSym32 ? kTileX * kTileX : kTile * kTile);
    const int per_tile = P / 256;
    const int64_t local = x - sg.item0;
    const int tile = (int)(local / per_tile);
    const int e = (int)(local - (int64_t)tile * per_tile) * 256 + threadIdx.x;
    const int nc = sg.ncomp;
    double s[4] = {0, 0, 0, 0};
    for (int set = 0; set < 2; ++set) {
        const int64_t W = set ? sg.n_chunks2 : sg.n_chunks;
        if (W <= 0) continue;
        int64_t s0 = 0, ns = 0;
        slot_range(Sched{sg.n_tiles, W, set ? sg.blocks2 : sg.blocks}, tile, s0, ns);
        const double* base = p.part + (set ? sg.part2 : sg.part) + e;
        for (int64_t slot = s0; slot < s0 + ns; ++slot) {
            const double* q = base + slot * nc * P;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c < nc) s[c] += q[c * P];
        }
    }
    double* st = sg.out + (int64_t)tile * nc * P + e;
#pragma unroll
    for (int c = 0; c < 4; ++c)
        if (c < nc) st[c * P] += s[c];
}

// S1 of a running accumulation: one block per channel adds the per-chunk means
// of a_0 of this push's chunks (real and imaginary parts and their squares)
// in a fixed tree order to the channel's four state sums.
__global__ __launch_bounds__(256) void k_accumulate_s1(const float2* s1, int64_t s1_cs, int64_t n_chunks,
                                                       double* state) {
    __shared__ double red[4][256];
    const int ch = blockIdx.x, tid = threadIdx.x;
    const float2* v = s1 + (int64_t)ch * s1_cs;
    double a[4] = {0, 0, 0, 0};
    for (int64_t c = tid; c < n_chunks; c += 256) {
        const float2 d = v[c];
        a[0] += d.x;
        a[1] += d.y;
        a[2] = fma((double)d.x, (double)d.x, a[2]);
        a[3] = fma((double)d.y, (double)d.y, a[3]);
    }
    for (int q = 0; q < 4; ++q) red[q][tid] = a[q];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h)
            for (int q = 0; q < 4; ++q) red[q][tid] += red[q][tid + h];
        __syncthreads();
    }
    if (tid < 4) state[4 * ch + tid] += red[tid][0];
}

// S1 from a running accumulation's state sums (one thread per channel).
__global__ void k_finalize_s1_sums(const double* state, int n_channels, int64_t n_chunks, double scale,
                                   double* out, double* err) {
    const int ch = threadIdx.x;
    if (ch >= n_channels) return;
    const double* q = state + 4 * ch;
    double mr, sr, mi, si;
    mean_sigma(q[0], q[2], (double)n_chunks, scale, mr, sr);
    mean_sigma(q[1], q[3], (double)n_chunks, scale, mi, si);
    if (out) {
        out[2 * ch] = mr;
        out[2 * ch + 1] = mi;
    }
    if (err) {
        err[2 * ch] = sr;
        err[2 * ch + 1] = si;
    }
}

// |a - b| / sqrt(sa^2 + sb^2) per real component.
__global__ void k_zscore(const double* a, const double* ae, const double* b, const double* be, int64_t n,
                         double* out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double d = fabs(a[i] - b[i]);
    out[i] = d / sqrt(ae[i] * ae[i] + be[i] * be[i]);
}

}  // namespace

hipError_t launch_accumulate(const AccumArgs& a, hipStream_t s) {
    if (a.n_items <= 0) return hipSuccess;
    k_accumulate<<<(unsigned)a.n_items, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_accumulate_s1(const float2* s1, int64_t s1_cs, int64_t n_chunks, int n_channels, double* state,
                                hipStream_t s) {
    if (n_chunks <= 0 || n_channels <= 0) return hipSuccess;
    k_accumulate_s1<<<(unsigned)n_channels, 256, 0, s>>>(s1, s1_cs, n_chunks, state);
    return hipGetLastError();
}

hipError_t launch_finalize_s1_sums(const double* state, int n_channels, int64_t n_chunks, double scale, double* out,
                                   double* err, hipStream_t s) {
    if (n_channels <= 0) return hipSuccess;
    k_finalize_s1_sums<<<1, 64, 0, s>>>(state, n_channels, n_chunks, scale, out, err);
    return hipGetLastError();
}

hipError_t launch_zscore(const double* a, const double* ae, const double* b, const double* be, int64_t n,
                         double* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_zscore<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a, ae, b, be, n, out);
    return hipGetLastError();
}

hipError_t launch_finalize_vec(const FinalizeArgs& a, hipStream_t s) {
    if (a.n_items <= 0) return hipSuccess;
    k_finalize_vec<<<(unsigned)(a.n_items * kVecGroups), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_finalize_grid(const FinalizeArgs& a, hipStream_t s) {
    if (a.n_items <= 0) return hipSuccess;
    k_finalize_tiles<<<(unsigned)a.n_items, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_finalize_s1(const FinalizeArgs& a, hipStream_t s) {
    if (a.n_items <= 0 || !a.s1) return hipSuccess;
    k_finalize_s1<<<(unsigned)a.n_items, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_fill_nan(double* p, int64_t n, hipStream_t s) {
    if (!p || n <= 0) return hipSuccess;
    k_fill_nan<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

}  // namespace ps
