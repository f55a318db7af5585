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

// S2: one block per (record, combination, 256-wide k block).
__global__ __launch_bounds__(256) void k_finalize_vec(FinalizeArgs p) {
    const int64_t x = blockIdx.x;
    if (x >= p.n_items) return;
    const Seg& sg = p.segs[find_seg(p.segs, p.n_segs, x)];
    const int64_t t = x - sg.item0;
    const int k = (int)t * 256 + threadIdx.x;
    if (k >= p.Nf) return;
    const double* part = p.part + sg.part + threadIdx.x;
    double s[4] = {0, 0, 0, 0};
    int64_t s0 = 0, ns = 0;
    if (sg.n_chunks > 0) slot_range(Sched{sg.n_tiles, sg.n_chunks, sg.blocks}, t, s0, ns);
    for (int64_t slot = s0; slot < s0 + ns; ++slot) {
        const double* q = part + slot * 4 * 256;
        for (int c = 0; c < 4; ++c) s[c] += q[c * 256];
    }
    const double np = (double)sg.n_chunks;
    double mr, sr, mi, si;
    mean_sigma(s[0], s[2], np, sg.scale, mr, sr);
    mean_sigma(s[1], s[3], np, sg.scale, mi, si);
    if (sg.out) {
        sg.out[2 * k] = mr;
        sg.out[2 * k + 1] = mi;
    }
    if (sg.err) {
        sg.err[2 * k] = sr;
        sg.err[2 * k + 1] = si;
    }
}

// S3 / S4: one block per (record, combination, tile, 256 grid points of the
// tile): adds the tile's slots in slot order and writes its grid points (all of
// them, or only k <= l for symmetric spectra) with coalesced accesses.
__global__ __launch_bounds__(256) void k_finalize_tiles(FinalizeArgs p) {
    const int64_t x = blockIdx.x;
    if (x >= p.n_items) return;
    const Seg& sg = p.segs[find_seg(p.segs, p.n_segs, x)];
    const int E = sg.tiles >= kSym32 ? kTileX : kTile;
    const int TT = E * E;
    const int per_tile = TT / 256;
    const int64_t local = x - sg.item0;
    const int tile = (int)(local / per_tile);
    const int2 t = p.tt.t[sg.tiles][tile];
    const int k0 = t.x * E, l0 = t.y * E;
    const double np = (double)sg.n_chunks;
    const int ncomp = sg.ncomp;
    int64_t s0 = 0, ns = 0;
    if (sg.n_chunks > 0) slot_range(Sched{sg.n_tiles, sg.n_chunks, sg.blocks}, tile, s0, ns);
    {
        const int idx = (int)(local - (int64_t)tile * per_tile) * 256 + threadIdx.x;
        const int k = k0 + idx / E, l = l0 + idx % E;
        if (k >= p.Nf || l >= p.Nf || (sg.sym && k > l)) return;
        double s[4] = {0, 0, 0, 0};
        for (int64_t slot = s0; slot < s0 + ns; ++slot) {
            const double* q = p.part + sg.part + slot * ncomp * TT + idx;
            for (int c = 0; c < ncomp; ++c) s[c] += q[c * TT];
        }
        double mr, sr, mi = 0.0, si = 0.0;
        if (ncomp == 4) {
            mean_sigma(s[0], s[2], np, sg.scale, mr, sr);
            mean_sigma(s[1], s[3], np, sg.scale, mi, si);
        } else {
            mean_sigma(s[0], s[1], np, sg.scale, mr, sr);
            if (np < 1.0) mi = mr;      // NaN
            if (np < 2.0) si = sr;      // NaN
        }
        const int64_t o = ((int64_t)k * p.Nf + l) * 2;
        if (sg.out) {
            sg.out[o] = mr;
            sg.out[o + 1] = mi;
        }
        if (sg.err) {
            sg.err[o] = sr;
            sg.err[o + 1] = si;
        }
    }
}

// Symmetric spectra: copy (k, l) -> (l, k) for k < l through an LDS transpose
// of 32 x 32 blocks of complex (16-byte) values; one block per (segment,
// destination block), for the spectrum and its error bars.
__device__ __forceinline__ void mirror_block(double* a, int Nf, int bx, int by, double2 (*sh)[33]) {
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    double2* v = reinterpret_cast<double2*>(a);
    // source block: rows bx*32.., columns by*32.. (upper triangle)
    for (int r = ty; r < 32; r += 8) {
        const int k = bx * 32 + r, l = by * 32 + tx;
        if (k < Nf && l < Nf) sh[r][tx] = v[(int64_t)k * Nf + l];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int k = by * 32 + r, l = bx * 32 + tx;    // destination (k, l) with k > l
        if (k < Nf && l < Nf && k > l) v[(int64_t)k * Nf + l] = sh[tx][r];
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_mirror(FinalizeArgs p) {
    __shared__ double2 sh[32][33];
    const int64_t x = blockIdx.x;
    if (x >= p.n_items) return;
    const Seg& sg = p.segs[find_seg(p.segs, p.n_segs, x)];
    const int nb = (p.Nf + 31) / 32;
    const int local = (int)(x - sg.item0);
    const int by = local / nb, bx = local % nb;   // destination block row by, column bx
    if (by < bx) return;
    if (sg.out) mirror_block(sg.out, p.Nf, bx, by, sh);
    if (sg.err) mirror_block(sg.err, p.Nf, bx, by, sh);
}

__global__ void k_fill_nan(double* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = __longlong_as_double(0x7ff8000000000000LL);
}

}  // namespace

hipError_t launch_finalize_vec(const FinalizeArgs& a, hipStream_t s) {
    if (a.n_items <= 0) return hipSuccess;
    k_finalize_vec<<<(unsigned)a.n_items, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_finalize_grid(const FinalizeArgs& a, hipStream_t s) {
    if (a.n_items <= 0) return hipSuccess;
    k_finalize_tiles<<<(unsigned)a.n_items, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_mirror(const FinalizeArgs& a, hipStream_t s) {
    if (a.n_items <= 0) return hipSuccess;
    k_mirror<<<(unsigned)a.n_items, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_fill_nan(double* p, int64_t n, hipStream_t s) {
    if (!p || n <= 0) return hipSuccess;
    k_fill_nan<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

}  // namespace ps
