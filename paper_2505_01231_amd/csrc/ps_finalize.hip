// Chunk average and error bars (Section 4.2), in FP64.
//
// The moment kernels leave, per grid point and chunk part, the sums over
// chunks of the un-scaled estimate x (its real and imaginary parts) and of
// their squares.  Here the parts are added in a fixed order and
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

__global__ __launch_bounds__(256) void k_finalize_vec(FinalizeVecArgs p) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= p.Nf) return;
    double s[4] = {0, 0, 0, 0};
    for (int sp = 0; sp < p.n_split; ++sp)
        for (int c = 0; c < 4; ++c) s[c] += p.part[((int64_t)sp * 4 + c) * p.Nf + k];
    const double np = (double)p.n_chunks;
    double mr, sr, mi, si;
    mean_sigma(s[0], s[2], np, p.scale, mr, sr);
    mean_sigma(s[1], s[3], np, p.scale, mi, si);
    if (p.out) {
        p.out[2 * k] = mr;
        p.out[2 * k + 1] = mi;
    }
    if (p.err) {
        p.err[2 * k] = sr;
        p.err[2 * k + 1] = si;
    }
}

// One block per partial tile: sums over the chunk parts in a fixed order and
// writes the tile's grid points (all of them, or only k <= l for symmetric
// spectra) with coalesced reads of the partials and coalesced row writes.
__global__ __launch_bounds__(256) void k_finalize_tiles(FinalizeGridArgs p, const int2* tiles) {
    const int tile = blockIdx.x;
    const int2 t = tiles[tile];
    const int E = p.edge;
    const int k0 = t.x * E, l0 = t.y * E;
    const int TT = E * E;
    const double np = (double)p.n_chunks;
    for (int idx = threadIdx.x; idx < TT; idx += 256) {
        const int k = k0 + idx / E, l = l0 + idx % E;
        if (k >= p.Nf || l >= p.Nf || (p.sym && k > l)) continue;
        double s[4] = {0, 0, 0, 0};
        for (int sp = 0; sp < p.n_split; ++sp) {
            const double* q = p.part + ((int64_t)sp * p.n_tiles + tile) * p.ncomp * TT + idx;
            for (int c = 0; c < p.ncomp; ++c) s[c] += q[c * TT];
        }
        double mr, sr, mi = 0.0, si = 0.0;
        if (p.ncomp == 4) {
            mean_sigma(s[0], s[2], np, p.scale, mr, sr);
            mean_sigma(s[1], s[3], np, p.scale, mi, si);
        } else {
            mean_sigma(s[0], s[1], np, p.scale, mr, sr);
            if (np < 1.0) mi = mr;      // NaN
            if (np < 2.0) si = sr;      // NaN
        }
        const int64_t o = ((int64_t)k * p.Nf + l) * 2;
        if (p.out) {
            p.out[o] = mr;
            p.out[o + 1] = mi;
        }
        if (p.err) {
            p.err[o] = sr;
            p.err[o + 1] = si;
        }
    }
}

// Symmetric spectra: copy (k, l) -> (l, k) for k < l through an LDS transpose
// of 32 x 32 blocks of complex (16-byte) values.
__global__ __launch_bounds__(256) void k_mirror(double* __restrict__ a, int Nf) {
    __shared__ double2 sh[32][33];
    const int bx = blockIdx.x, by = blockIdx.y;     // destination block (row by, column bx), by >= bx
    if (by < bx) return;
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
}

__global__ void k_fill_nan(double* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = __longlong_as_double(0x7ff8000000000000LL);
}

}  // namespace

hipError_t launch_finalize_vec(const FinalizeVecArgs& a, hipStream_t s) {
    k_finalize_vec<<<(a.Nf + 255) / 256, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_finalize_grid(const FinalizeGridArgs& a, const int2* tiles, hipStream_t s) {
    k_finalize_tiles<<<a.n_tiles, 256, 0, s>>>(a, tiles);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !a.sym) return e;
    const int nb = (a.Nf + 31) / 32;
    dim3 grid(nb, nb);
    if (a.out) k_mirror<<<grid, 256, 0, s>>>(a.out, a.Nf);
    if (a.err) k_mirror<<<grid, 256, 0, s>>>(a.err, a.Nf);
    return hipGetLastError();
}

hipError_t launch_fill_nan(double* p, int64_t n, hipStream_t s) {
    if (!p || n <= 0) return hipSuccess;
    k_fill_nan<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

}  // namespace ps
