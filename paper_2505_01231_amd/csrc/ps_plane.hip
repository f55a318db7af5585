// Full frequency plane of one channel combination (Section 9).
//
// For real signals a_{-k} = conj(a_k), so a spectrum at negative frequencies
// equals a positive-quadrant value of a related combination: the cumulant is
// symmetric in its arguments, and conjugating all of them conjugates it.  With
// K = -k > 0, L = -l > 0:
//   S2_ab(-K)          = conj S2_ab(K)
//   S3_abc(-K, -L)     = conj S3_abc(K, L)
//   S3_abc(-K, l)      = conj S3_acb(K, l - K)     (l >= K)
//                      =      S3_bca(l, K - l)     (l <  K)
//   S3_abc(k, -L)      = conj S3_bca(L, k - L)     (k >= L)
//                      =      S3_acb(k, L - k)     (k <  L)
//   S4_abcd(-K, l)     = S4_bacd(K, l),  S4_abcd(k, -L) = S4_abdc(k, L),
//   S4_abcd(-K, -L)    = S4_badc(K, L)
// (S3_abc(k, l) = C3(a_k, b_l, c*_{k+l}), S4_abcd(k, l) = C4(a_k, b*_k, c_l, d*_l)).
// Every source index stays inside [0, N_f)^2.  Error bars (sigma_re,
// sigma_im) are unchanged by conjugation and transposition.
#include "ps_internal.h"

namespace ps {
namespace {

__global__ __launch_bounds__(256) void k_full_plane(PlaneArgs a) {
    const int E = 2 * a.Nf - 1;
    const int64_t n = a.order == 2 ? E : (int64_t)E * E;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int k = (a.order == 2 ? (int)i : (int)(i / E)) - (a.Nf - 1);
    const int l = (a.order == 2 ? 0 : (int)(i % E)) - (a.Nf - 1);
    const int K = -k, L = -l;
    int s = 0, p = k, q = l;
    bool cj = false;
    if (a.order == 2) {
        if (k < 0) p = K, cj = true;
        q = 0;
    } else if (a.order == 3) {
        if (k >= 0 && l >= 0) {
        } else if (k < 0 && l < 0) {
            p = K, q = L, cj = true;
        } else if (k < 0) {
            if (l >= K) s = 1, p = K, q = l - K, cj = true;
            else s = 2, p = l, q = K - l;
        } else {
            if (k >= L) s = 2, p = L, q = k - L, cj = true;
            else s = 1, p = k, q = L - k;
        }
    } else {
        if (k < 0 && l < 0) s = 3, p = K, q = L;
        else if (k < 0) s = 1, p = K;
        else if (l < 0) s = 2, q = L;
    }
    const PlaneSrc src = a.src[s];
    if (src.conj) cj = !cj;
    int64_t at;
    if (a.order == 2) {
        at = (int64_t)src.idx * a.Nf + p;
    } else {
        const int r = src.transpose ? q : p, c = src.transpose ? p : q;
        at = ((int64_t)src.idx * a.Nf + r) * a.Nf + c;
    }
    if (a.out) {
        const double re = a.in[2 * at], im = a.in[2 * at + 1];
        a.out[2 * i] = re;
        a.out[2 * i + 1] = cj ? -im : im;
    }
    if (a.err) {
        a.err[2 * i] = a.in_err[2 * at];
        a.err[2 * i + 1] = a.in_err[2 * at + 1];
    }
}

}  // namespace

hipError_t launch_full_plane(const PlaneArgs& a, hipStream_t s) {
    const int E = 2 * a.Nf - 1;
    const int64_t n = a.order == 2 ? E : (int64_t)E * E;
    if (n <= 0 || (!a.out && !a.err)) return hipSuccess;
    k_full_plane<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace ps
