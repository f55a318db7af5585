// Internal interface between the host runtime (ps_api.cpp) and the kernel
// launchers (ps_fft.hip, ps_moments.hip, ps_finalize.hip).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ps {

// Output-tile edge of the S3/S4 moment kernels: a tile covers 64 x 64 (k, l)
// grid points; the 256 threads of a block each own a 4 x 4 sub-grid.
constexpr int kTile = 64;
// Tile edge of the cross-channel S4 kernel (20 frame sums per grid point leave
// room for 2 x 2 grid points per thread only).
constexpr int kTileX = 32;
// Frames staged in LDS at once by the moment kernels.
constexpr int kFrameBatch = 16;
constexpr int kFrameBatchSmall = 10;

// ---------------------------------------------------------------- stage a1
struct FftArgs {
    const void* x;          // sample 0 of channel 0 of the record
    int dtype;              // ps_dtype
    int64_t chan_stride;    // elements between channels
    int64_t frame0;         // first frame to transform
    int n_frames;           // frames per channel
    int n_channels;
    int log2n;              // log2(N), 8..13
    int K;                  // coefficients kept per frame
    const float* g;         // window [N]
    const float2* tw;       // exp(+2 pi j t / N), t < N
    float2* out;            // [C][out_frames][K], frame index (f - frame0_out)
    int64_t out_chan_stride;  // float2 elements between channels of `out`
    int64_t out_frame0;     // frame index subtracted before writing
};
hipError_t launch_window_rfft(const FftArgs& a, hipStream_t s);

// In-place centring: a_k(f) -= mean over the m frames of its chunk.
struct CentreArgs {
    float2* coef;           // [C][n_chunks * m][K]
    int64_t coef_chan_stride;
    int K, m;
    int n_chunks;
    int n_channels;
};
hipError_t launch_centre(const CentreArgs& a, hipStream_t s);

// ---------------------------------------------------------------- moments
// Chunk-centred coefficients a' = a - mean_f a (after launch_centre).
struct CoefView {
    const float2* coef;     // [C][frames][K]; chunk c starts at frame (c - coef_chunk0) * m
    int64_t coef_chan_stride;
    int K, m;
    int coef_chunk0;
};

struct S2Args {
    CoefView v;
    int Nf;
    int a, b;               // channels: C2(a_k, b*_k)
    int chunk0, chunk1;     // chunk range of this launch
    int n_split;
    double* part;           // [n_split][4][Nf]: sum re, sum im, sum re^2, sum im^2 of sum_f a' b'*
    int accumulate;
};
hipError_t launch_s2(const S2Args& a, hipStream_t s);

struct GridArgs {
    CoefView v;
    int Nf;
    int ch[4];              // channels of the combination
    const int2* tiles;      // [n_tiles] (kt, lt)
    int n_tiles;
    int chunk0, chunk1;
    int n_split;
    double* part;           // [n_split][n_tiles][ncomp][kTile*kTile]
    int accumulate;
    double gamma;           // S4: (m-1)/(m(m+1))
};
hipError_t launch_s3(const GridArgs& a, hipStream_t s);
hipError_t launch_s4_single(const GridArgs& a, hipStream_t s);
hipError_t launch_s4_mfma(const GridArgs& a, hipStream_t s);
hipError_t launch_s4_cross(const GridArgs& a, hipStream_t s);

int s3_blocks_per_cu();
int s4_blocks_per_cu();
int s4_mfma_blocks_per_cu();
int s4_cross_blocks_per_cu();

// ---------------------------------------------------------------- finalize
struct FinalizeVecArgs {
    const double* part;     // [n_split][4][Nf]
    int n_split, Nf;
    int64_t n_chunks;
    double scale;
    double* out;            // [Nf][2]
    double* err;            // [Nf][2]
};
hipError_t launch_finalize_vec(const FinalizeVecArgs& a, hipStream_t s);

struct FinalizeGridArgs {
    const double* part;     // [n_split][n_tiles][ncomp][edge*edge]
    int n_split, n_tiles, ncomp;
    int edge;               // tile edge (kTile or kTileX)
    int sym;                // only tiles kt <= lt exist; (k, l) with k > l is the mirror of (l, k)
    int Nf;
    int64_t n_chunks;
    double scale;
    double* out;            // [Nf][Nf][2]
    double* err;            // [Nf][Nf][2]
};
hipError_t launch_finalize_grid(const FinalizeGridArgs& a, const int2* tiles, hipStream_t s);

hipError_t launch_fill_nan(double* p, int64_t n, hipStream_t s);

}  // namespace ps
