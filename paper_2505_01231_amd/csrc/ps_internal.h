// Internal interface between the host runtime (ps_api.cpp) and the kernel
// launchers (ps_fft.hip, ps_moments.hip, ps_finalize.hip).  Not part of the ABI.
//
// Batching: one ps_execute runs each stage as ONE launch over every record and
// every channel combination.  The host describes the work as a table of
// segments (one per record and combination) that it copies into the
// workspace; each block finds its segment by binary search over the
// segments' first work-item index and derives its share of the segment's
// (tile, chunk) units and partial-sum slots from it (see Sched).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ps {

// Output-tile edge of the S3 / single-channel S4 kernels: a tile covers 64 x 64
// (k, l) grid points; the 256 threads of a block each own a 4 x 4 sub-grid.
constexpr int kTile = 64;
// Tile edge of the cross-channel S4 kernel (20 frame sums per grid point leave
// room for 2 x 2 grid points per thread only).
constexpr int kTileX = 32;
// Frames staged in LDS at once by the moment kernels.
constexpr int kFrameBatch = 16;
constexpr int kFrameBatchSmall = 10;
constexpr int kFrameBatchRow = 11;      // S3 only: chunks of 10 frames plus the c3^(opt) mean row

// Tile tables owned by the plan, one per kind and grid size.
enum TileKind { kSym64 = 0, kFull64 = 1, kSym32 = 2, kFull32 = 3 };

// ---------------------------------------------------------------- records (stage a1)
// Coefficient region of the workspace: [C][F_total][K] float2, records'
// frames concatenated in record order (chunk g of the batch = frames
// [g m, (g+1) m) of every channel).
struct RecDesc {
    const void* data;       // sample 0 of channel 0
    int64_t chan_stride;    // elements between channels
    int64_t frame0;         // first global frame of this record
    int32_t dtype;          // ps_dtype
    int32_t pad;
};

// Records of several frame lengths can share one launch: the frames of each
// frame length (a "class") are numbered on their own, and a launch carries up
// to kMaxClasses classes, each with its own window, twiddles, coefficient
// count and output region; a block finds its class by its index.
constexpr int kMaxClasses = 6;

struct FftClass {
    const RecDesc* recs;    // device table sorted by frame0 (the class's frames), or NULL: use `single`
    RecDesc single;
    int n_recs;
    int64_t g_lo, g_hi;     // the class's frames to transform
    int64_t out_g0;         // frame stored at row 0 of `out`
    int log2n;              // log2(N), 8..13 (complex signals: log2 of twice the frame length)
    int K;                  // coefficients kept per frame
    int jmax;               // complex signals: column c holds bin c - jmax
    const float* g;         // window [N]
    const float2* tw;       // twiddles, see fft_twiddle_count
    float2* out;            // [C][rows][K]
    int64_t out_chan_stride;
    int64_t block0;         // first block of the class in the launch
    // Frame length N when it is not a power of two (0: the FFT): the direct
    // transform with exp(+2 pi j t / N), t < N, from tw64 (FP64).
    int dft_n;
    const double2* tw64;
    // N = dft_n1 * (N / dft_n1) with dft_n1 <= N / dft_n1: the two-stage form
    // of the direct transform (0: one stage)
    int dft_n1;
};

struct FftArgs {
    FftClass cls[kMaxClasses];
    int n_cls;
    int n_channels;
    // Complex signals: frames of M = N/2 complex samples (dtype 3: complex
    // float32, 4: complex float64), transformed as they are; column c of the
    // output holds bin c - jmax.  Real signals: column c holds bin c.
    int cplx;
};
hipError_t launch_window_rfft(const FftArgs& a, hipStream_t s);

// Radices of the second and third pass of the frame transform (M = N/2 points:
// radix 16 first, then radix 16 while whole powers of 16 remain, then one
// radix 2/4/8 pass for the rest; 0 = no such pass).  The twiddle table `tw`
// holds exp(+2 pi j t / N), t < N, followed by one table per later pass of
// radix R and span Ns, laid out [r][k] (r < R, k < Ns): exp(+2 pi j r k / (R Ns)).
__host__ __device__ constexpr int fft_radix2(int log2n) {
    return (log2n - 1) / 4 >= 2 ? 16 : ((log2n - 1) % 4 ? 1 << ((log2n - 1) % 4) : 0);
}
__host__ __device__ constexpr int fft_radix3(int log2n) {
    return (log2n - 1) / 4 >= 3 ? 16 : ((log2n - 1) / 4 == 2 && (log2n - 1) % 4 ? 1 << ((log2n - 1) % 4) : 0);
}
__host__ __device__ constexpr int fft_twiddle_count(int log2n) {
    return (1 << log2n) + fft_radix2(log2n) * 16 + fft_radix3(log2n) * 16 * fft_radix2(log2n);
}

// Operand records of the matrix-core S4 kernel (scaled FP16 x 2): for each
// chunk and column, a power of two s > max_f (|Re a'|, |Im a'|) over the
// chunk's frames, and each of the values Re a' / s, Im a' / s, P / s^2
// (P = |a'|^2) of frames 0..9 split into two float16 terms x = h + l
// (h = fp16(x), l = fp16(x - h), both rounded to nearest).  Two frames make a
// 32-bit word (the earlier frame in the low half): h words 0..4, l words
// 0..4.  A value's record is kOpPieces 16-byte pieces, H = h words 0..3,
// L = l words 0..3, T = (h word 4, l word 4, 0, 0), frames >= m zero, stored
// piece-major over the columns; the column count is padded to a multiple of
// the 64-wide tile with zero records (op4_cols).
constexpr int kOpFrames = 10;
constexpr int kOpPieces = 3;
constexpr int kOpWords = 4 * kOpPieces;

// The smallest power of two strictly above a >= 0 (1 for a == 0).
__device__ __forceinline__ float pow2_above(float a) {
    if (!(a > 0.f)) return 1.0f;
    int e;
    (void)frexpf(a, &e);            // a = f 2^e, f in [0.5, 1)
    return ldexpf(1.0f, e);
}

// In-place centring: a_k(f) -= mean over the m frames of its chunk.  With
// `s1` set, the chunk's mean of a_0 (column s1_col; the first-order
// k-statistic) is also stored at s1[channel * s1_cs + s1_chunk0 + chunk].
// One class per frame length, as for the transform.
struct CentreClass {
    float2* coef;           // [C][n_chunks * m][K]
    int64_t coef_chan_stride;
    int K;
    int64_t n_chunks;
    int64_t s1_chunk0;
    // c3^(opt) rows for S3 (null: none): per chunk the m frames shifted by
    // alpha times the chunk mean, a - (1 - alpha) mean, then one row mu mean;
    // [C][n_chunks * (m + 1)][K]
    float2* out3;
    int64_t out3_cs;
    // Matrix-core S4 operands (null: none; chunks of m <= kOpFrames frames):
    // per chunk and column k < op4_cols of every channel, the split terms of
    // Re a' / s, Im a' / s and P / s^2 (see kOpWords), p = sum_f P and s^2;
    // op4_cols is N_f rounded up to a multiple of 64 (columns from K on: zero
    // records, p = 0, s = 1).
    uint32_t* op4;          // [C][n_chunks][3][kOpPieces][op4_cols][4]
    int64_t op4_cs;         // uint32 elements between channels
    double* p4;             // [C][n_chunks][op4_cols][2]: (p, s^2) per column
    int64_t p4_cs;          // double elements between channels
    int op4_cols;
    int64_t block0;         // first block of the class
};
struct CentreArgs {
    CentreClass cls[kMaxClasses];
    int n_cls;
    int m;
    int n_channels;
    float2* s1;
    int64_t s1_cs;
    int s1_col;
    float alpha, mu;
};
hipError_t launch_centre(const CentreArgs& a, hipStream_t s);

// ---------------------------------------------------------------- work decomposition
// A segment's work is T tiles x W chunks of (tile, chunk) units spread over B
// blocks.  Tiles [0, T1), T1 = (T / B) B, are processed whole: block j takes
// tiles j, j + B, j + 2B, ... (rounds), and the blocks of one round walk the
// chunks in the same order, so that their coefficient reads meet in L2.  The
// R = T - T1 remaining tiles hold U = R W units, taken in tile-major order and
// cut into Q = min(B, U) non-empty runs of equal length (stream-K); run j goes
// to block j, before its rounds, and touches at most two tiles since R < B.
// Every piece (one tile, one chunk range) writes its own partial-sum slot:
//   whole tile t              -> slot t
//   run j's piece of tile t   -> slot T1 + j + (t - T1)
// Runs are ordered and non-empty, so these are distinct and the slots of one
// tile are consecutive; the finalize kernels add them in slot order, so the
// result does not depend on timing.  The per-chunk schedule uses B = T (one
// tile per block, every launch the same slots).
struct Sched {
    int64_t T, W, B;
    __host__ __device__ int64_t T1() const { return (T / B) * B; }
    __host__ __device__ int64_t R() const { return T - T1(); }
    __host__ __device__ int64_t rounds() const { return T / B; }
    __host__ __device__ int64_t runs() const { return R() * W < B ? R() * W : B; }
    __host__ __device__ int64_t n_slots() const { return T1() + (R() > 0 ? runs() + R() : 0); }
    // first unit of run j (j <= runs(); later blocks have no run)
    __host__ __device__ int64_t run_begin(int64_t j) const {
        const int64_t Q = runs();
        return j >= Q ? R() * W : j * R() * W / Q;
    }
    // the run holding unit v (R > 0, W > 0)
    __host__ __device__ int64_t run_of(int64_t v) const {
        const int64_t U = R() * W;
        return ((v + 1) * runs() + U - 1) / U - 1;
    }
};

// ---------------------------------------------------------------- moments
// One segment = one (record, channel combination) of one stage.
struct Seg {
    int64_t item0;          // first work item (block) of the segment
    int64_t coef;           // float2 offset of the record's chunk 0 in the coefficient region
    int64_t cs;             // float2 elements between channels of the record's coefficient block
    int64_t op4, op4_cs;    // S4 operand records of the record's chunk 0 (uint32 offset), channel stride
    int64_t p4, p4_cs;      // and its (column sum of P, scale s^2) pairs (double offset), channel stride
    const int2* tile_tab;   // the grid's tile table (tile t -> (kt, lt)); by `tiles` and the grid size
    int32_t K;              // coefficients per frame of the record's frame length
    int32_t Nf;             // points per grid axis of the record's spectra
    int64_t part;           // double offset of the segment's partial sums
    int32_t n_tiles;        // tiles (S3/S4) or 256-wide k blocks (S2)
    int32_t blocks;         // B of the segment's Sched (blocks of the moment stage)
    int32_t n_chunks;       // Np of the record
    int32_t tiles;          // TileKind
    int32_t ch[4];          // channels of the combination
    double* out;            // finalize: spectrum slot, [Nf][2] or [Nf][Nf][2]
    double* err;
    double scale;           // finalize: prefactor * dt^(n-1) / sum g^n
    int32_t sym;            // finalize: mirror (k, l) -> (l, k)
    int32_t ncomp;          // finalize: 4 (complex) or 2 (real)
    // finalize with interlaced windows: the partial sums of the shifted frame
    // set (its own Sched{n_tiles, n_chunks2, blocks2}); n_chunks2 == 0: none
    int64_t part2;
    int32_t n_chunks2;
    int32_t blocks2;
};

struct BatchArgs {
    const Seg* segs;        // device table, sorted by item0
    int n_segs;
    int64_t n_items;
    const float2* coef;     // coefficient region
    const uint32_t* op4;    // S4 operand records (pre-split; null: the S4 kernel splits)
    const double* p4;
    double* part;           // partial-sum region
    int m;                  // rows per chunk
    int col0;               // column of grid index 0 for the first factors (see View)
    int col3;               // column of grid-sum index 0 for S3's third factor
    // Per-chunk schedule: only chunks [win_lo, win_hi) of each segment are
    // processed and chunk c sits at frame (c - win_lo) m of the region.
    int per_chunk, win_lo, win_hi;
    int accumulate;         // add to the partial sums instead of overwriting
    // S4 kernels form v = M4 - gamma (p_k p_l + |Q|^2 + |R|^2) in FP64:
    // gamma = (m-1)/(m(m+1)) for the k-statistic, 1/m for the natural estimator
    double gamma;
    int s4_shift;           // S4 planes: a, d at +q columns, b, c at -q (cross-channel kernels only)
    int s3_fb;              // S3 frames per LDS batch (10, 11 or 16); 0: chosen by the rows per chunk
};
hipError_t launch_s2(const BatchArgs& a, hipStream_t s);
hipError_t launch_s3(const BatchArgs& a, hipStream_t s);
hipError_t launch_s4_single(const BatchArgs& a, hipStream_t s);
hipError_t launch_s4_mfma(const BatchArgs& a, hipStream_t s);
hipError_t launch_s4_mfma_f16(const BatchArgs& a, hipStream_t s);
hipError_t launch_s4_cross(const BatchArgs& a, hipStream_t s);
hipError_t launch_s4_cross_mfma(const BatchArgs& a, hipStream_t s);

int s3_blocks_per_cu();
int s4_blocks_per_cu();
int s4_mfma_blocks_per_cu();
int s4_mfma_pre_blocks_per_cu();
int s4_mfma_f16_blocks_per_cu();
int s4_cross_blocks_per_cu();
int s4_cross_mfma_blocks_per_cu();

// ---------------------------------------------------------------- finalize
struct FinalizeArgs {
    const Seg* segs;        // items: S2 k blocks, or tiles (grid size and tile table per segment)
    int n_segs;
    int64_t n_items;
    const double* part;
    const float2* s1;       // per-chunk means of a_0, [C][s1_cs] (S1 only)
    int64_t s1_cs;
};
hipError_t launch_finalize_vec(const FinalizeArgs& a, hipStream_t s);
// Items are 16 x 16 sub-blocks of tiles; symmetric spectra are mirrored here.
hipError_t launch_finalize_grid(const FinalizeArgs& a, hipStream_t s);
// S1: one item per (record, channel); Seg.part (and part2) hold the index of
// the record's (and its interlaced twin's) first chunk in `s1`, Seg.ch[0] the
// channel.
hipError_t launch_finalize_s1(const FinalizeArgs& a, hipStream_t s);

hipError_t launch_fill_nan(double* p, int64_t n, hipStream_t s);

// Running accumulation (ps_stream_*): per combination, the batch's partial
// sums of up to two pieces (Seg.part / n_chunks / blocks and Seg.part2 /
// n_chunks2 / blocks2) added tile by tile to the state slots at Seg.out
// ([n_tiles][ncomp][points of a tile]; Seg.tiles < 0: the 256-point k blocks
// of S2).  Items: n_tiles x points per tile / 256 per segment.
struct AccumArgs {
    const Seg* segs;
    int n_segs;
    int64_t n_items;
    const double* part;
};
hipError_t launch_accumulate(const AccumArgs& a, hipStream_t s);
hipError_t launch_accumulate_s1(const float2* s1, int64_t s1_cs, int64_t n_chunks, int n_channels, double* state,
                                hipStream_t s);
hipError_t launch_finalize_s1_sums(const double* state, int n_channels, int64_t n_chunks, double scale, double* out,
                                   double* err, hipStream_t s);
hipError_t launch_zscore(const double* a, const double* ae, const double* b, const double* be, int64_t n,
                         double* out, hipStream_t s);

// ---------------------------------------------------------------- full plane
// One combination's spectrum on the signed grid (-N_f, N_f) gathered from the
// positive-quadrant outputs (see k_full_plane for the regions).  src[i] names
// the stored combination that serves raw combination i of the order's list
// (S2: ab; S3: abc, acb, bca; S4: abcd, bacd, abdc, badc) and how: conjugated
// and/or transposed.
struct PlaneSrc {
    int32_t idx;            // stored combination
    int32_t transpose;      // read (q, p) instead of (p, q)
    int32_t conj;
};
struct PlaneArgs {
    int order, Nf;
    const double* in;       // [stored combos][N_f] or [..][N_f][N_f] complex
    const double* in_err;   // same layout (sigma_re, sigma_im), or NULL
    PlaneSrc src[4];
    double* out;            // [2 N_f - 1] or [2 N_f - 1][2 N_f - 1] complex, or NULL
    double* err;
};
hipError_t launch_full_plane(const PlaneArgs& a, hipStream_t s);

// Static scratch of ps_execute_static (ps_static.hip): kStaticScratchBytes of
// device memory per GPU.  static_scratch_setup resolves the current device's
// copy (at plan creation); static_scratch_ptr returns it (NULL before).
constexpr size_t kStaticScratchBytes = size_t(256) << 20;
hipError_t static_scratch_setup();
void* static_scratch_ptr();

// The partial-sum slots of tile t: n consecutive slots from s0 (see Sched).
__device__ __forceinline__ void slot_range(const Sched& sc, int64_t t, int64_t& s0, int64_t& n) {
    const int64_t T1 = sc.T1();
    if (t < T1) {
        s0 = t;
        n = 1;
        return;
    }
    const int64_t v0 = (t - T1) * sc.W;
    const int64_t j0 = sc.run_of(v0), j1 = sc.run_of(v0 + sc.W - 1);
    s0 = T1 + j0 + (t - T1);
    n = j1 - j0 + 1;
}

// Workgroup barrier that orders LDS accesses only.  The threads of a block
// share data through LDS alone, so outstanding global loads (prefetches) may
// stay in flight across it; __syncthreads() would wait for them.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Segment lookup shared by the kernels: the last segment with item0 <= v.
__device__ __forceinline__ int find_seg(const Seg* segs, int n, int64_t v) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].item0 <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace ps
