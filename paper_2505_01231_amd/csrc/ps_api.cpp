// Host runtime behind the C ABI of include/polyspec.h: validation, the FP64
// window and FFT tables, the channel-combination lists, workspace layout, the
// choice of launch shapes, and the order of kernel launches per record.
// Release calls on teardown and clean-up paths, written (void)hip...(),
// discard their status on purpose: the objects are gone either way, and the
// error that led there, if any, is the one reported.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "polyspec.h"
#include "ps_internal.h"

namespace {

thread_local std::string g_last_error;

ps_status fail(ps_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define PS_HIP(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(PS_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));         \
    } while (0)

// Window g_i in FP64 (Section 3; approximate confined Gaussian of Appendix B).
void make_window(int kind, int N, double sigma_t, std::vector<double>& g) {
    g.resize(N);
    const double pi = 3.14159265358979323846;
    if (kind == PS_WIN_HANN) {
        for (int i = 0; i < N; ++i) {
            const double s = std::sin(pi * i / (N - 1));
            g[i] = s * s;
        }
    } else if (kind == PS_WIN_HANN_PERIODIC) {
        for (int i = 0; i < N; ++i) {
            const double s = std::sin(pi * i / N);
            g[i] = s * s;
        }
    } else {
        const double c = 0.5 * (N - 1);
        const double den = 4.0 * N * (double)N * sigma_t * sigma_t;
        auto G = [&](double x) { return std::exp(-(x - c) * (x - c) / den); };
        const double ratio = G(-0.5) / (G(-0.5 + N) + G(-0.5 - N));
        for (int i = 0; i < N; ++i) g[i] = G(i) - ratio * (G(i + N) + G(i - N));
    }
}

// Combination orbits under the grid-preserving symmetries (Section 9).
void all_combos(int C, std::vector<int8_t>& c2, std::vector<int8_t>& c3, std::vector<int8_t>& c4) {
    c2.clear();
    c3.clear();
    c4.clear();
    for (int a = 0; a < C; ++a)
        for (int b = a; b < C; ++b) c2.insert(c2.end(), {(int8_t)a, (int8_t)b});
    for (int a = 0; a < C; ++a)
        for (int b = a; b < C; ++b)
            for (int c = 0; c < C; ++c) c3.insert(c3.end(), {(int8_t)a, (int8_t)b, (int8_t)c});
    for (int a = 0; a < C; ++a)
        for (int b = 0; b < C; ++b)
            for (int c = 0; c < C; ++c)
                for (int d = 0; d < C; ++d) {
                    const int self = ((a * 4 + b) * 4 + c) * 4 + d;
                    const int badc = ((b * 4 + a) * 4 + d) * 4 + c;
                    const int cdab = ((c * 4 + d) * 4 + a) * 4 + b;
                    const int dcba = ((d * 4 + c) * 4 + b) * 4 + a;
                    if (self <= badc && self <= cdab && self <= dcba)
                        c4.insert(c4.end(), {(int8_t)a, (int8_t)b, (int8_t)c, (int8_t)d});
                }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr size_t kStagingBytes = 4u << 20;     // pinned work-table staging per buffer (two per plan)

// Output tiles: upper triangle (kt <= lt) for symmetric spectra, all
// otherwise, walked in G x G blocks of tiles: the consecutive tiles that one
// XCD processes at a time then share their k and l columns (and part of the
// k + l range) in that XCD's L2, instead of spanning whole tile rows.
void tile_order(int T, int G, std::vector<int2>& sym, std::vector<int2>& full) {
    sym.clear();
    full.clear();
    for (int bk = 0; bk < T; bk += G)
        for (int bl = 0; bl < T; bl += G)
            for (int kt = bk; kt < std::min(T, bk + G); ++kt)
                for (int lt = bl; lt < std::min(T, bl + G); ++lt) {
                    full.push_back(make_int2(kt, lt));
                    if (kt <= lt) sym.push_back(make_int2(kt, lt));
                }
}

}  // namespace

// One frame length of a plan: its window and FFT tables, grid and tile
// tables.  Class 0 is the plan's frame_len (its fields are also the plan's
// own); further classes come from ps_config.frame_len_set.
struct FrameClass {
    int N = 0, log2n_fft = 0, Nf = 0, Ng = 0, K = 0, jmax = 0;
    int T = 0, TX = 0;
    int n_tiles[4] = {0, 0, 0, 0};
    double sum_g[5] = {0, 0, 0, 0, 0};
    float* d_g = nullptr;
    float2* d_tw = nullptr;
    double2* d_tw64 = nullptr;      // exp(+2 pi j t / N), t < N (direct transform)
    int2* d_tiles[4] = {nullptr, nullptr, nullptr, nullptr};
};

struct ps_plan_s {
    int N = 0, log2n = 0, Nf = 0, K = 0, m = 0, C = 0;
    double dt = 1, f_max = 0, window_param = 0.14;
    uint32_t orders = 0;
    int window = 0, precision = 0, schedule = 0;
    int estimator = PS_EST_KSTAT;
    bool interlaced = false;
    // Complex signals: output grid Ng = 2 N_f - 1 (signed bins), coefficient
    // column c holds bin c - jmax, the first factors of grid index k' sit at
    // column k' + col0; the transform runs at twice the frame length's log2.
    bool cplx = false;
    int Ng = 0, col0 = 0, jmax = 0, log2n_fft = 0;
    int s4_shift = 0;       // S4 plane parallel to the cut (complex signals)
    // N not a power of two: the direct transform (k_window_dft) instead of the
    // FFT, in two stages N = dft_n1 (N / dft_n1) when N has a divisor of at least
    // 8 below its square root (k_window_dft2), else in one
    bool dft = false;
    int dft_n1 = 0;
    std::vector<int8_t> c2, c3, c4;
    double sum_g[5] = {0, 0, 0, 0, 0};
    int T = 0, TX = 0;
    int n_tiles[4] = {0, 0, 0, 0};   // per ps::TileKind
    float* d_g = nullptr;
    float2* d_tw = nullptr;
    int2* d_tiles[4] = {nullptr, nullptr, nullptr, nullptr};
    int n_cu = 256, bpc_s3 = 2, bpc_s4 = 2, bpc_s4x = 2;
    // Single-channel S4 on the matrix cores with operands scaled and split
    // once per column and chunk by the centring pass (scaled FP16 x 2, real
    // signals, the cut, m <= ps::kOpFrames).
    bool s4_pre = false;
    // Launch configuration (ps_plan_set_tuning / ps_plan_autotune).
    int tile_group = 8;     // tile order: tile_group x tile_group blocks
    int s3_fb = 0;          // S3 frame batch; 0: chosen by m
    // Pinned host staging of the per-execute work tables (two, used in turn;
    // an event guards reuse until the copy that read it has finished).
    char* h_stage[2] = {nullptr, nullptr};
    size_t h_cap[2] = {0, 0};
    hipEvent_t h_ev[2] = {nullptr, nullptr};
    int h_next = 0;
    // Stage timing (ps_profile_enable): event pairs recorded on the stream.
    bool prof = false;
    struct Timed {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Timed> timed;

    bool has(int order) const { return (orders >> order) & 1u; }
    bool c3opt() const { return estimator == PS_EST_C3OPT && has(3); }
    int n2() const { return has(2) ? (int)c2.size() / 2 : 0; }
    int n3() const { return has(3) ? (int)c3.size() / 3 : 0; }
    int n4() const { return has(4) ? (int)c4.size() / 4 : 0; }
    bool s3_sym(int i) const { return c3[3 * i] == c3[3 * i + 1]; }
    // A plane (s4_shift != 0) has neither the single-channel structure nor
    // the transposition symmetry of the cut: the cross-channel kernels on full
    // grids compute it.
    bool s4_single(int i) const {
        const int8_t* q = &c4[4 * i];
        return s4_shift == 0 && q[0] == q[1] && q[1] == q[2] && q[2] == q[3];
    }
    // S4_abcd(k,l) = S4_cdab(l,k): symmetric grid when (a,b) = (c,d).
    bool s4_sym(int i) const {
        const int8_t* q = &c4[4 * i];
        return s4_shift == 0 && q[0] == q[2] && q[1] == q[3];
    }
    // Frame lengths: fc[0] mirrors the fields above (same device tables);
    // fc[1..] are the further frame lengths records may carry.
    std::vector<FrameClass> fc;
    // class of a record's frame length (0: the plan's), -1 if not declared
    int class_of(int frame_len) const {
        if (frame_len == 0 || frame_len == N) return 0;
        for (size_t i = 1; i < fc.size(); ++i)
            if (fc[i].N == frame_len) return (int)i;
        return -1;
    }
};

namespace {

// Units (tile, chunk) per block of one stage in the batched schedule.  A block
// belongs to one segment, so a segment of U units gets ceil(U / L) blocks of at
// most L units.  L is chosen among candidates (whole waves of resident blocks
// over the stage's total, and even cuts of the largest segment) to minimise
// the makespan estimate waves x (L + 1), waves = ceil(blocks / slots): with
// many segments the plain ceil(U_stage / slots) leaves a nearly empty second
// wave of blocks.  The + 1 charges each block one unit for its partial-sum
// write, which favours fewer, longer blocks among equals.
int64_t units_per_block(const std::vector<int64_t>& U_seg, int64_t slots) {
    int64_t U = 0, U_max = 0;
    for (int64_t u : U_seg) {
        U += u;
        U_max = std::max(U_max, u);
    }
    if (U == 0) return 1;
    slots = std::max<int64_t>(slots, 1);
    auto cost = [&](int64_t L, int64_t& blocks) {
        blocks = 0;
        for (int64_t u : U_seg) blocks += (u + L - 1) / L;
        return (double)((blocks + slots - 1) / slots) * (double)(L + 1);
    };
    int64_t best_L = std::max<int64_t>(1, (U + slots - 1) / slots), best_blocks = 0;
    double best = cost(best_L, best_blocks);
    auto consider = [&](int64_t L) {
        if (L < 1) return;
        int64_t blocks = 0;
        const double c = cost(L, blocks);
        if (c < best || (c == best && blocks < best_blocks)) {
            best = c;
            best_L = L;
            best_blocks = blocks;
        }
    };
    for (int64_t w = 1; w <= 32; ++w) consider((U + slots * w - 1) / (slots * w));
    for (int64_t k = 1; k <= 64; ++k) consider((U_max + k - 1) / k);
    return best_L;
}
int32_t seg_blocks(int64_t T, int64_t Np, int64_t L, bool per_chunk) {
    if (per_chunk) return (int32_t)T;
    const int64_t U = T * Np;
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(U, (U + L - 1) / L));
}

// Window (FP64, its power sums kept), FFT twiddles exp(+2 pi j t / N2)
// rounded once to FP32 followed by the per-pass tables of a transform of
// 2^tw_log2 points, and the tile tables of one frame length, uploaded to the
// device (synchronous).  On failure the tables allocated so far stay in `c`
// for the caller to free.
hipError_t build_class_tables(const ps_plan_s* p, FrameClass& c, int tw_log2, int N2) {
    const int N = c.N;
    std::vector<double> g;
    make_window(p->window, N, p->window_param, g);
    for (int n = 0; n < 5; ++n) {
        double sum = 0;
        for (double v : g) sum += std::pow(v, n);
        c.sum_g[n] = sum;
    }
    std::vector<float> gf(N);
    for (int i = 0; i < N; ++i) gf[i] = (float)g[i];
    const double two_pi = 6.28318530717958647692;
    std::vector<float2> tw;
    tw.reserve(N2 + ps::fft_twiddle_count(tw_log2));
    for (int t = 0; t < N2; ++t) {
        const double ang = two_pi * t / N2;
        tw.push_back(make_float2((float)std::cos(ang), (float)std::sin(ang)));
    }
    // per-pass tables of the transform's later passes, [r][k]
    const int R2 = ps::fft_radix2(tw_log2), R3 = ps::fft_radix3(tw_log2);
    const int pass_r[2] = {R2, R3}, pass_ns[2] = {16, 16 * R2};
    for (int q = 0; q < 2; ++q)
        for (int r = 0; r < pass_r[q]; ++r)
            for (int k = 0; k < pass_ns[q]; ++k) {
                const double ang = two_pi * r * k / ((double)pass_r[q] * pass_ns[q]);
                tw.push_back(make_float2((float)std::cos(ang), (float)std::sin(ang)));
            }
    c.T = (c.Ng + ps::kTile - 1) / ps::kTile;
    c.TX = (c.Ng + ps::kTileX - 1) / ps::kTileX;
    std::vector<int2> tiles[4];
    tile_order(c.T, p->tile_group, tiles[ps::kSym64], tiles[ps::kFull64]);
    tile_order(c.TX, p->tile_group, tiles[ps::kSym32], tiles[ps::kFull32]);
    for (int i = 0; i < 4; ++i) c.n_tiles[i] = (int)tiles[i].size();
    auto upload = [&](void** dst, const void* src, size_t bytes) -> hipError_t {
        hipError_t e = hipMalloc(dst, std::max<size_t>(bytes, 16));
        if (e != hipSuccess) return e;
        return bytes ? hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
    };
    hipError_t e = upload((void**)&c.d_g, gf.data(), gf.size() * sizeof(float));
    if (e == hipSuccess) e = upload((void**)&c.d_tw, tw.data(), tw.size() * sizeof(float2));
    if (e == hipSuccess && p->dft) {
        // exp(+2 pi j t / N) for the direct transform: long double angle, one rounding
        std::vector<double2> t64(N);
        for (int t = 0; t < N; ++t) {
            const long double ang = 2.0L * 3.14159265358979323846264338327950288L * t / N;
            t64[t] = make_double2((double)std::cos(ang), (double)std::sin(ang));
        }
        e = upload((void**)&c.d_tw64, t64.data(), t64.size() * sizeof(double2));
    }
    for (int i = 0; i < 4 && e == hipSuccess; ++i)
        e = upload((void**)&c.d_tiles[i], tiles[i].data(), tiles[i].size() * sizeof(int2));
    return e;
}

// ------------------------------------------------------------ batch description
struct RecInfo {
    int64_t Np = 0, F = 0;
    int cls = 0;            // frame length (plan class)
    int bc = 0;             // its entry in Batch.bc
    int64_t frame0 = 0;     // first frame within its class's coefficient block
    int64_t chunk0c = 0;    // first chunk within its class
    int64_t chunk0 = 0;     // first chunk of the batch, class-major (per-chunk S1 means)
};

// The records of one frame length within a batch: their coefficient block
// [C][rows][K] (and, with c3^(opt), the block of S3 rows [C][rows3][K]).
struct BatchClass {
    int cls = 0;
    int64_t F = 0, chunks = 0;      // frames and chunks per channel
    int64_t chunk_base = 0;         // first chunk of the class in the batch
    int64_t rows = 0, rows3 = 0;    // rows per channel of its blocks
    size_t coef_off = 0, coef3_off = 0;     // byte offsets in the workspace
    // pre-split S4 operands: chunk slots per channel, byte offsets of the
    // operand records [C][op_chunks][3][kOpPieces][N_f'][4] and the FP64
    // (P sum, scale s^2) pairs [C][op_chunks][N_f'][2] (N_f' = N_f rounded up
    // to the tile edge)
    int64_t op_chunks = 0;
    size_t op4_off = 0, p4_off = 0;
    int rd0 = 0, n_rd = 0;          // its record descriptors in Batch.rd
};

struct SegTable {
    std::vector<ps::Seg> v;
    int64_t n_items = 0;
    size_t dev_off = 0;     // byte offset of the table inside the table region
    void add(ps::Seg s, int64_t items) {
        s.item0 = n_items;
        n_items += items;
        v.push_back(s);
    }
};

// One set of launches: every record (batched schedule) or one record
// (per-chunk schedule).
// (The list of tables is a function, not a stored array of pointers: groups
// live in a vector, and a copied group must not point into its original.)
struct Group {
    int rec = -1;           // record of a per-chunk group
    SegTable s2, s3, s4s, s4x, f2, f3, f4, f1;
    SegTable acc;           // running accumulation (ps_stream_push) instead of f2..f4
    std::array<SegTable*, 9> all() { return {&s2, &s3, &s4s, &s4x, &f2, &f3, &f4, &f1, &acc}; }
    std::array<const SegTable*, 9> all() const { return {&s2, &s3, &s4s, &s4x, &f2, &f3, &f4, &f1, &acc}; }
};

// With interlaced windows every caller record r becomes two internal records:
// 2r, its frames from sample 0, and 2r + 1, its frames from sample N/2 (stride
// 2); the finalize of 2r combines both.
// Columns of the S4 operand records: N_f rounded up to the tile edge.
inline int op_cols(int nf) { return (nf + ps::kTile - 1) / ps::kTile * ps::kTile; }

struct Batch {
    // single-channel S4 combinations of the plan (those the pre-split operands serve)
    static int n_s4_single(const ps_plan_s* p) {
        int n = 0;
        for (int i = 0; i < p->n4(); ++i) n += p->s4_single(i) ? 1 : 0;
        return n;
    }
    int stride = 1;                 // internal records per caller record
    std::vector<RecInfo> ri;        // per internal record
    std::vector<ps::RecDesc> rd;    // grouped by class, frame0 ascending within a class
    std::vector<BatchClass> bc;     // the frame lengths present, in plan class order
    int64_t F_tot = 0, chunks_tot = 0;
    std::vector<Group> groups;
    size_t coef_bytes = 0;          // coefficient blocks at the workspace's start
    size_t off_tab = 0, off_part = 0, off_s1 = 0, total = 0;
    size_t tab_bytes = 0;
    int64_t part_doubles = 0;
};

size_t align64(size_t x) { return (x + 63) & ~size_t(63); }

// Bytes per sample of a record's dtype.
size_t elem_size(int dtype) {
    return dtype == PS_F32 ? 4 : dtype == PS_F64 ? 8 : dtype == PS_I16 ? 2 : dtype == PS_C64 ? 8 : 16;
}

// Finalize scales of each order: the estimator's prefactor (k-statistics of
// Section 4.1, or the natural estimator of Section 6: c2 = s2 / m, c3 = t3 / m,
// c4 = (m M4 - pairs) / m^2) times dt^(n-1) / sum g^n (Sections 3 and 4);
// s4 goes with the kernels' form M4 - gamma (pairs).
struct Scales {
    double s1, s2, s3, s4;
};
Scales spectrum_scales(const ps_plan_s* p, const double* sum_g) {
    const int m = p->m;
    const double dt = p->dt;
    const bool nat = p->estimator == PS_EST_NATURAL;
    const double c4a = nat ? m : m * (m + 1.0);
    Scales sc;
    sc.s1 = 1.0 / sum_g[1];
    sc.s2 = dt / ((nat ? m : m - 1) * sum_g[2]);
    // c3^(opt): the S3 sum over the m + 1 rows of each chunk times (m+4)/((m+1) m)
    const double c3f = p->c3opt() ? (m + 4.0) / ((m + 1.0) * m) : nat ? 1.0 / m : m / ((double)(m - 1) * (m - 2));
    sc.s3 = dt * dt * c3f / sum_g[3];
    sc.s4 = dt * dt * dt * c4a / ((nat ? (double)m * m : (double)(m - 1) * (m - 2) * (m - 3)) * sum_g[4]);
    return sc;
}

void finish_layout(const ps_plan_s* p, Batch& B);

void build_batch(const ps_plan_s* p, const ps_record* recs, int n, const ps_output* outs, Batch& B) {
    const bool per_chunk = p->schedule == PS_SCHED_PER_CHUNK;
    const int m = p->m;
    const bool opt3 = p->c3opt();
    B.stride = p->interlaced ? 2 : 1;
    const int n_int = n * B.stride;
    B.ri.assign(n_int, RecInfo{});
    // chunk counts and frame lengths
    std::vector<int> bc_of(p->fc.size(), -1);
    for (int ir = 0; ir < n_int; ++ir) {
        const ps_record& rec = recs[ir / B.stride];
        RecInfo& q = B.ri[ir];
        q.cls = std::max(0, p->class_of(rec.frame_len));
        const int Nr = p->fc[q.cls].N;
        // the shifted frame set of interlaced windows starts T/2 = N/2 samples later
        const int64_t skip = (ir % B.stride) ? Nr / 2 : 0;
        q.Np = (std::max<int64_t>(0, rec.n_samples - skip) / Nr) / m;
        q.F = q.Np * m;
        bc_of[q.cls] = 0;
    }
    for (size_t c = 0; c < p->fc.size(); ++c)
        if (bc_of[c] == 0) {
            bc_of[c] = (int)B.bc.size();
            B.bc.push_back(BatchClass{});
            B.bc.back().cls = (int)c;
        }
    // frames and chunks numbered per class; descriptors grouped by class
    int64_t chunk_base = 0;
    for (size_t b = 0; b < B.bc.size(); ++b) {
        BatchClass& k = B.bc[b];
        k.rd0 = (int)B.rd.size();
        for (int ir = 0; ir < n_int; ++ir) {
            RecInfo& q = B.ri[ir];
            if (q.cls != k.cls) continue;
            const ps_record& rec = recs[ir / B.stride];
            const int64_t skip = (ir % B.stride) ? p->fc[q.cls].N / 2 : 0;
            q.bc = (int)b;
            q.frame0 = k.F;
            q.chunk0c = k.chunks;
            k.F += q.F;
            k.chunks += q.Np;
            ps::RecDesc d{};
            d.data = q.Np > 0 ? static_cast<const char*>(rec.d_data) + skip * elem_size(rec.dtype) : rec.d_data;
            d.chan_stride = rec.channel_stride;
            d.frame0 = q.frame0;
            d.dtype = rec.dtype;
            B.rd.push_back(d);
        }
        k.n_rd = (int)B.rd.size() - k.rd0;
        k.chunk_base = chunk_base;
        chunk_base += k.chunks;
        B.F_tot += k.F;
        B.chunks_tot += k.chunks;
    }
    for (RecInfo& q : B.ri) q.chunk0 = B.bc[q.bc].chunk_base + q.chunk0c;
    // coefficient blocks (the per-chunk schedule holds one chunk per class)
    size_t off = 0;
    for (BatchClass& k : B.bc) {
        k.rows = per_chunk ? m : k.F;
        k.coef_off = off;
        off = align256(off + (size_t)p->C * k.rows * p->fc[k.cls].K * sizeof(float2));
    }
    for (BatchClass& k : B.bc) {
        k.rows3 = opt3 ? (per_chunk ? 1 : k.chunks) * (m + 1) : 0;
        k.coef3_off = off;
        off = align256(off + (size_t)p->C * k.rows3 * p->fc[k.cls].K * sizeof(float2));
    }
    const bool op4 = p->s4_pre && B.n_s4_single(p) > 0;
    for (BatchClass& k : B.bc) {
        const int64_t ng = op_cols(p->fc[k.cls].Ng);
        k.op_chunks = op4 ? (per_chunk ? 1 : k.chunks) : 0;
        k.op4_off = off;
        off = align256(off + (size_t)p->C * k.op_chunks * 3 * ng * ps::kOpWords * sizeof(uint32_t));
        k.p4_off = off;
        off = align256(off + (size_t)p->C * k.op_chunks * 2 * ng * sizeof(double));
    }
    B.coef_bytes = off;

    // groups (interlaced windows: batched schedule only)
    if (per_chunk) {
        for (int r = 0; r < n; ++r)
            if (B.ri[r].Np > 0) {
                B.groups.emplace_back();
                B.groups.back().rec = r;
            }
    } else {
        B.groups.emplace_back();
    }
    const int64_t TT = (int64_t)ps::kTile * ps::kTile, TX = (int64_t)ps::kTileX * ps::kTileX;
    int64_t part = 0;
    for (Group& G : B.groups) {
        const int r_lo = per_chunk ? G.rec : 0, r_hi = per_chunk ? G.rec + 1 : n_int;
        // units of every segment per stage, for the block counts
        std::vector<int64_t> U2, U3, U4s, U4x;
        for (int r = r_lo; r < r_hi; ++r) {
            const int64_t Np = B.ri[r].Np;
            if (Np == 0) continue;
            const FrameClass& fc = p->fc[B.ri[r].cls];
            const int kblocks = (fc.Ng + 255) / 256;
            for (int i = 0; i < p->n2(); ++i) U2.push_back((int64_t)kblocks * Np);
            for (int i = 0; i < p->n3(); ++i) U3.push_back(fc.n_tiles[p->s3_sym(i) ? ps::kSym64 : ps::kFull64] * Np);
            for (int i = 0; i < p->n4(); ++i) {
                if (p->s4_single(i)) U4s.push_back(fc.n_tiles[ps::kSym64] * Np);
                else U4x.push_back(fc.n_tiles[p->s4_sym(i) ? ps::kSym32 : ps::kFull32] * Np);
            }
        }
        const int64_t L2 = units_per_block(U2, 4LL * p->n_cu);
        const int64_t L3 = units_per_block(U3, (int64_t)p->n_cu * p->bpc_s3);
        const int64_t L4s = units_per_block(U4s, (int64_t)p->n_cu * p->bpc_s4);
        const int64_t L4x = units_per_block(U4x, (int64_t)p->n_cu * p->bpc_s4x);
        // finalize segments of the last first-set record, per combination, for
        // its shifted twin (which follows it) to attach its partial sums to
        std::vector<size_t> fin2(p->n2()), fin3(p->n3()), fin4(p->n4()), fin1(p->C);
        for (int r = r_lo; r < r_hi; ++r) {
            const RecInfo& q = B.ri[r];
            if (q.Np == 0) continue;
            const FrameClass& fc = p->fc[q.cls];
            const BatchClass& k = B.bc[q.bc];
            const int K = fc.K, Nf = fc.Ng;     // Nf: points per output axis
            const int64_t nf2 = (int64_t)Nf * Nf;
            const int kblocks = (Nf + 255) / 256;
            const Scales scl = spectrum_scales(p, fc.sum_g);
            const bool twin = r % B.stride != 0;   // shifted set: no output of its own
            const ps_output* o = outs ? &outs[r / B.stride] : nullptr;
            // a finalize segment for the first set, or the twin's sums attached to it
            auto finalize = [&](SegTable& f, std::vector<size_t>& fin, int i, const ps::Seg& sg, int64_t items) {
                if (!twin) {
                    fin[i] = f.v.size();
                    f.add(sg, items);
                } else {
                    ps::Seg& a = f.v[fin[i]];
                    a.part2 = sg.part;
                    a.n_chunks2 = sg.n_chunks;
                    a.blocks2 = sg.blocks;
                }
            };
            ps::Seg base{};
            // the record's chunk 0 (per-chunk schedule: the class block holds the current chunk)
            base.coef = (int64_t)(k.coef_off / sizeof(float2)) + (per_chunk ? 0 : q.frame0 * K);
            base.cs = k.rows * K;
            base.K = K;
            base.Nf = Nf;
            base.n_chunks = (int32_t)q.Np;
            if (p->has(1)) {
                // S1 per channel: the record's per-chunk means of a_0 from index chunk0
                for (int c = 0; c < p->C; ++c) {
                    ps::Seg sg = base;
                    sg.part = q.chunk0;
                    sg.ch[0] = c;
                    sg.out = o && o->d_s1 ? o->d_s1 + 2 * c : nullptr;
                    sg.err = o && o->d_s1_err ? o->d_s1_err + 2 * c : nullptr;
                    sg.scale = scl.s1;
                    finalize(G.f1, fin1, c, sg, 1);
                }
            }
            for (int i = 0; i < p->n2(); ++i) {
                ps::Seg sg = base;
                sg.n_tiles = kblocks;
                sg.blocks = seg_blocks(kblocks, q.Np, L2, per_chunk);
                sg.tiles = 0;
                for (int j = 0; j < 2; ++j) sg.ch[j] = p->c2[2 * i + j];
                sg.part = part;
                part += ps::Sched{sg.n_tiles, q.Np, sg.blocks}.n_slots() * 4 * 256;
                sg.out = o && o->d_s2 ? o->d_s2 + 2 * (int64_t)i * Nf : nullptr;
                sg.err = o && o->d_s2_err ? o->d_s2_err + 2 * (int64_t)i * Nf : nullptr;
                sg.scale = scl.s2;
                sg.ncomp = 4;
                G.s2.add(sg, sg.blocks);
                finalize(G.f2, fin2, i, sg, kblocks);
            }
            for (int i = 0; i < p->n3(); ++i) {
                ps::Seg sg = base;
                const bool sym = p->s3_sym(i);
                sg.tiles = sym ? ps::kSym64 : ps::kFull64;
                sg.tile_tab = fc.d_tiles[sg.tiles];
                sg.n_tiles = fc.n_tiles[sg.tiles];
                sg.blocks = seg_blocks(sg.n_tiles, q.Np, L3, per_chunk);
                for (int j = 0; j < 3; ++j) sg.ch[j] = p->c3[3 * i + j];
                if (opt3) {     // the S3 rows of c3^(opt): m + 1 per chunk
                    sg.coef = (int64_t)(k.coef3_off / sizeof(float2)) + (per_chunk ? 0 : q.chunk0c * (m + 1) * K);
                    sg.cs = k.rows3 * K;
                }
                sg.part = part;
                part += ps::Sched{sg.n_tiles, q.Np, sg.blocks}.n_slots() * 4 * TT;
                sg.out = o && o->d_s3 ? o->d_s3 + 2 * i * nf2 : nullptr;
                sg.err = o && o->d_s3_err ? o->d_s3_err + 2 * i * nf2 : nullptr;
                sg.scale = scl.s3;
                sg.sym = sym;
                sg.ncomp = 4;
                G.s3.add(sg, sg.blocks);
                finalize(G.f3, fin3, i, sg, (int64_t)sg.n_tiles * (TT / 256));
            }
            for (int i = 0; i < p->n4(); ++i) {
                ps::Seg sg = base;
                const bool single = p->s4_single(i), sym = p->s4_sym(i);
                sg.tiles = single ? ps::kSym64 : (sym ? ps::kSym32 : ps::kFull32);
                sg.tile_tab = fc.d_tiles[sg.tiles];
                sg.n_tiles = fc.n_tiles[sg.tiles];
                sg.blocks = seg_blocks(sg.n_tiles, q.Np, single ? L4s : L4x, per_chunk);
                for (int j = 0; j < 4; ++j) sg.ch[j] = p->c4[4 * i + j];
                sg.ncomp = single ? 2 : 4;
                if (single && k.op_chunks > 0) {
                    const int64_t ngp = op_cols(Nf);
                    const int64_t rec = 3 * ngp * ps::kOpWords;       // uint32 per chunk
                    sg.op4 = (int64_t)(k.op4_off / sizeof(uint32_t)) + (per_chunk ? 0 : q.chunk0c * rec);
                    sg.op4_cs = k.op_chunks * rec;
                    sg.p4 = (int64_t)(k.p4_off / sizeof(double)) + (per_chunk ? 0 : q.chunk0c * 2 * ngp);
                    sg.p4_cs = k.op_chunks * 2 * ngp;
                }
                sg.part = part;
                part += ps::Sched{sg.n_tiles, q.Np, sg.blocks}.n_slots() * sg.ncomp * (single ? TT : TX);
                sg.out = o && o->d_s4 ? o->d_s4 + 2 * i * nf2 : nullptr;
                sg.err = o && o->d_s4_err ? o->d_s4_err + 2 * i * nf2 : nullptr;
                sg.scale = scl.s4;
                sg.sym = sym;
                (single ? G.s4s : G.s4x).add(sg, sg.blocks);
                finalize(G.f4, fin4, i, sg, (int64_t)sg.n_tiles * ((single ? TT : TX) / 256));
            }
        }
    }
    B.part_doubles = part;
    finish_layout(p, B);
}

// Table region and workspace offsets of a built batch (again after tables
// were added to its groups).
void finish_layout(const ps_plan_s* p, Batch& B) {
    // table region: record descriptors, then every segment table
    size_t tab = align64(sizeof(ps::RecDesc) * std::max<size_t>(1, B.rd.size()));
    for (Group& G : B.groups)
        for (SegTable* t : G.all()) {
            t->dev_off = tab;
            tab = align64(tab + sizeof(ps::Seg) * t->v.size());
        }
    B.tab_bytes = tab;
    size_t off = B.coef_bytes;
    B.off_tab = off;
    off = align256(off + B.tab_bytes);
    B.off_part = off;
    off = align256(off + (size_t)B.part_doubles * sizeof(double));
    B.off_s1 = off;
    if (p->has(1)) off = align256(off + (size_t)p->C * B.chunks_tot * sizeof(float2));
    B.total = std::max<size_t>(off, 256);
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Optional event pair around one stage launch (only while profiling).
struct StageTimer {
    ps_plan_s* p;
    hipStream_t st;
    int stage;
    hipEvent_t a = nullptr;
    StageTimer(ps_plan_s* p_, hipStream_t st_, int stage_) : p(p_), st(st_), stage(stage_) {
        if (p->prof && hipEventCreate(&a) == hipSuccess && hipEventRecord(a, st) != hipSuccess) {
            (void)hipEventDestroy(a);
            a = nullptr;
        }
    }
    ~StageTimer() {
        if (!a) return;
        hipEvent_t b = nullptr;
        if (hipEventCreate(&b) == hipSuccess && hipEventRecord(b, st) == hipSuccess) {
            p->timed.push_back({stage, a, b});
        } else {
            (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    }
};

ps_status check_record(const ps_plan_s* p, const ps_record* r) {
    if (!r) return fail(PS_E_INVALID_ARG, "record is NULL");
    if (r->dtype < PS_F32 || r->dtype > PS_C128) return fail(PS_E_INVALID_ARG, "bad dtype %d", r->dtype);
    if ((r->dtype >= PS_C64) != p->cplx)
        return fail(PS_E_INVALID_ARG, "dtype %d does not match the plan's %s signal", r->dtype,
                    p->cplx ? "complex" : "real");
    if (r->n_samples < 0) return fail(PS_E_INVALID_ARG, "n_samples < 0");
    const int cls = p->class_of(r->frame_len);
    if (cls < 0) return fail(PS_E_INVALID_ARG, "record frame_len %d is not among the plan's frame lengths", r->frame_len);
    if (p->C > 1 && r->channel_stride < r->n_samples)
        return fail(PS_E_INVALID_ARG, "channel_stride (%lld) < n_samples (%lld)",
                    (long long)r->channel_stride, (long long)r->n_samples);
    if ((r->n_samples / p->fc[cls].N) / p->m > INT32_MAX)
        return fail(PS_E_UNSUPPORTED, "record of %lld samples: at most 2^31 - 1 chunks per record",
                    (long long)r->n_samples);
    const size_t esz = elem_size(r->dtype);
    if (r->n_samples >= (int64_t)p->fc[cls].N * p->m) {
        if (!r->d_data) return fail(PS_E_INVALID_ARG, "record data is NULL");
        if (!aligned(r->d_data, esz)) return fail(PS_E_INVALID_ARG, "record data misaligned");
    }
    return PS_OK;
}

}  // namespace

extern "C" {

int32_t ps_abi_version(void) { return PS_ABI_VERSION; }

const char* ps_status_string(ps_status s) {
    switch (s) {
        case PS_OK: return "PS_OK";
        case PS_E_INVALID_ARG: return "PS_E_INVALID_ARG";
        case PS_E_UNSUPPORTED: return "PS_E_UNSUPPORTED";
        case PS_E_WORKSPACE: return "PS_E_WORKSPACE";
        case PS_E_HIP: return "PS_E_HIP";
        case PS_E_INTERNAL: return "PS_E_INTERNAL";
    }
    return "PS_E_UNKNOWN";
}

const char* ps_last_error(void) { return g_last_error.c_str(); }

ps_status ps_enumerate_combos(int32_t n_channels, int32_t order, int8_t* out, int32_t* n) {
    if (!n || n_channels < 1 || n_channels > 4 || order < 2 || order > 4)
        return fail(PS_E_INVALID_ARG, "bad argument");
    std::vector<int8_t> a2, a3, a4;
    all_combos(n_channels, a2, a3, a4);
    const std::vector<int8_t>& v = order == 2 ? a2 : order == 3 ? a3 : a4;
    const int32_t count = (int32_t)(v.size() / order);
    if (out) {
        if (*n < count) return fail(PS_E_INVALID_ARG, "capacity %d < %d", *n, count);
        std::memcpy(out, v.data(), v.size());
    }
    *n = count;
    return PS_OK;
}

ps_status ps_plan_destroy(ps_plan_t p) {
    if (!p) return PS_OK;
    for (auto& t : p->timed) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (int i = 0; i < 2; ++i) {
        if (p->h_ev[i]) {
            (void)hipEventSynchronize(p->h_ev[i]);
            (void)hipEventDestroy(p->h_ev[i]);
        }
        if (p->h_stage[i]) (void)hipHostFree(p->h_stage[i]);
    }
    for (FrameClass& c : p->fc) {
        (void)hipFree(c.d_g);
        (void)hipFree(c.d_tw);
        (void)hipFree(c.d_tw64);
        for (int i = 0; i < 4; ++i) (void)hipFree(c.d_tiles[i]);
    }
    delete p;
    return PS_OK;
}

ps_status ps_plan_create(const ps_config* cfg, ps_plan_t* out) {
    if (!out) return fail(PS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(PS_E_INVALID_ARG, "cfg is NULL");
    // (a ps_config without the trailing frame_len_set is accepted: no further frame lengths)
    if (cfg->struct_size < offsetof(ps_config, frame_len_set))
        return fail(PS_E_INVALID_ARG, "struct_size %u < %zu", cfg->struct_size, offsetof(ps_config, frame_len_set));
    const uint32_t fl_set = cfg->struct_size >= sizeof(ps_config) ? (uint32_t)cfg->frame_len_set : 0u;
    const uint32_t known = PS_ORDER_S1 | PS_ORDER_S2 | PS_ORDER_S3 | PS_ORDER_S4;
    if (cfg->orders == 0 || (cfg->orders & ~known))
        return fail(PS_E_INVALID_ARG, "orders must be a non-empty subset of {1,2,3,4}");
    if (cfg->n_channels < 1 || cfg->n_channels > 4)
        return fail(PS_E_INVALID_ARG, "n_channels must be 1..4");
    const int N = cfg->frame_len;
    // 256..8192: powers of two by the FFT, any other length by the direct transform
    if (N < 256 || N > 8192) return fail(PS_E_UNSUPPORTED, "frame_len %d outside 256..8192", N);
    const bool dft = (N & (N - 1)) != 0;
    if (dft && cfg->complex_signal)
        return fail(PS_E_UNSUPPORTED, "complex signals need a power-of-two frame_len (N = %d)", N);
    if (!(cfg->dt > 0) || !std::isfinite(cfg->dt)) return fail(PS_E_INVALID_ARG, "dt must be > 0");
    // c3^(opt) (S3 only) is defined from m = 2
    const int min_m = (cfg->orders & PS_ORDER_S4)   ? 4
                      : (cfg->orders & PS_ORDER_S3) ? (cfg->estimator == PS_EST_C3OPT ? 2 : 3)
                      : (cfg->orders & PS_ORDER_S2) ? 2
                                                    : 1;
    if (cfg->m < min_m) return fail(PS_E_INVALID_ARG, "m = %d < %d (k-statistic denominator)", cfg->m, min_m);
    if (cfg->window < PS_WIN_HANN || cfg->window > PS_WIN_ACG)
        return fail(PS_E_INVALID_ARG, "unknown window %d", cfg->window);
    if (cfg->window == PS_WIN_ACG && !(cfg->window_param > 0))
        return fail(PS_E_INVALID_ARG, "acG window needs sigma_t > 0");
    if (cfg->precision < PS_PREC_FP32 || cfg->precision > PS_PREC_FP16X2S)
        return fail(PS_E_INVALID_ARG, "unknown precision %d", cfg->precision);
    if (cfg->precision == PS_PREC_FP16X2S && (cfg->orders & PS_ORDER_S4) && cfg->m > 10)
        return fail(PS_E_UNSUPPORTED, "FP16X2S needs m <= 10 (one scale per chunk and column)");
    if (cfg->schedule != PS_SCHED_BATCHED && cfg->schedule != PS_SCHED_PER_CHUNK)
        return fail(PS_E_INVALID_ARG, "unknown schedule %d", cfg->schedule);
    if (cfg->interlaced != 0 && cfg->interlaced != 1) return fail(PS_E_INVALID_ARG, "interlaced must be 0 or 1");
    if (cfg->estimator != PS_EST_KSTAT && cfg->estimator != PS_EST_NATURAL && cfg->estimator != PS_EST_C3OPT)
        return fail(PS_E_INVALID_ARG, "unknown estimator %d", cfg->estimator);
    if (cfg->interlaced && cfg->schedule != PS_SCHED_BATCHED)
        return fail(PS_E_UNSUPPORTED, "interlaced windows need the batched schedule");
    if (cfg->complex_signal != 0 && cfg->complex_signal != 1) return fail(PS_E_INVALID_ARG, "complex_signal must be 0 or 1");
    if (cfg->s4_shift != 0 && !cfg->complex_signal)
        return fail(PS_E_UNSUPPORTED, "S4 planes (s4_shift != 0) need complex_signal = 1");
    if (cfg->complex_signal && cfg->frame_len > 4096)
        return fail(PS_E_UNSUPPORTED, "complex signals: frame_len up to 4096");
    int Nf = cfg->n_freq;
    if (Nf == 0) {
        if (!(cfg->f_max >= 0) || !std::isfinite(cfg->f_max))
            return fail(PS_E_INVALID_ARG, "n_freq == 0 needs f_max >= 0");
        Nf = (int)std::floor(cfg->f_max * N * cfg->dt) + 1;
    }
    if (Nf < 1) return fail(PS_E_INVALID_ARG, "n_freq must be >= 1");
    const bool s3 = cfg->orders & PS_ORDER_S3;
    if (s3 && 2 * (Nf - 1) > N / 2)
        return fail(PS_E_INVALID_ARG, "S3 needs 2 (N_f - 1) <= N/2 (N_f = %d, N = %d)", Nf, N);
    if (!s3 && Nf - 1 > N / 2)
        return fail(PS_E_INVALID_ARG, "N_f - 1 must be <= N/2 (N_f = %d, N = %d)", Nf, N);
    if (cfg->s4_shift != 0 && Nf - 1 + std::abs(cfg->s4_shift) > N / 2)
        return fail(PS_E_INVALID_ARG, "S4 plane needs N_f - 1 + |q| <= N/2 (q = %d)", cfg->s4_shift);

    // Further frame lengths (frame_len_set): powers of two 256..8192, real
    // signals; N_f scales with N when n_freq is given, else follows f_max.
    int class_nf[14] = {0};
    if (fl_set) {
        if (fl_set & ~0x3F00u) return fail(PS_E_INVALID_ARG, "frame_len_set holds bits outside 8..13 (256..8192)");
        if (cfg->complex_signal || dft)
            return fail(PS_E_UNSUPPORTED, "further frame lengths need real signals and a power-of-two frame_len");
        for (int q = 8; q <= 13; ++q) {
            if (!(fl_set >> q & 1u) || (1 << q) == N) continue;
            const int Nq = 1 << q;
            int nfq;
            if (cfg->n_freq > 0) {
                if (((int64_t)Nf * Nq) % N != 0)
                    return fail(PS_E_INVALID_ARG, "n_freq %d does not scale to frame length %d (n_freq * %d / %d)", Nf,
                                Nq, Nq, N);
                nfq = (int)((int64_t)Nf * Nq / N);
            } else {
                nfq = (int)std::floor(cfg->f_max * Nq * cfg->dt) + 1;
            }
            if (nfq < 1) return fail(PS_E_INVALID_ARG, "frame length %d: N_f < 1", Nq);
            if (s3 && 2 * (nfq - 1) > Nq / 2)
                return fail(PS_E_INVALID_ARG, "frame length %d: S3 needs 2 (N_f - 1) <= N/2 (N_f = %d)", Nq, nfq);
            if (!s3 && nfq - 1 > Nq / 2)
                return fail(PS_E_INVALID_ARG, "frame length %d: N_f - 1 must be <= N/2 (N_f = %d)", Nq, nfq);
            class_nf[q] = nfq;
        }
    }

    auto* p = new ps_plan_s();
    p->N = N;
    p->dft = dft;
    if (!dft)
        while ((1 << p->log2n) < N) ++p->log2n;
    if (dft) {
        for (int d = 1; d * d <= N; ++d)
            if (N % d == 0) p->dft_n1 = d;
        if (p->dft_n1 < 8) p->dft_n1 = 0;
    }
    p->Nf = Nf;
    p->cplx = cfg->complex_signal != 0;
    p->Ng = p->cplx ? 2 * Nf - 1 : Nf;
    p->s4_shift = cfg->s4_shift;
    p->jmax = p->cplx ? (s3 ? 2 * (Nf - 1) : Nf - 1) : 0;
    if (p->cplx && (cfg->orders & PS_ORDER_S4)) p->jmax = std::max(p->jmax, Nf - 1 + std::abs(p->s4_shift));
    p->K = p->cplx ? 2 * p->jmax + 1 : (s3 ? 2 * Nf - 1 : Nf);
    p->col0 = p->cplx ? p->jmax - (Nf - 1) : 0;
    p->log2n_fft = p->log2n + (p->cplx ? 1 : 0);
    p->m = cfg->m;
    p->C = cfg->n_channels;
    p->dt = cfg->dt;
    p->f_max = (Nf - 1) / (N * cfg->dt);
    p->orders = cfg->orders;
    p->window = cfg->window;
    p->window_param = cfg->window_param;
    p->precision = cfg->precision;
    p->schedule = cfg->schedule;
    p->interlaced = cfg->interlaced != 0;
    p->estimator = cfg->estimator;

    // Channel combinations: explicit lists or every orbit.
    std::vector<int8_t> a2, a3, a4;
    all_combos(p->C, a2, a3, a4);
    if (p->s4_shift != 0) {     // no symmetry reduces a plane's combinations
        a4.clear();
        for (int i = 0; i < p->C * p->C * p->C * p->C; ++i)
            a4.insert(a4.end(), {(int8_t)(i / (p->C * p->C * p->C)), (int8_t)(i / (p->C * p->C) % p->C),
                                 (int8_t)(i / p->C % p->C), (int8_t)(i % p->C)});
    }
    struct { int n; const int8_t* ptr; int arity; std::vector<int8_t>* dst; std::vector<int8_t>* dflt; } lists[3] = {
        {cfg->n_combos2, cfg->combos2, 2, &p->c2, &a2},
        {cfg->n_combos3, cfg->combos3, 3, &p->c3, &a3},
        {cfg->n_combos4, cfg->combos4, 4, &p->c4, &a4}};
    for (auto& l : lists) {
        if (l.n < 0) {
            delete p;
            return fail(PS_E_INVALID_ARG, "negative combination count");
        }
        if (l.n == 0) {
            *l.dst = *l.dflt;
            continue;
        }
        if (!l.ptr) {
            delete p;
            return fail(PS_E_INVALID_ARG, "combination list is NULL");
        }
        l.dst->assign(l.ptr, l.ptr + (size_t)l.n * l.arity);
        for (int8_t ch : *l.dst)
            if (ch < 0 || ch >= p->C) {
                delete p;
                return fail(PS_E_INVALID_ARG, "combination refers to channel %d of %d", ch, p->C);
            }
    }

    // Tables of the plan's frame length (class 0): the twiddle layout depends
    // on the transform (complex signals: the tables of a real transform of
    // twice the frame length, whose complex transform has the frame length;
    // a frame length that is not a power of two: the FP64 exponentials of the
    // direct transform, beside small unused FFT tables).
    FrameClass c0;
    c0.N = N;
    c0.log2n_fft = p->log2n_fft;
    c0.Nf = p->Nf;
    c0.Ng = p->Ng;
    c0.K = p->K;
    c0.jmax = p->jmax;
    hipError_t e = build_class_tables(p, c0, p->dft ? 8 : p->log2n_fft, p->dft ? N : 1 << p->log2n_fft);
    p->fc.push_back(c0);        // owns the device tables (also freed on failure)
    if (e == hipSuccess) {
        for (int n = 0; n < 5; ++n) p->sum_g[n] = c0.sum_g[n];
        p->T = c0.T;
        p->TX = c0.TX;
        for (int i = 0; i < 4; ++i) p->n_tiles[i] = c0.n_tiles[i];
        p->d_g = c0.d_g;
        p->d_tw = c0.d_tw;
        for (int i = 0; i < 4; ++i) p->d_tiles[i] = c0.d_tiles[i];
    }
    // Further frame lengths (real signals): N_f scaled with N (n_freq given)
    // or taken from f_max, K and the constraints as for class 0.
    for (int q = 8; q <= 13 && e == hipSuccess; ++q) {
        const int Nq = 1 << q;
        if (!(fl_set >> q & 1u) || Nq == N) continue;
        FrameClass c;
        c.N = Nq;
        c.log2n_fft = q;
        c.Nf = class_nf[q];
        c.Ng = c.Nf;
        c.K = s3 ? 2 * c.Nf - 1 : c.Nf;
        e = build_class_tables(p, c, q, Nq);
        p->fc.push_back(c);
    }
    if (e != hipSuccess) {
        ps_plan_destroy(p);
        return fail(PS_E_HIP, "device table setup failed: %s", hipGetErrorString(e));
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        p->n_cu = std::max(1, prop.multiProcessorCount);
    // Pinned staging of the work tables (two, used in turn) and their events,
    // allocated here so that executes need no allocation for batches whose
    // tables fit (larger ones enlarge them, except on the static-scratch path).
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipHostMalloc((void**)&p->h_stage[i], kStagingBytes, hipHostMallocDefault);
        if (e == hipSuccess) p->h_cap[i] = kStagingBytes;
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->h_ev[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = ps::static_scratch_setup();
    if (e != hipSuccess) {
        ps_plan_destroy(p);
        return fail(PS_E_HIP, "plan setup failed: %s", hipGetErrorString(e));
    }
    p->bpc_s3 = ps::s3_blocks_per_cu();
    p->s4_pre = p->precision == PS_PREC_FP16X2S && !p->cplx && p->s4_shift == 0 && p->m <= ps::kOpFrames;
    p->bpc_s4 = p->precision == PS_PREC_FP32     ? ps::s4_blocks_per_cu()
                : p->precision == PS_PREC_BF16X3 ? ps::s4_mfma_blocks_per_cu()
                : p->s4_pre                      ? ps::s4_mfma_pre_blocks_per_cu()
                                                 : ps::s4_mfma_f16_blocks_per_cu();
    p->bpc_s4x = p->precision == PS_PREC_BF16X3 ? ps::s4_cross_mfma_blocks_per_cu() : ps::s4_cross_blocks_per_cu();
    *out = p;
    return PS_OK;
}

// ------------------------------------------------------------ launch configuration
namespace {
hipError_t write_tiles(ps_plan_t p) {
    for (const FrameClass& c : p->fc) {
        std::vector<int2> tiles[4];
        tile_order(c.T, p->tile_group, tiles[ps::kSym64], tiles[ps::kFull64]);
        tile_order(c.TX, p->tile_group, tiles[ps::kSym32], tiles[ps::kFull32]);
        for (int i = 0; i < 4; ++i) {
            if (tiles[i].empty()) continue;
            const hipError_t e = hipMemcpy(c.d_tiles[i], tiles[i].data(), tiles[i].size() * sizeof(int2),
                                           hipMemcpyHostToDevice);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}
bool valid_tuning(const ps_tuning& t) {
    const bool g = t.tile_group == 1 || t.tile_group == 2 || t.tile_group == 4 || t.tile_group == 8 ||
                   t.tile_group == 16;
    const bool f = t.s3_frame_batch == 0 || t.s3_frame_batch == ps::kFrameBatchSmall ||
                   t.s3_frame_batch == ps::kFrameBatchRow || t.s3_frame_batch == ps::kFrameBatch;
    return g && f;
}
}  // namespace

ps_status ps_plan_get_tuning(ps_plan_t p, ps_tuning* t) {
    if (!p || !t) return fail(PS_E_INVALID_ARG, "NULL argument");
    t->tile_group = p->tile_group;
    t->s3_frame_batch = p->s3_fb;
    return PS_OK;
}

ps_status ps_plan_set_tuning(ps_plan_t p, const ps_tuning* t) {
    if (!p || !t) return fail(PS_E_INVALID_ARG, "NULL argument");
    if (!valid_tuning(*t))
        return fail(PS_E_INVALID_ARG, "tuning: tile_group %d (1, 2, 4, 8 or 16), s3_frame_batch %d (0, %d, %d or %d)",
                    t->tile_group, t->s3_frame_batch, ps::kFrameBatchSmall, ps::kFrameBatchRow, ps::kFrameBatch);
    p->s3_fb = t->s3_frame_batch;
    if (t->tile_group != p->tile_group) {
        p->tile_group = t->tile_group;
        PS_HIP(write_tiles(p));
    }
    return PS_OK;
}

ps_status ps_plan_autotune(ps_plan_t p, const ps_record* recs, int32_t n_rec, void* d_ws, size_t ws_bytes,
                           const ps_output* outs, int32_t reps, ps_stream_t stream, ps_tune_report* report) {
    if (!p || !recs || n_rec <= 0 || !outs) return fail(PS_E_INVALID_ARG, "autotune: NULL or empty argument");
    if (reps < 1 || reps > 100) return fail(PS_E_INVALID_ARG, "autotune: reps = %d (1..100)", reps);
    hipStream_t st = (hipStream_t)stream;
    ps_tuning cand[PS_TUNE_MAX];
    int n = 0;
    const int groups[4] = {1, 4, 8, 16};
    // The S3 frame batch matters when a chunk does not fit one small batch.
    const bool fb_choice = p->has(3) && p->m > ps::kFrameBatchSmall;
    for (int g : groups) {
        if (fb_choice) {                        // the default rule (0), then 10 and 16
            cand[n++] = ps_tuning{g, 0};
            cand[n++] = ps_tuning{g, ps::kFrameBatchSmall};
            cand[n++] = ps_tuning{g, ps::kFrameBatch};
        } else {
            cand[n++] = ps_tuning{g, 0};
        }
    }
    const ps_tuning orig{p->tile_group, p->s3_fb};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PS_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(PS_E_HIP, "autotune: hipEventCreate failed");
    }
    double ms[PS_TUNE_MAX];
    int best = 0;
    ps_status rc = PS_OK;
    for (int i = 0; i < n && rc == PS_OK; ++i) {
        if ((rc = ps_plan_set_tuning(p, &cand[i])) != PS_OK) break;
        if ((rc = ps_execute(p, recs, n_rec, d_ws, ws_bytes, outs, stream)) != PS_OK) break;     // warm-up
        if (hipEventRecord(e0, st) != hipSuccess) rc = fail(PS_E_HIP, "autotune: hipEventRecord failed");
        for (int r = 0; r < reps && rc == PS_OK; ++r) rc = ps_execute(p, recs, n_rec, d_ws, ws_bytes, outs, stream);
        if (rc != PS_OK) break;
        float el = 0.f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&el, e0, e1) != hipSuccess) {
            rc = fail(PS_E_HIP, "autotune: event timing failed");
            break;
        }
        ms[i] = el / reps;
        if (ms[i] < ms[best]) best = i;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != PS_OK) {
        // keep the configuration the plan had (the error detail stays the first failure's)
        if (orig.tile_group != p->tile_group) {
            p->tile_group = orig.tile_group;
            (void)write_tiles(p);
        }
        p->s3_fb = orig.s3_frame_batch;
        return rc;
    }
    if ((rc = ps_plan_set_tuning(p, &cand[best])) != PS_OK) return rc;
    if (report) {
        report->n = n;
        report->best = best;
        for (int i = 0; i < n; ++i) {
            report->cand[i] = cand[i];
            report->ms[i] = ms[i];
        }
    }
    return PS_OK;
}

ps_status ps_profile_enable(ps_plan_t p, int32_t on) {
    if (!p) return fail(PS_E_INVALID_ARG, "plan is NULL");
    p->prof = on != 0;
    return PS_OK;
}

ps_status ps_profile_read(ps_plan_t p, double* stage_ms, int32_t n) {
    if (!p || !stage_ms || n < 1) return fail(PS_E_INVALID_ARG, "bad argument");
    double ms[6] = {0, 0, 0, 0, 0, 0};
    double cnt[6] = {0, 0, 0, 0, 0, 0};
    ps_status status = PS_OK;
    for (auto& t : p->timed) {
        float e = 0.f;
        if (status == PS_OK) {
            hipError_t err = hipEventSynchronize(t.b);
            if (err == hipSuccess) err = hipEventElapsedTime(&e, t.a, t.b);
            if (err != hipSuccess) status = fail(PS_E_HIP, "event timing failed: %s", hipGetErrorString(err));
        }
        ms[t.stage] += e;
        cnt[t.stage] += 1;
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    p->timed.clear();
    for (int i = 0; i < n && i < 12; ++i) stage_ms[i] = i < 6 ? ms[i] : cnt[i - 6];
    return status;
}

ps_status ps_plan_query(ps_plan_t p, ps_plan_info* info) {
    if (!p || !info) return fail(PS_E_INVALID_ARG, "NULL argument");
    info->frame_len = p->N;
    info->n_freq = p->Nf;
    info->n_coef = p->K;
    info->m = p->m;
    info->n_combos2 = p->n2();
    info->n_combos3 = p->n3();
    info->n_combos4 = p->n4();
    info->grid = p->Ng;
    info->f_max = p->f_max;
    for (int n = 0; n < 5; ++n) info->sum_g[n] = p->sum_g[n];
    info->combos2 = p->c2.data();
    info->combos3 = p->c3.data();
    info->combos4 = p->c4.data();
    return PS_OK;
}

ps_status ps_record_info(ps_plan_t p, int64_t n_samples, int64_t* n_chunks, uint32_t* flags) {
    if (!p || n_samples < 0) return fail(PS_E_INVALID_ARG, "bad argument");
    const int64_t np = (n_samples / p->N) / p->m;
    if (n_chunks) *n_chunks = np;
    if (flags) *flags = (np == 0 ? PS_FLAG_EMPTY : 0u) | (np == 1 ? PS_FLAG_NO_ERRBAR : 0u);
    return PS_OK;
}

ps_status ps_record_chunks(ps_plan_t p, const ps_record* rec, int64_t* n_chunks, uint32_t* flags) {
    if (!p || !rec || rec->n_samples < 0) return fail(PS_E_INVALID_ARG, "bad argument");
    const int cls = p->class_of(rec->frame_len);
    if (cls < 0) return fail(PS_E_INVALID_ARG, "frame_len %d is not among the plan's frame lengths", rec->frame_len);
    const int64_t np = (rec->n_samples / p->fc[cls].N) / p->m;
    if (n_chunks) *n_chunks = np;
    if (flags) *flags = (np == 0 ? PS_FLAG_EMPTY : 0u) | (np == 1 ? PS_FLAG_NO_ERRBAR : 0u);
    return PS_OK;
}

ps_status ps_plan_frame_info(ps_plan_t p, int32_t frame_len, ps_plan_info* info) {
    if (!p || !info) return fail(PS_E_INVALID_ARG, "NULL argument");
    const int cls = p->class_of(frame_len);
    if (cls < 0) return fail(PS_E_INVALID_ARG, "frame_len %d is not among the plan's frame lengths", frame_len);
    ps_status s = ps_plan_query(p, info);
    if (s != PS_OK) return s;
    const FrameClass& fc = p->fc[cls];
    info->frame_len = fc.N;
    info->n_freq = fc.Nf;
    info->n_coef = fc.K;
    info->grid = fc.Ng;
    info->f_max = (fc.Nf - 1) / (fc.N * p->dt);
    for (int n = 0; n < 5; ++n) info->sum_g[n] = fc.sum_g[n];
    return PS_OK;
}

ps_status ps_workspace_size(ps_plan_t p, const ps_record* recs, int32_t n_rec, size_t* bytes) {
    if (!p || !bytes || n_rec < 0 || (n_rec > 0 && !recs)) return fail(PS_E_INVALID_ARG, "bad argument");
    for (int i = 0; i < n_rec; ++i) {
        ps_status s = check_record(p, &recs[i]);
        if (s != PS_OK) return s;
    }
    Batch B;
    build_batch(p, recs, n_rec, nullptr, B);
    *bytes = B.total;
    return PS_OK;
}

ps_status ps_coefficients(ps_plan_t p, const ps_record* rec, float* d_coef, ps_stream_t stream) {
    if (!p || !rec) return fail(PS_E_INVALID_ARG, "NULL argument");
    ps_status st = check_record(p, rec);
    if (st != PS_OK) return st;
    const FrameClass& fc = p->fc[p->class_of(rec->frame_len)];
    const int64_t F = ((rec->n_samples / fc.N) / p->m) * p->m;
    if (F == 0) return PS_OK;
    if (!d_coef || !aligned(d_coef, 8)) return fail(PS_E_INVALID_ARG, "coefficient buffer NULL or misaligned");
    ps::FftArgs a{};
    a.n_cls = 1;
    ps::FftClass& c = a.cls[0];
    c.recs = nullptr;
    c.single = ps::RecDesc{rec->d_data, rec->channel_stride, 0, rec->dtype, 0};
    c.n_recs = 1;
    c.g_lo = 0;
    c.g_hi = F;
    c.out_g0 = 0;
    c.log2n = fc.log2n_fft;
    c.jmax = fc.jmax;
    c.K = fc.K;
    c.g = fc.d_g;
    c.tw = fc.d_tw;
    c.dft_n = p->dft ? fc.N : 0;
    c.tw64 = fc.d_tw64;
    c.dft_n1 = p->dft_n1;
    c.out = reinterpret_cast<float2*>(d_coef);
    c.out_chan_stride = F * fc.K;
    a.n_channels = p->C;
    a.cplx = p->cplx;
    PS_HIP(ps::launch_window_rfft(a, (hipStream_t)stream));
    return PS_OK;
}

namespace {

// Copy the batch's record descriptors and segment tables into the workspace
// (one H2D copy from the plan's pinned staging buffer).
// `grow`: the staging buffer may be enlarged (a pinned host allocation);
// without it a batch whose tables exceed the buffer is refused.
ps_status upload_tables(ps_plan_t p, const Batch& B, char* d_tab, hipStream_t st, bool grow = true) {
    const int i = p->h_next;
    if (!grow && (p->h_cap[i] < B.tab_bytes || !p->h_ev[i]))
        return fail(PS_E_WORKSPACE, "work tables of %zu bytes exceed the plan's pinned staging of %zu bytes",
                    B.tab_bytes, p->h_cap[i]);
    p->h_next ^= 1;
    if (p->h_ev[i]) PS_HIP(hipEventSynchronize(p->h_ev[i]));
    if (p->h_cap[i] < B.tab_bytes) {
        if (p->h_stage[i]) (void)hipHostFree(p->h_stage[i]);
        p->h_stage[i] = nullptr;
        p->h_cap[i] = 0;
        const size_t cap = std::max<size_t>(B.tab_bytes, 1 << 20);
        PS_HIP(hipHostMalloc((void**)&p->h_stage[i], cap, hipHostMallocDefault));
        p->h_cap[i] = cap;
    }
    if (!p->h_ev[i]) PS_HIP(hipEventCreateWithFlags(&p->h_ev[i], hipEventDisableTiming));
    char* h = p->h_stage[i];
    std::memcpy(h, B.rd.data(), sizeof(ps::RecDesc) * B.rd.size());
    for (const Group& G : B.groups)
        for (const SegTable* t : G.all())
            if (!t->v.empty()) std::memcpy(h + t->dev_off, t->v.data(), sizeof(ps::Seg) * t->v.size());
    PS_HIP(hipMemcpyAsync(d_tab, h, B.tab_bytes, hipMemcpyHostToDevice, st));
    PS_HIP(hipEventRecord(p->h_ev[i], st));
    return PS_OK;
}

ps::BatchArgs batch_args(const ps_plan_s* p, const Batch& B, const SegTable& t, char* ws, const char* tab,
                         int per_chunk, int win_lo, int win_hi, int accumulate) {
    ps::BatchArgs a{};
    a.segs = reinterpret_cast<const ps::Seg*>(tab + t.dev_off);
    a.n_segs = (int)t.v.size();
    a.n_items = t.n_items;
    a.coef = reinterpret_cast<const float2*>(ws);     // segments hold offsets from the workspace start
    a.part = reinterpret_cast<double*>(ws + B.off_part);
    a.m = p->m;
    a.col0 = p->col0;
    a.col3 = p->cplx ? p->jmax - 2 * (p->Nf - 1) : 0;
    a.per_chunk = per_chunk;
    a.win_lo = win_lo;
    a.win_hi = win_hi;
    a.accumulate = accumulate;
    const bool nat = p->estimator == PS_EST_NATURAL;
    a.gamma = nat ? 1.0 / p->m : (p->m - 1.0) / (p->m * (p->m + 1.0));
    a.s4_shift = p->s4_shift;
    a.s3_fb = p->s3_fb;
    return a;
}

ps::FinalizeArgs fin_args(const ps_plan_s* p, const Batch& B, const SegTable& t, char* ws, const char* tab) {
    ps::FinalizeArgs f{};
    f.segs = reinterpret_cast<const ps::Seg*>(tab + t.dev_off);
    f.n_segs = (int)t.v.size();
    f.n_items = t.n_items;
    f.part = reinterpret_cast<const double*>(ws + B.off_part);
    f.s1 = p->has(1) ? reinterpret_cast<const float2*>(ws + B.off_s1) : nullptr;
    f.s1_cs = B.chunks_tot;
    return f;
}

// The moment stages of one group (one launch each).
ps_status launch_moments(ps_plan_t p, const Batch& B, const Group& G, char* ws, const char* tab, int per_chunk,
                         int win_lo, int win_hi, int accumulate, hipStream_t st) {
    if (G.s2.n_items) {
        StageTimer t(p, st, 2);
        PS_HIP(ps::launch_s2(batch_args(p, B, G.s2, ws, tab, per_chunk, win_lo, win_hi, accumulate), st));
    }
    if (G.s3.n_items) {
        StageTimer t(p, st, 3);
        ps::BatchArgs a = batch_args(p, B, G.s3, ws, tab, per_chunk, win_lo, win_hi, accumulate);
        // the c3^(opt) rows: m shifted frames and one mean row per chunk
        // (the segments point at their blocks)
        if (p->c3opt()) a.m = p->m + 1;
        PS_HIP(ps::launch_s3(a, st));
    }
    if (G.s4s.n_items) {
        StageTimer t(p, st, 4);
        ps::BatchArgs a = batch_args(p, B, G.s4s, ws, tab, per_chunk, win_lo, win_hi, accumulate);
        if (p->s4_pre) {                // operands split by the centring pass
            a.op4 = reinterpret_cast<const uint32_t*>(ws);
            a.p4 = reinterpret_cast<const double*>(ws);
        }
        if (p->precision == PS_PREC_FP32) {
            PS_HIP(ps::launch_s4_single(a, st));
        } else if (p->precision == PS_PREC_BF16X3) {
            PS_HIP(ps::launch_s4_mfma(a, st));
        } else {
            PS_HIP(ps::launch_s4_mfma_f16(a, st));
        }
    }
    if (G.s4x.n_items) {
        StageTimer t(p, st, 4);
        PS_HIP((p->precision == PS_PREC_BF16X3 ? ps::launch_s4_cross_mfma : ps::launch_s4_cross)(
            batch_args(p, B, G.s4x, ws, tab, per_chunk, win_lo, win_hi, accumulate), st));
    }
    return PS_OK;
}

ps_status launch_finalize(ps_plan_t p, const Batch& B, const Group& G, char* ws, const char* tab, hipStream_t st) {
    StageTimer t(p, st, 5);
    if (G.f2.n_items) PS_HIP(ps::launch_finalize_vec(fin_args(p, B, G.f2, ws, tab), st));
    if (G.f3.n_items) PS_HIP(ps::launch_finalize_grid(fin_args(p, B, G.f3, ws, tab), st));
    if (G.f4.n_items) PS_HIP(ps::launch_finalize_grid(fin_args(p, B, G.f4, ws, tab), st));
    if (G.f1.n_items) PS_HIP(ps::launch_finalize_s1(fin_args(p, B, G.f1, ws, tab), st));
    return PS_OK;
}

}  // namespace

namespace {

ps_status validate_execute(ps_plan_t p, const ps_record* recs, int32_t n_rec, void* d_ws,
                           const ps_output* outs) {
    if (!p || n_rec < 0 || (n_rec > 0 && (!recs || !outs))) return fail(PS_E_INVALID_ARG, "bad argument");
    if (!aligned(d_ws, 256)) return fail(PS_E_INVALID_ARG, "workspace must be 256-byte aligned");
    for (int r = 0; r < n_rec; ++r) {
        ps_status s = check_record(p, &recs[r]);
        if (s != PS_OK) return s;
        const ps_output& o = outs[r];
        const double* ptrs[8] = {o.d_s2, o.d_s2_err, o.d_s3, o.d_s3_err, o.d_s4, o.d_s4_err, o.d_s1, o.d_s1_err};
        for (const double* q : ptrs)
            if (q && !aligned(q, 8)) return fail(PS_E_INVALID_ARG, "output pointer misaligned");
    }
    return PS_OK;
}

// The running accumulation of a stream: state sums of S1 (per channel) for
// launch_accumulate_s1; the other orders' state slots are named by the
// group's accumulation table.
struct AccumTarget {
    double* s1_state;
};

// Every launch of one execution, given device tables at `tab`.  With `acc`
// the batch's sums are added to a stream's state (its group's accumulation
// table) instead of being finalized into outputs.
ps_status enqueue_all(ps_plan_t p, const Batch& B, const ps_record* recs, int32_t n_rec, const ps_output* outs,
                      char* ws, const char* tab, hipStream_t st, const AccumTarget* acc = nullptr) {
    const int m = p->m;
    for (int r = 0; r < n_rec && outs; ++r) {
        if (B.ri[r * B.stride].Np > 0) continue;
        const int Nf = p->fc[B.ri[r * B.stride].cls].Ng;
        const int64_t nf2 = (int64_t)Nf * Nf;
        const ps_output& o = outs[r];
        PS_HIP(ps::launch_fill_nan(o.d_s2, 2 * (int64_t)p->n2() * Nf, st));
        PS_HIP(ps::launch_fill_nan(o.d_s2_err, 2 * (int64_t)p->n2() * Nf, st));
        PS_HIP(ps::launch_fill_nan(o.d_s3, 2 * (int64_t)p->n3() * nf2, st));
        PS_HIP(ps::launch_fill_nan(o.d_s3_err, 2 * (int64_t)p->n3() * nf2, st));
        PS_HIP(ps::launch_fill_nan(o.d_s4, 2 * (int64_t)p->n4() * nf2, st));
        PS_HIP(ps::launch_fill_nan(o.d_s4_err, 2 * (int64_t)p->n4() * nf2, st));
        if (p->has(1)) {
            PS_HIP(ps::launch_fill_nan(o.d_s1, 2 * (int64_t)p->C, st));
            PS_HIP(ps::launch_fill_nan(o.d_s1_err, 2 * (int64_t)p->C, st));
        }
    }
    if (B.chunks_tot == 0) return PS_OK;

    ps::FftArgs fa{};
    fa.n_channels = p->C;
    fa.cplx = p->cplx;
    ps::CentreArgs ca{};
    ca.m = m;
    ca.n_channels = p->C;
    ca.s1 = p->has(1) ? reinterpret_cast<float2*>(ws + B.off_s1) : nullptr;
    ca.s1_cs = B.chunks_tot;
    ca.s1_col = p->jmax;
    if (p->c3opt()) {
        const double alpha = 4.0 / (m + 4.0);
        ca.alpha = (float)alpha;
        ca.mu = (float)std::cbrt(m * ((4.0 - 2.0 * m) / (m + 4.0) - alpha * alpha * alpha));
    }
    // The transform and centring arguments of one frame length's block.
    auto fft_class = [&](const BatchClass& k) {
        const FrameClass& fc = p->fc[k.cls];
        ps::FftClass c{};
        c.log2n = fc.log2n_fft;
        c.K = fc.K;
        c.jmax = fc.jmax;
        c.g = fc.d_g;
        c.tw = fc.d_tw;
        c.dft_n = p->dft ? fc.N : 0;
        c.tw64 = fc.d_tw64;
        c.dft_n1 = p->dft_n1;
        c.out = reinterpret_cast<float2*>(ws + k.coef_off);
        c.out_chan_stride = k.rows * fc.K;
        return c;
    };
    auto centre_class = [&](const BatchClass& k) {
        const FrameClass& fc = p->fc[k.cls];
        ps::CentreClass c{};
        c.coef = reinterpret_cast<float2*>(ws + k.coef_off);
        c.coef_chan_stride = k.rows * fc.K;
        c.K = fc.K;
        if (p->c3opt()) {
            c.out3 = reinterpret_cast<float2*>(ws + k.coef3_off);
            c.out3_cs = k.rows3 * fc.K;
        }
        if (k.op_chunks > 0) {
            const int ngp = op_cols(fc.Ng);
            c.op4 = reinterpret_cast<uint32_t*>(ws + k.op4_off);
            c.op4_cs = k.op_chunks * 3 * (int64_t)ngp * ps::kOpWords;
            c.p4 = reinterpret_cast<double*>(ws + k.p4_off);
            c.p4_cs = k.op_chunks * 2 * (int64_t)ngp;
            c.op4_cols = ngp;
        }
        return c;
    };
    ps_status s = PS_OK;

    if (p->schedule != PS_SCHED_PER_CHUNK) {
        // every frame length in one launch per stage
        int64_t fft_blocks = 0, centre_blocks = 0;
        for (const BatchClass& k : B.bc) {
            if (k.chunks == 0) continue;
            if (fa.n_cls == ps::kMaxClasses || ca.n_cls == ps::kMaxClasses)
                return fail(PS_E_INTERNAL, "more than %d frame lengths in one batch", ps::kMaxClasses);
            ps::FftClass c = fft_class(k);
            c.recs = reinterpret_cast<const ps::RecDesc*>(tab) + k.rd0;
            c.n_recs = k.n_rd;
            c.g_lo = 0;
            c.g_hi = k.F;
            c.out_g0 = 0;
            c.block0 = fft_blocks;
            fft_blocks += (k.F + (8192 / p->fc[k.cls].N) - 1) / (8192 / p->fc[k.cls].N);
            fa.cls[fa.n_cls++] = c;
            ps::CentreClass d = centre_class(k);
            d.n_chunks = k.chunks;
            d.s1_chunk0 = k.chunk_base;
            d.block0 = centre_blocks;
            centre_blocks += (int64_t)((p->fc[k.cls].K + 255) / 256) * k.chunks;
            ca.cls[ca.n_cls++] = d;
        }
        if (fa.n_cls == 1) fa.cls[0].block0 = 0;
        {
            StageTimer t(p, st, 0);
            PS_HIP(ps::launch_window_rfft(fa, st));
        }
        {
            StageTimer t(p, st, 1);
            PS_HIP(ps::launch_centre(ca, st));
        }
        s = launch_moments(p, B, B.groups[0], ws, tab, 0, 0, 0, 0, st);
        if (s != PS_OK) return s;
        if (acc) {
            const Group& G = B.groups[0];
            StageTimer t(p, st, 5);
            ps::AccumArgs aa{};
            aa.segs = reinterpret_cast<const ps::Seg*>(tab + G.acc.dev_off);
            aa.n_segs = (int)G.acc.v.size();
            aa.n_items = G.acc.n_items;
            aa.part = reinterpret_cast<const double*>(ws + B.off_part);
            PS_HIP(ps::launch_accumulate(aa, st));
            if (p->has(1))
                PS_HIP(ps::launch_accumulate_s1(reinterpret_cast<const float2*>(ws + B.off_s1), B.chunks_tot,
                                                B.chunks_tot, p->C, acc->s1_state, st));
            return PS_OK;
        }
        return launch_finalize(p, B, B.groups[0], ws, tab, st);
    }

    // Per-chunk schedule: one short-time estimate per launch set, record by record.
    for (const Group& G : B.groups) {
        const int r = G.rec;
        const BatchClass& k = B.bc[B.ri[r].bc];
        fa.n_cls = 1;
        ca.n_cls = 1;
        fa.cls[0] = fft_class(k);
        fa.cls[0].recs = nullptr;
        fa.cls[0].single = ps::RecDesc{recs[r].d_data, recs[r].channel_stride, 0, recs[r].dtype, 0};
        fa.cls[0].n_recs = 1;
        ca.cls[0] = centre_class(k);
        for (int64_t c = 0; c < B.ri[r].Np; ++c) {
            fa.cls[0].g_lo = c * m;
            fa.cls[0].g_hi = (c + 1) * m;
            fa.cls[0].out_g0 = c * m;
            {
                StageTimer t(p, st, 0);
                PS_HIP(ps::launch_window_rfft(fa, st));
            }
            ca.cls[0].n_chunks = 1;
            ca.cls[0].s1_chunk0 = B.ri[r].chunk0 + c;
            {
                StageTimer t(p, st, 1);
                PS_HIP(ps::launch_centre(ca, st));
            }
            s = launch_moments(p, B, G, ws, tab, 1, (int)c, (int)c + 1, c > 0 ? 1 : 0, st);
            if (s != PS_OK) return s;
        }
        s = launch_finalize(p, B, G, ws, tab, st);
        if (s != PS_OK) return s;
    }
    return PS_OK;
}

}  // namespace

ps_status ps_execute(ps_plan_t p, const ps_record* recs, int32_t n_rec, void* d_ws, size_t ws_bytes,
                     const ps_output* outs, ps_stream_t stream) {
    ps_status s = validate_execute(p, recs, n_rec, d_ws, outs);
    if (s != PS_OK || n_rec == 0) return s;
    hipStream_t st = (hipStream_t)stream;
    Batch B;
    build_batch(p, recs, n_rec, outs, B);
    if (!d_ws || ws_bytes < B.total) return fail(PS_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, B.total);
    char* ws = static_cast<char*>(d_ws);
    if (B.chunks_tot > 0) {
        s = upload_tables(p, B, ws + B.off_tab, st);
        if (s != PS_OK) return s;
    }
    return enqueue_all(p, B, recs, n_rec, outs, ws, ws + B.off_tab, st);
}

ps_status ps_execute_static(ps_plan_t p, const ps_record* recs, int32_t n_rec, const ps_output* outs,
                            ps_stream_t stream) {
    char* ws = static_cast<char*>(ps::static_scratch_ptr());
    if (!ws) return fail(PS_E_INVALID_ARG, "no static scratch on the current device (create a plan on it first)");
    ps_status s = validate_execute(p, recs, n_rec, ws, outs);
    if (s != PS_OK || n_rec == 0) return s;
    hipStream_t st = (hipStream_t)stream;
    Batch B;
    build_batch(p, recs, n_rec, outs, B);
    if (B.total > ps::kStaticScratchBytes)
        return fail(PS_E_WORKSPACE, "these records need %zu bytes of workspace; the static scratch holds %zu",
                    B.total, ps::kStaticScratchBytes);
    if (B.chunks_tot > 0) {
        s = upload_tables(p, B, ws + B.off_tab, st, /*grow=*/false);
        if (s != PS_OK) return s;
    }
    const bool prof = p->prof;
    p->prof = false;        // stage timing would create events
    s = enqueue_all(p, B, recs, n_rec, outs, ws, ws + B.off_tab, st);
    p->prof = prof;
    return s;
}

namespace {

// The stored combination serving raw combination `x` of `order` (orbit
// symmetries of Section 9): S2_ba = conj S2_ab; S3_bac(k, l) = S3_abc(l, k);
// S4_badc = conj S4_abcd, S4_cdab(k, l) = S4_abcd(l, k).  Returns false if
// no member of x's orbit is among the plan's combinations.
bool plane_source(const ps_plan_s* p, int order, const int8_t* x, ps::PlaneSrc& out) {
    const std::vector<int8_t>& list = order == 2 ? p->c2 : (order == 3 ? p->c3 : p->c4);
    const int n = (int)list.size() / order;
    struct Alt {
        int8_t c[4];
        int transpose, conj;
    };
    Alt alts[4];
    int n_alts = 0;
    if (order == 2) {
        alts[n_alts++] = Alt{{x[0], x[1], 0, 0}, 0, 0};
        alts[n_alts++] = Alt{{x[1], x[0], 0, 0}, 0, 1};
    } else if (order == 3) {
        alts[n_alts++] = Alt{{x[0], x[1], x[2], 0}, 0, 0};
        alts[n_alts++] = Alt{{x[1], x[0], x[2], 0}, 1, 0};
    } else {
        alts[n_alts++] = Alt{{x[0], x[1], x[2], x[3]}, 0, 0};
        alts[n_alts++] = Alt{{x[1], x[0], x[3], x[2]}, 0, 1};
        alts[n_alts++] = Alt{{x[2], x[3], x[0], x[1]}, 1, 0};
        alts[n_alts++] = Alt{{x[3], x[2], x[1], x[0]}, 1, 1};
    }
    for (int j = 0; j < n_alts; ++j)
        for (int i = 0; i < n; ++i)
            if (std::equal(alts[j].c, alts[j].c + order, list.begin() + (size_t)i * order)) {
                out = ps::PlaneSrc{i, alts[j].transpose, alts[j].conj};
                return true;
            }
    return false;
}

// One record of m N samples per chunk [chunk_lo, chunk_lo + n) of `rec`.
ps_status chunk_records(ps_plan_t p, const ps_record* rec, int64_t chunk_lo, int64_t n, std::vector<ps_record>& out) {
    if (!p || !rec) return fail(PS_E_INVALID_ARG, "NULL argument");
    const ps_status s = check_record(p, rec);
    if (s != PS_OK) return s;
    const int Nr = p->fc[p->class_of(rec->frame_len)].N;
    const int64_t np = (rec->n_samples / Nr) / p->m;
    if (chunk_lo < 0 || n < 0 || n > 0x7fffffff || chunk_lo > np - n)
        return fail(PS_E_INVALID_ARG, "chunks [%lld, %lld) outside the record's %lld", (long long)chunk_lo,
                    (long long)(chunk_lo + n), (long long)np);
    const int64_t esz = (int64_t)elem_size(rec->dtype);
    const int64_t span = (int64_t)p->m * Nr;
    out.assign((size_t)n, *rec);
    for (int64_t i = 0; i < n; ++i) {
        out[i].d_data = static_cast<const char*>(rec->d_data) + (chunk_lo + i) * span * esz;
        out[i].n_samples = span;
    }
    return PS_OK;
}

}  // namespace

ps_status ps_sequential_workspace_size(ps_plan_t p, const ps_record* rec, int64_t chunk_lo, int64_t n_chunks,
                                       size_t* bytes) {
    if (!bytes) return fail(PS_E_INVALID_ARG, "bytes is NULL");
    std::vector<ps_record> rs;
    const ps_status s = chunk_records(p, rec, chunk_lo, n_chunks, rs);
    if (s != PS_OK) return s;
    return ps_workspace_size(p, rs.data(), (int32_t)rs.size(), bytes);
}

ps_status ps_execute_sequential(ps_plan_t p, const ps_record* rec, int64_t chunk_lo, int64_t n_chunks, void* d_ws,
                                size_t ws_bytes, const ps_output* out, ps_stream_t stream) {
    std::vector<ps_record> rs;
    const ps_status s = chunk_records(p, rec, chunk_lo, n_chunks, rs);
    if (s != PS_OK) return s;
    if (n_chunks > 0 && !out) return fail(PS_E_INVALID_ARG, "out is NULL");
    // one output block per chunk, consecutive in each array
    const int64_t nf = p->fc[p->class_of(rec->frame_len)].Ng, nf2 = nf * nf;
    const int64_t e1 = 2LL * p->C, e2 = 2 * p->n2() * nf, e3 = 2 * p->n3() * nf2, e4 = 2 * p->n4() * nf2;
    auto at = [](double* base, int64_t i, int64_t n) { return base ? base + i * n : nullptr; };
    std::vector<ps_output> outs((size_t)n_chunks);
    for (int64_t i = 0; i < n_chunks; ++i)
        outs[i] = ps_output{at(out->d_s2, i, e2), at(out->d_s2_err, i, e2), at(out->d_s3, i, e3),
                            at(out->d_s3_err, i, e3), at(out->d_s4, i, e4), at(out->d_s4_err, i, e4),
                            at(out->d_s1, i, e1), at(out->d_s1_err, i, e1)};
    return ps_execute(p, rs.data(), (int32_t)rs.size(), d_ws, ws_bytes, outs.data(), stream);
}

ps_status ps_full_plane(ps_plan_t p, int32_t order, const int8_t* combo, const ps_output* in, double* d_out,
                        double* d_err, ps_stream_t stream) {
    if (!p || !combo || !in) return fail(PS_E_INVALID_ARG, "NULL argument");
    if (order < 2 || order > 4 || !p->has(order)) return fail(PS_E_INVALID_ARG, "order %d not computed", order);
    if (p->cplx) return fail(PS_E_UNSUPPORTED, "complex signals: the output grid is already the full plane");
    for (int i = 0; i < order; ++i)
        if (combo[i] < 0 || combo[i] >= p->C) return fail(PS_E_INVALID_ARG, "channel %d outside 0..%d", combo[i], p->C - 1);
    const double* src = order == 2 ? in->d_s2 : (order == 3 ? in->d_s3 : in->d_s4);
    const double* src_err = order == 2 ? in->d_s2_err : (order == 3 ? in->d_s3_err : in->d_s4_err);
    if ((d_out && !src) || (d_err && !src_err)) return fail(PS_E_INVALID_ARG, "input spectrum is NULL");
    const int8_t a = combo[0], b = combo[1];
    std::vector<std::vector<int8_t>> raw;
    if (order == 2) {
        raw = {{a, b}};
    } else if (order == 3) {
        const int8_t c = combo[2];
        raw = {{a, b, c}, {a, c, b}, {b, c, a}};
    } else {
        const int8_t c = combo[2], d = combo[3];
        raw = {{a, b, c, d}, {b, a, c, d}, {a, b, d, c}, {b, a, d, c}};
    }
    ps::PlaneArgs pa{};
    pa.order = order;
    pa.Nf = p->Nf;
    pa.in = src;
    pa.in_err = src_err;
    pa.out = d_out;
    pa.err = d_err;
    for (size_t i = 0; i < raw.size(); ++i)
        if (!plane_source(p, order, raw[i].data(), pa.src[i]))
            return fail(PS_E_UNSUPPORTED, "the plan does not hold the orbit of a combination needed for the full plane");
    PS_HIP(ps::launch_full_plane(pa, (hipStream_t)stream));
    return PS_OK;
}

// ------------------------------------------------------------------ graphs
struct ps_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* d_tab = nullptr;      // work tables owned by the graph
};

ps_status ps_graph_destroy(ps_graph_t g) {
    if (!g) return PS_OK;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->d_tab) (void)hipFree(g->d_tab);
    delete g;
    return PS_OK;
}

ps_status ps_graph_create(ps_plan_t p, const ps_record* recs, int32_t n_rec, void* d_ws, size_t ws_bytes,
                          const ps_output* outs, ps_graph_t* out) {
    if (!out) return fail(PS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    ps_status s = validate_execute(p, recs, n_rec, d_ws, outs);
    if (s != PS_OK) return s;
    Batch B;
    build_batch(p, recs, n_rec, outs, B);
    if (!d_ws || ws_bytes < B.total) return fail(PS_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, B.total);
    auto* g = new ps_graph_s();
    // Work tables: built once on the host, copied synchronously into device
    // memory that the graph owns (nothing is staged at replay time).
    std::vector<char> h(B.tab_bytes);
    std::memcpy(h.data(), B.rd.data(), sizeof(ps::RecDesc) * B.rd.size());
    for (const Group& G : B.groups)
        for (const SegTable* t : G.all())
            if (!t->v.empty()) std::memcpy(h.data() + t->dev_off, t->v.data(), sizeof(ps::Seg) * t->v.size());
    hipError_t e = hipMalloc(&g->d_tab, std::max<size_t>(B.tab_bytes, 256));
    if (e == hipSuccess) e = hipMemcpy(g->d_tab, h.data(), B.tab_bytes, hipMemcpyHostToDevice);
    hipStream_t cs = nullptr;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        if (cs) (void)hipStreamDestroy(cs);
        ps_graph_destroy(g);
        return fail(PS_E_HIP, "graph setup failed: %s", hipGetErrorString(e));
    }
    const bool prof = p->prof;
    p->prof = false;       // no timing events inside a graph
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        s = enqueue_all(p, B, recs, n_rec, outs, static_cast<char*>(d_ws), static_cast<const char*>(g->d_tab), cs);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &graph);
        g->graph = graph;
        if (s == PS_OK && e2 != hipSuccess) s = fail(PS_E_HIP, "stream capture failed: %s", hipGetErrorString(e2));
    } else {
        s = fail(PS_E_HIP, "stream capture failed: %s", hipGetErrorString(e));
    }
    p->prof = prof;
    (void)hipStreamDestroy(cs);
    if (s == PS_OK) {
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) s = fail(PS_E_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    if (s != PS_OK) {
        ps_graph_destroy(g);
        return s;
    }
    *out = g;
    return PS_OK;
}

ps_status ps_graph_launch(ps_graph_t g, ps_stream_t stream) {
    if (!g || !g->exec) return fail(PS_E_INVALID_ARG, "graph is NULL");
    PS_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return PS_OK;
}

// ------------------------------------------------------------------ streaming
struct ps_streamer_s {
    ps_plan_t plan = nullptr;
    int64_t window = 0;
    int dtype = 0, depth = 0, max_windows = 1;
    size_t esz = 0;
    hipStream_t copy = nullptr;
    std::vector<void*> stage;           // device staging slots
    std::vector<hipEvent_t> copied, done;
    std::vector<int> used;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int next = 0;
    std::vector<void*> allocs;
};

ps_status ps_streamer_destroy(ps_streamer_t s) {
    if (!s) return PS_OK;
    for (hipEvent_t e : s->done)
        if (e) (void)hipEventSynchronize(e);
    if (s->copy) (void)hipStreamSynchronize(s->copy);
    for (hipEvent_t e : s->copied)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : s->done)
        if (e) (void)hipEventDestroy(e);
    for (void* a : s->allocs) (void)hipFree(a);
    if (s->copy) (void)hipStreamDestroy(s->copy);
    delete s;
    return PS_OK;
}

ps_status ps_streamer_create_multi(ps_plan_t p, int64_t window_samples, int32_t max_windows, int32_t dtype,
                                   int32_t depth, ps_streamer_t* out) {
    if (!out) return fail(PS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!p || window_samples <= 0 || depth < 1 || depth > 16 || dtype < PS_F32 || dtype > PS_C128 ||
        (dtype >= PS_C64) != p->cplx || max_windows < 1 || max_windows > 64)
        return fail(PS_E_INVALID_ARG, "bad argument");
    auto* s = new ps_streamer_s();
    s->plan = p;
    s->window = window_samples;
    s->dtype = dtype;
    s->depth = depth;
    s->max_windows = max_windows;
    s->esz = elem_size(dtype);
    hipError_t e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
    auto alloc = [&](size_t bytes) -> void* {
        void* q = nullptr;
        if (e == hipSuccess && bytes > 0) {
            e = hipMalloc(&q, bytes);
            if (e == hipSuccess) s->allocs.push_back(q);
        }
        return q;
    };
    // workspace for the largest of the group sizes 1..max_windows
    std::vector<ps_record> rs(max_windows);
    for (ps_record& r : rs) {
        r = ps_record{};
        r.n_samples = window_samples;
        r.channel_stride = window_samples;
        r.dtype = dtype;
    }
    for (int n = 1; n <= max_windows; ++n) {
        Batch B;
        build_batch(p, rs.data(), n, nullptr, B);
        s->ws_bytes = std::max(s->ws_bytes, B.total);
    }
    s->ws = alloc(s->ws_bytes);
    for (int i = 0; i < depth && e == hipSuccess; ++i) {
        s->stage.push_back(alloc(s->esz * window_samples * p->C * max_windows));
        hipEvent_t a = nullptr, b = nullptr;
        if (e == hipSuccess) e = hipEventCreateWithFlags(&a, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b, hipEventDisableTiming);
        s->copied.push_back(a);
        s->done.push_back(b);
        s->used.push_back(0);
    }
    if (e != hipSuccess) {
        ps_streamer_destroy(s);
        return fail(PS_E_HIP, "streamer setup failed: %s", hipGetErrorString(e));
    }
    *out = s;
    return PS_OK;
}

ps_status ps_streamer_create(ps_plan_t p, int64_t window_samples, int32_t dtype, int32_t depth,
                             ps_streamer_t* out) {
    return ps_streamer_create_multi(p, window_samples, 1, dtype, depth, out);
}

ps_status ps_streamer_push_multi(ps_streamer_t s, const void* h_pinned, int32_t n_windows, const ps_output* outs,
                                 ps_stream_t compute, int32_t* slot) {
    if (!s || !h_pinned || !outs) return fail(PS_E_INVALID_ARG, "bad argument");
    if (n_windows < 1 || n_windows > s->max_windows)
        return fail(PS_E_INVALID_ARG, "n_windows %d outside 1..%d", n_windows, s->max_windows);
    const int i = s->next;
    s->next = (s->next + 1) % s->depth;
    hipStream_t cs = (hipStream_t)compute;
    const size_t win_bytes = s->esz * s->window * s->plan->C;
    // The slot's staging buffer may still be read by its previous computation.
    if (s->used[i]) PS_HIP(hipStreamWaitEvent(s->copy, s->done[i], 0));
    PS_HIP(hipMemcpyAsync(s->stage[i], h_pinned, win_bytes * n_windows, hipMemcpyHostToDevice, s->copy));
    PS_HIP(hipEventRecord(s->copied[i], s->copy));
    PS_HIP(hipStreamWaitEvent(cs, s->copied[i], 0));
    ps_record rs[64];
    for (int w = 0; w < n_windows; ++w) {
        rs[w] = ps_record{};
        rs[w].d_data = static_cast<char*>(s->stage[i]) + win_bytes * w;
        rs[w].n_samples = s->window;
        rs[w].channel_stride = s->window;
        rs[w].dtype = s->dtype;
    }
    ps_status st = ps_execute(s->plan, rs, n_windows, s->ws, s->ws_bytes, outs, compute);
    if (st != PS_OK) return st;
    PS_HIP(hipEventRecord(s->done[i], cs));
    s->used[i] = 1;
    if (slot) *slot = i;
    return PS_OK;
}

ps_status ps_streamer_push(ps_streamer_t s, const void* h_pinned, const ps_output* outs, ps_stream_t compute,
                           int32_t* slot) {
    return ps_streamer_push_multi(s, h_pinned, 1, outs, compute, slot);
}

ps_status ps_streamer_wait(ps_streamer_t s, int32_t slot) {
    if (!s || slot < 0 || slot >= s->depth) return fail(PS_E_INVALID_ARG, "bad argument");
    if (s->used[slot]) PS_HIP(hipEventSynchronize(s->done[slot]));
    return PS_OK;
}


}  // extern "C"

// ------------------------------------------------------------------ running accumulation
// (Section 4.2: the estimate depends on the chunks only through the sums over
// chunks of x, (Re x)^2, (Im x)^2 and their count, so these sums are the state.)
namespace {

// The state slots of every spectrum (FP64): per combination the tiles of its
// grid, [n_tiles][ncomp][points of a tile] (S2: 256-wide k blocks with 4
// components), then 4 sums per channel for S1.
struct StateLayout {
    std::vector<int64_t> off2, off3, off4;
    int64_t off1 = 0, doubles = 0;
};

int s4_kind(const ps_plan_s* p, int i) {
    return p->s4_single(i) ? ps::kSym64 : (p->s4_sym(i) ? ps::kSym32 : ps::kFull32);
}

StateLayout state_layout(const ps_plan_s* p) {
    StateLayout L;
    const int64_t TT = (int64_t)ps::kTile * ps::kTile, TX = (int64_t)ps::kTileX * ps::kTileX;
    const int64_t kblocks = (p->Ng + 255) / 256;
    int64_t o = 0;
    for (int i = 0; i < p->n2(); ++i) {
        L.off2.push_back(o);
        o += kblocks * 4 * 256;
    }
    for (int i = 0; i < p->n3(); ++i) {
        L.off3.push_back(o);
        o += (int64_t)p->n_tiles[p->s3_sym(i) ? ps::kSym64 : ps::kFull64] * 4 * TT;
    }
    for (int i = 0; i < p->n4(); ++i) {
        L.off4.push_back(o);
        const int kind = s4_kind(p, i);
        o += kind == ps::kSym64 ? (int64_t)p->n_tiles[kind] * 2 * TT : (int64_t)p->n_tiles[kind] * 4 * TX;
    }
    L.off1 = o;
    if (p->has(1)) o += 4LL * p->C;
    L.doubles = o;
    return L;
}

// FNV-1a over bytes (the configuration check of exported states).
uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ULL) {
    const unsigned char* b = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ULL;
    return h;
}

struct StateHeader {
    char magic[8];
    uint32_t header_bytes, version;
    int32_t N, Nf, m, C, K, Ng;
    uint32_t orders;
    int32_t window, precision, estimator, complex_signal, s4_shift, dtype, tile_group;
    int32_t n2, n3, n4;
    int32_t reserved;   // zero; keeps the doubles aligned without padding bytes
    double dt, window_param;
    int64_t n_chunks, n_samples, n_carry, state_doubles, carry_bytes;
    uint64_t combo_hash;
};
// The header is compared byte for byte on import: it must hold no padding.
static_assert(sizeof(StateHeader) == 8 + 2 * 4 + 6 * 4 + 4 + 7 * 4 + 4 * 4 + 2 * 8 + 5 * 8 + 8,
              "state header without padding");

}  // namespace

struct ps_accum_s {
    ps_plan_t plan = nullptr;
    int64_t max_push = 0, chunk_samples = 0;
    int dtype = 0, tile_group = 0;
    size_t esz = 0;
    StateLayout layout;
    double* d_state = nullptr;
    char* d_stage = nullptr;        // [C][stage_stride] samples: carry, then the pushed samples
    int64_t stage_stride = 0;
    void* d_ws = nullptr;
    size_t ws_bytes = 0;
    void* d_tab = nullptr;          // finalize tables of ps_stream_end
    size_t tab_bytes = 0;
    hipEvent_t done = nullptr;      // after the last enqueued push / end
    bool pending = false;
    int64_t n_chunks = 0, n_samples = 0, n_carry = 0;
};

namespace {

// The batch of one push: one record of `n` staged samples per channel, its
// accumulation table pointing at the state slots.
void build_stream_batch(const ps_accum_s* a, int64_t n, Batch& B) {
    const ps_plan_s* p = a->plan;
    ps_record r{};
    r.d_data = a->d_stage;
    r.n_samples = n;
    r.channel_stride = a->stage_stride;
    r.dtype = a->dtype;
    build_batch(p, &r, 1, nullptr, B);
    Group& G = B.groups[0];
    const int64_t TT = (int64_t)ps::kTile * ps::kTile, TX = (int64_t)ps::kTileX * ps::kTileX;
    auto add = [&](const SegTable& f, const std::vector<int64_t>& off, int64_t points, bool vec) {
        for (size_t i = 0; i < f.v.size(); ++i) {
            ps::Seg sg = f.v[i];
            sg.n_chunks2 = 0;
            sg.part2 = 0;
            sg.blocks2 = 0;
            sg.out = a->d_state + off[i];
            sg.err = nullptr;
            if (vec) sg.tiles = -1;
            const int64_t P = vec ? 256 : (sg.tiles >= ps::kSym32 ? TX : TT);
            (void)points;
            G.acc.add(sg, (int64_t)sg.n_tiles * (P / 256));
        }
    };
    add(G.f2, a->layout.off2, 256, true);
    add(G.f3, a->layout.off3, TT, false);
    add(G.f4, a->layout.off4, TT, false);
    finish_layout(p, B);
}

}  // namespace

extern "C" {

ps_status ps_stream_destroy(ps_accum_t a) {
    if (!a) return PS_OK;
    if (a->done) {
        (void)hipEventSynchronize(a->done);
        (void)hipEventDestroy(a->done);
    }
    (void)hipFree(a->d_state);
    (void)hipFree(a->d_stage);
    (void)hipFree(a->d_ws);
    (void)hipFree(a->d_tab);
    delete a;
    return PS_OK;
}

ps_status ps_stream_begin(ps_plan_t p, int64_t max_push_samples, int32_t dtype, ps_accum_t* out) {
    if (!out) return fail(PS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!p || max_push_samples < 1) return fail(PS_E_INVALID_ARG, "bad argument");
    if (dtype < PS_F32 || dtype > PS_C128 || (dtype >= PS_C64) != p->cplx)
        return fail(PS_E_INVALID_ARG, "dtype %d does not match the plan's %s signal", dtype,
                    p->cplx ? "complex" : "real");
    if (p->schedule != PS_SCHED_BATCHED) return fail(PS_E_UNSUPPORTED, "streams need the batched schedule");
    if (p->interlaced) return fail(PS_E_UNSUPPORTED, "streams do not take interlaced windows");
    auto* a = new ps_accum_s();
    a->plan = p;
    a->max_push = max_push_samples;
    a->chunk_samples = (int64_t)p->N * p->m;
    a->dtype = dtype;
    a->tile_group = p->tile_group;
    a->esz = elem_size(dtype);
    a->layout = state_layout(p);
    a->stage_stride = max_push_samples + a->chunk_samples;
    // Workspace: the largest over the chunk counts a push can complete
    // (sampled densely near both ends, log-spaced between), checked again at
    // every push.
    const int64_t np_max = a->stage_stride / a->chunk_samples;
    std::vector<int64_t> counts;
    for (int64_t c = 1; c <= std::min<int64_t>(np_max, 64); ++c) counts.push_back(c);
    for (int64_t c = std::max<int64_t>(1, np_max - 64); c <= np_max; ++c) counts.push_back(c);
    for (double c = 64; c < np_max; c *= 1.05) counts.push_back((int64_t)c);
    size_t ws = 256;
    for (int64_t c : counts) {
        Batch B;
        build_stream_batch(a, c * a->chunk_samples, B);
        ws = std::max(ws, B.total);
    }
    a->ws_bytes = align256(ws + ws / 16 + (1 << 20));
    // finalize tables of ps_stream_end: one segment per spectrum and combination,
    // plus the padding finish_layout may put in front of them
    a->tab_bytes = align256(sizeof(ps::Seg) * (size_t)(p->n2() + p->n3() + p->n4() + 1 + 64));
    hipError_t e = hipMalloc((void**)&a->d_state, sizeof(double) * std::max<int64_t>(1, a->layout.doubles));
    if (e == hipSuccess) e = hipMemset(a->d_state, 0, sizeof(double) * std::max<int64_t>(1, a->layout.doubles));
    if (e == hipSuccess) e = hipMalloc((void**)&a->d_stage, a->esz * a->stage_stride * p->C);
    if (e == hipSuccess) e = hipMalloc(&a->d_ws, a->ws_bytes);
    if (e == hipSuccess) e = hipMalloc(&a->d_tab, a->tab_bytes);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&a->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        ps_stream_destroy(a);
        return fail(PS_E_HIP, "stream setup failed: %s", hipGetErrorString(e));
    }
    *out = a;
    return PS_OK;
}

ps_status ps_stream_push(ps_accum_t a, const void* d_data, int64_t n, int64_t channel_stride, ps_stream_t stream) {
    if (!a) return fail(PS_E_INVALID_ARG, "stream is NULL");
    ps_plan_s* p = a->plan;
    if (n < 0 || n > a->max_push) return fail(PS_E_INVALID_ARG, "n_samples %lld outside 0..%lld", (long long)n,
                                              (long long)a->max_push);
    if (n == 0) return PS_OK;
    if (!d_data || !aligned(d_data, a->esz)) return fail(PS_E_INVALID_ARG, "data NULL or misaligned");
    if (p->C > 1 && channel_stride < n) return fail(PS_E_INVALID_ARG, "channel_stride < n_samples");
    if (p->tile_group != a->tile_group)
        return fail(PS_E_INVALID_ARG, "the plan's tile order changed since ps_stream_begin");
    hipStream_t st = (hipStream_t)stream;
    const int64_t have = a->n_carry + n;
    const int64_t chunks = have / a->chunk_samples;
    const int64_t used = chunks * a->chunk_samples, tail = have - used;
    if (a->n_chunks + chunks > INT32_MAX)
        return fail(PS_E_UNSUPPORTED, "a stream holds at most 2^31 - 1 chunks (%lld accumulated)",
                    (long long)a->n_chunks);
    // append the pushed samples after the carried ones
    PS_HIP(hipMemcpy2DAsync(a->d_stage + a->n_carry * a->esz, a->esz * a->stage_stride, d_data,
                            a->esz * (p->C > 1 ? channel_stride : n), a->esz * n, p->C, hipMemcpyDeviceToDevice,
                            st));
    if (chunks > 0) {
        Batch B;
        build_stream_batch(a, used, B);
        if (B.total > a->ws_bytes) return fail(PS_E_INTERNAL, "stream workspace %zu < %zu", a->ws_bytes, B.total);
        char* ws = static_cast<char*>(a->d_ws);
        ps_status s = upload_tables(p, B, ws + B.off_tab, st);
        if (s != PS_OK) return s;
        ps_record r{};
        r.d_data = a->d_stage;
        r.n_samples = used;
        r.channel_stride = a->stage_stride;
        r.dtype = a->dtype;
        AccumTarget t{a->d_state + a->layout.off1};
        s = enqueue_all(p, B, &r, 1, nullptr, ws, ws + B.off_tab, st, &t);
        if (s != PS_OK) return s;
        // the samples beyond the last complete chunk move to the front
        // (after the transform has read them; tail < m N <= used: no overlap)
        if (tail > 0)
            PS_HIP(hipMemcpy2DAsync(a->d_stage, a->esz * a->stage_stride, a->d_stage + used * a->esz,
                                    a->esz * a->stage_stride, a->esz * tail, p->C, hipMemcpyDeviceToDevice, st));
    }
    PS_HIP(hipEventRecord(a->done, st));
    a->pending = true;
    a->n_chunks += chunks;
    a->n_samples += n;
    a->n_carry = tail;
    return PS_OK;
}

ps_status ps_stream_end(ps_accum_t a, const ps_output* out, ps_stream_t stream) {
    if (!a || !out) return fail(PS_E_INVALID_ARG, "NULL argument");
    ps_plan_s* p = a->plan;
    const double* ptrs[8] = {out->d_s2, out->d_s2_err, out->d_s3, out->d_s3_err, out->d_s4, out->d_s4_err,
                             out->d_s1, out->d_s1_err};
    for (const double* q : ptrs)
        if (q && !aligned(q, 8)) return fail(PS_E_INVALID_ARG, "output pointer misaligned");
    hipStream_t st = (hipStream_t)stream;
    const int Nf = p->Ng;
    const int64_t nf2 = (int64_t)Nf * Nf;
    if (a->n_chunks == 0) {
        PS_HIP(ps::launch_fill_nan(out->d_s2, 2 * (int64_t)p->n2() * Nf, st));
        PS_HIP(ps::launch_fill_nan(out->d_s2_err, 2 * (int64_t)p->n2() * Nf, st));
        PS_HIP(ps::launch_fill_nan(out->d_s3, 2 * (int64_t)p->n3() * nf2, st));
        PS_HIP(ps::launch_fill_nan(out->d_s3_err, 2 * (int64_t)p->n3() * nf2, st));
        PS_HIP(ps::launch_fill_nan(out->d_s4, 2 * (int64_t)p->n4() * nf2, st));
        PS_HIP(ps::launch_fill_nan(out->d_s4_err, 2 * (int64_t)p->n4() * nf2, st));
        if (p->has(1)) {
            PS_HIP(ps::launch_fill_nan(out->d_s1, 2 * (int64_t)p->C, st));
            PS_HIP(ps::launch_fill_nan(out->d_s1_err, 2 * (int64_t)p->C, st));
        }
        PS_HIP(hipEventRecord(a->done, st));
        a->pending = true;
        return PS_OK;
    }
    // Finalize tables over the state: each tile is one slot (a schedule of
    // n_tiles blocks for n_tiles tiles), Np = chunks accumulated.
    const Scales scl = spectrum_scales(p, p->sum_g);
    const int64_t TT = (int64_t)ps::kTile * ps::kTile, TX = (int64_t)ps::kTileX * ps::kTileX;
    const int kblocks = (Nf + 255) / 256;
    SegTable f2, f3, f4;
    for (int i = 0; i < p->n2(); ++i) {
        ps::Seg sg{};
        sg.part = a->layout.off2[i];
        sg.Nf = Nf;
        sg.n_tiles = kblocks;
        sg.blocks = kblocks;
        sg.n_chunks = (int32_t)a->n_chunks;
        sg.out = out->d_s2 ? out->d_s2 + 2 * (int64_t)i * Nf : nullptr;
        sg.err = out->d_s2_err ? out->d_s2_err + 2 * (int64_t)i * Nf : nullptr;
        sg.scale = scl.s2;
        sg.ncomp = 4;
        f2.add(sg, kblocks);
    }
    for (int i = 0; i < p->n3(); ++i) {
        ps::Seg sg{};
        sg.tiles = p->s3_sym(i) ? ps::kSym64 : ps::kFull64;
        sg.tile_tab = p->d_tiles[sg.tiles];
        sg.Nf = Nf;
        sg.n_tiles = p->n_tiles[sg.tiles];
        sg.blocks = sg.n_tiles;
        sg.part = a->layout.off3[i];
        sg.n_chunks = (int32_t)a->n_chunks;
        sg.out = out->d_s3 ? out->d_s3 + 2 * i * nf2 : nullptr;
        sg.err = out->d_s3_err ? out->d_s3_err + 2 * i * nf2 : nullptr;
        sg.scale = scl.s3;
        sg.sym = p->s3_sym(i);
        sg.ncomp = 4;
        f3.add(sg, (int64_t)sg.n_tiles * (TT / 256));
    }
    for (int i = 0; i < p->n4(); ++i) {
        ps::Seg sg{};
        sg.tiles = s4_kind(p, i);
        sg.tile_tab = p->d_tiles[sg.tiles];
        sg.Nf = Nf;
        const bool single = sg.tiles == ps::kSym64;
        sg.n_tiles = p->n_tiles[sg.tiles];
        sg.blocks = sg.n_tiles;
        sg.part = a->layout.off4[i];
        sg.n_chunks = (int32_t)a->n_chunks;
        sg.out = out->d_s4 ? out->d_s4 + 2 * i * nf2 : nullptr;
        sg.err = out->d_s4_err ? out->d_s4_err + 2 * i * nf2 : nullptr;
        sg.scale = scl.s4;
        sg.sym = p->s4_sym(i);
        sg.ncomp = single ? 2 : 4;
        f4.add(sg, (int64_t)sg.n_tiles * ((single ? TT : TX) / 256));
    }
    // tables through the plan's pinned staging into the stream's table buffer
    Batch B;
    B.groups.emplace_back();
    B.groups[0].f2 = f2;
    B.groups[0].f3 = f3;
    B.groups[0].f4 = f4;
    finish_layout(p, B);
    if (B.tab_bytes > a->tab_bytes)
        return fail(PS_E_INTERNAL, "finalize tables of %zu bytes exceed the stream's %zu", B.tab_bytes, a->tab_bytes);
    char* tab = static_cast<char*>(a->d_tab);
    ps_status s = upload_tables(p, B, tab, st);
    if (s != PS_OK) return s;
    ps::FinalizeArgs fa{};
    fa.part = a->d_state;
    auto fin = [&](const SegTable& t, bool vec) -> hipError_t {
        fa.segs = reinterpret_cast<const ps::Seg*>(tab + t.dev_off);
        fa.n_segs = (int)t.v.size();
        fa.n_items = t.n_items;
        return vec ? ps::launch_finalize_vec(fa, st) : ps::launch_finalize_grid(fa, st);
    };
    if (!f2.v.empty()) PS_HIP(fin(B.groups[0].f2, true));
    if (!f3.v.empty()) PS_HIP(fin(B.groups[0].f3, false));
    if (!f4.v.empty()) PS_HIP(fin(B.groups[0].f4, false));
    if (p->has(1))
        PS_HIP(ps::launch_finalize_s1_sums(a->d_state + a->layout.off1, p->C, a->n_chunks, scl.s1, out->d_s1,
                                           out->d_s1_err, st));
    PS_HIP(hipEventRecord(a->done, st));
    a->pending = true;
    return PS_OK;
}

ps_status ps_stream_counts(ps_accum_t a, int64_t* n_chunks, int64_t* n_samples, int64_t* n_carry) {
    if (!a) return fail(PS_E_INVALID_ARG, "stream is NULL");
    if (n_chunks) *n_chunks = a->n_chunks;
    if (n_samples) *n_samples = a->n_samples;
    if (n_carry) *n_carry = a->n_carry;
    return PS_OK;
}

namespace {
StateHeader make_header(const ps_accum_s* a) {
    const ps_plan_s* p = a->plan;
    StateHeader h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, "PSSTATE1", 8);
    h.header_bytes = sizeof(StateHeader);
    h.version = 1;
    h.N = p->N;
    h.Nf = p->Nf;
    h.m = p->m;
    h.C = p->C;
    h.K = p->K;
    h.Ng = p->Ng;
    h.orders = p->orders;
    h.window = p->window;
    h.precision = p->precision;
    h.estimator = p->estimator;
    h.complex_signal = p->cplx;
    h.s4_shift = p->s4_shift;
    h.dtype = a->dtype;
    h.tile_group = a->tile_group;
    h.n2 = p->n2();
    h.n3 = p->n3();
    h.n4 = p->n4();
    h.dt = p->dt;
    h.window_param = p->window == PS_WIN_ACG ? p->window_param : 0.0;
    h.n_chunks = a->n_chunks;
    h.n_samples = a->n_samples;
    h.n_carry = a->n_carry;
    h.state_doubles = a->layout.doubles;
    h.carry_bytes = (int64_t)(a->esz * a->n_carry * p->C);
    uint64_t hh = fnv1a(p->c2.data(), p->c2.size());
    hh = fnv1a(p->c3.data(), p->c3.size(), hh);
    h.combo_hash = fnv1a(p->c4.data(), p->c4.size(), hh);
    return h;
}
}  // namespace

ps_status ps_stream_export_state(ps_accum_t a, void* h_buf, size_t* n_bytes) {
    if (!a || !n_bytes) return fail(PS_E_INVALID_ARG, "NULL argument");
    const StateHeader h = make_header(a);
    const size_t need = sizeof(StateHeader) + sizeof(double) * (size_t)h.state_doubles + (size_t)h.carry_bytes;
    if (!h_buf) {
        *n_bytes = need;
        return PS_OK;
    }
    if (*n_bytes < need) return fail(PS_E_INVALID_ARG, "buffer %zu < %zu bytes", *n_bytes, need);
    if (a->pending) PS_HIP(hipEventSynchronize(a->done));
    char* b = static_cast<char*>(h_buf);
    std::memcpy(b, &h, sizeof h);
    b += sizeof h;
    if (h.state_doubles > 0)
        PS_HIP(hipMemcpy(b, a->d_state, sizeof(double) * (size_t)h.state_doubles, hipMemcpyDeviceToHost));
    b += sizeof(double) * (size_t)h.state_doubles;
    if (a->n_carry > 0)
        PS_HIP(hipMemcpy2D(b, a->esz * a->n_carry, a->d_stage, a->esz * a->stage_stride, a->esz * a->n_carry,
                           a->plan->C, hipMemcpyDeviceToHost));
    *n_bytes = need;
    return PS_OK;
}

ps_status ps_stream_import_state(ps_accum_t a, const void* h_buf, size_t n_bytes) {
    if (!a || !h_buf) return fail(PS_E_INVALID_ARG, "NULL argument");
    if (n_bytes < sizeof(StateHeader)) return fail(PS_E_INVALID_ARG, "state too short");
    StateHeader h;
    std::memcpy(&h, h_buf, sizeof h);
    if (std::memcmp(h.magic, "PSSTATE1", 8) != 0 || h.header_bytes != sizeof(StateHeader) || h.version != 1)
        return fail(PS_E_INVALID_ARG, "not an exported stream state");
    StateHeader mine = make_header(a);
    // the configuration must match; the counters come from the import
    mine.n_chunks = h.n_chunks;
    mine.n_samples = h.n_samples;
    mine.n_carry = h.n_carry;
    mine.carry_bytes = h.carry_bytes;
    if (std::memcmp(&mine, &h, sizeof h) != 0)
        return fail(PS_E_INVALID_ARG, "the state was exported by a stream of another configuration");
    if (h.n_carry < 0 || h.n_carry >= a->chunk_samples || h.n_chunks < 0 || h.n_samples < 0 ||
        h.carry_bytes != (int64_t)(a->esz * h.n_carry * a->plan->C))
        return fail(PS_E_INVALID_ARG, "inconsistent state counters");
    const size_t need = sizeof(StateHeader) + sizeof(double) * (size_t)h.state_doubles + (size_t)h.carry_bytes;
    if (n_bytes < need) return fail(PS_E_INVALID_ARG, "state %zu < %zu bytes", n_bytes, need);
    if (a->pending) PS_HIP(hipEventSynchronize(a->done));
    const char* b = static_cast<const char*>(h_buf) + sizeof h;
    if (h.state_doubles > 0)
        PS_HIP(hipMemcpy(a->d_state, b, sizeof(double) * (size_t)h.state_doubles, hipMemcpyHostToDevice));
    b += sizeof(double) * (size_t)h.state_doubles;
    if (h.n_carry > 0)
        PS_HIP(hipMemcpy2D(a->d_stage, a->esz * a->stage_stride, b, a->esz * h.n_carry, a->esz * h.n_carry,
                           a->plan->C, hipMemcpyHostToDevice));
    a->n_chunks = h.n_chunks;
    a->n_samples = h.n_samples;
    a->n_carry = h.n_carry;
    a->pending = false;
    return PS_OK;
}

ps_status ps_spectra_zscore(const double* d_a, const double* d_a_err, const double* d_b, const double* d_b_err,
                            int64_t n_points, double* d_out, ps_stream_t stream) {
    if (n_points < 0) return fail(PS_E_INVALID_ARG, "n_points < 0");
    if (n_points == 0) return PS_OK;
    const double* ptrs[5] = {d_a, d_a_err, d_b, d_b_err, d_out};
    for (const double* q : ptrs)
        if (!q || !aligned(q, 8)) return fail(PS_E_INVALID_ARG, "pointer NULL or misaligned");
    PS_HIP(ps::launch_zscore(d_a, d_a_err, d_b, d_b_err, 2 * n_points, d_out, (hipStream_t)stream));
    return PS_OK;
}

}  // extern "C"
