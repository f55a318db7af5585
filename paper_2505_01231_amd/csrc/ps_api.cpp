// Host runtime behind the C ABI of include/polyspec.h: validation, the FP64
// window and FFT tables, the channel-combination lists, workspace layout, the
// choice of launch shapes, and the order of kernel launches per record.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
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

}  // namespace

struct ps_plan_s {
    int N = 0, log2n = 0, Nf = 0, K = 0, m = 0, C = 0;
    double dt = 1, f_max = 0, window_param = 0.14;
    uint32_t orders = 0;
    int window = 0, precision = 0, schedule = 0;
    std::vector<int8_t> c2, c3, c4;
    double sum_g[5] = {0, 0, 0, 0, 0};
    int T = 0, TX = 0;
    int n_tiles_sym = 0, n_tiles_full = 0, n_tilesx_sym = 0, n_tilesx_full = 0;
    float* d_g = nullptr;
    float2* d_tw = nullptr;
    int2* d_tiles_sym = nullptr;     // 64 x 64 tiles, kt <= lt
    int2* d_tiles_full = nullptr;    // 64 x 64 tiles, all
    int2* d_tilesx_sym = nullptr;    // 32 x 32 tiles (cross-channel S4), kt <= lt
    int2* d_tilesx_full = nullptr;
    int n_cu = 256, bpc_s3 = 2, bpc_s4 = 2, bpc_s4x = 2;
    // Stage timing (ps_profile_enable): event pairs recorded on the stream.
    bool prof = false;
    struct Timed {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Timed> timed;

    bool has(int order) const { return (orders >> order) & 1u; }
    int n2() const { return has(2) ? (int)c2.size() / 2 : 0; }
    int n3() const { return has(3) ? (int)c3.size() / 3 : 0; }
    int n4() const { return has(4) ? (int)c4.size() / 4 : 0; }
    bool s3_sym(int i) const { return c3[3 * i] == c3[3 * i + 1]; }
    bool s4_single(int i) const {
        const int8_t* q = &c4[4 * i];
        return q[0] == q[1] && q[1] == q[2] && q[2] == q[3];
    }
    // S4_abcd(k,l) = S4_cdab(l,k): symmetric grid when (a,b) = (c,d).
    bool s4_sym(int i) const {
        const int8_t* q = &c4[4 * i];
        return q[0] == q[2] && q[1] == q[3];
    }
};

namespace {

// Split of the chunk range over blocks: the smallest split count whose
// wave-quantised time is within 3% of the best for up to 64 parts.
int choose_split(int n_tiles, int64_t n_chunks, int slots) {
    if (n_chunks <= 1) return 1;
    const int smax = (int)std::min<int64_t>(64, n_chunks);
    auto cost = [&](int s) {
        const double waves = std::ceil((double)n_tiles * s / slots);
        return waves * std::ceil((double)n_chunks / s);
    };
    double best = 1e300;
    for (int s = 1; s <= smax; ++s) best = std::min(best, cost(s));
    for (int s = 1; s <= smax; ++s)
        if (cost(s) <= 1.03 * best) return s;
    return smax;
}

int choose_split_vec(int Nf, int64_t n_chunks, int n_cu) {
    const int blocks = (Nf + 255) / 256;
    int s = (4 * n_cu + blocks - 1) / blocks;
    s = std::max(1, std::min<int>(s, 256));
    return (int)std::min<int64_t>(s, std::max<int64_t>(1, n_chunks));
}

// Launch shape and partial-sum slot of one S4 channel combination.
struct S4Shape {
    bool single = true;   // a = b = c = d: real form, 64-tiles (FP32 vector or matrix cores)
    bool sym = true;      // only tiles kt <= lt
    int edge = 64;
    int n_tiles = 0;
    const int2* d_tiles = nullptr;
    int split = 1;
    int ncomp = 2;
    size_t off = 0;
};

struct Layout {
    int64_t Np = 0, F = 0;
    int chunk_frames = 0;   // frames resident in the coefficient buffer
    int split2 = 1, split3_sym = 1, split3_full = 1;
    size_t off_coef = 0, off_p2 = 0, off_p3 = 0, off_p4 = 0, total = 0;
    std::vector<size_t> p3_off;
    std::vector<S4Shape> s4;
    size_t p2_stride = 0;
};

Layout layout_for(const ps_plan_s* p, int64_t n_samples) {
    Layout L;
    L.Np = (n_samples / p->N) / p->m;
    L.F = L.Np * p->m;
    const bool per_chunk = p->schedule == PS_SCHED_PER_CHUNK;
    L.chunk_frames = per_chunk ? p->m : (int)L.F;
    if (!per_chunk) {
        L.split2 = choose_split_vec(p->Nf, L.Np, p->n_cu);
        L.split3_sym = choose_split(p->n_tiles_sym, L.Np, p->n_cu * p->bpc_s3);
        L.split3_full = choose_split(p->n_tiles_full, L.Np, p->n_cu * p->bpc_s3);
    }
    size_t off = 0;
    L.off_coef = off;
    off = align256(off + (size_t)p->C * L.chunk_frames * p->K * sizeof(float2));
    L.off_p2 = off;
    L.p2_stride = align256((size_t)L.split2 * 4 * p->Nf * sizeof(double));
    off += (size_t)p->n2() * L.p2_stride;
    L.off_p3 = off;
    const size_t TT = (size_t)ps::kTile * ps::kTile;
    for (int i = 0; i < p->n3(); ++i) {
        L.p3_off.push_back(off);
        const bool sym = p->s3_sym(i);
        const size_t n = (size_t)(sym ? L.split3_sym : L.split3_full) *
                         (sym ? p->n_tiles_sym : p->n_tiles_full) * 4 * TT;
        off = align256(off + n * sizeof(double));
    }
    L.off_p4 = off;
    for (int i = 0; i < p->n4(); ++i) {
        S4Shape sh;
        sh.single = p->s4_single(i);
        sh.sym = p->s4_sym(i);
        if (sh.single) {
            sh.edge = ps::kTile;
            sh.n_tiles = p->n_tiles_sym;
            sh.d_tiles = p->d_tiles_sym;
            sh.ncomp = 2;
            if (!per_chunk) sh.split = choose_split(sh.n_tiles, L.Np, p->n_cu * p->bpc_s4);
        } else {
            sh.edge = ps::kTileX;
            sh.n_tiles = sh.sym ? p->n_tilesx_sym : p->n_tilesx_full;
            sh.d_tiles = sh.sym ? p->d_tilesx_sym : p->d_tilesx_full;
            sh.ncomp = 4;
            if (!per_chunk) sh.split = choose_split(sh.n_tiles, L.Np, p->n_cu * p->bpc_s4x);
        }
        sh.off = off;
        const size_t n = (size_t)sh.split * sh.n_tiles * sh.ncomp * sh.edge * sh.edge;
        off = align256(off + n * sizeof(double));
        L.s4.push_back(sh);
    }
    L.total = std::max<size_t>(off, 256);
    return L;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Optional event pair around one stage launch (only while profiling).
struct StageTimer {
    ps_plan_s* p;
    hipStream_t st;
    int stage;
    hipEvent_t a = nullptr;
    StageTimer(ps_plan_s* p_, hipStream_t st_, int stage_) : p(p_), st(st_), stage(stage_) {
        if (p->prof && hipEventCreate(&a) == hipSuccess) hipEventRecord(a, st);
    }
    ~StageTimer() {
        if (!a) return;
        hipEvent_t b = nullptr;
        if (hipEventCreate(&b) == hipSuccess && hipEventRecord(b, st) == hipSuccess) {
            p->timed.push_back({stage, a, b});
        } else {
            hipEventDestroy(a);
            if (b) hipEventDestroy(b);
        }
    }
};

ps_status check_record(const ps_plan_s* p, const ps_record* r) {
    if (!r) return fail(PS_E_INVALID_ARG, "record is NULL");
    if (r->dtype < PS_F32 || r->dtype > PS_I16) return fail(PS_E_INVALID_ARG, "bad dtype %d", r->dtype);
    if (r->n_samples < 0) return fail(PS_E_INVALID_ARG, "n_samples < 0");
    if (r->reserved != 0) return fail(PS_E_INVALID_ARG, "record.reserved must be 0");
    if (p->C > 1 && r->channel_stride < r->n_samples)
        return fail(PS_E_INVALID_ARG, "channel_stride (%lld) < n_samples (%lld)",
                    (long long)r->channel_stride, (long long)r->n_samples);
    const size_t esz = r->dtype == PS_F32 ? 4 : (r->dtype == PS_F64 ? 8 : 2);
    if (r->n_samples >= (int64_t)p->N * p->m) {
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
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
    }
    hipFree(p->d_g);
    hipFree(p->d_tw);
    hipFree(p->d_tiles_sym);
    hipFree(p->d_tiles_full);
    hipFree(p->d_tilesx_sym);
    hipFree(p->d_tilesx_full);
    delete p;
    return PS_OK;
}

ps_status ps_plan_create(const ps_config* cfg, ps_plan_t* out) {
    if (!out) return fail(PS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(PS_E_INVALID_ARG, "cfg is NULL");
    if (cfg->struct_size < sizeof(ps_config))
        return fail(PS_E_INVALID_ARG, "struct_size %u < %zu", cfg->struct_size, sizeof(ps_config));
    const uint32_t known = PS_ORDER_S2 | PS_ORDER_S3 | PS_ORDER_S4;
    if (cfg->orders == 0 || (cfg->orders & ~known))
        return fail(PS_E_INVALID_ARG, "orders must be a non-empty subset of {2,3,4}");
    if (cfg->n_channels < 1 || cfg->n_channels > 4)
        return fail(PS_E_INVALID_ARG, "n_channels must be 1..4");
    const int N = cfg->frame_len;
    if (N < 2 || (N & (N - 1)))
        return fail(PS_E_UNSUPPORTED, "frame_len %d is not a power of two", N);
    if (N < 256 || N > 8192) return fail(PS_E_UNSUPPORTED, "frame_len %d outside 256..8192", N);
    if (!(cfg->dt > 0) || !std::isfinite(cfg->dt)) return fail(PS_E_INVALID_ARG, "dt must be > 0");
    const int min_m = (cfg->orders & PS_ORDER_S4) ? 4 : (cfg->orders & PS_ORDER_S3) ? 3 : 2;
    if (cfg->m < min_m) return fail(PS_E_INVALID_ARG, "m = %d < %d (k-statistic denominator)", cfg->m, min_m);
    if (cfg->window < PS_WIN_HANN || cfg->window > PS_WIN_ACG)
        return fail(PS_E_INVALID_ARG, "unknown window %d", cfg->window);
    if (cfg->window == PS_WIN_ACG && !(cfg->window_param > 0))
        return fail(PS_E_INVALID_ARG, "acG window needs sigma_t > 0");
    if (cfg->precision < PS_PREC_FP32 || cfg->precision > PS_PREC_FP16X2S)
        return fail(PS_E_INVALID_ARG, "unknown precision %d", cfg->precision);
    if (cfg->precision == PS_PREC_FP16X2S)
        return fail(PS_E_UNSUPPORTED, "precision %d not available in this build", cfg->precision);
    if (cfg->schedule != PS_SCHED_BATCHED && cfg->schedule != PS_SCHED_PER_CHUNK)
        return fail(PS_E_INVALID_ARG, "unknown schedule %d", cfg->schedule);
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

    auto* p = new ps_plan_s();
    p->N = N;
    while ((1 << p->log2n) < N) ++p->log2n;
    p->Nf = Nf;
    p->K = s3 ? 2 * Nf - 1 : Nf;
    p->m = cfg->m;
    p->C = cfg->n_channels;
    p->dt = cfg->dt;
    p->f_max = (Nf - 1) / (N * cfg->dt);
    p->orders = cfg->orders;
    p->window = cfg->window;
    p->window_param = cfg->window_param;
    p->precision = cfg->precision;
    p->schedule = cfg->schedule;

    // Channel combinations: explicit lists or every orbit.
    std::vector<int8_t> a2, a3, a4;
    all_combos(p->C, a2, a3, a4);
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

    // Window and sums (FP64); FFT twiddles exp(+2 pi j t/N) rounded once to FP32.
    std::vector<double> g;
    make_window(p->window, N, p->window_param, g);
    for (int n = 0; n < 5; ++n) {
        double s = 0;
        for (double v : g) s += std::pow(v, n);
        p->sum_g[n] = s;
    }
    std::vector<float> gf(N);
    for (int i = 0; i < N; ++i) gf[i] = (float)g[i];
    std::vector<float2> tw(N);
    const double two_pi = 6.28318530717958647692;
    for (int t = 0; t < N; ++t) {
        const double ang = two_pi * t / N;
        tw[t] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }

    // Output tiles: upper triangle (kt <= lt) for symmetric spectra, all otherwise.
    auto make_tiles = [](int T, std::vector<int2>& sym, std::vector<int2>& full) {
        for (int kt = 0; kt < T; ++kt)
            for (int lt = 0; lt < T; ++lt) {
                full.push_back(make_int2(kt, lt));
                if (kt <= lt) sym.push_back(make_int2(kt, lt));
            }
    };
    p->T = (Nf + ps::kTile - 1) / ps::kTile;
    p->TX = (Nf + ps::kTileX - 1) / ps::kTileX;
    std::vector<int2> ts, tf, txs, txf;
    make_tiles(p->T, ts, tf);
    make_tiles(p->TX, txs, txf);
    p->n_tiles_sym = (int)ts.size();
    p->n_tiles_full = (int)tf.size();
    p->n_tilesx_sym = (int)txs.size();
    p->n_tilesx_full = (int)txf.size();

    auto upload = [&](void** dst, const void* src, size_t bytes) -> hipError_t {
        hipError_t e = hipMalloc(dst, bytes);
        if (e != hipSuccess) return e;
        return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = upload((void**)&p->d_g, gf.data(), gf.size() * sizeof(float));
    if (e == hipSuccess) e = upload((void**)&p->d_tw, tw.data(), tw.size() * sizeof(float2));
    if (e == hipSuccess) e = upload((void**)&p->d_tiles_sym, ts.data(), ts.size() * sizeof(int2));
    if (e == hipSuccess) e = upload((void**)&p->d_tiles_full, tf.data(), tf.size() * sizeof(int2));
    if (e == hipSuccess) e = upload((void**)&p->d_tilesx_sym, txs.data(), txs.size() * sizeof(int2));
    if (e == hipSuccess) e = upload((void**)&p->d_tilesx_full, txf.data(), txf.size() * sizeof(int2));
    if (e != hipSuccess) {
        ps_plan_destroy(p);
        return fail(PS_E_HIP, "device table setup failed: %s", hipGetErrorString(e));
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        p->n_cu = std::max(1, prop.multiProcessorCount);
    p->bpc_s3 = ps::s3_blocks_per_cu();
    p->bpc_s4 = p->precision == PS_PREC_FP32 ? ps::s4_blocks_per_cu() : ps::s4_mfma_blocks_per_cu();
    p->bpc_s4x = ps::s4_cross_blocks_per_cu();
    *out = p;
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
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
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
    info->reserved = 0;
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

ps_status ps_workspace_size(ps_plan_t p, const ps_record* recs, int32_t n_rec, size_t* bytes) {
    if (!p || !bytes || n_rec < 0 || (n_rec > 0 && !recs)) return fail(PS_E_INVALID_ARG, "bad argument");
    size_t need = 256;
    for (int i = 0; i < n_rec; ++i) {
        ps_status s = check_record(p, &recs[i]);
        if (s != PS_OK) return s;
        need = std::max(need, layout_for(p, recs[i].n_samples).total);
    }
    *bytes = need;
    return PS_OK;
}

ps_status ps_coefficients(ps_plan_t p, const ps_record* rec, float* d_coef, ps_stream_t stream) {
    if (!p || !rec) return fail(PS_E_INVALID_ARG, "NULL argument");
    ps_status st = check_record(p, rec);
    if (st != PS_OK) return st;
    const int64_t F = ((rec->n_samples / p->N) / p->m) * p->m;
    if (F == 0) return PS_OK;
    if (!d_coef || !aligned(d_coef, 8)) return fail(PS_E_INVALID_ARG, "coefficient buffer NULL or misaligned");
    ps::FftArgs a{};
    a.x = rec->d_data;
    a.dtype = rec->dtype;
    a.chan_stride = rec->channel_stride;
    a.frame0 = 0;
    a.n_frames = (int)F;
    a.n_channels = p->C;
    a.log2n = p->log2n;
    a.K = p->K;
    a.g = p->d_g;
    a.tw = p->d_tw;
    a.out = reinterpret_cast<float2*>(d_coef);
    a.out_chan_stride = F * p->K;
    a.out_frame0 = 0;
    PS_HIP(ps::launch_window_rfft(a, (hipStream_t)stream));
    return PS_OK;
}

ps_status ps_execute(ps_plan_t p, const ps_record* recs, int32_t n_rec, void* d_ws, size_t ws_bytes,
                     const ps_output* outs, ps_stream_t stream) {
    if (!p || n_rec < 0 || (n_rec > 0 && (!recs || !outs))) return fail(PS_E_INVALID_ARG, "bad argument");
    if (!aligned(d_ws, 256)) return fail(PS_E_INVALID_ARG, "workspace must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    // Validate everything before enqueueing anything.
    for (int r = 0; r < n_rec; ++r) {
        ps_status s = check_record(p, &recs[r]);
        if (s != PS_OK) return s;
        const Layout L = layout_for(p, recs[r].n_samples);
        if (!d_ws || ws_bytes < L.total)
            return fail(PS_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.total);
        const ps_output& o = outs[r];
        const double* need[6] = {p->n2() ? o.d_s2 : nullptr, p->n2() ? o.d_s2_err : nullptr,
                                 p->n3() ? o.d_s3 : nullptr, p->n3() ? o.d_s3_err : nullptr,
                                 p->n4() ? o.d_s4 : nullptr, p->n4() ? o.d_s4_err : nullptr};
        for (const double* q : need)
            if (q && !aligned(q, 8)) return fail(PS_E_INVALID_ARG, "output pointer misaligned");
    }
    const int Nf = p->Nf, m = p->m;
    const double dt = p->dt;
    const double scale2 = dt / ((m - 1) * p->sum_g[2]);
    const double scale3 = dt * dt * m / ((double)(m - 1) * (m - 2) * p->sum_g[3]);
    const double scale4 = dt * dt * dt * m * (m + 1.0) / ((double)(m - 1) * (m - 2) * (m - 3) * p->sum_g[4]);
    const double gamma = (m - 1.0) / (m * (m + 1.0));
    const int64_t nf2 = (int64_t)Nf * Nf;

    for (int r = 0; r < n_rec; ++r) {
        const ps_record& rec = recs[r];
        const ps_output& o = outs[r];
        const Layout L = layout_for(p, rec.n_samples);
        if (L.Np == 0) {
            PS_HIP(ps::launch_fill_nan(o.d_s2, 2 * (int64_t)p->n2() * Nf, st));
            PS_HIP(ps::launch_fill_nan(o.d_s2_err, 2 * (int64_t)p->n2() * Nf, st));
            PS_HIP(ps::launch_fill_nan(o.d_s3, 2 * (int64_t)p->n3() * nf2, st));
            PS_HIP(ps::launch_fill_nan(o.d_s3_err, 2 * (int64_t)p->n3() * nf2, st));
            PS_HIP(ps::launch_fill_nan(o.d_s4, 2 * (int64_t)p->n4() * nf2, st));
            PS_HIP(ps::launch_fill_nan(o.d_s4_err, 2 * (int64_t)p->n4() * nf2, st));
            continue;
        }
        char* ws = static_cast<char*>(d_ws);
        float2* coef = reinterpret_cast<float2*>(ws + L.off_coef);
        const int64_t coef_cs = (int64_t)L.chunk_frames * p->K;
        const bool per_chunk = p->schedule == PS_SCHED_PER_CHUNK;
        const int64_t n_steps = per_chunk ? L.Np : 1;

        for (int64_t step = 0; step < n_steps; ++step) {
            const int c_lo = per_chunk ? (int)step : 0;
            const int c_hi = per_chunk ? (int)step + 1 : (int)L.Np;
            ps::FftArgs fa{};
            fa.x = rec.d_data;
            fa.dtype = rec.dtype;
            fa.chan_stride = rec.channel_stride;
            fa.frame0 = (int64_t)c_lo * m;
            fa.n_frames = (c_hi - c_lo) * m;
            fa.n_channels = p->C;
            fa.log2n = p->log2n;
            fa.K = p->K;
            fa.g = p->d_g;
            fa.tw = p->d_tw;
            fa.out = coef;
            fa.out_chan_stride = coef_cs;
            fa.out_frame0 = (int64_t)c_lo * m;
            {
                StageTimer t(p, st, 0);
                PS_HIP(ps::launch_window_rfft(fa, st));
            }

            ps::CentreArgs ca{};
            ca.coef = coef;
            ca.coef_chan_stride = coef_cs;
            ca.K = p->K;
            ca.m = m;
            ca.n_chunks = c_hi - c_lo;
            ca.n_channels = p->C;
            {
                StageTimer t(p, st, 1);
                PS_HIP(ps::launch_centre(ca, st));
            }

            ps::CoefView cv{coef, coef_cs, p->K, m, c_lo};
            const int acc = step > 0 ? 1 : 0;
            for (int i = 0; i < p->n2(); ++i) {
                ps::S2Args a{};
                a.v = cv;
                a.Nf = Nf;
                a.a = p->c2[2 * i];
                a.b = p->c2[2 * i + 1];
                a.chunk0 = c_lo;
                a.chunk1 = c_hi;
                a.n_split = L.split2;
                a.part = reinterpret_cast<double*>(ws + L.off_p2 + i * L.p2_stride);
                a.accumulate = acc;
                StageTimer t(p, st, 2);
                PS_HIP(ps::launch_s2(a, st));
            }
            for (int i = 0; i < p->n3(); ++i) {
                const bool sym = p->s3_sym(i);
                ps::GridArgs a{};
                a.v = cv;
                a.Nf = Nf;
                for (int j = 0; j < 3; ++j) a.ch[j] = p->c3[3 * i + j];
                a.tiles = sym ? p->d_tiles_sym : p->d_tiles_full;
                a.n_tiles = sym ? p->n_tiles_sym : p->n_tiles_full;
                a.chunk0 = c_lo;
                a.chunk1 = c_hi;
                a.n_split = sym ? L.split3_sym : L.split3_full;
                a.part = reinterpret_cast<double*>(ws + L.p3_off[i]);
                a.accumulate = acc;
                StageTimer t(p, st, 3);
                PS_HIP(ps::launch_s3(a, st));
            }
            for (int i = 0; i < p->n4(); ++i) {
                const S4Shape& sh = L.s4[i];
                ps::GridArgs a{};
                a.v = cv;
                a.Nf = Nf;
                for (int j = 0; j < 4; ++j) a.ch[j] = p->c4[4 * i + j];
                a.tiles = sh.d_tiles;
                a.n_tiles = sh.n_tiles;
                a.chunk0 = c_lo;
                a.chunk1 = c_hi;
                a.n_split = sh.split;
                a.part = reinterpret_cast<double*>(ws + sh.off);
                a.accumulate = acc;
                a.gamma = gamma;
                StageTimer t(p, st, 4);
                if (!sh.single) {
                    PS_HIP(ps::launch_s4_cross(a, st));
                } else if (p->precision == PS_PREC_FP32) {
                    PS_HIP(ps::launch_s4_single(a, st));
                } else {
                    PS_HIP(ps::launch_s4_mfma(a, st));
                }
            }
        }

        for (int i = 0; i < p->n2(); ++i) {
            ps::FinalizeVecArgs f{};
            f.part = reinterpret_cast<const double*>(ws + L.off_p2 + i * L.p2_stride);
            f.n_split = L.split2;
            f.Nf = Nf;
            f.n_chunks = L.Np;
            f.scale = scale2;
            f.out = o.d_s2 ? o.d_s2 + 2 * (int64_t)i * Nf : nullptr;
            f.err = o.d_s2_err ? o.d_s2_err + 2 * (int64_t)i * Nf : nullptr;
            StageTimer t(p, st, 5);
            PS_HIP(ps::launch_finalize_vec(f, st));
        }
        for (int i = 0; i < p->n3(); ++i) {
            const bool sym = p->s3_sym(i);
            ps::FinalizeGridArgs f{};
            f.part = reinterpret_cast<const double*>(ws + L.p3_off[i]);
            f.n_split = sym ? L.split3_sym : L.split3_full;
            f.n_tiles = sym ? p->n_tiles_sym : p->n_tiles_full;
            f.ncomp = 4;
            f.edge = ps::kTile;
            f.sym = sym;
            f.Nf = Nf;
            f.n_chunks = L.Np;
            f.scale = scale3;
            f.out = o.d_s3 ? o.d_s3 + 2 * i * nf2 : nullptr;
            f.err = o.d_s3_err ? o.d_s3_err + 2 * i * nf2 : nullptr;
            StageTimer t(p, st, 5);
            PS_HIP(ps::launch_finalize_grid(f, sym ? p->d_tiles_sym : p->d_tiles_full, st));
        }
        for (int i = 0; i < p->n4(); ++i) {
            const S4Shape& sh = L.s4[i];
            ps::FinalizeGridArgs f{};
            f.part = reinterpret_cast<const double*>(ws + sh.off);
            f.n_split = sh.split;
            f.n_tiles = sh.n_tiles;
            f.ncomp = sh.ncomp;
            f.edge = sh.edge;
            f.sym = sh.sym;
            f.Nf = Nf;
            f.n_chunks = L.Np;
            f.scale = scale4;
            f.out = o.d_s4 ? o.d_s4 + 2 * i * nf2 : nullptr;
            f.err = o.d_s4_err ? o.d_s4_err + 2 * i * nf2 : nullptr;
            StageTimer t(p, st, 5);
            PS_HIP(ps::launch_finalize_grid(f, sh.d_tiles, st));
        }
    }
    return PS_OK;
}

}  // extern "C"
