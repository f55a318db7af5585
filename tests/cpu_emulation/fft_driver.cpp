// Host driver of the emulated transform kernels (test infrastructure only).
//
//   fft_driver P LOG2M2 FRAMES K DTYPE MISALIGN OUT.f32
//
// Runs k_window_rfft_pf<LOG2M2, P> (P = 3 or 5; N = 2 P 2^LOG2M2) on FRAMES
// frames of one channel with the launch shape and the argument fields the
// library uses for that frame length (pf_c, pf_d, the twiddle table of N
// entries plus the pass tables, K coefficients per frame), every buffer
// allocated to its exact size, and writes the K x FRAMES complex outputs.
// DTYPE 0 float32, 1 float64, 2 int16; MISALIGN 1 starts the samples one
// element past an aligned address.  Samples and window are deterministic.
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "ps_fft_extract.inc"

thread_local emu_idx threadIdx, blockIdx;
std::barrier<>* emu_block_barrier = nullptr;

template <typename KernelFn>
static void emu_launch(KernelFn fn, dim3 grid, int threads) {
    for (unsigned by = 0; by < grid.y; ++by)
        for (unsigned bx = 0; bx < grid.x; ++bx) {
            // threads that return early leave the barrier (as finished waves do)
            std::barrier<> bar(threads);
            emu_block_barrier = &bar;
            std::vector<std::thread> ts;
            ts.reserve(threads);
            for (int t = 0; t < threads; ++t)
                ts.emplace_back([&, t] {
                    threadIdx = emu_idx{(unsigned)t, 0, 0};
                    blockIdx = emu_idx{bx, by, 0};
                    fn();
                    bar.arrive_and_drop();
                });
            for (auto& th : ts) th.join();
        }
}

template <int LOG2M2, int P>
static void run(ps::FftArgs a, int64_t frames) {
    constexpr int T2 = (1 << LOG2M2) / 16, F = ps::pf_frames<LOG2M2, P>();
    const dim3 grid((unsigned)((frames + F - 1) / F), 1);
    emu_launch([a] { ps::k_window_rfft_pf<LOG2M2, P>(a); }, grid, F * P * T2);
}

int main(int argc, char** argv) {
    if (argc != 8) return 2;
    const int P = atoi(argv[1]), log2m2 = atoi(argv[2]);
    const int64_t frames = atoll(argv[3]);
    const int K = atoi(argv[4]), dtype = atoi(argv[5]), mis = atoi(argv[6]);
    const int M2 = 1 << log2m2, M = P * M2, N = 2 * M;
    const size_t esz = dtype == 0 ? 4 : dtype == 1 ? 8 : 2;
    // samples: exactly frames * N elements (+ the misalignment element)
    char* raw = (char*)malloc(esz * (size_t)(frames * N + mis));
    uint64_t st = 12345;
    for (int64_t i = 0; i < frames * N + mis; ++i) {
        st = st * 6364136223846793005ULL + 1442695040888963407ULL;
        const double v = ((double)(st >> 11) / 9007199254740992.0 - 0.5) * 2000.0;
        if (dtype == 0) ((float*)raw)[i] = (float)v;
        else if (dtype == 1) ((double*)raw)[i] = v;
        else ((int16_t*)raw)[i] = (int16_t)v;
    }
    const void* data = raw + esz * mis;
    // window (a smooth positive bump) and twiddles in the library's layout
    std::vector<float>* g = new std::vector<float>(N);
    for (int i = 0; i < N; ++i) (*g)[i] = (float)(0.5 - 0.5 * std::cos(2 * M_PI * (i + 0.5) / N));
    const int tw_log2 = log2m2 + 1;
    const int R2 = ps::fft_radix2(tw_log2), R3 = ps::fft_radix3(tw_log2);
    std::vector<float2>* tw = new std::vector<float2>();
    for (int t = 0; t < N; ++t)
        tw->push_back(make_float2((float)std::cos(2 * M_PI * t / N), (float)std::sin(2 * M_PI * t / N)));
    const int pass_r[2] = {R2, R3}, pass_ns[2] = {16, 16 * R2};
    for (int q = 0; q < 2; ++q)
        for (int r = 0; r < pass_r[q]; ++r)
            for (int k = 0; k < pass_ns[q]; ++k) {
                const double ang = 2 * M_PI * r * k / ((double)pass_r[q] * pass_ns[q]);
                tw->push_back(make_float2((float)std::cos(ang), (float)std::sin(ang)));
            }
    // exact-size heap copies (vectors may over-allocate)
    float* d_g = (float*)malloc(sizeof(float) * N);
    memcpy(d_g, g->data(), sizeof(float) * N);
    float2* d_tw = (float2*)malloc(sizeof(float2) * tw->size());
    memcpy(d_tw, tw->data(), sizeof(float2) * tw->size());
    float2* out = (float2*)malloc(sizeof(float2) * (size_t)(frames * K));
    int pf_c = 0, pf_d = 0;
    for (int c = 0; c < M; c += M2)
        if (c % P == 1) pf_c = c;
    for (int d = 0; d < M; d += P)
        if (d % M2 == 1) pf_d = d;
    ps::FftArgs a{};
    a.n_cls = 1;
    ps::FftClass& c = a.cls[0];
    c.recs = nullptr;
    c.single = ps::RecDesc{data, frames * N, 0, dtype, 0};
    c.n_recs = 1;
    c.g_lo = 0;
    c.g_hi = frames;
    c.out_g0 = 0;
    c.log2n = log2m2;
    c.K = K;
    c.g = d_g;
    c.tw = d_tw;
    c.out = out;
    c.out_chan_stride = frames * K;
    a.n_channels = 1;
    a.pf = P;
    a.pf_c = pf_c;
    a.pf_d = pf_d;
    const int key = P * 16 + log2m2;
    switch (key) {
        case 3 * 16 + 7: run<7, 3>(a, frames); break;
        case 3 * 16 + 8: run<8, 3>(a, frames); break;
        case 3 * 16 + 9: run<9, 3>(a, frames); break;
        case 3 * 16 + 10: run<10, 3>(a, frames); break;
        case 5 * 16 + 7: run<7, 5>(a, frames); break;
        case 5 * 16 + 8: run<8, 5>(a, frames); break;
        case 5 * 16 + 9: run<9, 5>(a, frames); break;
        default: return 3;
    }
    FILE* f = fopen(argv[7], "wb");
    if (!f) return 4;
    fwrite(out, sizeof(float2), (size_t)(frames * K), f);
    fclose(f);
    // the samples and window the kernel saw, for the reference transform
    std::vector<double> samp((size_t)(frames * N));
    for (int64_t i = 0; i < frames * N; ++i)
        samp[i] = dtype == 0 ? ((const float*)data)[i] : dtype == 1 ? ((const double*)data)[i]
                                                                   : ((const int16_t*)data)[i];
    std::string p2 = std::string(argv[7]) + ".in";
    f = fopen(p2.c_str(), "wb");
    fwrite(samp.data(), sizeof(double), samp.size(), f);
    fwrite(d_g, sizeof(float), N, f);
    fclose(f);
    free(raw);
    free(d_g);
    free(d_tw);
    free(out);
    delete g;
    delete tw;
    return 0;
}
