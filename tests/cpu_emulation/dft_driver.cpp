// Host driver of the emulated direct transform kernel (test infrastructure
// only).
//
//   dft_driver N FRAMES K DTYPE MISALIGN N1 OUT.f32
//
// Runs k_window_dft (N1 = 0) or its two-stage form k_window_dft2 (N = N1 N2)
// for frame length N (not a power of two) on FRAMES frames of one channel with
// the launch shape and the argument fields the library uses (the FP64 table
// exp(+2 pi j t / N) of N entries, K coefficients per frame), every buffer,
// the dynamic LDS included, allocated to its exact size, and writes the
// FRAMES x K complex outputs.  DTYPE 0 float32, 1 float64, 2 int16; MISALIGN 1 starts the
// samples one element past an aligned address.  Samples and window are
// deterministic; OUT.f32.in receives the samples (float64) and the window
// (float32) for the reference.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <thread>
#include <vector>

#include "ps_fft_extract.inc"

thread_local emu_idx threadIdx, blockIdx;
std::barrier<>* emu_block_barrier = nullptr;
char* emu_dyn_smem = nullptr;

template <typename KernelFn>
static void emu_launch(KernelFn fn, dim3 grid, int threads) {
    for (unsigned bz = 0; bz < grid.z; ++bz)
        for (unsigned by = 0; by < grid.y; ++by)
            for (unsigned bx = 0; bx < grid.x; ++bx) {
                std::barrier<> bar(threads);
                emu_block_barrier = &bar;
                std::vector<std::thread> ts;
                ts.reserve(threads);
                for (int t = 0; t < threads; ++t)
                    ts.emplace_back([&, t] {
                        threadIdx = emu_idx{(unsigned)t, 0, 0};
                        blockIdx = emu_idx{bx, by, bz};
                        fn();
                        bar.arrive_and_drop();
                    });
                for (auto& th : ts) th.join();
            }
}

int main(int argc, char** argv) {
    if (argc != 8) return 2;
    const int N = atoi(argv[1]);
    const int64_t frames = atoll(argv[2]);
    const int K = atoi(argv[3]), dtype = atoi(argv[4]), mis = atoi(argv[5]), N1 = atoi(argv[6]);
    const char* out_path = argv[7];
    if (N < 2 || K < 1 || K > N / 2 + 1 || frames < 1) return 2;
    const size_t esz = dtype == 0 ? 4 : dtype == 1 ? 8 : 2;
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
    float* d_g = (float*)malloc(sizeof(float) * N);
    for (int i = 0; i < N; ++i) d_g[i] = (float)(0.5 - 0.5 * std::cos(2 * M_PI * (i + 0.5) / N));
    double2* d_tw64 = (double2*)malloc(sizeof(double2) * N);
    for (int t = 0; t < N; ++t) {
        const long double ang = 2.0L * 3.14159265358979323846264338327950288L * t / N;
        d_tw64[t] = make_double2((double)std::cos(ang), (double)std::sin(ang));
    }
    float2* out = (float2*)malloc(sizeof(float2) * (size_t)(frames * K));
    ps::FftArgs a{};
    a.n_cls = 1;
    ps::FftClass& c = a.cls[0];
    c.recs = nullptr;
    c.single = ps::RecDesc{data, frames * N, 0, dtype, 0};
    c.n_recs = 1;
    c.g_lo = 0;
    c.g_hi = frames;
    c.out_g0 = 0;
    c.K = K;
    c.g = d_g;
    c.tw = nullptr;
    c.dft_n = N;
    c.tw64 = d_tw64;
    c.dft_n1 = N1;
    c.out = out;
    c.out_chan_stride = frames * K;
    a.n_channels = 1;
    // the library's launch shapes (launch_dft)
    if (N1 > 0) {
        if (N % N1 != 0 || N1 > N / N1) return 2;
        const size_t lds = ps::dft2_lds_bytes(N, N1);
        emu_dyn_smem = (char*)malloc(lds);
        emu_launch([a] { ps::k_window_dft2(a); }, dim3((unsigned)frames, 1), 256);
        free(emu_dyn_smem);
    } else {
        const dim3 grid((unsigned)((frames + ps::kDftFrames - 1) / ps::kDftFrames), 1,
                        (unsigned)((K + ps::kDftBins - 1) / ps::kDftBins));
        emu_launch([a] { ps::k_window_dft(a); }, grid, 256);
    }
    FILE* f = fopen(out_path, "wb");
    if (!f) return 4;
    fwrite(out, sizeof(float2), (size_t)(frames * K), f);
    fclose(f);
    std::vector<double> samp((size_t)(frames * N));
    for (int64_t i = 0; i < frames * N; ++i)
        samp[i] = dtype == 0 ? ((const float*)data)[i] : dtype == 1 ? ((const double*)data)[i]
                                                                   : ((const int16_t*)data)[i];
    std::string p2 = std::string(out_path) + ".in";
    f = fopen(p2.c_str(), "wb");
    fwrite(samp.data(), sizeof(double), samp.size(), f);
    fwrite(d_g, sizeof(float), N, f);
    fclose(f);
    free(raw);
    free(d_g);
    free(d_tw64);
    free(out);
    return 0;
}
