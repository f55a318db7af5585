/* A C99 client of libpolyspec: the whole estimator through the C ABI alone,
 * with device memory from the HIP runtime (no PyTorch).
 *
 *   ps_c_client IN.f32 OUT.f64 N N_F M PRECISION
 *
 * IN.f32 holds one channel of float32 samples; the program copies them to the
 * device, runs ps_execute for S2, S3 and S4 with an acG window, and writes to
 * OUT.f64 the FP64 outputs in the order S2, S2 error, S3, S3 error, S4, S4
 * error (the layouts of ps_output), preceded by the chunk count as a double.
 * PRECISION is 0 (FP32), 1 (split BF16 x 3) or 2 (scaled FP16 x 2).  Exit
 * status 0 on success; every failure prints the library's or the runtime's
 * message and exits non-zero.
 *
 *   ps_c_client stream IN.f32 OUT.f64 N N_F M PRECISION PIECE SPLIT STATE
 *
 * The same record through the running accumulation (ps_stream_*), pushed in
 * pieces of PIECE samples.  With SPLIT > 0 the accumulation stops after
 * SPLIT pieces: its state is exported to the file STATE, the accumulator is
 * destroyed, a new one (of a new plan) imports the file and takes the
 * remaining pieces.  OUT.f64 as above. */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "polyspec.h"

#define HIP_CHECK(call)                                                               \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));         \
            return 2;                                                                 \
        }                                                                             \
    } while (0)

#define PS_CHECK(call)                                                                \
    do {                                                                              \
        ps_status s_ = (call);                                                        \
        if (s_ != PS_OK) {                                                            \
            fprintf(stderr, "%s: %s: %s\n", #call, ps_status_string(s_), ps_last_error()); \
            return 3;                                                                 \
        }                                                                             \
    } while (0)

static int write_outputs(const char* path, int64_t n_chunks, double* const* d_out, const size_t* sizes) {
    FILE* g = fopen(path, "wb");
    if (!g) {
        fprintf(stderr, "cannot open %s\n", path);
        return 1;
    }
    const double header = (double)n_chunks;
    fwrite(&header, sizeof(double), 1, g);
    for (int i = 0; i < 6; ++i) {
        double* h = (double*)malloc(sizes[i] * sizeof(double));
        HIP_CHECK(hipMemcpy(h, d_out[i], sizes[i] * sizeof(double), hipMemcpyDeviceToHost));
        fwrite(h, sizeof(double), sizes[i], g);
        free(h);
    }
    fclose(g);
    return 0;
}

static float* read_f32(const char* path, int64_t* n) {
    FILE* f = fopen(path, "rb");
    if (!f) return NULL;
    fseek(f, 0, SEEK_END);
    const long bytes = ftell(f);
    fseek(f, 0, SEEK_SET);
    *n = bytes / (long)sizeof(float);
    float* h = (float*)malloc((size_t)*n * sizeof(float));
    if (h && fread(h, sizeof(float), (size_t)*n, f) != (size_t)*n) {
        free(h);
        h = NULL;
    }
    fclose(f);
    return h;
}

static ps_config make_config(int N, int nf, int m, int precision) {
    ps_config cfg = {0};
    cfg.struct_size = sizeof(ps_config);
    cfg.orders = PS_ORDER_S2 | PS_ORDER_S3 | PS_ORDER_S4;
    cfg.n_channels = 1;
    cfg.frame_len = N;
    cfg.n_freq = nf;
    cfg.m = m;
    cfg.dt = 1.0;
    cfg.window = PS_WIN_ACG;
    cfg.window_param = 0.14;
    cfg.precision = precision;
    cfg.schedule = PS_SCHED_BATCHED;
    return cfg;
}

static int run_stream(char** argv) {
    int64_t n = 0;
    float* h_z = read_f32(argv[2], &n);
    if (!h_z) {
        fprintf(stderr, "cannot read %s\n", argv[2]);
        return 1;
    }
    const ps_config cfg = make_config(atoi(argv[4]), atoi(argv[5]), atoi(argv[6]), atoi(argv[7]));
    const int64_t piece = atoll(argv[8]);
    const int split = atoi(argv[9]);
    const char* state_path = argv[10];
    if (piece < 1) return 1;
    ps_plan_t plan = NULL;
    PS_CHECK(ps_plan_create(&cfg, &plan));
    ps_plan_info info;
    PS_CHECK(ps_plan_query(plan, &info));
    float* d_z = NULL;
    HIP_CHECK(hipMalloc((void**)&d_z, (size_t)n * sizeof(float)));
    HIP_CHECK(hipMemcpy(d_z, h_z, (size_t)n * sizeof(float), hipMemcpyHostToDevice));
    hipStream_t stream;
    HIP_CHECK(hipStreamCreate(&stream));
    ps_accum_t acc = NULL;
    PS_CHECK(ps_stream_begin(plan, piece, PS_F32, &acc));
    int pushed = 0;
    for (int64_t at = 0; at < n; at += piece, ++pushed) {
        if (split > 0 && pushed == split) {
            /* checkpoint: state to a file, everything torn down and rebuilt */
            size_t bytes = 0;
            PS_CHECK(ps_stream_export_state(acc, NULL, &bytes));
            void* buf = malloc(bytes);
            PS_CHECK(ps_stream_export_state(acc, buf, &bytes));
            FILE* f = fopen(state_path, "wb");
            if (!f || fwrite(buf, 1, bytes, f) != bytes) return 1;
            fclose(f);
            free(buf);
            PS_CHECK(ps_stream_destroy(acc));
            PS_CHECK(ps_plan_destroy(plan));
            plan = NULL;
            acc = NULL;
            PS_CHECK(ps_plan_create(&cfg, &plan));
            PS_CHECK(ps_stream_begin(plan, piece, PS_F32, &acc));
            f = fopen(state_path, "rb");
            if (!f) return 1;
            buf = malloc(bytes);
            if (fread(buf, 1, bytes, f) != bytes) return 1;
            fclose(f);
            PS_CHECK(ps_stream_import_state(acc, buf, bytes));
            free(buf);
        }
        const int64_t len = n - at < piece ? n - at : piece;
        PS_CHECK(ps_stream_push(acc, d_z + at, len, len, stream));
    }
    const size_t nf = (size_t)info.n_freq;
    const size_t sizes[6] = {2 * nf, 2 * nf, 2 * nf * nf, 2 * nf * nf, 2 * nf * nf, 2 * nf * nf};
    double* d_out[6];
    for (int i = 0; i < 6; ++i) HIP_CHECK(hipMalloc((void**)&d_out[i], sizes[i] * sizeof(double)));
    ps_output out = {d_out[0], d_out[1], d_out[2], d_out[3], d_out[4], d_out[5], NULL, NULL};
    PS_CHECK(ps_stream_end(acc, &out, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    int64_t n_chunks = 0, n_samples = 0, n_carry = 0;
    PS_CHECK(ps_stream_counts(acc, &n_chunks, &n_samples, &n_carry));
    if (write_outputs(argv[3], n_chunks, d_out, sizes)) return 1;
    for (int i = 0; i < 6; ++i) HIP_CHECK(hipFree(d_out[i]));
    PS_CHECK(ps_stream_destroy(acc));
    PS_CHECK(ps_plan_destroy(plan));
    HIP_CHECK(hipStreamDestroy(stream));
    HIP_CHECK(hipFree(d_z));
    free(h_z);
    printf("ps_c_client stream: chunks=%lld samples=%lld carry=%lld split=%d ok\n", (long long)n_chunks,
           (long long)n_samples, (long long)n_carry, split);
    return 0;
}

int main(int argc, char** argv) {
    if (argc == 11 && strcmp(argv[1], "stream") == 0) return run_stream(argv);
    if (argc != 7) {
        fprintf(stderr, "usage: %s IN.f32 OUT.f64 N N_F M PRECISION\n"
                        "       %s stream IN.f32 OUT.f64 N N_F M PRECISION PIECE SPLIT STATE\n", argv[0], argv[0]);
        return 1;
    }
    FILE* f = fopen(argv[1], "rb");
    if (!f) {
        fprintf(stderr, "cannot open %s\n", argv[1]);
        return 1;
    }
    fseek(f, 0, SEEK_END);
    const long bytes = ftell(f);
    fseek(f, 0, SEEK_SET);
    const int64_t n = bytes / (long)sizeof(float);
    float* h_z = (float*)malloc((size_t)n * sizeof(float));
    if (!h_z || fread(h_z, sizeof(float), (size_t)n, f) != (size_t)n) {
        fprintf(stderr, "cannot read %s\n", argv[1]);
        return 1;
    }
    fclose(f);

    ps_config cfg = {0};
    cfg.struct_size = sizeof(ps_config);
    cfg.orders = PS_ORDER_S2 | PS_ORDER_S3 | PS_ORDER_S4;
    cfg.n_channels = 1;
    cfg.frame_len = atoi(argv[3]);
    cfg.n_freq = atoi(argv[4]);
    cfg.m = atoi(argv[5]);
    cfg.dt = 1.0;
    cfg.window = PS_WIN_ACG;
    cfg.window_param = 0.14;
    cfg.precision = atoi(argv[6]);
    cfg.schedule = PS_SCHED_BATCHED;

    ps_plan_t plan = NULL;
    PS_CHECK(ps_plan_create(&cfg, &plan));
    ps_plan_info info;
    PS_CHECK(ps_plan_query(plan, &info));
    int64_t n_chunks = 0;
    uint32_t flags = 0;
    PS_CHECK(ps_record_info(plan, n, &n_chunks, &flags));

    float* d_z = NULL;
    HIP_CHECK(hipMalloc((void**)&d_z, (size_t)n * sizeof(float)));
    HIP_CHECK(hipMemcpy(d_z, h_z, (size_t)n * sizeof(float), hipMemcpyHostToDevice));
    ps_record rec = {d_z, n, n, PS_F32, 0};

    size_t ws_bytes = 0;
    PS_CHECK(ps_workspace_size(plan, &rec, 1, &ws_bytes));
    void* d_ws = NULL;
    HIP_CHECK(hipMalloc(&d_ws, ws_bytes));

    const size_t nf = (size_t)info.n_freq;
    const size_t sizes[6] = {2 * nf, 2 * nf, 2 * nf * nf, 2 * nf * nf, 2 * nf * nf, 2 * nf * nf};
    double* d_out[6];
    for (int i = 0; i < 6; ++i) HIP_CHECK(hipMalloc((void**)&d_out[i], sizes[i] * sizeof(double)));
    ps_output out = {d_out[0], d_out[1], d_out[2], d_out[3], d_out[4], d_out[5]};

    hipStream_t stream;
    HIP_CHECK(hipStreamCreate(&stream));
    PS_CHECK(ps_execute(plan, &rec, 1, d_ws, ws_bytes, &out, stream));
    HIP_CHECK(hipStreamSynchronize(stream));

    FILE* g = fopen(argv[2], "wb");
    if (!g) {
        fprintf(stderr, "cannot open %s\n", argv[2]);
        return 1;
    }
    const double header = (double)n_chunks;
    fwrite(&header, sizeof(double), 1, g);
    for (int i = 0; i < 6; ++i) {
        double* h = (double*)malloc(sizes[i] * sizeof(double));
        HIP_CHECK(hipMemcpy(h, d_out[i], sizes[i] * sizeof(double), hipMemcpyDeviceToHost));
        fwrite(h, sizeof(double), sizes[i], g);
        free(h);
        HIP_CHECK(hipFree(d_out[i]));
    }
    fclose(g);
    HIP_CHECK(hipStreamDestroy(stream));
    HIP_CHECK(hipFree(d_ws));
    HIP_CHECK(hipFree(d_z));
    PS_CHECK(ps_plan_destroy(plan));
    free(h_z);
    printf("ps_c_client: N=%d N_f=%d m=%d chunks=%lld precision=%d ok\n", cfg.frame_len, info.n_freq, cfg.m,
           (long long)n_chunks, cfg.precision);
    return 0;
}
