// Issue cost of vector instructions on the SIMDs of one GPU: each thread runs
// ITER iterations of 8 independent chains of one instruction kind, with 1, 2,
// 4 and 8 waves per SIMD (256-thread blocks, 256 x wps blocks).  Printed:
// SIMD cycles per wave64 chain step at 2.4 GHz (kernel time over the steps
// one SIMD runs).  Build and run:
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//       paper_2505_01231_amd/csrc/examples/valu_issue_rate.hip -o /tmp/valu_issue_rate
//   /tmp/valu_issue_rate
#include <hip/hip_runtime.h>
#include <cstdio>
#include <vector>
constexpr int ITER = 2048;
__global__ __launch_bounds__(256) void k_cvt(const float* in, double* out) {
    float x[8]; double a[8];
    for (int i = 0; i < 8; ++i) { x[i] = in[threadIdx.x + i]; a[i] = 0.0; }
    for (int it = 0; it < ITER; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const double c = (double)x[i];          // v_cvt_f64_f32
            a[i] = fma(c, c, a[i]);                 // v_fma_f64
            x[i] = __builtin_bit_cast(float, __builtin_bit_cast(int, x[i]) + 1);   // v_add_u32
        }
    }
    double s = 0; for (int i = 0; i < 8; ++i) s += a[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ __launch_bounds__(256) void k_nocvt(const float* in, double* out) {
    double x[8], a[8];
    for (int i = 0; i < 8; ++i) { x[i] = in[threadIdx.x + i]; a[i] = 0.0; }
    for (int it = 0; it < ITER; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            a[i] = fma(x[i], x[i], a[i]);           // v_fma_f64
            x[i] = __builtin_bit_cast(double, __builtin_bit_cast(long, x[i]) + 1);   // 64-bit add (2 ops)
        }
    }
    double s = 0; for (int i = 0; i < 8; ++i) s += a[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ __launch_bounds__(256) void k_fma64(const float* in, double* out) {
    double x[8], a[8];
    for (int i = 0; i < 8; ++i) { x[i] = in[threadIdx.x + i]; a[i] = 1.0; }
    for (int it = 0; it < ITER; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = fma(a[i], x[i], 0.5);
    }
    double s = 0; for (int i = 0; i < 8; ++i) s += a[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ __launch_bounds__(256) void k_fma32(const float* in, double* out) {
    float x[8], a[8];
    for (int i = 0; i < 8; ++i) { x[i] = in[threadIdx.x + i]; a[i] = 1.0f; }
    for (int it = 0; it < ITER; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = fmaf(a[i], x[i], 0.5f);
    }
    double s = 0; for (int i = 0; i < 8; ++i) s += a[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}
template <typename K>
float run(K k, const float* in, double* out, int blocks) {
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, 0, in, out);
    (void)hipEventRecord(a);
    for (int r = 0; r < 5; ++r) hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, 0, in, out);
    (void)hipEventRecord(b);
    (void)hipEventSynchronize(b);
    float ms;
    (void)hipEventElapsedTime(&ms, a, b);
    return ms / 5;
}
int main() {
    float* in; double* out;
    (void)hipMalloc(&in, 1024 * sizeof(float));
    (void)hipMalloc(&out, (size_t)256 * 8 * 256 * sizeof(double));
    std::vector<float> h(1024, 1.0001f);
    (void)hipMemcpy(in, h.data(), 1024 * 4, hipMemcpyHostToDevice);
    const char* names[4] = {"cvt+fma64+add32", "fma64+add64", "fma_f64", "fma_f32"};
    for (int wps : {1, 2, 4, 8}) {
        const int blocks = 256 * wps;              // wps waves per SIMD (one block of 4 waves per CU per wps)
        const double steps = (double)wps * ITER * 8;
        float t[4] = {run(k_cvt, in, out, blocks), run(k_nocvt, in, out, blocks), run(k_fma64, in, out, blocks),
                      run(k_fma32, in, out, blocks)};
        for (int i = 0; i < 4; ++i)
            printf("waves/SIMD %d  %-18s %.4f ms  %.2f SIMD cycles per chain step\n", wps, names[i], t[i],
                   t[i] * 1e-3 * 2.4e9 / steps);
    }
    return 0;
}
