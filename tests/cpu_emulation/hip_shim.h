// A minimal host stand-in for the HIP runtime header, for compiling the
// library's transform kernels as plain C++ (test infrastructure only): every
// GPU thread of a block becomes a std::thread, LDS arrays become static
// arrays shared by those threads, and the workgroup barrier becomes a
// std::barrier.  Built with AddressSanitizer, an out-of-bounds access to any
// global buffer or LDS array of the emulated launch is reported.
#pragma once
#include <barrier>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
// dynamic LDS of the emulated launch: a buffer of exactly the launch's size
extern char* emu_dyn_smem;
#define HIP_DYNAMIC_SHARED(type, var) type* var = reinterpret_cast<type*>(emu_dyn_smem);
#define __restrict__ __restrict

struct dim3 {
    unsigned x = 1, y = 1, z = 1;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct emu_idx {
    unsigned x, y, z;
};
extern thread_local emu_idx threadIdx, blockIdx;

struct float2 {
    float x, y;
};
struct double2 {
    double x, y;
};
struct short2 {
    short x, y;
};
struct int2 {
    int x, y;
};
inline float2 make_float2(float a, float b) { return float2{a, b}; }
inline double2 make_double2(double a, double b) { return double2{a, b}; }
inline int2 make_int2(int a, int b) { return int2{a, b}; }

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorInvalidConfiguration = 9, hipErrorInvalidDevice = 101,
       hipErrorInvalidSymbol = 701 };
typedef void* hipStream_t;
inline hipError_t hipGetLastError() { return hipSuccess; }

// the workgroup barrier of the emulated block
extern std::barrier<>* emu_block_barrier;
inline void emu_barrier() { emu_block_barrier->arrive_and_wait(); }
#define __builtin_amdgcn_s_barrier() emu_barrier()
#define __builtin_amdgcn_fence(...) ((void)0)
