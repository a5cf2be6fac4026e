// CPU stand-in for the parts of the HIP runtime the sweep kernels use: each
// GPU thread of a block is a std::thread, __syncthreads is a std::barrier,
// shuffles go through a per-block exchange buffer.  Bounds are checked by
// ASan on the host.
#pragma once
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <algorithm>
#include <cstdio>
using std::min; using std::max;
using std::isfinite; using std::sqrt; using std::fma; using std::rint; using std::exp;
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __restrict__
struct dim3 { unsigned x = 1, y = 1, z = 1; dim3() {} dim3(unsigned a, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {} };
extern thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;
extern thread_local unsigned char *g_lds;
struct BlockCtx { std::barrier<> *bar; unsigned char *xch; };
extern thread_local BlockCtx g_blk;
inline void __syncthreads() { g_blk.bar->arrive_and_wait(); }
struct float2 { float x, y; };
struct double2 { double x, y; };
struct float4 { float x, y, z, w; };
typedef int hipError_t; typedef void *hipStream_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1 };
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipGetDevice(int *d) { *d = 0; return 0; }
inline hipError_t hipSetDevice(int) { return 0; }
inline const char *hipGetErrorString(hipError_t) { return "emu"; }
#define hipLaunchKernelGGL(...) ((void)0)
template <typename T> T shfl_xch(T v, int src, int lane)
{
    // every lane of the wavefront calls this together
    static_assert(sizeof(T) <= 16, "");
    std::memcpy(g_blk.xch + 16 * lane, &v, sizeof v);
    __syncthreads();
    T r = v;
    if (src >= 0 && src < 64) std::memcpy(&r, g_blk.xch + 16 * src, sizeof r);
    __syncthreads();
    return r;
}
template <typename T> T __shfl_up(T v, unsigned d, int w = 64) { int l = threadIdx.x % 64; return shfl_xch(v, l >= (int)d ? l - (int)d : l, l); }
template <typename T> T __shfl_down(T v, unsigned d, int w = 64) { int l = threadIdx.x % 64; return shfl_xch(v, l + (int)d < 64 ? l + (int)d : l, l); }
template <typename T> T __shfl(T v, int s, int w = 64) { int l = threadIdx.x % 64; return shfl_xch(v, s, l); }
