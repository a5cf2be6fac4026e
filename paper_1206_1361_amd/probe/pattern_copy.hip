// pattern_copy.hip -- the memory access patterns of the strided sweeps,
// without their arithmetic: an in-place pass over a 512x512x384 complex128
// array in which each block takes XT neighbouring columns across a plane
// and the whole line of every column along y or z (P chunks of C points per
// column, as the chunked y/z sweeps hold them), loads the tile, waits at a
// barrier and stores it back, scaled by a factor known only at run time (1)
// so that no load-store pair can be folded away.  Plain streaming passes over
// the same array (E elements per thread, consecutive threads on consecutive
// elements) are timed beside it as the copy ceiling.  A shape may pad the
// array: PAD extra elements after every plane (z lines) or every row (y
// lines), so that the line stride is no longer a power of two; the bytes
// counted stay those of the unpadded array.  An optional argument sets nx
// (default 512): with 256 the 16-byte elements stand for pairs of complex64
// columns, so the shapes are those of the complex64 sweeps of 512x512x384,
// which hold two neighbouring columns per thread.  Prints one line per shape:
// time per pass (HIP events, mean of 10 after 3 warm-up passes), GB/s of
// one read and one write of the array, and the fraction of 8 TB/s.
//
// Built by paper_1206_1361_amd/build.py as paper_1206_1361_amd/probe/pattern_copy;
// a measurement tool, not part of the library.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

typedef double d2 __attribute__((ext_vector_type(2)));

#define CHECK(x)                                                                   \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                              \
        }                                                                          \
    } while (0)

// Tile t of XT columns (t = b, or with xcd_ranges t = (b mod 8) G/8 + b/8,
// as the y sweep maps its blocks); thread (tx, pc) holds points
// pc C .. pc C + C - 1 of column col0 + tx.  Every grid here has nx a
// multiple of XT, so no thread leaves before the barrier.
template <int C>
__global__ void __launch_bounds__(1024) tile_pass(d2 *psi, int nx, int n, long stride, long outer_stride, int ncol,
                                                  int ntiles, int xcd_ranges, double scale)
{
    const int b = blockIdx.x, G = gridDim.x;
    const int tile = xcd_ranges && G % 8 == 0 ? (b % 8) * (G / 8) + b / 8 : b;
    const int outer = tile / ncol;
    const int i = (tile - outer * ncol) * (int)blockDim.x + (int)threadIdx.x;
    const int pos0 = (int)threadIdx.y * C;
    d2 *base = psi + (long)outer * outer_stride + i + (long)pos0 * stride;
    d2 u[C];
#pragma unroll
    for (int c = 0; c < C; ++c) u[c] = pos0 + c < n ? __builtin_nontemporal_load(base + (long)c * stride) : d2{0, 0};
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c)
        if (pos0 + c < n) __builtin_nontemporal_store(u[c] * scale, base + (long)c * stride);
}

// Block b (T threads) covers elements [b T E, (b + 1) T E); thread t takes
// t, t + T, ... within it.  Dynamic LDS, when asked for, only limits how
// many blocks share a CU.
template <int E>
__global__ void __launch_bounds__(256) stream_pass(d2 *psi, long n, double scale)
{
    const long T = blockDim.x;
    const long base = (long)blockIdx.x * T * E + threadIdx.x;
    d2 u[E];
#pragma unroll
    for (int e = 0; e < E; ++e) u[e] = base + T * e < n ? __builtin_nontemporal_load(psi + base + T * e) : d2{0, 0};
#pragma unroll
    for (int e = 0; e < E; ++e)
        if (base + T * e < n) __builtin_nontemporal_store(u[e] * scale, psi + base + T * e);
}

int main(int argc, char **argv)
{
    const double scale = argc > 99 ? 2.0 : 1.0;
    const int nx = argc > 1 ? std::atoi(argv[1]) : 512, ny = 512, nz = 384;
    if (nx < 64 || nx > 4096 || nx % 64 != 0) {
        std::printf("nx must be a multiple of 64 in 64..4096\n");
        return 1;
    }
    const long N = (long)nx * ny * nz;
    d2 *psi = nullptr;
    CHECK(hipMalloc(&psi, N * sizeof(d2)));
    CHECK(hipMemset(psi, 0, N * sizeof(d2)));
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    const double bytes = 2.0 * (double)N * sizeof(d2);
    auto report = [&](const char *name, float ms) {
        std::printf("%-46s %8.4f ms %7.0f GB/s %6.3f\n", name, ms, bytes / (ms * 1e-3) / 1e9,
                    bytes / (ms * 1e-3) / 8e12);
        std::fflush(stdout);
    };
    auto time_it = [&](auto launch) -> float {
        for (int w = 0; w < 3; ++w) launch();
        (void)hipEventRecord(a, nullptr);
        for (int r = 0; r < 10; ++r) launch();
        (void)hipEventRecord(b, nullptr);
        (void)hipEventSynchronize(b);
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, a, b);
        return ms / 10.0f;
    };
    if (nx == 256)
        std::printf("512x512x384 complex64 as 256x512x384 pairs of columns (16 bytes), one read + one write of %.3f GiB per pass\n",
                    N * 16.0 / (1 << 30));
    else
        std::printf("%dx512x384 complex128, one read + one write of %.3f GiB per pass\n", nx, N * 16.0 / (1 << 30));
    report("stream, 1 element per thread", time_it([&] {
               hipLaunchKernelGGL(stream_pass<1>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, nullptr, psi, N, scale);
           }));
    report("stream, 4 elements per thread", time_it([&] {
               hipLaunchKernelGGL(stream_pass<4>, dim3((unsigned)((N + 1023) / 1024)), dim3(256), 0, nullptr, psi, N, scale);
           }));
    report("stream, 16 elements per thread", time_it([&] {
               hipLaunchKernelGGL(stream_pass<16>, dim3((unsigned)((N + 4095) / 4096)), dim3(256), 0, nullptr, psi, N, scale);
           }));
    // one-wavefront blocks taking one 512-element row each, as the x sweep
    // moves a complex128 line, with at most W blocks per CU (LDS-limited)
    for (int w : {0, 32, 16, 8, 4}) {
        const size_t lds = w ? (160 * 1024) / w - 64 : 0;
        char name[96];
        std::snprintf(name, sizeof name, "stream, 64-thread blocks x 8 elements%s%d", w ? ", <= waves/CU " : "", w);
        if (!w) std::snprintf(name, sizeof name, "stream, 64-thread blocks x 8 elements");
        report(name, time_it([&] {
                   hipLaunchKernelGGL(stream_pass<8>, dim3((unsigned)((N + 511) / 512)), dim3(64), lds, nullptr, psi, N, scale);
               }));
    }
    // one-wavefront blocks taking 256 16-byte elements each, as the x sweep
    // moves a 512-point complex64 line
    report("stream, 64-thread blocks x 4 elements", time_it([&] {
               hipLaunchKernelGGL(stream_pass<4>, dim3((unsigned)((N + 255) / 256)), dim3(64), 0, nullptr, psi, N, scale);
           }));
    report("stream, 64-thread blocks x 1 element", time_it([&] {
               hipLaunchKernelGGL(stream_pass<1>, dim3((unsigned)((N + 63) / 64)), dim3(64), 0, nullptr, psi, N, scale);
           }));
    report("stream, 256-thread blocks x 2 elements", time_it([&] {
               hipLaunchKernelGGL(stream_pass<2>, dim3((unsigned)((N + 511) / 512)), dim3(256), 0, nullptr, psi, N, scale);
           }));
    for (int w : {16, 12}) {
        const size_t lds = (160 * 1024) / (w / 4) - 64;   // at most 64 KiB per block
        char name[96];
        std::snprintf(name, sizeof name, "stream, 256-thread blocks x 1 element, <= waves/CU %d", w);
        report(name, time_it([&] {
                   hipLaunchKernelGGL(stream_pass<1>, dim3((unsigned)((N + 255) / 256)), dim3(256), lds, nullptr, psi, N, scale);
               }));
    }
    struct Shape {
        int axis, xt, c, xcd, pad;
    };
    const std::vector<Shape> shapes = {
        {1, 8, 4, 1, 0},  {1, 16, 8, 1, 0},  {1, 16, 8, 0, 0}, {1, 16, 16, 1, 0}, {1, 16, 16, 0, 0},
        {1, 32, 16, 1, 0}, {1, 32, 24, 1, 0}, {1, 16, 16, 1, 16}, {1, 16, 16, 1, 64},
        {2, 8, 8, 0, 0},  {2, 16, 8, 0, 0},  {2, 16, 8, 1, 0}, {2, 16, 16, 0, 0}, {2, 32, 16, 0, 0},
        {2, 64, 24, 0, 0}, {2, 32, 24, 0, 0}, {2, 16, 8, 0, 16}, {2, 16, 8, 0, 64}, {2, 16, 8, 0, 512},
        {2, 16, 8, 0, 4096}, {2, 16, 6, 0, 0}, {2, 16, 12, 0, 0}, {2, 32, 12, 0, 0}, {1, 16, 12, 1, 0},
        {1, 32, 12, 1, 0}, {1, 16, 6, 1, 0},
    };
    // the largest padded array any shape addresses
    long need = N;
    for (const Shape &s : shapes) {
        const long padded = s.axis == 2 ? (long)nz * ((long)nx * ny + s.pad) : (long)nz * ny * (nx + s.pad);
        need = padded > need ? padded : need;
    }
    CHECK(hipFree(psi));
    CHECK(hipMalloc(&psi, need * sizeof(d2)));
    CHECK(hipMemset(psi, 0, need * sizeof(d2)));
    for (const Shape &s : shapes) {
        const int n = s.axis == 2 ? nz : ny;
        const int P = (n + s.c - 1) / s.c;
        if (s.xt * P > 1024 || nx % s.xt != 0) continue;
        const long row = s.axis == 2 ? nx : nx + s.pad;
        const long plane = s.axis == 2 ? (long)nx * ny + s.pad : (long)ny * row;
        const long stride = s.axis == 2 ? plane : row;
        const long outer_stride = s.axis == 2 ? row : plane;
        const int nouter = s.axis == 2 ? ny : nz;
        const int ncol = nx / s.xt, ntiles = ncol * nouter;
        const dim3 grid((unsigned)ntiles), block((unsigned)s.xt, (unsigned)P);
        char name[96];
        char padtxt[32] = "";
        if (s.pad) std::snprintf(padtxt, sizeof padtxt, ", pad %d", s.pad);
        std::snprintf(name, sizeof name, "%c lines: %2d cols x %2d chunks of %2d%s%s", s.axis == 2 ? 'z' : 'y', s.xt,
                      P, s.c, s.xcd ? ", XCD tile ranges" : "", padtxt);
        auto run = [&] {
            switch (s.c) {
            case 4: hipLaunchKernelGGL(tile_pass<4>, grid, block, 0, nullptr, psi, nx, n, stride, outer_stride, ncol, ntiles, s.xcd, scale); break;
            case 6: hipLaunchKernelGGL(tile_pass<6>, grid, block, 0, nullptr, psi, nx, n, stride, outer_stride, ncol, ntiles, s.xcd, scale); break;
            case 12: hipLaunchKernelGGL(tile_pass<12>, grid, block, 0, nullptr, psi, nx, n, stride, outer_stride, ncol, ntiles, s.xcd, scale); break;
            case 8: hipLaunchKernelGGL(tile_pass<8>, grid, block, 0, nullptr, psi, nx, n, stride, outer_stride, ncol, ntiles, s.xcd, scale); break;
            case 16: hipLaunchKernelGGL(tile_pass<16>, grid, block, 0, nullptr, psi, nx, n, stride, outer_stride, ncol, ntiles, s.xcd, scale); break;
            case 24: hipLaunchKernelGGL(tile_pass<24>, grid, block, 0, nullptr, psi, nx, n, stride, outer_stride, ncol, ntiles, s.xcd, scale); break;
            }
        };
        report(name, time_it(run));
    }
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    CHECK(hipFree(psi));
    return 0;
}
