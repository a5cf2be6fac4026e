// yz_small.cpp -- the fused small-grid y/z kernel (calclu_yz_small_kernel)
// against the separate y and z launches (calclu_strided_kernel, one column
// per thread), on the CPU under AddressSanitizer: one imaginary-time step
// (norm partials on) and one real-time step of each small grid, complex128
// and complex64, and one imaginary-time step on float64 and float32 storage,
// from seeded random states.  Prints, per case, whether psi
// and the z partials agree bit for bit.  Built and run by run.py --yz-small.
#include "hip/hip_runtime.h"
thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;
thread_local BlockCtx g_blk;
thread_local unsigned char *g_lds;
#include <functional>
#include <random>
#include <thread>
#include <vector>
#include "sweep_yz.cpp"
#include "reduce.cpp"
#include "solve_host.h"
using namespace gpssc_host;
using gpssc::cx;
using gpssc::value_t;

static unsigned char *g_lds_block = nullptr;   // the running block's LDS

// every block of a launch, one after another; bx*by host threads stand for
// the block's GPU threads, each block with its own zero-filled LDS
static void launch(int nblocks, int bx, int by, size_t lds, const std::function<void()> &body)
{
    const int nt = bx * by;
    std::barrier<> bar(nt);
    std::vector<unsigned char> xch(16 * 64 * ((nt + 63) / 64) + 16);
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            for (int b = 0; b < nblocks; ++b) {
                threadIdx = dim3(t % bx, t / bx);
                blockIdx = dim3(b);
                blockDim = dim3(bx, by);
                gridDim = dim3(nblocks);
                g_blk = BlockCtx{&bar, xch.data() + 16 * 64 * (t / 64)};
                if (t == 0) {
                    std::free(g_lds_block);
                    g_lds_block = lds ? (unsigned char *)std::malloc(lds) : nullptr;
                    if (lds) std::memset(g_lds_block, 0xCD, lds);
                }
                bar.arrive_and_wait();
                g_lds = g_lds_block;
                body();
                bar.arrive_and_wait();   // the block is done before the next one starts
            }
        });
    for (auto &x : th) x.join();
    std::free(g_lds_block);
    g_lds_block = nullptr;
}

template <typename S, typename A, bool REAL, int CY, int CZ>
static bool run_case(const int64_t grid[3], gp_dtype dtype, unsigned seed)
{
    SolveDesc x;
    std::mt19937 rng(seed);
    std::uniform_real_distribution<double> U(0.5, 3.0);
    for (int a = 0; a < 3; ++a) { x.grid[a] = grid[a]; x.dx[a] = 0.3; x.omega[a] = U(rng); }
    x.dt = 0.02; x.g = 25.0; x.real = REAL;
    const ClassShape c = class_shape(x.grid, dtype);
    if (c.chunk[1] != CY || c.chunk[2] != CZ) { std::printf("chunk mismatch\n"); return false; }
    build_solve(x, c);
    std::vector<unsigned char> tab(table_bytes(c, dtype));
    pack_solve_tables(x, c, dtype, tab.data());
    gpssc::XBatchArgs<A> xa; gpssc::SBatchArgs<A> ya, za;
    fill_solve_args<A>(x, c, tab.data(), xa, ya, za);
    const int nx = (int)grid[0], ny = (int)grid[1], nz = (int)grid[2];
    std::vector<S> psi0((size_t)x.elems);
    std::normal_distribution<double> N(0.0, 1.0);
    for (auto &v : psi0) {
        if constexpr (std::is_same<S, double>::value || std::is_same<S, float>::value) {
            v = (S)N(rng);
        } else {
            v.x = N(rng);
            v.y = REAL ? N(rng) : 0.0;
        }
    }
    constexpr bool NORM = !REAL;

    // separate launches, one column per thread, as launch_strided shapes them
    std::vector<S> p1 = psi0;
    std::vector<double> q1((size_t)nx * ny, -1.0);
    for (int ax = 1; ax < 3; ++ax) {
        const gpssc::SArgs<A> &a = ax == 1 ? ya.s : za.s;
        const cx<A> *zt = ax == 1 ? ya.zt : za.zt;
        const int xt = class_columns(c, ax, 1, dtype), P = a.lanes, nouter = ax == 1 ? nz : ny;
        const int ncol = (nx + xt - 1) / xt, ntiles = ncol * nouter;
        const size_t lds = 2 * (size_t)xt * P * sizeof(value_t<S, A>);
        launch(ntiles, xt, P, lds, [&] {
            if (ax == 1)
                gpssc::calclu_strided_kernel<S, A, CY, REAL, false, 1>(p1.data(), a, zt, nullptr, ncol, ntiles, 1);
            else
                gpssc::calclu_strided_kernel<S, A, CZ, REAL, NORM, 1>(p1.data(), a, zt, NORM ? q1.data() : nullptr,
                                                                      ncol, ntiles, 0);
        });
    }

    // one launch: the plan's 2 columns per block, and 4 (two rounds of tiles
    // per phase on the 64^3 grid)
    bool all = true;
    for (int cols : {2, 4}) {
        std::vector<S> p2 = psi0;
        std::vector<double> q2((size_t)nx * ny, -1.0);
        const int xw = (int)std::min<int64_t>(cols, nx);
        const int64_t need = std::max((int64_t)xw * ya.s.lanes * nz, (int64_t)xw * za.s.lanes * ny);
        const int threads = (int)std::min<int64_t>((need + 63) / 64 * 64, 1024);
        size_t slot = 2 * (size_t)xw * (size_t)std::max(ya.s.lanes, za.s.lanes) * sizeof(value_t<S, A>);
        if (NORM) slot = std::max(slot, (size_t)xw * za.s.lanes * sizeof(double));
        const size_t nslots = (size_t)std::max(threads / (xw * ya.s.lanes), threads / (xw * za.s.lanes));
        launch((nx + xw - 1) / xw, threads, 1, nslots * slot, [&] {
            gpssc::calclu_yz_small_kernel<S, A, CY, CZ, REAL, NORM>(p2.data(), ya.s, ya.zt, nz, za.s, za.zt, ny,
                                                                    NORM ? q2.data() : nullptr, xw, (int)slot);
        });
        const bool same = std::memcmp(p1.data(), p2.data(), sizeof(S) * p1.size()) == 0;
        const bool qsame = std::memcmp(q1.data(), q2.data(), sizeof(double) * q1.size()) == 0;
        std::printf("%dx%dx%d %s %s, %d cols: %d threads x %d blocks, psi equal %d, partials equal %d\n", nx, ny,
                    nz, gpssc::storage_traits<S>::complex ? (sizeof(A) == 8 ? "c128" : "c64") : (sizeof(A) == 8 ? "r64" : "r32"),
                    REAL ? "real" : "imag", xw, threads, (nx + xw - 1) / xw,
                    (int)same, (int)qsame);
        std::fflush(stdout);
        all = all && same && qsame;
    }
    return all;
}

template <typename S, typename A, bool REAL>
static bool run_grid(const int64_t g[3], gp_dtype dtype, unsigned seed)
{
    const ClassShape c = class_shape(g, dtype);
#define GP_C(CY, CZ) \
    if (c.chunk[1] == CY && c.chunk[2] == CZ) return run_case<S, A, REAL, CY, CZ>(g, dtype, seed);
    GP_C(1, 1) GP_C(1, 2) GP_C(1, 4) GP_C(1, 8) GP_C(2, 1) GP_C(2, 2) GP_C(2, 4) GP_C(2, 8)
    GP_C(4, 1) GP_C(4, 2) GP_C(4, 4) GP_C(4, 8) GP_C(8, 1) GP_C(8, 2) GP_C(8, 4) GP_C(8, 8)
#undef GP_C
    std::printf("no kernel for chunks %d, %d\n", c.chunk[1], c.chunk[2]);
    return false;
}

int main()
{
    const int64_t grids[][3] = {{32, 32, 32}, {16, 20, 24}, {24, 20, 16}, {9, 17, 33}, {33, 17, 9},
                                {5, 3, 7},    {3, 4, 1},    {7, 1, 5},    {64, 64, 64}};
    int bad = 0;
    unsigned seed = 1;
    for (const auto &g : grids) {
        bad += !run_grid<double2, double, false>(g, GP_C128, seed++);
        bad += !run_grid<double2, double, true>(g, GP_C128, seed++);
        bad += !run_grid<float2, float, false>(g, GP_C64, seed++);
        bad += !run_grid<float2, float, true>(g, GP_C64, seed++);
        bad += !run_grid<double, double, false>(g, GP_R64, seed++);
        bad += !run_grid<float, float, false>(g, GP_R32, seed++);
    }
    std::printf("cases differing: %d\n", bad);
    return bad ? 1 : 0;
}
