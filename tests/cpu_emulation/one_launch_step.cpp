// one_launch_step.cpp -- the batch kernels on the CPU: one imaginary-time
// (or, with the argument "real", real-time) step of the complex64 batch of
// test_one_launch_matches_per_class_launches_bitwise (the shapes of
// specs_wide, every solve active, or with a second argument the mask of that
// test) through the per-class kernels and through the kernels of
// GP_BATCH_ONE_LAUNCH, compiled for the host against the stand-in
// hip/hip_runtime.h and run under AddressSanitizer.  Prints whether the two
// forms leave the same bits.  Environment: ALL=1 runs every block (else the
// first two and last two blocks of every class and every 97th block, which
// checks bounds but leaves the comparison meaningless); SKIPX=1 / SKIPYZ=1
// leave out the x or the y/z sweeps.  Built and run by run.py.
#include "hip/hip_runtime.h"
thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;
thread_local BlockCtx g_blk;
thread_local unsigned char *g_lds;
#include <thread>
#include <vector>
#include <functional>
#include <random>
#include <map>
#include <tuple>
#include "sweep_x.cpp"
#include "sweep_yz.cpp"
#include "reduce.cpp"
#include "solve_host.h"
using namespace gpssc_host;

static std::vector<int> g_starts;   // class boundaries of the current launch (block0 values)
static bool g_all = false;          // run every block

// run the blocks with a pool of bx*by persistent threads (one per GPU
// thread of a block), the blocks one after another, each with its own LDS
static void launch(int nblocks, int bx, int by, size_t lds, const std::function<void()> &body)
{
    std::vector<int> pick;
    std::vector<int> st = g_starts; st.push_back(nblocks);
    if (g_starts.empty()) st = {0, nblocks};
    for (size_t k = 0; k + 1 < st.size(); ++k)
        for (int b : {st[k], st[k] + 1, st[k + 1] - 2, st[k + 1] - 1})
            if (b >= st[k] && b < st[k + 1]) pick.push_back(b);
    for (int b = 0; b < nblocks; b += (g_all ? 1 : 97)) pick.push_back(b);
    std::sort(pick.begin(), pick.end());
    pick.erase(std::unique(pick.begin(), pick.end()), pick.end());
    const int nt = bx * by;
    std::barrier<> bar(nt);
    std::vector<unsigned char> xch(16 * 64 * ((nt + 63) / 64) + 16);
    std::vector<unsigned char *> ldsbufs(pick.size(), nullptr);
    for (size_t q = 0; q < pick.size(); ++q)
        if (lds) { ldsbufs[q] = (unsigned char *)std::malloc(lds); std::memset(ldsbufs[q], 0xCD, lds); }
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            for (size_t q = 0; q < pick.size(); ++q) {
                threadIdx = dim3(t % bx, t / bx);
                blockIdx = dim3(pick[q]);
                blockDim = dim3(bx, by);
                gridDim = dim3(nblocks);
                g_blk = BlockCtx{&bar, xch.data() + 16 * 64 * (t / 64)};
                g_lds = ldsbufs[q];
                body();
                bar.arrive_and_wait();   // the block is done before the next one starts
            }
        });
    for (auto &x : th) x.join();
    for (auto *p : ldsbufs) std::free(p);
}

int main(int argc, char **argv)
{
    const gp_dtype dtype = GP_C64;
    using S = float2; using A = float;
    const bool real = argc > 1 && argv[1][0] == 'r';
    const bool skip_x = getenv("SKIPX") != nullptr;
    const bool skip_yz = getenv("SKIPYZ") != nullptr;
    g_all = getenv("ALL") != nullptr;
    std::vector<std::array<int64_t, 3>> shapes = {{24, 20, 16}, {96, 40, 300}, {130, 66, 48}, {300, 24, 20}, {48, 130, 96}, {24, 20, 16}};
    std::vector<int> mask = {1, 1, 1, 1, 1, 1};
    if (argc > 2) mask = {1, 0, 1, 1, 0, 1};
    const int n = (int)shapes.size();
    std::mt19937 rng(5);
    std::uniform_real_distribution<double> U(0.5, 3.0);
    struct Sol : SolveDesc { int cls; int64_t part_off; size_t tab_off; };
    std::vector<Sol> s(n);
    std::vector<ClassShape> cls;
    std::vector<std::vector<int>> members;
    std::map<std::tuple<int64_t, int64_t, int64_t>, int> index;
    int64_t part = 0; size_t tabb = 0;
    for (int i = 0; i < n; ++i) {
        Sol &x = s[i];
        for (int a = 0; a < 3; ++a) { x.grid[a] = shapes[i][a]; x.dx[a] = 0.25; x.omega[a] = U(rng); }
        x.dt = 0.01; x.g = 37.0 + i; x.real = real;
        auto key = std::make_tuple(x.grid[0], x.grid[1], x.grid[2]);
        auto it = index.find(key);
        if (it == index.end()) { it = index.emplace(key, (int)cls.size()).first; cls.push_back(class_shape(x.grid, dtype)); members.emplace_back(); }
        x.cls = it->second; members[x.cls].push_back(i);
        build_solve(x, cls[x.cls]);
        x.tab_off = tabb; tabb += table_bytes(cls[x.cls], dtype);
        x.part_off = part; part += x.grid[0] * x.grid[1];
    }
    std::vector<unsigned char> tab(tabb);
    for (auto &x : s) pack_solve_tables(x, cls[x.cls], dtype, tab.data() + x.tab_off);
    std::vector<gpssc::XBatchArgs<A>> xa(n); std::vector<gpssc::SBatchArgs<A>> ya(n), za(n);
    for (int i = 0; i < n; ++i) fill_solve_args<A>(s[i], cls[s[i].cls], tab.data() + s[i].tab_off, xa[i], ya[i], za[i]);
    std::vector<std::vector<S>> psi0(n);
    std::normal_distribution<float> N(0.f, 1.f);
    for (int i = 0; i < n; ++i) { psi0[i].resize(s[i].elems); for (auto &v : psi0[i]) v = S{N(rng), real ? N(rng) : 0.f}; }
    std::vector<int64_t> part_off(n); std::vector<double> dv(n), scales(n, 1.0); std::vector<int> flags(n, 0);
    for (int i = 0; i < n; ++i) { part_off[i] = s[i].part_off; dv[i] = 0.25 * 0.25 * 0.25; }
    std::vector<std::vector<int>> act(cls.size());
    for (size_t k = 0; k < cls.size(); ++k) for (int m : members[k]) if (mask[m]) act[k].push_back(m);

    // ---- per-class launches ----
    auto run_per_class = [&](std::vector<std::vector<S>> &psi, std::vector<double> &partials) {
        std::vector<S *> ptr(n); for (int i = 0; i < n; ++i) ptr[i] = psi[i].data();
        for (size_t k = 0; k < cls.size(); ++k) {
            const ClassShape &c = cls[k]; const int nact = (int)act[k].size(); if (!nact) continue;
            const int *ac = act[k].data();
            const int total = nact * c.nlines; const int L = gpssc::x_lines_per_wave(c.chunk[0], total);
            const int xb = (total + L - 1) / L;
#define XCASE(CC, LL) if (c.chunk[0] == CC && L == LL) launch(xb, 64, 1, 0, [&] { if (real) gpssc::calcnu_lux_batch_kernel<S, A, CC, LL, true>(ptr.data(), xa.data(), ac, c.nlines, total, nullptr); else gpssc::calcnu_lux_batch_kernel<S, A, CC, LL, false>(ptr.data(), xa.data(), ac, c.nlines, total, scales.data()); });
            if (!skip_x) { XCASE(1, 1) XCASE(1, 2) XCASE(1, 4) XCASE(2, 1) XCASE(2, 2) XCASE(2, 4) XCASE(3, 1) XCASE(3, 2) XCASE(5, 1) }
            for (int ax = 1; ax < 3 && !skip_yz; ++ax) {
                const int xt = ax == 1 ? c.xt_y : c.xt_z, cols = ax == 1 ? c.cols_y : c.cols_z;
                const int ncol = ax == 1 ? c.ncol_y : c.ncol_z, nt = ax == 1 ? c.ntiles_y : c.ntiles_z;
                const int la = c.lanes[ax], ch = c.chunk[ax];
                const size_t lds = 2 * (size_t)xt * la * (cols == 2 ? 16 : 8);
                double *pp = (ax == 2 && !real) ? partials.data() : nullptr;
                auto *ar = ax == 1 ? ya.data() : za.data();
#define YCASE(CC, WW) if (ch == CC && cols == WW) launch(nact * nt, xt, la, lds, [&] { if (real) gpssc::calclu_strided_batch_kernel<S, A, CC, true, false, WW>(ptr.data(), ar, ac, ncol, nt, nullptr, part_off.data()); else if (pp) gpssc::calclu_strided_batch_kernel<S, A, CC, false, true, WW>(ptr.data(), ar, ac, ncol, nt, pp, part_off.data()); else gpssc::calclu_strided_batch_kernel<S, A, CC, false, false, WW>(ptr.data(), ar, ac, ncol, nt, nullptr, part_off.data()); });
                YCASE(1, 1) YCASE(2, 1) YCASE(4, 1) YCASE(8, 1) YCASE(16, 1) YCASE(1, 2) YCASE(2, 2) YCASE(4, 2) YCASE(8, 2) YCASE(16, 2)
            }
        }
        std::printf("per-class step done\n"); std::fflush(stdout);
    };
    // ---- one launch ----
    auto run_one = [&](std::vector<std::vector<S>> &psi, std::vector<double> &partials) {
        std::vector<S *> ptr(n); for (int i = 0; i < n; ++i) ptr[i] = psi[i].data();
        std::vector<gpssc::XClassDesc> hx; std::vector<gpssc::YZClassDesc> hy, hz;
        int xblocks = 0, yblocks = 0, zblocks = 0, cmax_x = 1, cmax_y = 1, cmax_z = 1, lds_x = 0, thr_y = 0, thr_z = 0;
        size_t lds_y = 0, lds_z = 0;
        for (size_t k = 0; k < cls.size(); ++k) {
            const ClassShape &c = cls[k]; const int nact = (int)act[k].size(); if (!nact) continue;
            const int total = nact * c.nlines; const int L = gpssc::x_lines_per_wave(c.chunk[0], total);
            hx.push_back({xblocks, c.nlines, total, c.chunk[0], L, act[k].data()}); xblocks += (total + L - 1) / L;
            cmax_x = std::max(cmax_x, c.chunk[0]); lds_x = std::max(lds_x, L * (64 * c.chunk[0] + 64));
            hy.push_back({yblocks, c.ntiles_y, c.ncol_y, c.xt_y, c.lanes[1], c.chunk[1], c.cols_y, act[k].data()}); yblocks += nact * c.ntiles_y;
            cmax_y = std::max(cmax_y, c.chunk[1]); thr_y = std::max(thr_y, c.xt_y * c.lanes[1]); lds_y = std::max(lds_y, 2 * (size_t)c.xt_y * c.lanes[1] * (c.cols_y == 2 ? 16 : 8));
            hz.push_back({zblocks, c.ntiles_z, c.ncol_z, c.xt_z, c.lanes[2], c.chunk[2], c.cols_z, act[k].data()}); zblocks += nact * c.ntiles_z;
            cmax_z = std::max(cmax_z, c.chunk[2]); thr_z = std::max(thr_z, c.xt_z * c.lanes[2]); lds_z = std::max(lds_z, 2 * (size_t)c.xt_z * c.lanes[2] * (c.cols_z == 2 ? 16 : 8));
        }
        const int ncls = (int)hx.size();
        std::printf("one launch: x %d blocks (cmax %d, lds %d), y %d blocks of %d (cmax %d, lds %zu), z %d of %d (cmax %d, lds %zu)\n", xblocks, cmax_x, lds_x, yblocks, thr_y, cmax_y, lds_y, zblocks, thr_z, cmax_z, lds_z);
        std::fflush(stdout);
        g_starts.clear(); for (auto &d : hx) g_starts.push_back(d.block0);
        if (!skip_x) launch(xblocks, 64, 1, (size_t)lds_x * sizeof(S), [&] { if (real) gpssc::calcnu_lux_classes_kernel<S, A, 8, true>(ptr.data(), xa.data(), hx.data(), ncls, nullptr); else gpssc::calcnu_lux_classes_kernel<S, A, 8, false>(ptr.data(), xa.data(), hx.data(), ncls, scales.data()); });
        std::printf("  x done\n"); std::fflush(stdout);
        g_starts.clear(); for (auto &d : hy) g_starts.push_back(d.block0);
        if (!skip_yz) launch(yblocks, thr_y, 1, lds_y, [&] { if (real) gpssc::calclu_strided_classes_kernel<S, A, 16, true, false>(ptr.data(), ya.data(), hy.data(), ncls, nullptr, nullptr); else gpssc::calclu_strided_classes_kernel<S, A, 16, false, false>(ptr.data(), ya.data(), hy.data(), ncls, nullptr, nullptr); });
        std::printf("  y done\n"); std::fflush(stdout);
        g_starts.clear(); for (auto &d : hz) g_starts.push_back(d.block0);
        if (!skip_yz) launch(zblocks, thr_z, 1, lds_z, [&] { if (real) gpssc::calclu_strided_classes_kernel<S, A, 16, true, false>(ptr.data(), za.data(), hz.data(), ncls, nullptr, nullptr); else gpssc::calclu_strided_classes_kernel<S, A, 16, false, true>(ptr.data(), za.data(), hz.data(), ncls, partials.data(), part_off.data()); });
        std::printf("  z done\n"); std::fflush(stdout);
    };
    auto p1 = psi0, p2 = psi0;
    std::vector<double> q1(part, 0.0), q2(part, 0.0);
    g_starts.clear();
    run_per_class(p1, q1);
    run_one(p2, q2);
    long diff = 0;
    for (int i = 0; i < n; ++i) diff += std::memcmp(p1[i].data(), p2[i].data(), sizeof(S) * p1[i].size()) != 0;
    std::printf("solves differing: %ld, partials equal: %d\n", diff, (int)(q1 == q2));
    return 0;
}
