// The batch's host code (batch.hip) against the host-runtime stand-in, its
// kernels stubbed (kernel_stubs.h): batches of uneven solves in every storage
// type and mode, with graph replay on and off, the y/z shape tuner, the FP64
// finish of FP32 batches, active masks, rebinding psi (including an 8-byte
// aligned complex64 view, which gives up the column pairs) and the stopping
// rule of gp_batch_solve_imag.  Built with -fsanitize=address by run.py
// --batch.
#include "hip/hip_runtime.h"
thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;
thread_local BlockCtx g_blk;
thread_local unsigned char *g_lds;
#include <string>
namespace gpssc_host { thread_local std::string g_last_error; }
#include "batch.hip"
#include "kernel_stubs.h"

struct Case {
    gp_dtype dtype;
    gp_mode mode;
    int flags;
    bool offset_psi;   // bind psi 8 bytes past an allocation (complex64: no column pairs)
};

static int run_case(const Case &k)
{
    for (auto &c : gpssc::g_obs_calls) c = 0;   // every case runs its stopping rule from the start
    const int64_t shapes[][3] = {{16, 20, 24}, {9, 17, 33}, {24, 32, 40}, {16, 20, 24}, {64, 8, 130}, {9, 17, 33}};
    const int n = 6;
    std::vector<int64_t> grids;
    std::vector<double> dx, dt, traps, g;
    for (int i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            grids.push_back(shapes[i][a]);
            dx.push_back(0.3);
            traps.push_back(1.0 + 0.5 * a + 0.1 * i);
        }
        dt.push_back(0.01);
        g.push_back(10.0 + i);
    }
    gp_batch *b = nullptr;
    if (gp_batch_create(n, grids.data(), dx.data(), dt.data(), traps.data(), g.data(), k.mode, k.dtype, k.flags,
                        nullptr, &b) != GP_OK) {
        std::printf("create failed: %s\n", gpssc_host::g_last_error.c_str());
        return 1;
    }
    const size_t eb = storage_bytes(k.dtype);
    std::vector<void *> mem(n), psi(n);
    std::vector<int64_t> elems(n);
    for (int i = 0; i < n; ++i) {
        elems[i] = shapes[i][0] * shapes[i][1] * shapes[i][2];
        (void)hipMalloc(&mem[i], (size_t)elems[i] * eb + 16);
        psi[i] = static_cast<unsigned char *>(mem[i]) + (k.offset_psi ? 8 : 0);
    }
    int bad = 0;
    auto ok = [&](gp_status s, const char *what) {
        if (s != GP_OK && s != GP_ERR_NONFINITE) {
            std::printf("%s: status %d, %s\n", what, (int)s, gpssc_host::g_last_error.c_str());
            ++bad;
        }
    };
    ok(gp_batch_set_psi(b, psi.data(), elems.data()), "set_psi");
    std::vector<gp_obs> out(n);
    ok(gp_batch_step(b, 5), "step");
    ok(gp_batch_observables(b, out.data()), "observables");
    const unsigned char mask[n] = {1, 0, 1, 1, 0, 1};
    ok(gp_batch_set_active(b, mask), "set_active");
    ok(gp_batch_step(b, 3), "step (masked)");
    ok(gp_batch_observables(b, out.data()), "observables (masked)");
    ok(gp_batch_set_active(b, nullptr), "set_active (all)");
    ok(gp_batch_set_psi(b, psi.data(), elems.data()), "set_psi (again)");
    if (k.mode == GP_MODE_IMAG) {
        std::vector<int64_t> steps(n);
        std::vector<unsigned char> conv(n);
        ok(gp_batch_solve_imag(b, 1e-3, 10, 400, out.data(), steps.data(), conv.data()), "solve_imag");
    } else {
        ok(gp_batch_step(b, 11), "step (real)");
    }
    char buf[4096];
    ok(gp_batch_describe(b, buf, sizeof buf), "describe");
    ok(gp_batch_destroy(b), "destroy");
    for (void *p : mem) (void)hipFree(p);
    return bad;
}

int main(int argc, char **argv)
{
    const int iters = argc > 1 ? std::atoi(argv[1]) : 3;
    const int G = GP_BATCH_GRAPH, T = GP_BATCH_TUNE, F = GP_BATCH_FINISH_F64;
    const Case cases[] = {
        {GP_C64, GP_MODE_IMAG, G | T, false},  {GP_C64, GP_MODE_IMAG, G, true},      {GP_C64, GP_MODE_REAL, G, false},
        {GP_C128, GP_MODE_IMAG, G | T, false}, {GP_C128, GP_MODE_REAL, 0, false},     {GP_R32, GP_MODE_IMAG, G | F, false},
        {GP_C64, GP_MODE_IMAG, G | T | F, false}, {GP_R64, GP_MODE_IMAG, 0, false},   {GP_C64_F64, GP_MODE_IMAG, G, false},
    };
    int bad = 0;
    for (int it = 0; it < iters; ++it)
        for (const Case &k : cases) bad += run_case(k);
    std::printf("iterations %d, cases failing %d\n", iters, bad);
    return bad ? 1 : 0;
}
