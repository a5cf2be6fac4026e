// The server's host code (server.hip) against the host-runtime stand-in, its
// kernels stubbed with the reads and writes of their index arrays, driven by
// the request patterns of the server tests from the main thread while the
// engine thread runs rounds.  Built with -fsanitize=address or =thread.
#include "hip/hip_runtime.h"
thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;
thread_local BlockCtx g_blk;
thread_local unsigned char *g_lds;
#include <chrono>
#include <random>
#include <thread>
#include <string>
namespace gpssc_host { thread_local std::string g_last_error; }
#include "server.hip"

#include "kernel_stubs.h"

struct Req { int64_t grid[3]; gp_mode mode; bool real_state; int steps; double tol; };

static int scenario(gp_dtype sdt, uint64_t budget, int slots, int flags, const std::vector<Req> &rs, std::mt19937 &rng)
{
    gp_server *S = nullptr;
    if (gp_server_create(sdt, budget, slots, 10, flags, &S) != GP_OK) { std::printf("create failed: %s\n", gpssc_host::g_last_error.c_str()); return 1; }
    std::vector<std::vector<unsigned char>> in(rs.size()), out(rs.size());
    std::uniform_int_distribution<int> us(0, 300);
    int submitted = 0;
    for (size_t i = 0; i < rs.size(); ++i) {
        const Req &q = rs[i];
        const int64_t n = q.grid[0] * q.grid[1] * q.grid[2];
        const size_t eb = q.real_state ? (sdt == GP_C64 ? 4 : 8) : storage_bytes(sdt);
        in[i].assign(n * eb, 0);
        out[i].assign(n * eb, 0);
        for (size_t k = 0; k < n * eb; k += eb) in[i][k] = 1;   // nonzero real parts
        gp_request r{};
        for (int a = 0; a < 3; ++a) { r.grid[a] = q.grid[a]; r.dx[a] = 0.3; r.trap[a] = 1.0 + a; }
        r.dt = 0.01; r.g = 10.0; r.mode = q.mode; r.steps = q.steps; r.tol = q.tol; r.psi_in = in[i].data();
        r.psi_out = out[i].data(); r.tag = (int64_t)i; r.real_state = q.real_state ? 1 : 0;
        uint64_t id = 0;
        if (gp_server_submit(S, &r, &id) == GP_OK) ++submitted;
        std::this_thread::sleep_for(std::chrono::microseconds(us(rng)));
    }
    int got = 0;
    gp_result res[64];
    for (int it = 0; got < submitted && it < 20000; ++it) {
        int n = 0;
        gp_server_poll(S, res, 64, 0.001, &n);
        got += n;
    }
    gp_server_destroy(S);
    return got == submitted ? 0 : 2;
}

int main(int argc, char **argv)
{
    const int iters = argc > 1 ? std::atoi(argv[1]) : 20;
    std::mt19937 rng(7);
    const int64_t s0[3] = {16, 20, 24}, s1[3] = {9, 17, 33}, s2[3] = {24, 32, 40};
    auto R = [](const int64_t *g, gp_mode m, bool rs, int steps, double tol) { return Req{{g[0], g[1], g[2]}, m, rs, steps, tol}; };
    int bad = 0;
    for (int it = 0; it < iters; ++it) {
        // real states beside complex ones (complex64 and complex128 servers)
        std::vector<Req> mix = {R(s0, GP_MODE_IMAG, true, 400, 1e-7), R(s1, GP_MODE_IMAG, false, 400, 1e-7),
                                R(s2, GP_MODE_REAL, false, 45, 0.0), R(s0, GP_MODE_IMAG, false, 400, 1e-7),
                                R(s1, GP_MODE_IMAG, true, 400, 1e-7), R(s2, GP_MODE_REAL, false, 45, 0.0)};
        bad += scenario(GP_C64, 256u << 20, 16, GP_SERVER_GRAPH, mix, rng);
        bad += scenario(GP_C128, 256u << 20, 16, GP_SERVER_GRAPH, mix, rng);
        // a float64-storage server
        std::vector<Req> r64 = {R(s0, GP_MODE_IMAG, false, 300, 1e-9), R(s1, GP_MODE_IMAG, false, 300, 1e-9),
                                R(s0, GP_MODE_IMAG, false, 300, 1e-9)};
        bad += scenario(GP_R64, 64u << 20, 8, GP_SERVER_GRAPH, r64, rng);
        // automatic real storage, graph off, a slot limit
        std::vector<Req> all;
        for (int k = 0; k < 12; ++k) all.push_back(R(k % 2 ? s0 : s1, k % 3 == 2 ? GP_MODE_REAL : GP_MODE_IMAG, false, 30 + k, 1e-7));
        bad += scenario(GP_C64, 64u << 20, 4, GP_SERVER_GRAPH | GP_SERVER_REAL_AUTO, all, rng);
        bad += scenario(GP_C64, 64u << 20, 3, 0, all, rng);
    }
    std::printf("iterations %d, scenarios failing %d\n", iters, bad);
    return bad ? 1 : 0;
}
