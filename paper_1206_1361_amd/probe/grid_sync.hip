// grid_sync.hip -- the cost of a device-wide barrier: a cooperative launch of
// G blocks of 256 threads that pass ITERS grid barriers (cooperative groups)
// and do nothing else.  Prints the time per launch (HIP events, mean of 5
// after one warm-up launch) for 1 and 1001 barriers; the difference over 1000
// is the cost of one barrier at that grid size.
//
// Built by paper_1206_1361_amd/build.py as paper_1206_1361_amd/probe/grid_sync;
// a measurement tool, not part of the library.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <cstdio>

namespace cg = cooperative_groups;

__global__ void __launch_bounds__(256) barrier_loop(int iters, int *out)
{
    cg::grid_group grid = cg::this_grid();
    int acc = 0;
    for (int i = 0; i < iters; ++i) {
        acc += (int)blockIdx.x;
        grid.sync();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

int main()
{
    int dev = 0, coop = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    (void)hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, barrier_loop, 256, 0);
    std::printf("cooperative launch %d, %d CUs, %d resident blocks of 256 threads per CU\n", coop, ncu, per_cu);
    if (!coop) return 1;
    int *out = nullptr;
    if (hipMalloc(&out, sizeof(int) * 4096) != hipSuccess) return 1;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return 1;
    for (int G : {8, 32, 64, 128, 256}) {
        if (G > per_cu * ncu) continue;   // every block must be resident
        float us[2] = {0, 0};
        int k = 0;
        for (int iters : {1, 1001}) {
            void *args[] = {&iters, &out};
            hipError_t e = hipLaunchCooperativeKernel((const void *)barrier_loop, dim3(G), dim3(256), args, 0, nullptr);
            if (e == hipSuccess) e = hipDeviceSynchronize();
            if (e != hipSuccess) {
                std::printf("launch failed: %s\n", hipGetErrorString(e));
                return 1;
            }
            (void)hipEventRecord(a, nullptr);
            for (int r = 0; r < 5; ++r)
                (void)hipLaunchCooperativeKernel((const void *)barrier_loop, dim3(G), dim3(256), args, 0, nullptr);
            (void)hipEventRecord(b, nullptr);
            (void)hipEventSynchronize(b);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, a, b);
            us[k++] = ms * 1000.0f / 5.0f;
        }
        std::printf("%4d blocks: launch with 1 barrier %8.2f us, with 1001 %9.2f us; one barrier %.2f us\n", G, us[0],
                    us[1], (us[1] - us[0]) / 1000.0f);
        std::fflush(stdout);
    }
    hipError_t e = hipGetLastError();
    (void)hipFree(out);
    return e == hipSuccess ? 0 : 1;
}
