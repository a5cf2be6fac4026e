// Stubs of the library's kernel launchers for the host-code harnesses: each
// reads and writes the index arrays, pointer tables and per-solve scalars its
// kernels would, and the observables stub writes sums whose chemical
// potential settles over successive calls, so the stopping rules run.
#pragma once
#include <atomic>
namespace gpssc {
inline std::atomic<long> g_obs_calls[4096];
int obs_num_blocks(int nx, int ny) { return ((nx + 63) / 64) * ((ny + 3) / 4); }
hipError_t launch_nu_x_batch(Prec, bool, int, int nact, int, void *const *psis, const void *, const int *active,
                             const double *scales, hipStream_t, int)
{
    mock_do([=] { for (int a = 0; a < nact; ++a) { volatile void *p = psis[active[a]]; (void)p; if (scales) (void)scales[active[a]]; } });
    return hipSuccess;
}
hipError_t launch_strided_batch(Prec, bool, int, int, int, int, int nact, int, int, void *const *psis, const void *,
                                const int *active, double *partials, const int64_t *part_off, hipStream_t)
{
    mock_do([=] { for (int a = 0; a < nact; ++a) { volatile void *p = psis[active[a]]; (void)p; if (partials) partials[part_off[active[a]]] = 1.0; } });
    return hipSuccess;
}
hipError_t launch_norm_finalize_batch(int nact, const int *active, const double *partials, const int64_t *part_off,
                                      int npart, const double *dv, double *scales, int *flags, hipStream_t)
{
    mock_do([=] {
        for (int a = 0; a < nact; ++a) {
            const int si = active[a];
            double s = 0; for (int q = 0; q < npart; ++q) s += partials[part_off[si] + q];
            (void)s; (void)dv[si]; scales[si] = 1.0; flags[si] = 0;
        }
    });
    return hipSuccess;
}
hipError_t launch_scale_batch(Prec, int nact, const int *active, void *const *psis, int64_t, double *scales, hipStream_t)
{
    mock_do([=] { for (int a = 0; a < nact; ++a) { volatile void *p = psis[active[a]]; (void)p; scales[active[a]] = 1.0; } });
    return hipSuccess;
}
hipError_t launch_observables_batch(Prec, int nact, const int *active, void *const *psis, const ObsArgs<double> *args,
                                    int nx, int ny, double *partials, const int64_t *obs_off, double *sums, hipStream_t)
{
    mock_do([=] {
        const int nb = obs_num_blocks(nx, ny);
        for (int a = 0; a < nact; ++a) {
            const int si = active[a];
            volatile void *p = psis[si]; (void)p;
            for (int q = 0; q < nb * OBS_NSUMS; ++q) partials[obs_off[si] + q] = 0.5;
            const ObsArgs<double> &o = args[si];
            const double dv = o.dx * o.dy * o.dz;
            for (int q = 0; q < OBS_NSUMS; ++q) sums[(int64_t)si * OBS_NSUMS + q] = 1.0;
            sums[(int64_t)si * OBS_NSUMS + OBS_POT] = 1.0 + 1.0 / (double)(1 + g_obs_calls[si % 4096]++);
            sums[(int64_t)si * OBS_NSUMS + OBS_DENS] = 1.0 / dv;
            sums[(int64_t)si * OBS_NSUMS + OBS_M1X] = 0.0;
            sums[(int64_t)si * OBS_NSUMS + OBS_M1Y] = 0.0;
            sums[(int64_t)si * OBS_NSUMS + OBS_M1Z] = 0.0;
        }
    });
    return hipSuccess;
}
hipError_t launch_convert(Prec to, Prec from, void *dst, const void *src, int64_t elems, hipStream_t)
{
    const size_t bt = storage_bytes(to), bf = storage_bytes(from);
    mock_do([=] { std::memset(dst, 0, bt * elems); volatile unsigned char x = 0; for (size_t i = 0; i < bf * elems; ++i) x ^= ((const unsigned char *)src)[i]; });
    return hipSuccess;
}
hipError_t launch_nu_x_classes(Prec, bool, int, int, int, void *const *, const void *, const XClassDesc *, int,
                               const double *, hipStream_t) { return hipSuccess; }
hipError_t launch_strided_classes(Prec, bool, int, int, size_t, int, void *const *, const void *, const YZClassDesc *,
                                  int, double *, const int64_t *, hipStream_t) { return hipSuccess; }
hipError_t launch_norm_finalize_classes(int, const NormClassDesc *, int, const double *, const int64_t *,
                                        const double *, double *, int *, hipStream_t) { return hipSuccess; }
}  // namespace gpssc
