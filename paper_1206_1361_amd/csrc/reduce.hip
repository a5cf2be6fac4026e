// reduce.hip -- calcnorm finalisation, the end-of-call scaling, and the
// calcmuen / calcrms sums.
//
// Paper: "Summary of revisions" names calcnorm (normalisation) and calcmuen,
// calcrms (chemical potential, energy and rms sizes) among the routines that
// carry a time step and its diagnostics.  Every sum here is FP64 and formed
// in a fixed order (per thread, then a fixed LDS tree per block, then a
// fixed-order sum over the blocks), so results are bitwise reproducible.
#include "gp_internal.h"

namespace gpssc {

constexpr int kReduceThreads = 256;

// Fixed-order sum of v over a block of kReduceThreads threads; the result is
// valid in thread 0.
__device__ double block_sum(double v, double *red)
{
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int h = kReduceThreads / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Thread t's share of a norm sum: p[b] (times w[b], the product rounded on
// its own) added for b = t, t + kReduceThreads, ... in that order.  The loads
// of kSumAhead terms are issued before they are added, so the thread does
// not wait on each load in turn; the order of the additions is unchanged.
constexpr int kSumAhead = 8;

__device__ __forceinline__ double strided_sum(const double *__restrict__ p, const double *__restrict__ w, int n,
                                              int t)
{
#pragma clang fp contract(off)
    double acc = 0.0;
    for (int b0 = t; b0 < n; b0 += kSumAhead * kReduceThreads) {
        double v[kSumAhead];
#pragma unroll
        for (int u = 0; u < kSumAhead; ++u) {
            const int b = b0 + u * kReduceThreads;
            v[u] = b < n ? (w ? w[b] * p[b] : p[b]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kSumAhead; ++u)
            if (b0 + u * kReduceThreads < n) acc += v[u];
    }
    return acc;
}

__global__ void __launch_bounds__(kReduceThreads)
calcnorm_finalize_kernel(const double *__restrict__ partials, int n, double dv,
                         double *__restrict__ scale, int *__restrict__ flag,
                         const double *__restrict__ weights)
{
    __shared__ double red[kReduceThreads];
    const double acc = strided_sum(partials, weights, n, threadIdx.x);
    const double sum = block_sum(acc, red);
    if (threadIdx.x == 0) {
        const double norm = dv * sum;
        const bool ok = norm > 0.0 && isfinite(norm);
        *scale = ok ? 1.0 / sqrt(norm) : (double)NAN;
        if (!ok) flag[0] = 1;
    }
}

// Solve si's 1/sqrt(N) from its ntiles partials (one block).
__device__ __forceinline__ void finalize_solve(int si, const double *__restrict__ partials,
                                               const int64_t *__restrict__ part_off, int ntiles,
                                               const double *__restrict__ dv, double *__restrict__ scales,
                                               int *__restrict__ flags, double *red)
{
    const double acc = strided_sum(partials + part_off[si], nullptr, ntiles, threadIdx.x);
    const double sum = block_sum(acc, red);
    if (threadIdx.x == 0) {
        const double norm = dv[si] * sum;
        const bool ok = norm > 0.0 && isfinite(norm);
        scales[si] = ok ? 1.0 / sqrt(norm) : (double)NAN;
        if (!ok) flags[si] = 1;
    }
}

// Batched: block b finalises solve active[b].
__global__ void __launch_bounds__(kReduceThreads)
calcnorm_finalize_batch_kernel(const int *__restrict__ active, const double *__restrict__ partials,
                               const int64_t *__restrict__ part_off, int ntiles,
                               const double *__restrict__ dv, double *__restrict__ scales,
                               int *__restrict__ flags)
{
    __shared__ double red[kReduceThreads];
    finalize_solve(active[blockIdx.x], partials, part_off, ntiles, dv, scales, flags, red);
}

// Every class in one launch: class k's blocks from cls[k].block0 on, one
// per active solve of the class.
__global__ void __launch_bounds__(kReduceThreads)
calcnorm_finalize_classes_kernel(const NormClassDesc *__restrict__ cls, int ncls,
                                 const double *__restrict__ partials, const int64_t *__restrict__ part_off,
                                 const double *__restrict__ dv, double *__restrict__ scales,
                                 int *__restrict__ flags)
{
    __shared__ double red[kReduceThreads];
    const int b = blockIdx.x;
    const NormClassDesc c = cls[class_of_block(cls, ncls, b)];
    finalize_solve(c.active[b - c.block0], partials, part_off, c.npart, dv, scales, flags, red);
}

// Batched: blockIdx.y picks the solve; afterwards its scale is reset to 1 by
// reset_scales_kernel (a separate launch, once every block has read it).
template <typename S>
__global__ void __launch_bounds__(kReduceThreads)
scale_batch_kernel(S *const *__restrict__ psis, const int *__restrict__ active, int64_t elems,
                   const double *__restrict__ scales)
{
    using R = typename storage_traits<S>::real;
    const int si = active[blockIdx.y];
    const R s = (R)scales[si];
    S *psi = psis[si];
    const int64_t stride = (int64_t)gridDim.x * kReduceThreads;
    for (int64_t p = (int64_t)blockIdx.x * kReduceThreads + threadIdx.x; p < elems; p += stride) {
        psi[p] = sscale(psi[p], s);
    }
}

__global__ void __launch_bounds__(kReduceThreads)
reset_scales_kernel(const int *__restrict__ active, int nact, double *__restrict__ scales)
{
    for (int b = threadIdx.x; b < nact; b += kReduceThreads) scales[active[b]] = 1.0;
}

template <typename S>
__global__ void __launch_bounds__(kReduceThreads)
scale_kernel(S *__restrict__ psi, int64_t elems, const double *__restrict__ scale)
{
    using R = typename storage_traits<S>::real;
    const R s = (R)(*scale);
    const int64_t stride = (int64_t)gridDim.x * kReduceThreads;
    for (int64_t p = (int64_t)blockIdx.x * kReduceThreads + threadIdx.x; p < elems; p += stride) {
        psi[p] = sscale(psi[p], s);
    }
}

// Observables: block (64, 4) covers 64 x 4 columns (i, j) and walks z.  Each
// point adds |psi|^2, V|psi|^2, |psi|^4, x|psi|^2 ..., z^2|psi|^2 and the
// squared difference to the next node along each axis (zero beyond the
// last node); the link to the zero before the first node is added at the
// first node.
constexpr int kObsX = 64, kObsY = 4;
// z planes loaded ahead per step of the walk: 2 for 16-byte elements, 4 for
// smaller ones (measured on 512x512x384: complex128 359 / 363 / 440 us at
// 1 / 2 / 4 planes, complex64 549 / 400 / 370 us).
template <typename S>
constexpr int obs_planes() { return sizeof(S) >= 16 ? 2 : 4; }

template <typename S>
__device__ __forceinline__ void obs_block(const S *__restrict__ psi, const ObsArgs<double> &a,
                                          double *__restrict__ out, double *red, int bx, int by)
{
    const int tx = threadIdx.x % kObsX, ty = threadIdx.x / kObsX;
    const int i = bx * kObsX + tx;
    const int j = by * kObsY + ty;
    double acc[OBS_NSUMS];
#pragma unroll
    for (int q = 0; q < OBS_NSUMS; ++q) acc[q] = 0.0;

    if (i < a.nx && j < a.ny) {
        // every product and sum rounded on its own (no fused multiply-add),
        // so the sums do not depend on whether the storage is complex or real
#pragma clang fp contract(off)
        const int64_t plane = (int64_t)a.nx * a.ny;
        const double x = ((double)i - a.c0x) * a.dx;
        const double y = ((double)j - a.c0y) * a.dy;
        const double vxy = a.hgx * x * x + a.hgy * y * y;
        double prev_re = 0.0, prev_im = 0.0;  // node k-1 (zero before the first)
        const S *col = psi + (int64_t)j * a.nx + i;
        // kObsZ planes at a time: their loads (the node and its x and y
        // partners; zero past the grid) are all issued before the sums, which
        // then run plane by plane in order, as one plane at a time would
        constexpr int kObsZ = obs_planes<S>();
        for (int k0 = 0; k0 < a.nz; k0 += kObsZ) {
            S v[kObsZ], vx[kObsZ], vy[kObsZ];
#pragma unroll
            for (int u = 0; u < kObsZ; ++u) {
                const int64_t at = (int64_t)(k0 + u) * plane;
                v[u] = szero<S>();
                vx[u] = szero<S>();
                vy[u] = szero<S>();
                if (k0 + u < a.nz) {
                    v[u] = col[at];
                    if (i + 1 < a.nx) vx[u] = col[at + 1];
                    if (j + 1 < a.ny) vy[u] = col[at + a.nx];
                }
            }
#pragma unroll
            for (int u = 0; u < kObsZ; ++u) {
                const int k = k0 + u;
                if (k >= a.nz) break;
                const double re = sre(v[u]), im = sim(v[u]);
                const double w = re * re + im * im;
                const double z = ((double)k - a.c0z) * a.dz;
                acc[OBS_DENS] += w;
                acc[OBS_POT] += (vxy + a.hgz * z * z) * w;
                acc[OBS_QUART] += w * w;
                acc[OBS_M1X] += x * w;
                acc[OBS_M1Y] += y * w;
                acc[OBS_M1Z] += z * w;
                acc[OBS_M2X] += x * x * w;
                acc[OBS_M2Y] += y * y * w;
                acc[OBS_M2Z] += z * z * w;
                // x link to i+1 (and the ghost link before i = 0)
                double nre = sre(vx[u]), nim = sim(vx[u]);
                acc[OBS_LINKX] += (nre - re) * (nre - re) + (nim - im) * (nim - im);
                if (i == 0) acc[OBS_LINKX] += w;
                // y link to j+1
                nre = sre(vy[u]);
                nim = sim(vy[u]);
                acc[OBS_LINKY] += (nre - re) * (nre - re) + (nim - im) * (nim - im);
                if (j == 0) acc[OBS_LINKY] += w;
                // z link from k-1 (the k = 0 term is the ghost link)
                acc[OBS_LINKZ] += (re - prev_re) * (re - prev_re) + (im - prev_im) * (im - prev_im);
                prev_re = re;
                prev_im = im;
            }
        }
        acc[OBS_LINKZ] += prev_re * prev_re + prev_im * prev_im;  // ghost beyond the last node
    }

#pragma unroll
    for (int q = 0; q < OBS_NSUMS; ++q) {
        const double s = block_sum(acc[q], red);
        if (threadIdx.x == 0) out[q] = s;
    }
}

template <typename S>
__global__ void __launch_bounds__(kObsX * kObsY)
calcmuen_rms_kernel(const S *__restrict__ psi, const ObsArgs<double> a,
                    double *__restrict__ partials)
{
    __shared__ double red[kReduceThreads];
    const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    obs_block(psi, a, partials + b * OBS_NSUMS, red, blockIdx.x, blockIdx.y);
}

// Batched: blockIdx.z picks the solve; its partials start at
// partials + solve * (gridDim.x * gridDim.y) * OBS_NSUMS.
template <typename S>
__global__ void __launch_bounds__(kObsX * kObsY)
calcmuen_rms_batch_kernel(S *const *__restrict__ psis, const int *__restrict__ active,
                          const ObsArgs<double> *__restrict__ args, double *__restrict__ partials,
                          const int64_t *__restrict__ obs_off)
{
    __shared__ double red[kReduceThreads];
    const int si = active[blockIdx.z];
    const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    obs_block<S>(psis[si], args[si], partials + obs_off[si] + b * OBS_NSUMS, red, blockIdx.x, blockIdx.y);
}

__global__ void __launch_bounds__(kReduceThreads)
obs_finalize_kernel(const double *__restrict__ partials, int nblocks, double *__restrict__ sums)
{
    __shared__ double red[kReduceThreads];
    for (int q = 0; q < OBS_NSUMS; ++q) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += kReduceThreads)
            acc += partials[(int64_t)b * OBS_NSUMS + q];
        const double s = block_sum(acc, red);
        if (threadIdx.x == 0) sums[q] = s;
    }
}

// Batched: block b sums solve active[b]'s partials into sums[si].
__global__ void __launch_bounds__(kReduceThreads)
obs_finalize_batch_kernel(const int *__restrict__ active, const double *__restrict__ partials,
                          const int64_t *__restrict__ obs_off, int nblocks, double *__restrict__ sums)
{
    __shared__ double red[kReduceThreads];
    const int si = active[blockIdx.x];
    const double *p = partials + obs_off[si];
    for (int q = 0; q < OBS_NSUMS; ++q) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += kReduceThreads) acc += p[(int64_t)b * OBS_NSUMS + q];
        const double s = block_sum(acc, red);
        if (threadIdx.x == 0) sums[(int64_t)si * OBS_NSUMS + q] = s;
    }
}

// Calls f with a value of the storage type of prec (the type selects the
// kernel instantiation).
template <typename F>
hipError_t with_storage(Prec prec, F f)
{
    switch (prec) {
    case PREC_C128: return f(double2{});
    case PREC_C64:
    case PREC_C64_F64: return f(float2{});
    case PREC_R64: return f(double{});
    case PREC_R32: return f(float{});
    }
    return hipErrorInvalidValue;
}

hipError_t launch_norm_finalize_batch(int nact, const int *active, const double *partials,
                                      const int64_t *part_off, int ntiles, const double *dv,
                                      double *scales, int *flags, hipStream_t stream)
{
    if (nact <= 0) return hipSuccess;
    hipLaunchKernelGGL(calcnorm_finalize_batch_kernel, dim3((unsigned)nact), dim3(kReduceThreads), 0,
                       stream, active, partials, part_off, ntiles, dv, scales, flags);
    return hipGetLastError();
}

hipError_t launch_norm_finalize_classes(int nblocks, const NormClassDesc *cls, int ncls, const double *partials,
                                        const int64_t *part_off, const double *dv, double *scales, int *flags,
                                        hipStream_t stream)
{
    if (nblocks <= 0 || ncls <= 0) return hipSuccess;
    hipLaunchKernelGGL(calcnorm_finalize_classes_kernel, dim3((unsigned)nblocks), dim3(kReduceThreads), 0, stream,
                       cls, ncls, partials, part_off, dv, scales, flags);
    return hipGetLastError();
}

hipError_t launch_scale_batch(Prec prec, int nact, const int *active, void *const *psis, int64_t elems,
                              double *scales, hipStream_t stream)
{
    if (nact <= 0) return hipSuccess;
    int64_t blocks = (elems + kReduceThreads - 1) / kReduceThreads;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    const dim3 grid((unsigned)blocks, (unsigned)nact);
    hipError_t e = with_storage(prec, [&](auto tag) {
        using S = decltype(tag);
        hipLaunchKernelGGL(scale_batch_kernel<S>, grid, dim3(kReduceThreads), 0, stream,
                           reinterpret_cast<S *const *>(psis), active, elems, scales);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reset_scales_kernel, dim3(1), dim3(kReduceThreads), 0, stream, active, nact, scales);
    return hipGetLastError();
}

hipError_t launch_observables_batch(Prec prec, int nact, const int *active, void *const *psis,
                                    const ObsArgs<double> *args, int nx, int ny, double *partials,
                                    const int64_t *obs_off, double *sums, hipStream_t stream)
{
    if (nact <= 0) return hipSuccess;
    const dim3 grid((unsigned)((nx + kObsX - 1) / kObsX), (unsigned)((ny + kObsY - 1) / kObsY),
                    (unsigned)nact);
    const dim3 block(kObsX * kObsY);
    hipError_t e = with_storage(prec, [&](auto tag) {
        using S = decltype(tag);
        hipLaunchKernelGGL(calcmuen_rms_batch_kernel<S>, grid, block, 0, stream,
                           reinterpret_cast<S *const *>(psis), active, args, partials, obs_off);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(obs_finalize_batch_kernel, dim3((unsigned)nact), dim3(kReduceThreads), 0, stream,
                       active, partials, obs_off, (int)(grid.x * grid.y), sums);
    return hipGetLastError();
}

hipError_t launch_norm_finalize(const double *partials, int n, double dv, double *scale,
                                int *flag, hipStream_t stream, const double *weights)
{
    hipLaunchKernelGGL(calcnorm_finalize_kernel, dim3(1), dim3(kReduceThreads), 0, stream,
                       partials, n, dv, scale, flag, weights);
    return hipGetLastError();
}

hipError_t launch_scale(Prec prec, void *psi, int64_t elems, const double *scale,
                        hipStream_t stream)
{
    int64_t blocks = (elems + kReduceThreads - 1) / kReduceThreads;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    return with_storage(prec, [&](auto tag) {
        using S = decltype(tag);
        hipLaunchKernelGGL(scale_kernel<S>, dim3((unsigned)blocks), dim3(kReduceThreads), 0, stream,
                           static_cast<S *>(psi), elems, scale);
        return hipGetLastError();
    });
}

// psi copied between storage types: float <-> double of one kind (exact
// upwards, rounded to nearest downwards), or complex <-> real of one
// precision (the real part; a zero imaginary part).
template <typename D, typename S>
__global__ void __launch_bounds__(kReduceThreads)
convert_kernel(D *__restrict__ dst, const S *__restrict__ src, int64_t elems)
{
    using R = typename storage_traits<D>::real;
    for (int64_t p = (int64_t)blockIdx.x * kReduceThreads + threadIdx.x; p < elems;
         p += (int64_t)gridDim.x * kReduceThreads) {
        const S v = src[p];
        if constexpr (storage_traits<D>::complex) {
            D d;
            if constexpr (storage_traits<S>::complex) {
                d.x = (R)v.x;
                d.y = (R)v.y;
            } else {
                d.x = (R)v;
                d.y = (R)0;
            }
            dst[p] = d;
        } else if constexpr (storage_traits<S>::complex) {
            dst[p] = (R)v.x;
        } else {
            dst[p] = (R)v;
        }
    }
}

hipError_t launch_convert(Prec to, Prec from, void *dst, const void *src, int64_t elems, hipStream_t stream)
{
    int64_t blocks = (elems + kReduceThreads - 1) / kReduceThreads;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    const dim3 grid((unsigned)blocks), block(kReduceThreads);
#define GP_CONV(DT, ST)                                                                                       \
    hipLaunchKernelGGL((convert_kernel<DT, ST>), grid, block, 0, stream, static_cast<DT *>(dst),              \
                       static_cast<const ST *>(src), elems);                                                  \
    return hipGetLastError();
    if (to == PREC_C128 && from == PREC_C64) { GP_CONV(double2, float2) }
    if (to == PREC_C64 && from == PREC_C128) { GP_CONV(float2, double2) }
    if (to == PREC_R64 && from == PREC_R32) { GP_CONV(double, float) }
    if (to == PREC_R32 && from == PREC_R64) { GP_CONV(float, double) }
    if (to == PREC_R32 && from == PREC_C64) { GP_CONV(float, float2) }
    if (to == PREC_C64 && from == PREC_R32) { GP_CONV(float2, float) }
    if (to == PREC_R64 && from == PREC_C128) { GP_CONV(double, double2) }
    if (to == PREC_C128 && from == PREC_R64) { GP_CONV(double2, double) }
#undef GP_CONV
    return hipErrorInvalidValue;
}

int obs_num_blocks(int nx, int ny)
{
    return ((nx + kObsX - 1) / kObsX) * ((ny + kObsY - 1) / kObsY);
}

hipError_t launch_observables(Prec prec, const void *psi, const ObsArgs<double> &args,
                              double *partials, double *sums, hipStream_t stream)
{
    const dim3 grid((unsigned)((args.nx + kObsX - 1) / kObsX),
                    (unsigned)((args.ny + kObsY - 1) / kObsY));
    const dim3 block(kObsX * kObsY);
    hipError_t e = with_storage(prec, [&](auto tag) {
        using S = decltype(tag);
        hipLaunchKernelGGL(calcmuen_rms_kernel<S>, grid, block, 0, stream, static_cast<const S *>(psi), args,
                           partials);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(obs_finalize_kernel, dim3(1), dim3(kReduceThreads), 0, stream,
                       partials, (int)grid.x * (int)grid.y, sums);
    return hipGetLastError();
}

}  // namespace gpssc

namespace gpssc {

// Density profiles: the density integrated over the other two axes, per
// node of each axis.  One block per node of the profiled axis; its threads
// stride over the other two in a fixed order, then a fixed tree.
template <typename S>
__global__ void __launch_bounds__(kReduceThreads)
profile_kernel(const S *__restrict__ psi, int nx, int ny, int nz, int axis, double w, double *__restrict__ out)
{
    __shared__ double red[kReduceThreads];
    const int node = blockIdx.x;
    const int64_t m = axis == 0 ? (int64_t)ny * nz : (axis == 1 ? (int64_t)nx * nz : (int64_t)nx * ny);
    double acc = 0.0;
    for (int64_t q = threadIdx.x; q < m; q += kReduceThreads) {
#pragma clang fp contract(off)
        int64_t p;
        if (axis == 0) {
            p = q * nx + node;                               // q = k*ny + j
        } else if (axis == 1) {
            const int64_t k = q / nx, i = q - k * nx;
            p = (k * ny + node) * nx + i;
        } else {
            p = (int64_t)node * nx * ny + q;                 // q = j*nx + i
        }
        const S v = psi[p];
        acc += sre(v) * sre(v) + sim(v) * sim(v);
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) out[node] = w * s;
}

hipError_t launch_profiles(Prec prec, const void *psi, int nx, int ny, int nz, const double w[3], double *out,
                           hipStream_t stream)
{
    const int n[3] = {nx, ny, nz};
    double *dst = out;
    for (int axis = 0; axis < 3; ++axis) {
        hipError_t e = with_storage(prec, [&](auto tag) {
            using S = decltype(tag);
            hipLaunchKernelGGL(profile_kernel<S>, dim3((unsigned)n[axis]), dim3(kReduceThreads), 0, stream,
                               static_cast<const S *>(psi), nx, ny, nz, axis, w[axis], dst);
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
        dst += n[axis];
    }
    return hipSuccess;
}

}  // namespace gpssc
