// sweep_x.hip -- calcnu fused with calclux: the pointwise potential +
// nonlinear sub-step followed by the Crank-Nicolson solve along x.
//
// Paper: "Summary of revisions" names calcnu (the nonlinear/potential part of
// the time evolution) and calclux (the x part of the Crank-Nicolson split);
// "Method of solution" of summaries (v) and (xiv) fixes the split-step
// Crank-Nicolson propagation in imaginary or real time.
//
// One wavefront solves one x line (j, k) at a time: Nx contiguous points.
// The line is read with coalesced loads, staged through LDS, and lane l takes
// the contiguous chunk
// [l*C, l*C + C) into registers.  The Crank-Nicolson system of the line is
// solved through the constant-coefficient factorisation of its Toeplitz
// matrix (SweepCoef): the forward and the backward recurrence
//     w_i = m r_i + a w_{i-1},        y_i = w_i + a y_{i+1}
// have the same coefficient at every node, so each lane runs its chunk with a
// zero carry, the carries between chunks come from a Kogge-Stone scan across
// the 64 lanes (stage multipliers a^(C 2^s)), each lane reruns its chunk from
// its carry, and the rank-one boundary term is added from the first node's
// value.  The result equals the Thomas solution up to rounding.
#include "sweep_common.h"

namespace gpssc {

// One x line: psi values in row order (element r*64 + lane) -> solved line,
// in row order, written back through the same LDS buffer.
template <typename S, typename A, int C, bool REAL>
__device__ __forceinline__ void solve_x_line(S (&row_vals)[C], S *buf, const XArgs<A> &a,
                                             const cx<A> *__restrict__ zt, A s, int line)
{
    using V = value_t<S, A>;
    const int lane = threadIdx.x;
    const int j = line % a.ny;
    const int k = line / a.ny;
    const int pos0 = lane * C;

#pragma unroll
    for (int r = 0; r < C; ++r) buf[xslot<C>(r * kWave + lane)] = row_vals[r];
    __syncthreads();
    V u[C];
#pragma unroll
    for (int c = 0; c < C; ++c) u[c] = ldv<V>(buf[lane * (C + 1) + c]);

    // calcnu: pending renormalisation, then exp(-tau (V + g|psi|^2)).
    const A y = ((A)j - a.c0y) * a.dy;
    const A z = ((A)k - a.c0z) * a.dz;
    const A vyz = a.hgy * y * y + a.hgz * z * z;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const V v = vscale(u[c], s);
        const A x = ((A)(pos0 + c) - a.c0x) * a.dx;
        const A theta = fma(a.hgx * x, x, vyz) + a.g * cabs2(v);
        u[c] = nu_factor<REAL>(v, a.dt * theta);   // padding stays 0
    }

    // right-hand side with zero ghosts; neighbours across chunk borders come
    // from the adjacent lanes
    V left = shfl_up_c(u[C - 1], 1);
    V right = shfl_down_c(u[0], 1);
    if (lane == 0) left = V{};
    if (lane == kWave - 1) right = V{};
    chunk_rhs<REAL>(u, left, right, a.k);

    // forward: local pass with zero carry, Kogge-Stone across lanes, rerun
    V t = chunk_forward<REAL, false>(u, V{}, a.k);
#pragma unroll
    for (int st = 0; st < kMaxStages; ++st) {
        if (st < a.k.nst) {
            const V from = shfl_up_c(t, 1 << st);
            if (lane >= (1 << st)) t = kfma<REAL>(a.k.stage[st], from, t);
        }
    }
    t = shfl_up_c(t, 1);
    if (lane == 0) t = V{};
    chunk_forward<REAL, true>(u, t, a.k);
    if (a.nx < kWave * C) chunk_clear_padding(u, pos0, a.nx);

    // backward: the same from the right
    t = chunk_backward<REAL, false>(u, V{}, a.k);
#pragma unroll
    for (int st = 0; st < kMaxStages; ++st) {
        if (st < a.k.nst) {
            const V from = shfl_down_c(t, 1 << st);
            if (lane + (1 << st) < kWave) t = kfma<REAL>(a.k.stage[st], from, t);
        }
    }
    t = shfl_down_c(t, 1);
    if (lane == kWave - 1) t = V{};
    chunk_backward<REAL, true>(u, t, a.k);

    // boundary correction from the first node
    const V y0 = shfl_c(u[0], 0);
    if (pos0 < a.k.nzc) chunk_correct<REAL>(u, y0, zt, pos0, a.k.nzc);

    // chunk order -> LDS -> row order
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c) buf[lane * (C + 1) + c] = stv<S>(u[c]);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < C; ++r) row_vals[r] = buf[xslot<C>(r * kWave + lane)];
}

// partials: NULL, or one double per line receiving sum |psi|^2 of the stored
// line (the norm partials of imaginary time when x is the only variable),
// summed per lane in row order, then over the lanes by a fixed tree.
template <typename S, typename A, int C, bool REAL>
__global__ void __launch_bounds__(kWave)
calcnu_lux_kernel(S *__restrict__ psi, const XArgs<A> a, const cx<A> *__restrict__ zt,
                  const double *__restrict__ scale, double *__restrict__ partials)
{
    __shared__ S buf[kWave * C + kWave];
    const int lane = threadIdx.x;
    const int nlines = a.ny * a.nz;
    const A s = scale ? (A)(*scale) : (A)1;
    for (int line = blockIdx.x; line < nlines; line += gridDim.x) {
        S *row = psi + (int64_t)line * a.nx;
        S v[C];
        load_x_row(v, row, a.nx);
        solve_x_line<S, A, C, REAL>(v, buf, a, zt, s, line);
#pragma unroll
        for (int r = 0; r < C; ++r) {
            const int e = r * kWave + lane;
            if (e < a.nx) stream_store(row + e, v[r]);
        }
        if (partials) {
            double acc = 0.0;
#pragma unroll
            for (int r = 0; r < C; ++r) {
                if (r * kWave + lane < a.nx) {
#pragma clang fp contract(off)
                    acc += sre(v[r]) * sre(v[r]) + sim(v[r]) * sim(v[r]);
                }
            }
#pragma unroll
            for (int d = kWave / 2; d > 0; d >>= 1) acc += __shfl_down(acc, d, kWave);
            if (lane == 0) partials[line] = acc;
        }
        __syncthreads();  // buf is free for the next line
    }
}

// Batched: block b advances line b % nlines of solve active[b / nlines].
template <typename S, typename A, int C, bool REAL>
__global__ void __launch_bounds__(kWave)
calcnu_lux_batch_kernel(S *const *__restrict__ psis, const XBatchArgs<A> *__restrict__ args,
                        const int *__restrict__ active, int nlines, const double *__restrict__ scales)
{
    __shared__ S buf[kWave * C + kWave];
    const int lane = threadIdx.x;
    const int slot = blockIdx.x / nlines;
    const int line = blockIdx.x - slot * nlines;
    const int si = active[slot];
    const XArgs<A> &a = args[si].x;
    const A s = scales ? (A)scales[si] : (A)1;
    S *row = psis[si] + (int64_t)line * a.nx;
    S v[C];
    load_x_row(v, row, a.nx);
    solve_x_line<S, A, C, REAL>(v, buf, a, args[si].zt, s, line);
#pragma unroll
    for (int r = 0; r < C; ++r) {
        const int e = r * kWave + lane;
        if (e < a.nx) stream_store(row + e, v[r]);
    }
}

template <typename S, typename A, bool REAL>
static hipError_t launch_batch_c(int chunk, int nact, int nlines, void *const *psis, const void *args,
                                 const int *active, const double *scales, hipStream_t stream)
{
    const dim3 grid((unsigned)((int64_t)nact * nlines));
    const dim3 block(kWave);
    S *const *p = reinterpret_cast<S *const *>(psis);
    const XBatchArgs<A> *a = static_cast<const XBatchArgs<A> *>(args);
#define GP_XB_CASE(CC)                                                                        \
    case CC:                                                                                  \
        hipLaunchKernelGGL((calcnu_lux_batch_kernel<S, A, CC, REAL>), grid, block, 0, stream,  \
                           p, a, active, nlines, scales);                                     \
        break;
    switch (chunk) {
        GP_XB_CASE(1) GP_XB_CASE(2) GP_XB_CASE(3) GP_XB_CASE(4)
        GP_XB_CASE(5) GP_XB_CASE(6) GP_XB_CASE(7) GP_XB_CASE(8)
        GP_XB_CASE(10) GP_XB_CASE(12) GP_XB_CASE(14) GP_XB_CASE(16)
    default:
        return hipErrorInvalidValue;
    }
#undef GP_XB_CASE
    return hipGetLastError();
}

hipError_t launch_nu_x_batch(Prec prec, bool real, int chunk, int nact, int nlines, void *const *psis,
                             const void *args, const int *active, const double *scales,
                             hipStream_t stream)
{
    if (real && (prec == PREC_R64 || prec == PREC_R32)) return hipErrorInvalidValue;  // real storage is imaginary time only
    if (nact <= 0) return hipSuccess;
#define GP_XB_PREC(S, A)                                                                      \
    return real ? launch_batch_c<S, A, true>(chunk, nact, nlines, psis, args, active, scales, stream) \
                : launch_batch_c<S, A, false>(chunk, nact, nlines, psis, args, active, scales, stream);
    switch (prec) {
    case PREC_C64: GP_XB_PREC(float2, float)
    case PREC_C64_F64: GP_XB_PREC(float2, double)
    case PREC_C128: GP_XB_PREC(double2, double)
    // real storage: imaginary time only (real time was refused above)
    case PREC_R64: return launch_batch_c<double, double, false>(chunk, nact, nlines, psis, args, active, scales, stream);
    case PREC_R32: return launch_batch_c<float, float, false>(chunk, nact, nlines, psis, args, active, scales, stream);
    }
#undef GP_XB_PREC
    return hipErrorInvalidValue;
}

template <typename S, typename A, bool REAL>
static hipError_t launch_c(int chunk, int nblocks, void *psi, const void *args, const void *zt,
                           const double *scale, double *partials, hipStream_t stream)
{
    const XArgs<A> &a = *static_cast<const XArgs<A> *>(args);
    const int nlines = a.ny * a.nz;
    const dim3 grid((unsigned)(nblocks > 0 && nblocks < nlines ? nblocks : nlines));
    const dim3 block(kWave);
    S *p = static_cast<S *>(psi);
    const cx<A> *z = static_cast<const cx<A> *>(zt);
#define GP_X_CASE(CC)                                                                  \
    case CC:                                                                           \
        hipLaunchKernelGGL((calcnu_lux_kernel<S, A, CC, REAL>), grid, block, 0, stream, \
                           p, a, z, scale, partials);                                  \
        break;
    switch (chunk) {
        GP_X_CASE(1) GP_X_CASE(2) GP_X_CASE(3) GP_X_CASE(4)
        GP_X_CASE(5) GP_X_CASE(6) GP_X_CASE(7) GP_X_CASE(8)
        GP_X_CASE(10) GP_X_CASE(12) GP_X_CASE(14) GP_X_CASE(16)
    default:
        return hipErrorInvalidValue;
    }
#undef GP_X_CASE
    return hipGetLastError();
}

hipError_t launch_nu_x(Prec prec, bool real, int chunk, int nblocks, void *psi, const void *args,
                       const void *zt, const double *scale, double *partials, hipStream_t stream)
{
    if (real && (prec == PREC_R64 || prec == PREC_R32)) return hipErrorInvalidValue;  // real storage is imaginary time only
#define GP_X_PREC(S, A)                                                                   \
    return real ? launch_c<S, A, true>(chunk, nblocks, psi, args, zt, scale, partials, stream)  \
                : launch_c<S, A, false>(chunk, nblocks, psi, args, zt, scale, partials, stream);
    switch (prec) {
    case PREC_C64: GP_X_PREC(float2, float)
    case PREC_C64_F64: GP_X_PREC(float2, double)
    case PREC_C128: GP_X_PREC(double2, double)
    // real storage: imaginary time only (real time was refused above)
    case PREC_R64: return launch_c<double, double, false>(chunk, nblocks, psi, args, zt, scale, partials, stream);
    case PREC_R32: return launch_c<float, float, false>(chunk, nblocks, psi, args, zt, scale, partials, stream);
    }
#undef GP_X_PREC
    return hipErrorInvalidValue;
}

}  // namespace gpssc
