// sweep_x.hip -- calcnu fused with calclux: the pointwise potential +
// nonlinear sub-step followed by the Crank-Nicolson solve along x.
//
// Paper: "Summary of revisions" names calcnu (the nonlinear/potential part of
// the time evolution) and calclux (the x part of the Crank-Nicolson split);
// "Method of solution" of summaries (v) and (xiv) fixes the split-step
// Crank-Nicolson propagation in imaginary or real time.
//
// One wavefront owns one x line (j, k): Nx contiguous points.  The line is
// read with coalesced loads into LDS, then lane l takes the contiguous chunk
// [l*C, l*C + C) into registers.  The constant-coefficient Thomas recursion
//     forward   d'_i = m_i q_i + a_i d'_{i-1},      a_i = -o m_i
//     backward  x_i  = d'_i   + a_i x_{i+1}
// is a first-order linear recurrence in both directions, so each lane runs
// it over its chunk with a zero carry, the carries between chunks come from
// a Kogge-Stone scan across the 64 lanes (the stage multipliers are products
// of a_i and are precomputed on the host), and each lane reruns its chunk
// from the true carry.  The result is the Thomas solution up to rounding.
#include "gp_internal.h"

namespace gpssc {

template <typename A>
__device__ __forceinline__ cx<A> shfl_up_c(cx<A> v, int d)
{
    return cx<A>{__shfl_up(v.re, d, kWave), __shfl_up(v.im, d, kWave)};
}

template <typename A>
__device__ __forceinline__ cx<A> shfl_down_c(cx<A> v, int d)
{
    return cx<A>{__shfl_down(v.re, d, kWave), __shfl_down(v.im, d, kWave)};
}

template <typename A> __device__ __forceinline__ void sincos_t(A x, A *s, A *c);
template <> __device__ __forceinline__ void sincos_t<double>(double x, double *s, double *c) { sincos(x, s, c); }
template <> __device__ __forceinline__ void sincos_t<float>(float x, float *s, float *c) { sincosf(x, s, c); }
template <typename A> __device__ __forceinline__ A exp_t(A x);
template <> __device__ __forceinline__ double exp_t<double>(double x) { return exp(x); }
template <> __device__ __forceinline__ float exp_t<float>(float x) { return expf(x); }

// LDS slot of line element e: one padding slot after every C elements keeps
// the chunk-order reads (stride C+1 elements between lanes) off one bank.
template <int C>
__device__ __forceinline__ int xslot(int e) { return e + e / C; }

template <typename S, typename A, int C, bool REAL>
__global__ void __launch_bounds__(kWave)
calcnu_lux_kernel(S *__restrict__ psi, const XArgs<A> a, const cx<A> *__restrict__ mtab,
                  const cx<A> *__restrict__ scan, const double *__restrict__ scale)
{
    __shared__ S buf[kWave * C + kWave];
    const int lane = threadIdx.x;
    const int line = blockIdx.x;            // j + Ny * k
    const int j = line % a.ny;
    const int k = line / a.ny;
    S *row = psi + (int64_t)line * a.nx;

    // coalesced load of the line into LDS
#pragma unroll
    for (int r = 0; r < C; ++r) {
        const int e = r * kWave + lane;
        S v;
        v.x = 0;
        v.y = 0;
        if (e < a.nx) v = row[e];
        buf[xslot<C>(e)] = v;
    }
    __syncthreads();

    cx<A> u[C];
#pragma unroll
    for (int c = 0; c < C; ++c) u[c] = ld<A>(buf[lane * (C + 1) + c]);

    // calcnu: pending renormalisation, then exp(-tau (V + g|psi|^2)).
    const A s = scale ? (A)(*scale) : (A)1;
    const A y = ((A)j - a.c0y) * a.dy;
    const A z = ((A)k - a.c0z) * a.dz;
    const A vyz = a.hgy * y * y + a.hgz * z * z;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int i = lane * C + c;
        if (i < a.nx) {
            cx<A> v = cx<A>{u[c].re * s, u[c].im * s};
            const A x = ((A)i - a.c0x) * a.dx;
            const A theta = fma(a.hgx * x, x, vyz) + a.g * cabs2(v);
            if (REAL) {
                A sn, cs;
                sincos_t<A>(a.dt * theta, &sn, &cs);
                v = cx<A>{fma(v.re, cs, v.im * sn), fma(v.im, cs, -v.re * sn)};
            } else {
                const A f = exp_t<A>(-a.dt * theta);
                v = cx<A>{v.re * f, v.im * f};
            }
            u[c] = v;
        }
    }

    // right-hand side (1 - tau/2 T) psi with zero ghosts; neighbours across
    // chunk borders come from the adjacent lanes.
    cx<A> left = shfl_up_c(u[C - 1], 1);
    cx<A> right = shfl_down_c(u[0], 1);
    if (lane == 0) left = cx<A>{0, 0};
    if (lane == kWave - 1) right = cx<A>{0, 0};

    cx<A> q[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const cx<A> lo = c > 0 ? u[c - 1] : left;
        const cx<A> hi = c < C - 1 ? u[c + 1] : right;
        q[c] = cfma(a.ro, cadd(lo, hi), cmul(a.rd, u[c]));
    }

    // Thomas coefficients of this lane's chunk: m_i and a_i = -o m_i.
    const cx<A> mo = cx<A>{-a.o.re, -a.o.im};
    cx<A> am[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const cx<A> m = mtab[c * kWave + lane];
        q[c] = cmul(m, q[c]);
        am[c] = cmul(mo, m);
    }

    // forward elimination: local pass with zero carry, scan, rerun
    cx<A> t = cx<A>{0, 0};
#pragma unroll
    for (int c = 0; c < C; ++c) t = cfma(am[c], t, q[c]);
    for (int st = 0; st < a.nst_f; ++st) {
        const cx<A> from = shfl_up_c(t, 1 << st);
        t = cfma(scan[st * kWave + lane], from, t);
    }
    t = shfl_up_c(t, 1);
    if (lane == 0) t = cx<A>{0, 0};
#pragma unroll
    for (int c = 0; c < C; ++c) {
        t = cfma(am[c], t, q[c]);
        q[c] = t;  // q now holds d'
    }

    // back substitution: same pattern from the right
    t = cx<A>{0, 0};
#pragma unroll
    for (int c = C - 1; c >= 0; --c) t = cfma(am[c], t, q[c]);
    for (int st = 0; st < a.nst_b; ++st) {
        const cx<A> from = shfl_down_c(t, 1 << st);
        t = cfma(scan[(kMaxStages + st) * kWave + lane], from, t);
    }
    t = shfl_down_c(t, 1);
    if (lane == kWave - 1) t = cx<A>{0, 0};
#pragma unroll
    for (int c = C - 1; c >= 0; --c) {
        t = cfma(am[c], t, q[c]);
        q[c] = t;  // q now holds the solution
    }

    // chunk order -> LDS -> coalesced store
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c) buf[lane * (C + 1) + c] = st<S>(q[c]);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < C; ++r) {
        const int e = r * kWave + lane;
        if (e < a.nx) row[e] = buf[xslot<C>(e)];
    }
}

template <typename S, typename A, bool REAL>
static hipError_t launch_c(int chunk, void *psi, const void *args, const void *m,
                           const void *scan, const double *scale, hipStream_t stream)
{
    const XArgs<A> &a = *static_cast<const XArgs<A> *>(args);
    const dim3 grid((unsigned)(a.ny * a.nz));
    const dim3 block(kWave);
    S *p = static_cast<S *>(psi);
    const cx<A> *mt = static_cast<const cx<A> *>(m);
    const cx<A> *sc = static_cast<const cx<A> *>(scan);
#define GP_X_CASE(CC)                                                                  \
    case CC:                                                                           \
        hipLaunchKernelGGL((calcnu_lux_kernel<S, A, CC, REAL>), grid, block, 0, stream, \
                           p, a, mt, sc, scale);                                       \
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

hipError_t launch_nu_x(Prec prec, bool real, int chunk, void *psi, const void *args,
                       const void *m, const void *scan, const double *scale,
                       hipStream_t stream)
{
    switch (prec) {
    case PREC_C64:
        return real ? launch_c<float2, float, true>(chunk, psi, args, m, scan, scale, stream)
                    : launch_c<float2, float, false>(chunk, psi, args, m, scan, scale, stream);
    case PREC_C64_F64:
        return real ? launch_c<float2, double, true>(chunk, psi, args, m, scan, scale, stream)
                    : launch_c<float2, double, false>(chunk, psi, args, m, scan, scale, stream);
    case PREC_C128:
        return real ? launch_c<double2, double, true>(chunk, psi, args, m, scan, scale, stream)
                    : launch_c<double2, double, false>(chunk, psi, args, m, scan, scale, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace gpssc
