// sweep_radial.hip -- calcnu fused with the Crank-Nicolson solve along a
// radial variable, and the physical quantities of the symmetric traps.
//
// Paper: program summaries (iv) imagtimecir, (ix) imagtimesph, (vii)
// imagtimeaxial and their real-time counterparts: the circularly and
// spherically symmetric traps (one radial variable) and the axially
// symmetric trap (rho, z), each propagated by the split-step Crank-Nicolson
// method.  The radial Laplacian is the conservative finite-volume form on
// r_i = (i + 1/2) h (no flux through r = 0, zero past the last node), so the
// Crank-Nicolson matrix along r is tridiagonal with position-dependent but
// time-constant coefficients.
//
// One wavefront per radial line, lane l holding the chunk [l*C, l*C + C) as
// in the x kernel.  The Thomas recurrences
//     d_i = m_i q_i + a_i d_{i-1},        x_i = d_i + b_i x_{i+1}
// now have a coefficient per position, so a chunk is an affine map of its
// carry, t_out = A t_in + B (A the product of the chunk's a or b, B the
// value from a zero carry); a Kogge-Stone scan over the 64 lanes composes
// the maps, and every lane reruns its chunk from the carry it receives.
#include "sweep_common.h"

namespace gpssc {

template <typename S, typename A, int C, bool REAL>
__global__ void __launch_bounds__(kWave)
calcnu_lur_kernel(S *__restrict__ psi, const RadialArgs<A> ra, const double *__restrict__ scale,
                  double *__restrict__ dens)
{
    __shared__ S buf[kWave * C + kWave];
    const XArgs<A> &a = ra.x;
    const int lane = threadIdx.x;
    const int line = blockIdx.x;
    const int j = line % a.ny;
    const int k = line / a.ny;
    const int pos0 = lane * C;
    const int np = ra.npad;
    const cx<A> *rd = ra.tab, *rl = rd + np, *ru = rl + np, *mm = ru + np, *am = mm + np, *bm = am + np;
    S *row = psi + (int64_t)line * a.nx;

    S v[C];
    load_x_row(v, row, a.nx);
#pragma unroll
    for (int r = 0; r < C; ++r) buf[xslot<C>(r * kWave + lane)] = v[r];
    __syncthreads();
    cx<A> u[C];
#pragma unroll
    for (int c = 0; c < C; ++c) u[c] = ld<A>(buf[lane * (C + 1) + c]);

    // calcnu: pending renormalisation, then exp(-tau (V + g|psi|^2)); the
    // radial coordinate is (i + 1/2) h (c0x = -1/2)
    const A s = scale ? (A)(*scale) : (A)1;
    const A y = ((A)j - a.c0y) * a.dy;
    const A z = ((A)k - a.c0z) * a.dz;
    const A vyz = trap_yz(a.hgy, y, a.hgz, z);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const cx<A> w = cx<A>{u[c].re * s, u[c].im * s};
        const A x = ((A)(pos0 + c) - a.c0x) * a.dx;
        const A theta = nu_theta(a.hgx, x, vyz, a.g, w);
        u[c] = nu_factor<REAL>(w, a.dt * theta);
    }

    // right side q_i = rd_i u_i + rl_i u_{i-1} + ru_i u_{i+1} (zero beyond the
    // line; the padding has zero coefficients)
    cx<A> left = shfl_up_c(u[C - 1], 1);
    cx<A> right = shfl_down_c(u[0], 1);
    if (lane == 0) left = cx<A>{0, 0};
    if (lane == kWave - 1) right = cx<A>{0, 0};
    {
        cx<A> prev = left;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int p = pos0 + c;
            const cx<A> cur = u[c];
            const cx<A> nxt = c < C - 1 ? u[c + 1] : right;
            u[c] = kfma<REAL>(ru[p], nxt, kfma<REAL>(rl[p], prev, kmul<REAL>(rd[p], cur)));
            prev = cur;
        }
    }

    // forward: chunk map from a zero carry, scan of the maps, rerun
    cx<A> A_ = cx<A>{1, 0}, B_ = cx<A>{0, 0};
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int p = pos0 + c;
        B_ = kfma<REAL>(am[p], B_, kmul<REAL>(mm[p], u[c]));
        A_ = kmul<REAL>(am[p], A_);
    }
#pragma unroll
    for (int st = 0; st < kMaxStages; ++st) {
        const int d = 1 << st;
        const cx<A> fa = shfl_up_c(A_, d), fb = shfl_up_c(B_, d);
        if (lane >= d) {
            B_ = kfma<REAL>(A_, fb, B_);
            A_ = kmul<REAL>(A_, fa);
        }
    }
    cx<A> t = shfl_up_c(B_, 1);
    if (lane == 0) t = cx<A>{0, 0};
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int p = pos0 + c;
        t = kfma<REAL>(am[p], t, kmul<REAL>(mm[p], u[c]));
        u[c] = t;
    }
    if (a.nx < kWave * C) chunk_clear_padding(u, pos0, a.nx);

    // backward: the same from the right
    A_ = cx<A>{1, 0};
    B_ = cx<A>{0, 0};
#pragma unroll
    for (int c = C - 1; c >= 0; --c) {
        const int p = pos0 + c;
        B_ = kfma<REAL>(bm[p], B_, u[c]);
        A_ = kmul<REAL>(bm[p], A_);
    }
#pragma unroll
    for (int st = 0; st < kMaxStages; ++st) {
        const int d = 1 << st;
        const cx<A> fa = shfl_down_c(A_, d), fb = shfl_down_c(B_, d);
        if (lane + d < kWave) {
            B_ = kfma<REAL>(A_, fb, B_);
            A_ = kmul<REAL>(A_, fa);
        }
    }
    t = shfl_down_c(B_, 1);
    if (lane == kWave - 1) t = cx<A>{0, 0};
#pragma unroll
    for (int c = C - 1; c >= 0; --c) {
        const int p = pos0 + c;
        t = kfma<REAL>(bm[p], t, u[c]);
        u[c] = t;
    }

    // density of what is stored, per position (the imaginary-time norm of
    // a one-line state)
    if (dens) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (pos0 + c < a.nx) {
#pragma clang fp contract(off)
                const S sv = st<S>(u[c]);
                dens[(int64_t)line * a.nx + pos0 + c] = sre(sv) * sre(sv) + sim(sv) * sim(sv);
            }
        }
    }

    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; ++c) buf[lane * (C + 1) + c] = st<S>(u[c]);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < C; ++r) {
        const int e = r * kWave + lane;
        if (e < a.nx) stream_store(row + e, buf[xslot<C>(e)]);
    }
}

template <typename S, typename A, bool REAL>
static hipError_t launch_r(int chunk, int nlines, void *psi, const void *args, const double *scale,
                           double *dens, hipStream_t stream)
{
    const RadialArgs<A> &a = *static_cast<const RadialArgs<A> *>(args);
    S *p = static_cast<S *>(psi);
#define GP_R_CASE(CC)                                                                              \
    case CC:                                                                                       \
        hipLaunchKernelGGL((calcnu_lur_kernel<S, A, CC, REAL>), dim3((unsigned)nlines), dim3(kWave), 0, \
                           stream, p, a, scale, dens);                                             \
        break;
    switch (chunk) {
        GP_R_CASE(1) GP_R_CASE(2) GP_R_CASE(3) GP_R_CASE(4)
        GP_R_CASE(5) GP_R_CASE(6) GP_R_CASE(7) GP_R_CASE(8)
        GP_R_CASE(10) GP_R_CASE(12) GP_R_CASE(14) GP_R_CASE(16)
    default:
        return hipErrorInvalidValue;
    }
#undef GP_R_CASE
    return hipGetLastError();
}

hipError_t launch_nu_r(Prec prec, bool real, int chunk, int nlines, void *psi, const void *args,
                       const double *scale, double *dens, hipStream_t stream)
{
    if (nlines <= 0) return hipSuccess;
    if (real && (prec == PREC_R64 || prec == PREC_R32)) return hipErrorInvalidValue;
#define GP_R_PREC(S, A)                                                                         \
    return real ? launch_r<S, A, true>(chunk, nlines, psi, args, scale, dens, stream)           \
                : launch_r<S, A, false>(chunk, nlines, psi, args, scale, dens, stream);
    switch (prec) {
    case PREC_C64: GP_R_PREC(float2, float)
    case PREC_C64_F64: GP_R_PREC(float2, double)
    case PREC_C128: GP_R_PREC(double2, double)
    case PREC_R64: GP_R_PREC(double, double)
    case PREC_R32: GP_R_PREC(float, float)
    }
#undef GP_R_PREC
    return hipErrorInvalidValue;
}

// ---- physical quantities of the symmetric traps ----
//
// Block k takes row k (one z node of the axial trap; the single line of the
// circular and spherical ones) and sums, over the radial index in a fixed
// order, the weighted terms
//   DENS  v_i |psi|^2          POT   v_i V |psi|^2     QUART v_i |psi|^4
//   LINKX s_i |psi_{i+1} - psi_i|^2 (zero beyond the last node)
//   LINKY v_i |psi_{k+1} - psi_k|^2 (and the ghost link before k = 0)
//   M1X, M2X  v_i r |psi|^2, v_i r^2 |psi|^2;  M1Y, M2Y the same in z,
// with v the cell and s the face weights of the radial axis.
constexpr int kRadObsThreads = 256;

__device__ double rad_block_sum(double v, double *red)
{
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int h = kRadObsThreads / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

template <typename S>
__global__ void __launch_bounds__(kRadObsThreads)
radial_obs_kernel(const S *__restrict__ psi, const RadialObsArgs o, double *__restrict__ partials)
{
    __shared__ double red[kRadObsThreads];
    const int k = blockIdx.x;
    double acc[OBS_NSUMS];
#pragma unroll
    for (int q = 0; q < OBS_NSUMS; ++q) acc[q] = 0.0;
    const double z = ((double)k - o.c0z) * o.dz;
    for (int i = threadIdx.x; i < o.nr; i += kRadObsThreads) {
#pragma clang fp contract(off)
        const S v = psi[(int64_t)k * o.nr + i];
        const double re = sre(v), im = sim(v);
        const double w = re * re + im * im;
        const double r = ((double)i + 0.5) * o.dr;
        const double cw = o.v[i];
        acc[OBS_DENS] += cw * w;
        acc[OBS_POT] += cw * (o.hgr * r * r + o.hgz * z * z) * w;
        acc[OBS_QUART] += cw * w * w;
        acc[OBS_M1X] += cw * r * w;
        acc[OBS_M2X] += cw * r * r * w;
        acc[OBS_M1Y] += cw * z * w;
        acc[OBS_M2Y] += cw * z * z * w;
        double nre = 0.0, nim = 0.0;
        if (i + 1 < o.nr) {
            const S n = psi[(int64_t)k * o.nr + i + 1];
            nre = sre(n);
            nim = sim(n);
        }
        acc[OBS_LINKX] += o.s[i] * ((nre - re) * (nre - re) + (nim - im) * (nim - im));
        if (o.nz > 1) {
            double ure = 0.0, uim = 0.0;
            if (k + 1 < o.nz) {
                const S n = psi[(int64_t)(k + 1) * o.nr + i];
                ure = sre(n);
                uim = sim(n);
            }
            double links = (ure - re) * (ure - re) + (uim - im) * (uim - im);
            if (k == 0) links += w;
            acc[OBS_LINKY] += cw * links;
        }
    }
#pragma unroll
    for (int q = 0; q < OBS_NSUMS; ++q) {
        const double sum = rad_block_sum(acc[q], red);
        if (threadIdx.x == 0) partials[(int64_t)k * OBS_NSUMS + q] = sum;
    }
}

__global__ void __launch_bounds__(kRadObsThreads)
radial_obs_finalize_kernel(const double *__restrict__ partials, int nrows, double *__restrict__ sums)
{
    __shared__ double red[kRadObsThreads];
    for (int q = 0; q < OBS_NSUMS; ++q) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < nrows; b += kRadObsThreads) acc += partials[(int64_t)b * OBS_NSUMS + q];
        const double s = rad_block_sum(acc, red);
        if (threadIdx.x == 0) sums[q] = s;
    }
}

hipError_t launch_radial_observables(Prec prec, const void *psi, const RadialObsArgs &args, double *partials,
                                     double *sums, hipStream_t stream)
{
    const dim3 grid((unsigned)args.nz);
    switch (prec) {
    case PREC_C128:
        hipLaunchKernelGGL(radial_obs_kernel<double2>, grid, dim3(kRadObsThreads), 0, stream,
                           static_cast<const double2 *>(psi), args, partials);
        break;
    case PREC_C64:
    case PREC_C64_F64:
        hipLaunchKernelGGL(radial_obs_kernel<float2>, grid, dim3(kRadObsThreads), 0, stream,
                           static_cast<const float2 *>(psi), args, partials);
        break;
    case PREC_R64:
        hipLaunchKernelGGL(radial_obs_kernel<double>, grid, dim3(kRadObsThreads), 0, stream,
                           static_cast<const double *>(psi), args, partials);
        break;
    case PREC_R32:
        hipLaunchKernelGGL(radial_obs_kernel<float>, grid, dim3(kRadObsThreads), 0, stream,
                           static_cast<const float *>(psi), args, partials);
        break;
    default:
        return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(radial_obs_finalize_kernel, dim3(1), dim3(kRadObsThreads), 0, stream, partials, args.nz,
                       sums);
    return hipGetLastError();
}

}  // namespace gpssc
