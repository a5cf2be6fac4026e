// sweep_common.h -- pieces shared by the x and the y/z Crank-Nicolson sweep
// kernels: the right-hand side, the passes of the constant-coefficient
// factorisation over a chunk, and the phase factor of calcnu.  Internal to
// libgpssc.
#pragma once

#include "gp_internal.h"

namespace gpssc {

// coef * v for a Crank-Nicolson coefficient.  In imaginary time every
// coefficient is real (tau = dt), so only the real part is used.
template <bool REAL, typename A>
__device__ __forceinline__ cx<A> kmul(cx<A> coef, cx<A> v)
{
    if (REAL) return cmul(coef, v);
    return cx<A>{coef.re * v.re, coef.re * v.im};
}

// coef * t + v
template <bool REAL, typename A>
__device__ __forceinline__ cx<A> kfma(cx<A> coef, cx<A> t, cx<A> v)
{
    if (REAL) return cfma(coef, t, v);
    return cx<A>{fma(coef.re, t.re, v.re), fma(coef.re, t.im, v.im)};
}

// Real values (real storage, imaginary time): the coefficients are real, and
// these are the real parts of the complex forms above.
template <bool REAL, typename A>
__device__ __forceinline__ A kmul(cx<A> coef, A v)
{
    static_assert(!REAL, "real values carry imaginary-time states only");
    return coef.re * v;
}

template <bool REAL, typename A>
__device__ __forceinline__ A kfma(cx<A> coef, A t, A v)
{
    static_assert(!REAL, "real values carry imaginary-time states only");
    return fma(coef.re, t, v);
}

template <typename A>
__device__ __forceinline__ A cabs2(A a) { return a * a; }

// Column pairs (y/z sweeps of complex64): each column on its own.
template <bool REAL, typename A>
__device__ __forceinline__ cx2<A> kmul(cx<A> coef, cx2<A> v)
{
    return cx2<A>{kmul<REAL>(coef, v.p), kmul<REAL>(coef, v.q)};
}

template <bool REAL, typename A>
__device__ __forceinline__ cx2<A> kfma(cx<A> coef, cx2<A> t, cx2<A> v)
{
    return cx2<A>{kfma<REAL>(coef, t.p, v.p), kfma<REAL>(coef, t.q, v.q)};
}

// Right-hand side (1 - tau/2 T) psi at one point from its neighbours:
//   (1 - kappa) u + kappa/2 (lo + hi) = u + kappa w,  w = (lo + hi)/2 - u,
// with kappa = dt/(2 dx^2) (imaginary time) or i dt/(2 dx^2) (real time).
// lo + hi is rounded on its own: the compiler may not fuse it with the
// multiplication that produced a neighbour, whose choice would otherwise
// depend on the shape of the surrounding code.
template <bool REAL, typename A>
__device__ __forceinline__ cx<A> cn_rhs(A kap, cx<A> lo, cx<A> u, cx<A> hi)
{
#pragma clang fp contract(off)
    const cx<A> w = cx<A>{fma((A)0.5, lo.re + hi.re, -u.re), fma((A)0.5, lo.im + hi.im, -u.im)};
    if (REAL) return cx<A>{fma(-kap, w.im, u.re), fma(kap, w.re, u.im)};
    return cx<A>{fma(kap, w.re, u.re), fma(kap, w.im, u.im)};
}

template <bool REAL, typename A>
__device__ __forceinline__ A cn_rhs(A kap, A lo, A u, A hi)
{
#pragma clang fp contract(off)
    static_assert(!REAL, "real values carry imaginary-time states only");
    return fma(kap, fma((A)0.5, lo + hi, -u), u);
}

template <bool REAL, typename A>
__device__ __forceinline__ cx2<A> cn_rhs(A kap, cx2<A> lo, cx2<A> u, cx2<A> hi)
{
    return cx2<A>{cn_rhs<REAL>(kap, lo.p, u.p, hi.p), cn_rhs<REAL>(kap, lo.q, u.q, hi.q)};
}

// Passes over one chunk of C points held in registers.  The coefficients
// are the same at every position (SweepCoef), so they live in scalar
// registers.

// u <- m (1 - tau/2 T) u, with the points either side of the chunk.
template <bool REAL, int C, typename A, typename V>
__device__ __forceinline__ void chunk_rhs(V (&u)[C], V left, V right, const SweepCoef<A> &k)
{
    V prev = left;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const V cur = u[c];
        const V rhs = cn_rhs<REAL>(k.kap, prev, cur, c < C - 1 ? u[c + 1] : right);
        prev = cur;
        u[c] = kmul<REAL>(k.m, rhs);
    }
}

// Forward recurrence t <- u_c + a t from carry t; returns the last value
// and, if STORE, leaves every value in u.
template <bool REAL, bool STORE, int C, typename A, typename V>
__device__ __forceinline__ V chunk_forward(V (&u)[C], V t, const SweepCoef<A> &k)
{
#pragma unroll
    for (int c = 0; c < C; ++c) {
        t = kfma<REAL>(k.a, t, u[c]);
        if (STORE) u[c] = t;
    }
    return t;
}

// Backward recurrence t <- u_c + a t from the chunk end.
template <bool REAL, bool STORE, int C, typename A, typename V>
__device__ __forceinline__ V chunk_backward(V (&u)[C], V t, const SweepCoef<A> &k)
{
#pragma unroll
    for (int c = C - 1; c >= 0; --c) {
        t = kfma<REAL>(k.a, t, u[c]);
        if (STORE) u[c] = t;
    }
    return t;
}

// Zero the values at positions >= n (the padding after the end of a line),
// so nothing past the last node feeds the back substitution.
template <int C, typename V>
__device__ __forceinline__ void chunk_clear_padding(V (&u)[C], int pos0, int n)
{
#pragma unroll
    for (int c = 0; c < C; ++c)
        if (pos0 + c >= n) u[c] = V{};
}

// Boundary correction x_i = y_i + y_0 zt_i for positions < nzc.
template <bool REAL, int C, typename A, typename V>
__device__ __forceinline__ void chunk_correct(V (&u)[C], V y0, const cx<A> *__restrict__ zt, int pos0, int nzc)
{
#pragma unroll
    for (int c = 0; c < C; ++c)
        if (pos0 + c < nzc) u[c] = kfma<REAL>(zt[pos0 + c], y0, u[c]);
}

template <typename A> __device__ __forceinline__ A exp_lib(A x);
template <> __device__ __forceinline__ double exp_lib<double>(double x) { return exp(x); }
template <> __device__ __forceinline__ float exp_lib<float>(float x) { return expf(x); }

// sin and cos for |x| <= pi/4 from their Taylor series, evaluated by
// Horner's rule in z = x^2.  The first omitted terms, x^17/17! and x^18/18!
// (FP64) or x^11/11! and x^12/12! (FP32), are below half an ulp of the
// result on that interval.
__device__ __forceinline__ void sincos_taylor(double x, double *s, double *c)
{
    const double z = x * x;
    double ps = 1.0 / 1307674368000.0;                  // 1/15!
    ps = fma(ps, -z, 1.0 / 6227020800.0);               // 1/13!
    ps = fma(ps, -z, 1.0 / 39916800.0);                 // 1/11!
    ps = fma(ps, -z, 1.0 / 362880.0);                   // 1/9!
    ps = fma(ps, -z, 1.0 / 5040.0);                     // 1/7!
    ps = fma(ps, -z, 1.0 / 120.0);                      // 1/5!
    ps = fma(ps, -z, 1.0 / 6.0);                        // 1/3!
    *s = fma(-x * z, ps, x);
    double pc = 1.0 / 20922789888000.0;                 // 1/16!
    pc = fma(pc, -z, 1.0 / 87178291200.0);              // 1/14!
    pc = fma(pc, -z, 1.0 / 479001600.0);                // 1/12!
    pc = fma(pc, -z, 1.0 / 3628800.0);                  // 1/10!
    pc = fma(pc, -z, 1.0 / 40320.0);                    // 1/8!
    pc = fma(pc, -z, 1.0 / 720.0);                      // 1/6!
    pc = fma(pc, -z, 1.0 / 24.0);                       // 1/4!
    pc = fma(pc, -z, 0.5);                              // 1/2!
    *c = fma(-z, pc, 1.0);
}

__device__ __forceinline__ void sincos_taylor(float x, float *s, float *c)
{
    const float z = x * x;
    float ps = 1.0f / 362880.0f;                        // 1/9!
    ps = fmaf(ps, -z, 1.0f / 5040.0f);                  // 1/7!
    ps = fmaf(ps, -z, 1.0f / 120.0f);                   // 1/5!
    ps = fmaf(ps, -z, 1.0f / 6.0f);                     // 1/3!
    *s = fmaf(-x * z, ps, x);
    float pc = 1.0f / 3628800.0f;                       // 1/10!
    pc = fmaf(pc, -z, 1.0f / 40320.0f);                 // 1/8!
    pc = fmaf(pc, -z, 1.0f / 720.0f);                   // 1/6!
    pc = fmaf(pc, -z, 1.0f / 24.0f);                    // 1/4!
    pc = fmaf(pc, -z, 0.5f);                            // 1/2!
    *c = fmaf(-z, pc, 1.0f);
}

// sin and cos of any phase: Cody-Waite reduction x = k pi/2 + r,
// |r| <= pi/4, with pi/2 split into three parts (each the correctly rounded
// remainder of pi/2 after the previous ones) applied by fused multiply-adds,
// then the Taylor polynomials on r and the rotation by the quadrant k mod 4.
// The remainder keeps a few ulps for |x| up to about 1e5 (FP64) or 1e3
// (FP32), far beyond any meaningful phase per step.  It is written inline:
// a library call here would make the sweep reserve registers for the call.
template <typename A> struct half_pi;
template <> struct half_pi<double> {
    static constexpr double inv = 0.6366197723675814;             // 2/pi
    static constexpr double p1 = 0x1.921fb54442d18p+0;
    static constexpr double p2 = 0x1.1a62633145c07p-54;
    static constexpr double p3 = -0x1.f1976b7ed8fbcp-110;
};
template <> struct half_pi<float> {
    static constexpr float inv = 0.63661975f;
    static constexpr float p1 = 1.5707963705062866f;
    static constexpr float p2 = -4.371138828673793e-08f;
    static constexpr float p3 = -1.7151245100058819e-15f;
};

template <typename A>
__device__ __forceinline__ void sincos_reduced(A x, A *s, A *c)
{
    using H = half_pi<A>;
    const A k = rint(x * H::inv);
    const A r = fma(-k, H::p3, fma(-k, H::p2, fma(-k, H::p1, x)));
    A sr, cr;
    sincos_taylor(r, &sr, &cr);
    const int q = (int)k & 3;   // |k| < 2^31 for every phase the reduction serves
    A ss = (q & 1) ? cr : sr;
    A cc = (q & 1) ? sr : cr;
    if (q & 2) ss = -ss;
    if ((q + 1) & 2) cc = -cc;
    *s = ss;
    *c = cc;
}

// calcnu phase factor: v * exp(-i phi) (real time) or v * exp(-phi)
// (imaginary time), phi = dt * (V + g|v|^2).
template <bool REAL, typename A>
__device__ __forceinline__ cx<A> nu_factor(cx<A> v, A phi)
{
    if (REAL) {
        // one path for every phase: for |phi| < pi/4 the reduction leaves
        // k = 0 and r = phi exactly
        A sn, cs;
        sincos_reduced(phi, &sn, &cs);
        return cx<A>{fma(v.re, cs, v.im * sn), fma(v.im, cs, -v.re * sn)};
    }
    const A f = exp_lib<A>(-phi);
    return cx<A>{v.re * f, v.im * f};
}

// Real values: imaginary time only, v * exp(-phi).
template <bool REAL, typename A>
__device__ __forceinline__ A nu_factor(A v, A phi)
{
    static_assert(!REAL, "real values carry imaginary-time states only");
    return v * exp_lib<A>(-phi);
}

// calcnu exponent theta = V(x, y, z) + g |v|^2 from the (y, z) trap part of
// the line, each rounding written out (no contraction left to the compiler),
// so a real state held as real or as complex values rounds the same way in
// every kernel shape.
template <typename A>
__device__ __forceinline__ A trap_yz(A hgy, A y, A hgz, A z) { return fma(hgy * y, y, hgz * z * z); }
template <typename A, typename V>
__device__ __forceinline__ A nu_theta(A hgx, A x, A vyz, A g, V v)
{
    return fma(g, cabs2(v), fma(hgx * x, x, vyz));
}

// v * s for either value kind.
template <typename A>
__device__ __forceinline__ cx<A> vscale(cx<A> v, A s) { return cx<A>{v.re * s, v.im * s}; }
template <typename A>
__device__ __forceinline__ A vscale(A v, A s) { return v * s; }

// ---- one x line per wavefront: lane l holds the chunk [l*C, l*C + C) ----

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

template <typename A>
__device__ __forceinline__ A shfl_up_c(A v, int d) { return __shfl_up(v, d, kWave); }
template <typename A>
__device__ __forceinline__ A shfl_down_c(A v, int d) { return __shfl_down(v, d, kWave); }
template <typename A>
__device__ __forceinline__ cx<A> shfl_c(cx<A> v, int src) { return cx<A>{__shfl(v.re, src, kWave), __shfl(v.im, src, kWave)}; }
template <typename A>
__device__ __forceinline__ A shfl_c(A v, int src) { return __shfl(v, src, kWave); }

// LDS slot of line element e: one padding slot after every C elements keeps
// the chunk-order reads (stride C+1 elements between lanes) off one bank.
template <int C>
__device__ __forceinline__ int xslot(int e) { return e + e / C; }

template <typename S, int C>
__device__ __forceinline__ void load_x_row(S (&v)[C], const S *__restrict__ row, int nx)
{
    const int lane = threadIdx.x;
#pragma unroll
    for (int r = 0; r < C; ++r) {
        const int e = r * kWave + lane;
        v[r] = szero<S>();
        if (e < nx) v[r] = stream_load(row + e);
    }
}

}  // namespace gpssc
