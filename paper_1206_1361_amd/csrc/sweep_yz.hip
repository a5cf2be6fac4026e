// sweep_yz.hip -- calcluy / calcluz: the Crank-Nicolson solves along y and z.
//
// Paper: "Summary of revisions" names calcluy and calcluz (the y and z parts
// of the split-step Crank-Nicolson time evolution) and calcnorm; the z kernel
// also produces the per-block partial sums the imaginary-time
// renormalisation needs.
//
// Lines run across memory with stride Nx (y) or Nx*Ny (z), so lanes are laid
// along x: a block covers XT neighbouring lines (one per threadIdx.x, so every
// load and store of a row of the block is one contiguous segment) and cuts
// each line into P = blockDim.y contiguous chunks of C points held in
// registers.  Thomas runs per chunk with a zero carry; the carries between
// chunks come from a Kogge-Stone scan through LDS whose stage multipliers are
// precomputed on the host; each chunk then reruns from its true carry.
#include "gp_internal.h"

namespace gpssc {

template <typename S, typename A, int C, bool NORM>
__global__ void __launch_bounds__(kMaxBlockYZ)
calclu_strided_kernel(S *__restrict__ psi, const SArgs<A> a, const cx<A> *__restrict__ mtab,
                      const cx<A> *__restrict__ scan, double *__restrict__ partials)
{
    extern __shared__ unsigned char smem_raw[];
    const int XT = blockDim.x;
    const int P = blockDim.y;
    const int tx = threadIdx.x;
    const int pc = threadIdx.y;
    cx<A> *b0 = reinterpret_cast<cx<A> *>(smem_raw);
    cx<A> *b1 = b0 + P * XT;
    const int me = pc * XT + tx;

    const int i = blockIdx.x * XT + tx;
    const bool act = i < a.nx;
    S *base = psi + (int64_t)blockIdx.y * a.outer_stride + i;

    cx<A> u[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int pos = pc * C + c;
        u[c] = cx<A>{0, 0};
        if (act && pos < a.n) u[c] = ld<A>(base[(int64_t)pos * a.stride]);
    }

    // neighbours across chunk borders
    b0[me] = u[0];
    b1[me] = u[C - 1];
    __syncthreads();
    const cx<A> left = pc > 0 ? b1[me - XT] : cx<A>{0, 0};
    const cx<A> right = pc < P - 1 ? b0[me + XT] : cx<A>{0, 0};

    cx<A> q[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const cx<A> lo = c > 0 ? u[c - 1] : left;
        const cx<A> hi = c < C - 1 ? u[c + 1] : right;
        q[c] = cfma(a.ro, cadd(lo, hi), cmul(a.rd, u[c]));
    }

    const cx<A> mo = cx<A>{-a.o.re, -a.o.im};
    cx<A> am[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const cx<A> m = mtab[pc * C + c];
        q[c] = cmul(m, q[c]);
        am[c] = cmul(mo, m);
    }

    // forward elimination
    cx<A> t = cx<A>{0, 0};
#pragma unroll
    for (int c = 0; c < C; ++c) t = cfma(am[c], t, q[c]);
    __syncthreads();  // every thread has read its neighbours from b0/b1
    cx<A> *cur = b0, *nxt = b1;
    cur[me] = t;
    __syncthreads();
    for (int stg = 0; stg < a.nst_f; ++stg) {
        const int d = 1 << stg;
        if (pc >= d) t = cfma(scan[stg * P + pc], cur[me - d * XT], t);
        nxt[me] = t;
        __syncthreads();
        cx<A> *tmp = cur; cur = nxt; nxt = tmp;
    }
    t = pc > 0 ? cur[me - XT] : cx<A>{0, 0};
#pragma unroll
    for (int c = 0; c < C; ++c) {
        t = cfma(am[c], t, q[c]);
        q[c] = t;
    }

    // back substitution
    t = cx<A>{0, 0};
#pragma unroll
    for (int c = C - 1; c >= 0; --c) t = cfma(am[c], t, q[c]);
    __syncthreads();  // every thread has read its forward carry
    nxt[me] = t;
    __syncthreads();
    { cx<A> *tmp = cur; cur = nxt; nxt = tmp; }
    for (int stg = 0; stg < a.nst_b; ++stg) {
        const int d = 1 << stg;
        if (pc + d < P) t = cfma(scan[(kMaxStages + stg) * P + pc], cur[me + d * XT], t);
        nxt[me] = t;
        __syncthreads();
        cx<A> *tmp = cur; cur = nxt; nxt = tmp;
    }
    t = pc < P - 1 ? cur[me + XT] : cx<A>{0, 0};
#pragma unroll
    for (int c = C - 1; c >= 0; --c) {
        t = cfma(am[c], t, q[c]);
        q[c] = t;
    }

#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int pos = pc * C + c;
        if (act && pos < a.n) base[(int64_t)pos * a.stride] = st<S>(q[c]);
    }

    if (NORM) {
        // sum |psi|^2 of what was stored (rounded to storage), fixed order
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int pos = pc * C + c;
            if (act && pos < a.n) {
                const S v = st<S>(q[c]);
                acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
            }
        }
        // block sum by a fixed LDS tree (the block size need not be a
        // multiple of the wavefront)
        __syncthreads();  // LDS reuse
        double *red = reinterpret_cast<double *>(smem_raw);
        const int nthreads = XT * P;
        int npow2 = 1;
        while (npow2 < nthreads) npow2 <<= 1;
        red[me] = acc;
        for (int idx = me + nthreads; idx < npow2; idx += nthreads) red[idx] = 0.0;
        __syncthreads();
        for (int h = npow2 >> 1; h > 0; h >>= 1) {
            if (me < h) red[me] += red[me + h];
            __syncthreads();
        }
        if (me == 0) partials[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = red[0];
    }
}

template <typename S, typename A>
static hipError_t launch_t(int chunk, int xt, int nouter, void *psi, const void *args,
                           const void *m, const void *scan, double *partials,
                           hipStream_t stream)
{
    const SArgs<A> &a = *static_cast<const SArgs<A> *>(args);
    const int P = a.lanes;
    if (xt * P > kMaxBlockYZ || P > kMaxLanesYZ) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((a.nx + xt - 1) / xt), (unsigned)nouter);
    const dim3 block((unsigned)xt, (unsigned)P);
    const size_t lds = 2 * (size_t)xt * P * sizeof(cx<A>);
    S *p = static_cast<S *>(psi);
    const cx<A> *mt = static_cast<const cx<A> *>(m);
    const cx<A> *sc = static_cast<const cx<A> *>(scan);
#define GP_S_CASE(CC)                                                                     \
    case CC:                                                                              \
        if (partials)                                                                     \
            hipLaunchKernelGGL((calclu_strided_kernel<S, A, CC, true>), grid, block, lds, \
                               stream, p, a, mt, sc, partials);                           \
        else                                                                              \
            hipLaunchKernelGGL((calclu_strided_kernel<S, A, CC, false>), grid, block, lds, \
                               stream, p, a, mt, sc, partials);                           \
        break;
    switch (chunk) {
        GP_S_CASE(1) GP_S_CASE(2) GP_S_CASE(4) GP_S_CASE(8) GP_S_CASE(16)
    default:
        return hipErrorInvalidValue;
    }
#undef GP_S_CASE
    return hipGetLastError();
}

hipError_t launch_strided(Prec prec, int chunk, int xt, int nouter, void *psi,
                          const void *args, const void *m, const void *scan,
                          double *partials, hipStream_t stream)
{
    switch (prec) {
    case PREC_C64:
        return launch_t<float2, float>(chunk, xt, nouter, psi, args, m, scan, partials, stream);
    case PREC_C64_F64:
        return launch_t<float2, double>(chunk, xt, nouter, psi, args, m, scan, partials, stream);
    case PREC_C128:
        return launch_t<double2, double>(chunk, xt, nouter, psi, args, m, scan, partials, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace gpssc
