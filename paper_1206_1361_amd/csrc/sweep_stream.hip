// sweep_stream.hip -- calcluy / calcluz by streaming along the lines.
//
// Paper: "Summary of revisions" names calcluy and calcluz (the y and z parts
// of the split-step Crank-Nicolson time evolution) and calcnorm; the last
// sweep also leaves the per-line partial sums of the imaginary-time
// renormalisation.
//
// One lane per line (or per pair of neighbouring complex64 lines): the 64
// lanes of a wavefront take 64 neighbouring columns of the plane across the
// lines, so every load and store of a row is one contiguous segment (1 KiB
// for complex128), and the wavefront walks along its lines in blocks of B
// points.  It solves the constant-coefficient factorisation of the chunked
// kernel (SweepCoef): the forward recurrence w_i = m r_i + a w_{i-1} runs
// exactly, in order; the backward recurrence y_i = w_i + a y_{i+1} of a block
// starts B - 1 points past the block's end from y = 0.  Its true start value
// reaches the block's last point multiplied by a^B, and the plan takes this
// strategy only when |a|^B is below 2^-60 (FP64 arithmetic) or 2^-30 (FP32)
// -- far below the rounding of the result -- so the lines are solved to
// rounding, as by the chunked scan.  No LDS and no barriers: waves run
// independently, each keeping the next block's loads in flight while it
// solves the current one.
#include "sweep_common.h"

// Threads per block (independent wavefronts; blocks only group them for
// dispatch) and the fewest wavefronts per SIMD the register allocation must
// allow.
#ifndef GPSSC_STREAM_THREADS
#define GPSSC_STREAM_THREADS 256
#endif
#ifndef GPSSC_STREAM_MIN_WAVES
#define GPSSC_STREAM_MIN_WAVES 1
#endif

namespace gpssc {

namespace {

template <typename S, typename A, int W>
using scol_t = typename std::conditional<W == 2, cx2<A>, value_t<S, A>>::type;

// psi is addressed through a buffer resource whose base moves with the
// block: the lane's column offset is the one per-lane register, the offset
// of a point inside the block is uniform (a scalar register), so the loads
// and stores of a block need no per-lane address arithmetic.  The resource
// spans exactly the rest of psi after its base; the hardware returns zero
// for a load and drops a store past it.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBufNT = GPSSC_NT_LOAD ? 2 : 0;     // nontemporal
constexpr int kBufNTStore = GPSSC_NT_STORE ? 2 : 0;

template <typename S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t psi_rsrc(S *base, int64_t bytes_left)
{
    const int n = bytes_left > 0x7fffffffLL ? 0x7fffffff : (int)bytes_left;
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, n, 0x00020000);
}

template <typename V, int W, typename S>
__device__ __forceinline__ V bload(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    if constexpr (W == 2) {
        const f32x4 v = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, kBufNT));
        return V{cx<float>{v.x, v.y}, cx<float>{v.z, v.w}};
    } else if constexpr (std::is_same<S, double2>::value) {
        const f64x2 v = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, kBufNT));
        return ldv<V>(double2{v.x, v.y});
    } else if constexpr (std::is_same<S, float2>::value) {
        const f32x2 v = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, kBufNT));
        float2 f;
        f.x = v.x;
        f.y = v.y;
        return ldv<V>(f);
    } else if constexpr (std::is_same<S, double>::value) {
        return ldv<V>(__builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, kBufNT)));
    } else {
        return ldv<V>(__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, kBufNT)));
    }
}

template <int W, typename S, typename V>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, int voff, int soff, V v)
{
    if constexpr (W == 2) {
        const f32x4 q = {v.p.re, v.p.im, v.q.re, v.q.im};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, q), r, voff, soff, kBufNTStore);
    } else if constexpr (std::is_same<S, double2>::value) {
        const double2 d = stv<S>(v);
        const f64x2 q = {d.x, d.y};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, q), r, voff, soff, kBufNTStore);
    } else if constexpr (std::is_same<S, float2>::value) {
        const float2 f = stv<S>(v);
        const f32x2 q = {f.x, f.y};
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, q), r, voff, soff, kBufNTStore);
    } else if constexpr (std::is_same<S, double>::value) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, stv<S>(v)), r, voff, soff, kBufNTStore);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, stv<S>(v)), r, voff, soff,
                                              kBufNTStore);
    }
}

// The lanes' view of psi for one block of B points starting at p0: the
// resource based at the wave's first column and point p0, the lane's column
// offset in bytes, the point stride in bytes.
template <typename S>
struct BlockView {
    __amdgpu_buffer_rsrc_t r;
    int voff;
    int sstride;
};

template <typename S>
__device__ __forceinline__ BlockView<S> block_view(S *wave_base, int64_t wave_elem0, int64_t total, int voff,
                                                   int64_t stride, int p0)
{
    const int64_t e0 = wave_elem0 + (int64_t)p0 * stride;
    return BlockView<S>{psi_rsrc(wave_base + (int64_t)p0 * stride, (total - e0) * (int64_t)sizeof(S)), voff,
                        (int)(stride * (int64_t)sizeof(S))};
}

template <typename V, int W, typename S, int B>
__device__ __forceinline__ void load_block(V (&dst)[B], const BlockView<S> &bv, int p0, int n, bool act)
{
    if (act && p0 + B <= n) {
#pragma unroll
        for (int c = 0; c < B; ++c) dst[c] = bload<V, W, S>(bv.r, bv.voff, c * bv.sstride);
    } else {
#pragma unroll
        for (int c = 0; c < B; ++c) {
            dst[c] = V{};
            if (act && p0 + c < n) dst[c] = bload<V, W, S>(bv.r, bv.voff, c * bv.sstride);
        }
    }
}

// |psi|^2 of a stored value, rounded to storage, term by term (no fused
// multiply-add) as in the chunked kernel.
template <typename S, typename A, int W>
__device__ __forceinline__ void add_norm(double (&acc)[W], scol_t<S, A, W> v)
{
#pragma clang fp contract(off)
    if constexpr (W == 2) {
        const float2 v0 = st<float2>(v.p), v1 = st<float2>(v.q);
        acc[0] += sre(v0) * sre(v0) + sim(v0) * sim(v0);
        acc[1] += sre(v1) * sre(v1) + sim(v1) * sim(v1);
    } else {
        const S s = stv<S>(v);
        acc[0] += sre(s) * sre(s) + sim(s) * sim(s);
    }
}

// One block step.  On entry:
//   cur[0 .. B-2]  w of block b (positions b B ...), cur[B-1] the raw value
//                  of its last position (its right neighbour was not loaded);
//   nxt[]          the raw values of block b + 1;
//   um2, wm2       raw value and w at position b B + B - 2;
//   fut[]          free: receives the loads of block b + 2.
// On exit cur holds the solved block b (stored), nxt the w of block b + 1 in
// the same form as cur on entry, fut the raw block b + 2.
template <typename S, typename A, int B, bool REAL, bool NORM, int W, typename V>
__device__ __forceinline__ void stream_block(V (&cur)[B], V (&nxt)[B], V (&fut)[B], V &um2, V &wm2, V &y0,
                                             double (&acc)[W], S *wave_base, int64_t wave_elem0, int64_t total,
                                             int voff, int64_t stride, int b, int n, bool act,
                                             const SweepCoef<A> &k, const cx<A> *__restrict__ zt)
{
    const int p0 = b * B;
    const int nb = (n + B - 1) / B;
    if (b + 2 < nb)
        load_block<V, W, S, B>(fut, block_view(wave_base, wave_elem0, total, voff, stride, p0 + 2 * B), p0 + 2 * B,
                               n, act);
    else {
#pragma unroll
        for (int c = 0; c < B; ++c) fut[c] = V{};
    }

    // finish the last position of block b: its right neighbour is nxt[0]
    const V ulast = cur[B - 1];
    {
        const V r = kmul<REAL>(k.m, cn_rhs<REAL>(k.kap, um2, ulast, nxt[0]));
        cur[B - 1] = p0 + B - 1 < n ? kfma<REAL>(k.a, wm2, r) : V{};
    }
    // right-hand side and forward recurrence of block b + 1 except its last
    // position; zero past the end of the line
    V prev = ulast, w = cur[B - 1];
#pragma unroll
    for (int c = 0; c < B - 1; ++c) {
        const V u = nxt[c];
        const V r = kmul<REAL>(k.m, cn_rhs<REAL>(k.kap, prev, u, nxt[c + 1]));
        prev = u;
        w = p0 + B + c < n ? kfma<REAL>(k.a, w, r) : V{};
        nxt[c] = w;
    }
    um2 = prev;
    wm2 = w;

    // backward recurrence: from y = 0 at position b B + 2B - 1 down through
    // the first B - 1 points of block b + 1, then block b
    V t{};
#pragma unroll
    for (int c = B - 2; c >= 0; --c) t = kfma<REAL>(k.a, t, nxt[c]);
#pragma unroll
    for (int c = B - 1; c >= 0; --c) {
        t = kfma<REAL>(k.a, t, cur[c]);
        cur[c] = t;
    }

    // boundary correction from the first node
    if (b == 0) y0 = cur[0];
    if (p0 < k.nzc) {
#pragma unroll
        for (int c = 0; c < B; ++c)
            if (p0 + c < k.nzc) cur[c] = kfma<REAL>(zt[p0 + c], y0, cur[c]);
    }

    const BlockView<S> bv = block_view(wave_base, wave_elem0, total, voff, stride, p0);
    if (act && p0 + B <= n) {
#pragma unroll
        for (int c = 0; c < B; ++c) bstore<W, S>(bv.r, bv.voff, c * bv.sstride, cur[c]);
    } else {
#pragma unroll
        for (int c = 0; c < B; ++c)
            if (act && p0 + c < n) bstore<W, S>(bv.r, bv.voff, c * bv.sstride, cur[c]);
    }
    if (NORM) {
#pragma unroll
        for (int c = 0; c < B; ++c)
            if (p0 + c < n) add_norm<S, A, W>(acc, cur[c]);
    }
}

// The lines of column `col` (W columns from it): column c of the plane across
// the lines starts at element (c / nx) * outer_stride + c % nx.  col0 is the
// wave's first column (the same in every lane).
template <typename S, typename A, int B, bool REAL, bool NORM, int W>
__device__ __forceinline__ void stream_columns(S *__restrict__ psi, const SArgs<A> &a, const cx<A> *__restrict__ zt,
                                               double *__restrict__ partials, int64_t col, int64_t col0,
                                               int64_t ncols, int64_t total)
{
    using V = scol_t<S, A, W>;
    const bool act = col < ncols;
    const int64_t cc = act ? col : col0;
    const int64_t elem0 = (col0 / a.nx) * a.outer_stride + col0 % a.nx;
    const int64_t elem = (cc / a.nx) * a.outer_stride + cc % a.nx;
    S *wave_base = psi + elem0;
    const int voff = (int)((elem - elem0) * (int64_t)sizeof(S));
    const int n = a.n;
    const int64_t stride = a.stride;
    const SweepCoef<A> &k = a.k;

    V P[B], Q[B], R[B];
    load_block<V, W, S, B>(P, block_view(wave_base, elem0, total, voff, stride, 0), 0, n, act);
    if (B < n)
        load_block<V, W, S, B>(Q, block_view(wave_base, elem0, total, voff, stride, B), B, n, act);
    else {
#pragma unroll
        for (int c = 0; c < B; ++c) Q[c] = V{};
    }
    // block 0 except its last position, from the zero ghost and zero carry
    V prev{}, w{};
#pragma unroll
    for (int c = 0; c < B - 1; ++c) {
        const V u = P[c];
        const V r = kmul<REAL>(k.m, cn_rhs<REAL>(k.kap, prev, u, P[c + 1]));
        prev = u;
        w = c < n ? kfma<REAL>(k.a, w, r) : V{};
        P[c] = w;
    }
    V um2 = prev, wm2 = w, y0{};
    double acc[W];
#pragma unroll
    for (int q = 0; q < W; ++q) acc[q] = 0.0;

    const int nb = (n + B - 1) / B;
    for (int b = 0;;) {
        stream_block<S, A, B, REAL, NORM, W>(P, Q, R, um2, wm2, y0, acc, wave_base, elem0, total, voff, stride, b, n,
                                             act, k, zt);
        if (++b >= nb) break;
        stream_block<S, A, B, REAL, NORM, W>(Q, R, P, um2, wm2, y0, acc, wave_base, elem0, total, voff, stride, b, n,
                                             act, k, zt);
        if (++b >= nb) break;
        stream_block<S, A, B, REAL, NORM, W>(R, P, Q, um2, wm2, y0, acc, wave_base, elem0, total, voff, stride, b, n,
                                             act, k, zt);
        if (++b >= nb) break;
    }
    if (NORM && act) {
#pragma unroll
        for (int q = 0; q < W; ++q) partials[cc + q] = acc[q];
    }
}

}  // namespace

// Thread t of the grid takes columns W t .. W t + W - 1 of the ncols columns
// across the lines (ncols = nx * nouter).
template <typename S, typename A, int B, bool REAL, bool NORM, int W>
__global__ void __launch_bounds__(GPSSC_STREAM_THREADS, GPSSC_STREAM_MIN_WAVES)
calclu_stream_kernel(S *__restrict__ psi, const SArgs<A> a, const cx<A> *__restrict__ zt,
                     double *__restrict__ partials, int64_t ncols, int64_t total)
{
    const int64_t col = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * W;
    const int64_t col0 = ((int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(kWave - 1))) * W;
    stream_columns<S, A, B, REAL, NORM, W>(psi, a, zt, partials, col, col0, ncols, total);
}

template <typename S, typename A, bool REAL, int W>
static hipError_t launch_stream_tw(int blk, int nouter, void *psi, const void *args, const void *zt,
                                   double *partials, hipStream_t stream)
{
    const SArgs<A> &a = *static_cast<const SArgs<A> *>(args);
    if (W == 2 && (a.nx % 2 != 0 || a.stride % 2 != 0 || a.outer_stride % 2 != 0 ||
                   reinterpret_cast<uintptr_t>(psi) % 16 != 0))
        return hipErrorInvalidValue;
    const int64_t ncols = (int64_t)a.nx * nouter;
    const int64_t total = ncols * a.n;   // elements of psi: nx * n * nouter
    const int64_t threads = (ncols + W - 1) / W;
    const dim3 block(GPSSC_STREAM_THREADS);
    const dim3 grid((unsigned)((threads + GPSSC_STREAM_THREADS - 1) / GPSSC_STREAM_THREADS));
    S *p = static_cast<S *>(psi);
    const cx<A> *z = static_cast<const cx<A> *>(zt);
#define GP_ST_CASE(BB)                                                                                             \
    case BB:                                                                                                       \
        if (partials)                                                                                              \
            hipLaunchKernelGGL((calclu_stream_kernel<S, A, BB, REAL, true, W>), grid, block, 0, stream, p, a, z,   \
                               partials, ncols, total);                                                            \
        else                                                                                                       \
            hipLaunchKernelGGL((calclu_stream_kernel<S, A, BB, REAL, false, W>), grid, block, 0, stream, p, a, z,  \
                               partials, ncols, total);                                                            \
        break;
    switch (blk) {
        GP_ST_CASE(8) GP_ST_CASE(12) GP_ST_CASE(16)
    default:
        return hipErrorInvalidValue;
    }
#undef GP_ST_CASE
    return hipGetLastError();
}

template <typename S, typename A, bool REAL>
static hipError_t launch_stream_t(int blk, int cols, int nouter, void *psi, const void *args, const void *zt,
                                  double *partials, hipStream_t stream)
{
    if (cols == 2) {
        if constexpr (std::is_same<S, float2>::value && std::is_same<A, float>::value)
            return launch_stream_tw<S, A, REAL, 2>(blk, nouter, psi, args, zt, partials, stream);
        return hipErrorInvalidValue;
    }
    if (cols != 1) return hipErrorInvalidValue;
    return launch_stream_tw<S, A, REAL, 1>(blk, nouter, psi, args, zt, partials, stream);
}

hipError_t launch_stream(Prec prec, bool real, int blk, int cols, int nouter, void *psi, const void *args,
                         const void *zt, double *partials, hipStream_t stream)
{
    if (real && (prec == PREC_R64 || prec == PREC_R32)) return hipErrorInvalidValue;  // real storage is imaginary time only
#define GP_ST_PREC(S, A)                                                                                  \
    return real ? launch_stream_t<S, A, true>(blk, cols, nouter, psi, args, zt, partials, stream)        \
                : launch_stream_t<S, A, false>(blk, cols, nouter, psi, args, zt, partials, stream);
    switch (prec) {
    case PREC_C64: GP_ST_PREC(float2, float)
    case PREC_C64_F64: GP_ST_PREC(float2, double)
    case PREC_C128: GP_ST_PREC(double2, double)
    // real storage: imaginary time only (real time was refused above)
    case PREC_R64:
        return launch_stream_t<double, double, false>(blk, cols, nouter, psi, args, zt, partials, stream);
    case PREC_R32:
        return launch_stream_t<float, float, false>(blk, cols, nouter, psi, args, zt, partials, stream);
    }
#undef GP_ST_PREC
    return hipErrorInvalidValue;
}

}  // namespace gpssc
