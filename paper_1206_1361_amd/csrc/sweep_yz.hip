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
// registers.  The solve is the constant-coefficient factorisation of the x
// kernel: per-chunk recurrences with a zero carry, the carries between chunks
// from a Kogge-Stone scan through LDS, a rerun from the true carry, and the
// rank-one boundary term from the first node.
#include "sweep_common.h"

namespace gpssc {

// Column values of one thread: one column (W = 1) or two neighbouring
// complex64 columns (W = 2, one 16-byte access per row).
template <typename S, typename A, int W>
using col_t = typename std::conditional<W == 2, cx2<A>, value_t<S, A>>::type;

template <typename V, int W, typename S>
__device__ __forceinline__ V load_cols(const S *at)
{
    if constexpr (W == 2) {
        static_assert(std::is_same<S, float2>::value, "column pairs are complex64");
        return stream_load_pair(at);
    } else {
        return ldv<V>(stream_load(at));
    }
}

template <int W, typename S, typename V>
__device__ __forceinline__ void store_cols(S *at, V v)
{
    if constexpr (W == 2)
        stream_store_pair(at, v);
    else
        stream_store(at, stv<S>(v));
}

// Where a thread sits in a tile: xt threads across the columns, p chunks
// along the lines; thread (tx, pc) holds the chunk pc of column tx.  A
// thread with on == false (a block larger than the tile, as in the launch
// over every class of a batch) touches no memory but takes part in every
// barrier of the tile.
struct TileShape {
    int xt, p;
    int tx, pc;
    bool on;
};

// One tile: XT*W neighbouring lines (columns) starting at column `col0`, at
// outer index `outer` (z for the y sweep, y for the z sweep); thread tx holds
// columns col0 + W tx .. col0 + W tx + W - 1 (W = 2 needs an even nx).  Every
// thread of the block executes the same barriers whatever its shape entry.
template <typename S, typename A, int C, bool REAL, bool NORM, int W>
__device__ __forceinline__ void solve_tile_at(S *__restrict__ psi, const SArgs<A> &a,
                                              const cx<A> *__restrict__ zt, double *__restrict__ partials,
                                              unsigned char *smem_raw, int col0, int outer, TileShape sh)
{
    using V = col_t<S, A, W>;
    const int XT = sh.xt;
    const int P = sh.p;
    const int tx = sh.tx;
    const int pc = sh.pc;
    const bool on = sh.on;
    V *b0 = reinterpret_cast<V *>(smem_raw);
    V *b1 = b0 + P * XT;
    const int me = pc * XT + tx;

    const int i = col0 + W * tx;
    const bool act = on && i < a.nx;
    const int pos0 = pc * C;
    const bool full = act && pos0 + C <= a.n;   // whole chunk inside the line
    S *base = psi + (int64_t)outer * a.outer_stride + i + (int64_t)pos0 * a.stride;

    V u[C];
    if (full) {
#pragma unroll
        for (int c = 0; c < C; ++c) u[c] = load_cols<V, W>(base + (int64_t)c * a.stride);
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            u[c] = V{};
            if (act && pos0 + c < a.n) u[c] = load_cols<V, W>(base + (int64_t)c * a.stride);
        }
    }

    // neighbours across chunk borders
    if (on) {
        b0[me] = u[0];
        b1[me] = u[C - 1];
    }
    __syncthreads();
    const V zero = V{};
    const V left = on && pc > 0 ? b1[me - XT] : zero;
    const V right = on && pc < P - 1 ? b0[me + XT] : zero;
    chunk_rhs<REAL>(u, left, right, a.k);

    // forward: local pass, Kogge-Stone over the chunks through LDS, rerun
    V t = chunk_forward<REAL, false>(u, zero, a.k);
    __syncthreads();  // every thread has read its neighbours from b0/b1
    V *cur = b0, *nxt = b1;
    if (on) cur[me] = t;
    __syncthreads();
#pragma unroll
    for (int stg = 0; stg < kMaxStages; ++stg) {
        if (stg < a.k.nst) {
            const int d = 1 << stg;
            if (on && pc >= d) t = kfma<REAL>(a.k.stage[stg], cur[me - d * XT], t);
            if (on) nxt[me] = t;
            __syncthreads();
            V *tmp = cur; cur = nxt; nxt = tmp;
        }
    }
    t = on && pc > 0 ? cur[me - XT] : zero;
    chunk_forward<REAL, true>(u, t, a.k);
    if (pos0 + C > a.n) chunk_clear_padding(u, pos0, a.n);

    // backward
    t = chunk_backward<REAL, false>(u, zero, a.k);
    __syncthreads();  // every thread has read its forward carry
    if (on) nxt[me] = t;
    __syncthreads();
    { V *tmp = cur; cur = nxt; nxt = tmp; }
#pragma unroll
    for (int stg = 0; stg < kMaxStages; ++stg) {
        if (stg < a.k.nst) {
            const int d = 1 << stg;
            if (on && pc + d < P) t = kfma<REAL>(a.k.stage[stg], cur[me + d * XT], t);
            if (on) nxt[me] = t;
            __syncthreads();
            V *tmp = cur; cur = nxt; nxt = tmp;
        }
    }
    t = on && pc < P - 1 ? cur[me + XT] : zero;
    chunk_backward<REAL, true>(u, t, a.k);

    // boundary correction from the first node of each line
    __syncthreads();  // every thread has read its backward carry
    if (on && pc == 0) nxt[tx] = u[0];
    __syncthreads();
    if (on && pos0 < a.k.nzc) chunk_correct<REAL>(u, nxt[tx], zt, pos0, a.k.nzc);

    if (full) {
#pragma unroll
        for (int c = 0; c < C; ++c) store_cols<W>(base + (int64_t)c * a.stride, u[c]);
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (act && pos0 + c < a.n) store_cols<W>(base + (int64_t)c * a.stride, u[c]);
    }

    if (NORM) {
        // sum |psi|^2 of what was stored (rounded to storage), one partial
        // per line (column): over its chunks in order, so the sum does not
        // depend on how many columns a block or a thread holds
        double acc[W];
#pragma unroll
        for (int w = 0; w < W; ++w) acc[w] = 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (act && pos0 + c < a.n) {
                // rounded term by term (no fused multiply-add), the same for
                // complex and real storage
#pragma clang fp contract(off)
                if constexpr (W == 2) {
                    const float2 v0 = st<float2>(u[c].p), v1 = st<float2>(u[c].q);
                    acc[0] += sre(v0) * sre(v0) + sim(v0) * sim(v0);
                    acc[1] += sre(v1) * sre(v1) + sim(v1) * sim(v1);
                } else {
                    const S v = stv<S>(u[c]);
                    acc[0] += sre(v) * sre(v) + sim(v) * sim(v);
                }
            }
        }
        __syncthreads();  // LDS reuse
        double *red = reinterpret_cast<double *>(smem_raw);
        if (on) {
#pragma unroll
            for (int w = 0; w < W; ++w) red[w * P * XT + me] = acc[w];
        }
        __syncthreads();
        if (pc == 0 && act) {
#pragma unroll
            for (int w = 0; w < W; ++w) {
                double col = 0.0;
                for (int q = 0; q < P; ++q) col += red[w * P * XT + q * XT + tx];
                partials[(int64_t)outer * a.nx + i + w] = col;
            }
        }
    }
}

// The tile as the block's own shape: blockDim.x columns, blockDim.y chunks.
template <typename S, typename A, int C, bool REAL, bool NORM, int W>
__device__ __forceinline__ void solve_tile(S *__restrict__ psi, const SArgs<A> &a,
                                           const cx<A> *__restrict__ zt, double *__restrict__ partials,
                                           unsigned char *smem_raw, int col0, int outer)
{
    solve_tile_at<S, A, C, REAL, NORM, W>(
        psi, a, zt, partials, smem_raw, col0, outer,
        TileShape{(int)blockDim.x, (int)blockDim.y, (int)threadIdx.x, (int)threadIdx.y, true});
}

// Tiles are numbered column-tile fastest; the grid has one block per tile
// (G = gridDim.x blocks) and block b solves tile t = b, or with xcd_ranges
// (and G a multiple of 8) t = (b mod 8) G/8 + b/8: blocks are handed to the
// 8 XCDs in turn, so this gives each XCD a contiguous range of tiles, and the
// blocks running on one XCD read neighbouring column tiles (whole rows)
// rather than every eighth one.  A block takes one tile and no more: a loop
// over tiles would keep every argument live across its iterations, more
// uniform values than the scalar registers hold, and the spills into vector
// lanes would cost about an eighth of the kernel's vector instructions.
template <typename S, typename A, int C, bool REAL, bool NORM, int W>
__global__ void __launch_bounds__(kMaxBlockYZ)
calclu_strided_kernel(S *__restrict__ psi, const SArgs<A> a, const cx<A> *__restrict__ zt,
                      double *__restrict__ partials, int ncol_tiles, int ntiles, int xcd_ranges)
{
    extern __shared__ unsigned char smem_raw[];
    const int b = blockIdx.x, G = gridDim.x;
    const int tile = xcd_ranges && G % 8 == 0 ? (b % 8) * (G / 8) + b / 8 : b;
    if (tile >= ntiles) return;
    const int outer = tile / ncol_tiles;
    const int col0 = (tile - outer * ncol_tiles) * (int)blockDim.x * W;
    solve_tile<S, A, C, REAL, NORM, W>(psi, a, zt, partials, smem_raw, col0, outer);
}

// Batched: block b solves tile b % ntiles of solve active[b / ntiles].
// With W = 2 (complex64 column pairs) every solve's psi must be 16-byte
// aligned and its nx even; the host checks both.
template <typename S, typename A, int C, bool REAL, bool NORM, int W>
__global__ void __launch_bounds__(kMaxBlockYZ)
calclu_strided_batch_kernel(S *const *__restrict__ psis, const SBatchArgs<A> *__restrict__ args,
                            const int *__restrict__ active, int ncol_tiles, int ntiles,
                            double *__restrict__ partials, const int64_t *__restrict__ part_off)
{
    extern __shared__ unsigned char smem_raw[];
    const int slot = blockIdx.x / ntiles;
    const int tile = blockIdx.x - slot * ntiles;
    const int si = active[slot];
    const int outer = tile / ncol_tiles;
    const int col0 = (tile - outer * ncol_tiles) * (int)blockDim.x * W;
    solve_tile<S, A, C, REAL, NORM, W>(psis[si], args[si].s, args[si].zt,
                                       NORM ? partials + part_off[si] : partials, smem_raw, col0, outer);
}

// Batched, every class in one launch: class k owns the blocks from
// cls[k].block0 on; a block solves tile b % ntiles of solve active[b /
// ntiles] of its class, with the class's chunking and tile shape, as
// calclu_strided_batch_kernel does.  The block (one dimension) is as large
// as the largest class tile; threads past the class's tile join the
// barriers only.  Registers are those of the largest variant (chunks of at
// most CMAX points).
template <typename S, typename A, int CMAX, bool REAL, bool NORM>
__global__ void __launch_bounds__(kMaxBlockYZ)
calclu_strided_classes_kernel(S *const *__restrict__ psis, const SBatchArgs<A> *__restrict__ args,
                              const YZClassDesc *__restrict__ cls, int ncls, double *__restrict__ partials,
                              const int64_t *__restrict__ part_off)
{
    extern __shared__ unsigned char smem_raw[];
    const int b = blockIdx.x;
    const YZClassDesc c = cls[class_of_block(cls, ncls, b)];
    const int rel = b - c.block0;
    const int slot = rel / c.ntiles;
    const int tile = rel - slot * c.ntiles;
    const int si = c.active[slot];
    const int outer = tile / c.ncol;
    const int col0 = (tile - outer * c.ncol) * c.xt * c.cols;
    const int lin = threadIdx.x;
    const TileShape sh{c.xt, c.lanes, lin % c.xt, lin / c.xt, lin < c.xt * c.lanes};
    double *part = NORM ? partials + part_off[si] : partials;
    constexpr bool kPairs = std::is_same<S, float2>::value && std::is_same<A, float>::value;
#define GP_YC(CC, WW)                                                                                         \
    case CC * 4 + WW:                                                                                         \
        if constexpr (CC <= CMAX && (WW == 1 || kPairs))                                                      \
            solve_tile_at<S, A, CC, REAL, NORM, WW>(psis[si], args[si].s, args[si].zt, part, smem_raw, col0,  \
                                                    outer, sh);                                               \
        break;
    switch (c.chunk * 4 + c.cols) {
        GP_YC(1, 1) GP_YC(2, 1) GP_YC(4, 1) GP_YC(8, 1) GP_YC(16, 1)
        GP_YC(1, 2) GP_YC(2, 2) GP_YC(4, 2) GP_YC(8, 2) GP_YC(16, 2)
    default:
        break;
    }
#undef GP_YC
}

template <typename S, typename A, bool REAL>
static hipError_t launch_classes_yz(int cmax, int threads, size_t lds, int nblocks, hipStream_t stream,
                                    void *const *psis, const void *args, const YZClassDesc *cls, int ncls,
                                    double *partials, const int64_t *part_off)
{
    S *const *p = reinterpret_cast<S *const *>(psis);
    const SBatchArgs<A> *a = static_cast<const SBatchArgs<A> *>(args);
    const dim3 grid((unsigned)nblocks), block((unsigned)threads);
#define GP_YCL(CM)                                                                                           \
    if (partials)                                                                                            \
        hipLaunchKernelGGL((calclu_strided_classes_kernel<S, A, CM, REAL, true>), grid, block, lds, stream, p, \
                           a, cls, ncls, partials, part_off);                                                \
    else                                                                                                     \
        hipLaunchKernelGGL((calclu_strided_classes_kernel<S, A, CM, REAL, false>), grid, block, lds, stream,  \
                           p, a, cls, ncls, partials, part_off);
    if (cmax <= 4) {
        GP_YCL(4)
    } else if (cmax <= 8) {
        GP_YCL(8)
    } else {
        GP_YCL(16)
    }
#undef GP_YCL
    return hipGetLastError();
}

hipError_t launch_strided_classes(Prec prec, bool real, int cmax, int threads, size_t lds_bytes, int nblocks,
                                  void *const *psis, const void *args, const YZClassDesc *cls, int ncls,
                                  double *partials, const int64_t *part_off, hipStream_t stream)
{
    if (real && (prec == PREC_R64 || prec == PREC_R32)) return hipErrorInvalidValue;  // real storage is imaginary time only
    if (nblocks <= 0 || ncls <= 0) return hipSuccess;
    if (cmax < 1 || cmax > 16 || threads < 1 || threads > kMaxBlockYZ || lds_bytes > 65536)
        return hipErrorInvalidValue;
#define GP_YCP(S, A)                                                                                            \
    return real ? launch_classes_yz<S, A, true>(cmax, threads, lds_bytes, nblocks, stream, psis, args, cls, ncls, \
                                                partials, part_off)                                             \
                : launch_classes_yz<S, A, false>(cmax, threads, lds_bytes, nblocks, stream, psis, args, cls, ncls, \
                                                 partials, part_off);
    switch (prec) {
    case PREC_C64: GP_YCP(float2, float)
    case PREC_C64_F64: GP_YCP(float2, double)
    case PREC_C128: GP_YCP(double2, double)
    case PREC_R64:
        return launch_classes_yz<double, double, false>(cmax, threads, lds_bytes, nblocks, stream, psis, args, cls,
                                                        ncls, partials, part_off);
    case PREC_R32:
        return launch_classes_yz<float, float, false>(cmax, threads, lds_bytes, nblocks, stream, psis, args, cls,
                                                      ncls, partials, part_off);
    }
#undef GP_YCP
    return hipErrorInvalidValue;
}

template <typename S, typename A, bool REAL, int W>
static hipError_t launch_batch_tw(int chunk, int xt, int lanes, int nact, int ncol, int ntiles,
                                  void *const *psis, const void *args, const int *active,
                                  double *partials, const int64_t *part_off, hipStream_t stream)
{
    if (xt * lanes > kMaxBlockYZ || lanes > kMaxLanesYZ) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((int64_t)nact * ntiles));
    const dim3 block((unsigned)xt, (unsigned)lanes);
    const size_t lds = 2 * (size_t)xt * lanes * sizeof(col_t<S, A, W>);
    S *const *p = reinterpret_cast<S *const *>(psis);
    const SBatchArgs<A> *a = static_cast<const SBatchArgs<A> *>(args);
#define GP_SB_CASE(CC)                                                                                    \
    case CC:                                                                                              \
        if (partials)                                                                                     \
            hipLaunchKernelGGL((calclu_strided_batch_kernel<S, A, CC, REAL, true, W>), grid, block, lds,   \
                               stream, p, a, active, ncol, ntiles, partials, part_off);                   \
        else                                                                                              \
            hipLaunchKernelGGL((calclu_strided_batch_kernel<S, A, CC, REAL, false, W>), grid, block, lds,  \
                               stream, p, a, active, ncol, ntiles, partials, part_off);                   \
        break;
    switch (chunk) {
        GP_SB_CASE(1) GP_SB_CASE(2) GP_SB_CASE(4) GP_SB_CASE(8) GP_SB_CASE(16)
    default:
        return hipErrorInvalidValue;
    }
#undef GP_SB_CASE
    return hipGetLastError();
}

template <typename S, typename A, bool REAL>
static hipError_t launch_batch_t(int chunk, int xt, int cols, int lanes, int nact, int ncol, int ntiles,
                                 void *const *psis, const void *args, const int *active,
                                 double *partials, const int64_t *part_off, hipStream_t stream)
{
    if (cols == 2) {
        if constexpr (std::is_same<S, float2>::value && std::is_same<A, float>::value)
            return launch_batch_tw<S, A, REAL, 2>(chunk, xt, lanes, nact, ncol, ntiles, psis, args, active,
                                                  partials, part_off, stream);
        return hipErrorInvalidValue;
    }
    if (cols != 1) return hipErrorInvalidValue;
    return launch_batch_tw<S, A, REAL, 1>(chunk, xt, lanes, nact, ncol, ntiles, psis, args, active, partials,
                                          part_off, stream);
}

hipError_t launch_strided_batch(Prec prec, bool real, int chunk, int xt, int cols, int lanes, int nact,
                                int ncol, int ntiles, void *const *psis, const void *args,
                                const int *active, double *partials, const int64_t *part_off,
                                hipStream_t stream)
{
    if (real && (prec == PREC_R64 || prec == PREC_R32)) return hipErrorInvalidValue;  // real storage is imaginary time only
    if (nact <= 0) return hipSuccess;
#define GP_SB_PREC(S, A)                                                                                    \
    return real ? launch_batch_t<S, A, true>(chunk, xt, cols, lanes, nact, ncol, ntiles, psis, args, active, \
                                             partials, part_off, stream)                                    \
                : launch_batch_t<S, A, false>(chunk, xt, cols, lanes, nact, ncol, ntiles, psis, args, active, \
                                              partials, part_off, stream);
    switch (prec) {
    case PREC_C64: GP_SB_PREC(float2, float)
    case PREC_C64_F64: GP_SB_PREC(float2, double)
    case PREC_C128: GP_SB_PREC(double2, double)
    // real storage: imaginary time only (real time was refused above)
    case PREC_R64:
        return launch_batch_t<double, double, false>(chunk, xt, cols, lanes, nact, ncol, ntiles, psis, args,
                                                     active, partials, part_off, stream);
    case PREC_R32:
        return launch_batch_t<float, float, false>(chunk, xt, cols, lanes, nact, ncol, ntiles, psis, args,
                                                   active, partials, part_off, stream);
    }
#undef GP_SB_PREC
    return hipErrorInvalidValue;
}

template <typename S, typename A, bool REAL, int W>
static hipError_t launch_tw(int chunk, int xt, int nouter, void *psi, const void *args,
                            const void *zt, double *partials, int xcd, hipStream_t stream)
{
    const SArgs<A> &a = *static_cast<const SArgs<A> *>(args);
    const int P = a.lanes;
    if (xt * P > kMaxBlockYZ || P > kMaxLanesYZ) return hipErrorInvalidValue;
    if (W == 2 && (a.nx % 2 != 0 || a.stride % 2 != 0 || a.outer_stride % 2 != 0 ||
                   reinterpret_cast<uintptr_t>(psi) % 16 != 0))
        return hipErrorInvalidValue;
    const int ncol = (a.nx + xt * W - 1) / (xt * W);
    const int ntiles = ncol * nouter;
    const dim3 grid((unsigned)ntiles);
    const dim3 block((unsigned)xt, (unsigned)P);
    const size_t lds = 2 * (size_t)xt * P * sizeof(col_t<S, A, W>);
    S *p = static_cast<S *>(psi);
    const cx<A> *z = static_cast<const cx<A> *>(zt);
#define GP_S_CASE(CC)                                                                              \
    case CC:                                                                                       \
        if (partials)                                                                              \
            hipLaunchKernelGGL((calclu_strided_kernel<S, A, CC, REAL, true, W>), grid, block, lds,  \
                               stream, p, a, z, partials, ncol, ntiles, xcd);                      \
        else                                                                                       \
            hipLaunchKernelGGL((calclu_strided_kernel<S, A, CC, REAL, false, W>), grid, block, lds, \
                               stream, p, a, z, partials, ncol, ntiles, xcd);                      \
        break;
    switch (chunk) {
        GP_S_CASE(1) GP_S_CASE(2) GP_S_CASE(4) GP_S_CASE(8) GP_S_CASE(16)
    default:
        return hipErrorInvalidValue;
    }
#undef GP_S_CASE
    return hipGetLastError();
}

template <typename S, typename A, bool REAL>
static hipError_t launch_t(int chunk, int xt, int cols, int nouter, void *psi, const void *args,
                           const void *zt, double *partials, int xcd, hipStream_t stream)
{
    if (cols == 2) {
        if constexpr (std::is_same<S, float2>::value && std::is_same<A, float>::value)
            return launch_tw<S, A, REAL, 2>(chunk, xt, nouter, psi, args, zt, partials, xcd, stream);
        return hipErrorInvalidValue;
    }
    if (cols != 1) return hipErrorInvalidValue;
    return launch_tw<S, A, REAL, 1>(chunk, xt, nouter, psi, args, zt, partials, xcd, stream);
}

hipError_t launch_strided(Prec prec, bool real, int chunk, int xt, int cols, int nouter,
                          void *psi, const void *args, const void *zt, double *partials, bool xcd_ranges,
                          hipStream_t stream)
{
    if (real && (prec == PREC_R64 || prec == PREC_R32)) return hipErrorInvalidValue;  // real storage is imaginary time only
    const int xcd = xcd_ranges ? 1 : 0;
#define GP_S_PREC(S, A)                                                                                      \
    return real ? launch_t<S, A, true>(chunk, xt, cols, nouter, psi, args, zt, partials, xcd, stream) \
                : launch_t<S, A, false>(chunk, xt, cols, nouter, psi, args, zt, partials, xcd, stream);
    switch (prec) {
    case PREC_C64: GP_S_PREC(float2, float)
    case PREC_C64_F64: GP_S_PREC(float2, double)
    case PREC_C128: GP_S_PREC(double2, double)
    // real storage: imaginary time only (real time was refused above)
    case PREC_R64:
        return launch_t<double, double, false>(chunk, xt, cols, nouter, psi, args, zt, partials, xcd,
                                               stream);
    case PREC_R32:
        return launch_t<float, float, false>(chunk, xt, cols, nouter, psi, args, zt, partials, xcd,
                                             stream);
    }
#undef GP_S_PREC
    return hipErrorInvalidValue;
}

}  // namespace gpssc
