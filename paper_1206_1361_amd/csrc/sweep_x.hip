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
// in row order, written back through the same LDS buffer.  solve_x_lines
// below runs the same steps on several lines at once; this one-line form is
// kept apart because at 8-point FP64 chunks its register allocation stays
// within 128 VGPRs (four wavefronts per SIMD) where the several-line form's
// does not.
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
    const A vyz = trap_yz(a.hgy, y, a.hgz, z);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const V v = vscale(u[c], s);
        const A x = ((A)(pos0 + c) - a.c0x) * a.dx;
        const A theta = nu_theta(a.hgx, x, vyz, a.g, v);
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

// L x lines at once: psi values in row order (line l, element r*64 + lane)
// -> solved lines, in row order, written back through LDS (one slice of
// 64*C + 64 elements per line).  The lines are independent; a wavefront runs
// them in one instruction stream so that their loads, shuffles and LDS
// round trips overlap, and every line sees exactly the arithmetic of a line
// solved alone.
template <typename A>
struct XLine {
    const cx<A> *zt;           // boundary correction of the line's grid
    A s;                       // pending renormalisation factor
    int line;                  // j + ny k
};

// args_of(l): the XArgs of line l's grid (sizes, trap, coefficients);
// ln(l): its XLine.
template <typename S, typename A, int C, int L, bool REAL, typename ArgsOf, typename LineOf>
__device__ __forceinline__ void solve_x_lines(S (&rows)[L][C], S *buf, ArgsOf args_of, LineOf ln)
{
    using V = value_t<S, A>;
    constexpr int SL = kWave * C + kWave;
    const int lane = threadIdx.x;
    const int pos0 = lane * C;

#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
        for (int r = 0; r < C; ++r) buf[l * SL + xslot<C>(r * kWave + lane)] = rows[l][r];
    __syncthreads();
    V u[L][C];
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
        for (int c = 0; c < C; ++c) u[l][c] = ldv<V>(buf[l * SL + lane * (C + 1) + c]);

    // calcnu: pending renormalisation, then exp(-tau (V + g|psi|^2)).
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const XArgs<A> &a = args_of(l);
        const int j = ln(l).line % a.ny;
        const int k = ln(l).line / a.ny;
        const A y = ((A)j - a.c0y) * a.dy;
        const A z = ((A)k - a.c0z) * a.dz;
        const A vyz = trap_yz(a.hgy, y, a.hgz, z);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const V v = vscale(u[l][c], ln(l).s);
            const A x = ((A)(pos0 + c) - a.c0x) * a.dx;
            const A theta = nu_theta(a.hgx, x, vyz, a.g, v);
            u[l][c] = nu_factor<REAL>(v, a.dt * theta);   // padding stays 0
        }
    }

    // right-hand side with zero ghosts; neighbours across chunk borders come
    // from the adjacent lanes
#pragma unroll
    for (int l = 0; l < L; ++l) {
        V left = shfl_up_c(u[l][C - 1], 1);
        V right = shfl_down_c(u[l][0], 1);
        if (lane == 0) left = V{};
        if (lane == kWave - 1) right = V{};
        chunk_rhs<REAL>(u[l], left, right, args_of(l).k);
    }

    // forward: local pass with zero carry, Kogge-Stone across lanes, rerun
    V t[L];
#pragma unroll
    for (int l = 0; l < L; ++l) t[l] = chunk_forward<REAL, false>(u[l], V{}, args_of(l).k);
#pragma unroll
    for (int st = 0; st < kMaxStages; ++st) {
#pragma unroll
        for (int l = 0; l < L; ++l) {
            if (st < args_of(l).k.nst) {
                const V from = shfl_up_c(t[l], 1 << st);
                if (lane >= (1 << st)) t[l] = kfma<REAL>(args_of(l).k.stage[st], from, t[l]);
            }
        }
    }
#pragma unroll
    for (int l = 0; l < L; ++l) {
        t[l] = shfl_up_c(t[l], 1);
        if (lane == 0) t[l] = V{};
        chunk_forward<REAL, true>(u[l], t[l], args_of(l).k);
        if (args_of(l).nx < kWave * C) chunk_clear_padding(u[l], pos0, args_of(l).nx);
    }

    // backward: the same from the right
#pragma unroll
    for (int l = 0; l < L; ++l) t[l] = chunk_backward<REAL, false>(u[l], V{}, args_of(l).k);
#pragma unroll
    for (int st = 0; st < kMaxStages; ++st) {
#pragma unroll
        for (int l = 0; l < L; ++l) {
            if (st < args_of(l).k.nst) {
                const V from = shfl_down_c(t[l], 1 << st);
                if (lane + (1 << st) < kWave) t[l] = kfma<REAL>(args_of(l).k.stage[st], from, t[l]);
            }
        }
    }
#pragma unroll
    for (int l = 0; l < L; ++l) {
        t[l] = shfl_down_c(t[l], 1);
        if (lane == kWave - 1) t[l] = V{};
        chunk_backward<REAL, true>(u[l], t[l], args_of(l).k);
    }

    // boundary correction from the first node
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const V y0 = shfl_c(u[l][0], 0);
        if (pos0 < args_of(l).k.nzc) chunk_correct<REAL>(u[l], y0, ln(l).zt, pos0, args_of(l).k.nzc);
    }

    // chunk order -> LDS -> row order
    __syncthreads();
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
        for (int c = 0; c < C; ++c) buf[l * SL + lane * (C + 1) + c] = stv<S>(u[l][c]);
    __syncthreads();
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
        for (int r = 0; r < C; ++r) rows[l][r] = buf[l * SL + xslot<C>(r * kWave + lane)];
}

template <typename S, int C>
__device__ __forceinline__ void store_x_row(S *__restrict__ row, const S (&v)[C], int nx)
{
    const int lane = threadIdx.x;
#pragma unroll
    for (int r = 0; r < C; ++r) {
        const int e = r * kWave + lane;
        if (e < nx) stream_store(row + e, v[r]);
    }
}

// One wavefront per block; block b solves line b (the grid has one block
// per line).  A block takes one line and no more: a loop over lines would
// keep every argument live across its iterations, more uniform values than
// the scalar registers hold, and the spills into vector lanes would cost
// about a fifth of the kernel's vector instructions.
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
    const int line = blockIdx.x;
    if (line >= nlines) return;
    {
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
    }
}

// Short lines (chunk <= 4): one wavefront per block; block b solves lines
// bL .. bL + L - 1 together (one block per L lines, for the reason given
// above).  Past the last line a slot solves the last line again and stores
// nothing.
// partials as in calcnu_lux_kernel.
template <typename S, typename A, int C, int L, bool REAL>
__global__ void __launch_bounds__(kWave)
calcnu_lux_lines_kernel(S *__restrict__ psi, const XArgs<A> a, const cx<A> *__restrict__ zt,
                        const double *__restrict__ scale, double *__restrict__ partials)
{
    __shared__ S buf[L * (kWave * C + kWave)];
    const int lane = threadIdx.x;
    const int nx = a.nx;
    const int nlines = a.ny * a.nz;
    const A s = scale ? (A)(*scale) : (A)1;
    const int base = blockIdx.x * L;
    if (base >= nlines) return;
    {
        auto ln = [&](int l) { return XLine<A>{zt, s, min(base + l, nlines - 1)}; };
        S v[L][C];
#pragma unroll
        for (int l = 0; l < L; ++l) load_x_row(v[l], psi + (int64_t)ln(l).line * nx, nx);
        solve_x_lines<S, A, C, L, REAL>(v, buf, [&](int) -> const XArgs<A> & { return a; }, ln);
#pragma unroll
        for (int l = 0; l < L; ++l) {
            if (base + l >= nlines) break;
            store_x_row(psi + (int64_t)ln(l).line * nx, v[l], nx);
            if (partials) {
                double acc = 0.0;
#pragma unroll
                for (int r = 0; r < C; ++r) {
                    if (r * kWave + lane < nx) {
#pragma clang fp contract(off)
                        acc += sre(v[l][r]) * sre(v[l][r]) + sim(v[l][r]) * sim(v[l][r]);
                    }
                }
#pragma unroll
                for (int d = kWave / 2; d > 0; d >>= 1) acc += __shfl_down(acc, d, kWave);
                if (lane == 0) partials[ln(l).line] = acc;
            }
        }
    }
}

// Batched: lines g = g0 .. g0 + L - 1 of the list of active solves, line
// g % nlines of solve active[g / nlines], for g below total = nact * nlines
// (past it, the last line again, not stored).  buf: L (64 C + 64) elements
// of LDS.
template <typename S, typename A, int C, int L, bool REAL>
__device__ __forceinline__ void x_batch_lines(S *const *__restrict__ psis, const XBatchArgs<A> *__restrict__ args,
                                              const int *__restrict__ active, int nlines, int total,
                                              const double *__restrict__ scales, int g0, S *buf)
{
    const XArgs<A> *ap[L];
    XLine<A> ln[L];
    S *rows[L];
    S v[L][C];
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const int g = min(g0 + l, total - 1);
        const int slot = g / nlines;
        const int si = active[slot];
        ap[l] = &args[si].x;
        ln[l] = XLine<A>{args[si].zt, scales ? (A)scales[si] : (A)1, g - slot * nlines};
        rows[l] = psis[si] + (int64_t)ln[l].line * ap[l]->nx;
        load_x_row(v[l], rows[l], ap[l]->nx);
    }
    solve_x_lines<S, A, C, L, REAL>(v, buf, [&](int l) -> const XArgs<A> & { return *ap[l]; }, [&](int l) { return ln[l]; });
#pragma unroll
    for (int l = 0; l < L; ++l)
        if (g0 + l < total) store_x_row(rows[l], v[l], ap[l]->nx);
}

// Batched, one class: block b advances lines bL .. bL + L - 1 of the list.
template <typename S, typename A, int C, int L, bool REAL>
__global__ void __launch_bounds__(kWave)
calcnu_lux_batch_kernel(S *const *__restrict__ psis, const XBatchArgs<A> *__restrict__ args,
                        const int *__restrict__ active, int nlines, int total,
                        const double *__restrict__ scales)
{
    __shared__ S buf[L * (kWave * C + kWave)];
    x_batch_lines<S, A, C, L, REAL>(psis, args, active, nlines, total, scales, (int)blockIdx.x * L, buf);
}

// Batched, every class in one launch: class k owns the blocks from
// cls[k].block0 on and advances its list as calcnu_lux_batch_kernel does,
// with its own chunk and lines per wavefront (at most CMAX points per lane;
// the kernel's registers are those of its largest variant).  LDS: the
// largest class's L (64 C + 64) elements, dynamic.
template <typename S, typename A, int CMAX, bool REAL>
__global__ void __launch_bounds__(kWave)
calcnu_lux_classes_kernel(S *const *__restrict__ psis, const XBatchArgs<A> *__restrict__ args,
                          const XClassDesc *__restrict__ cls, int ncls, const double *__restrict__ scales)
{
    extern __shared__ unsigned char xsmem[];
    S *buf = reinterpret_cast<S *>(xsmem);
    const int b = blockIdx.x;
    const XClassDesc c = cls[class_of_block(cls, ncls, b)];
    const int g0 = (b - c.block0) * c.lines;
#define GP_XC(CC, LL)                                                                                  \
    case CC * 8 + LL:                                                                                  \
        if constexpr (CC <= CMAX && LL <= x_max_lines_per_wave(CC))                                   \
            x_batch_lines<S, A, CC, LL, REAL>(psis, args, c.active, c.nlines, c.total, scales, g0, buf); \
        break;
    switch (c.chunk * 8 + c.lines) {
        GP_XC(1, 1) GP_XC(1, 2) GP_XC(1, 4) GP_XC(2, 1) GP_XC(2, 2) GP_XC(2, 4)
        GP_XC(3, 1) GP_XC(3, 2) GP_XC(4, 1) GP_XC(4, 2)
        GP_XC(5, 1) GP_XC(6, 1) GP_XC(7, 1) GP_XC(8, 1)
        GP_XC(10, 1) GP_XC(12, 1) GP_XC(14, 1) GP_XC(16, 1)
    default:
        break;
    }
#undef GP_XC
}

template <typename S, typename A, bool REAL>
static hipError_t launch_classes_x(int cmax, int nblocks, size_t lds, hipStream_t stream, void *const *psis,
                                   const void *args, const XClassDesc *cls, int ncls, const double *scales)
{
    S *const *p = reinterpret_cast<S *const *>(psis);
    const XBatchArgs<A> *a = static_cast<const XBatchArgs<A> *>(args);
    const dim3 grid((unsigned)nblocks);
    if (cmax <= 4)
        hipLaunchKernelGGL((calcnu_lux_classes_kernel<S, A, 4, REAL>), grid, dim3(kWave), lds, stream, p, a, cls,
                           ncls, scales);
    else if (cmax <= 8)
        hipLaunchKernelGGL((calcnu_lux_classes_kernel<S, A, 8, REAL>), grid, dim3(kWave), lds, stream, p, a, cls,
                           ncls, scales);
    else
        hipLaunchKernelGGL((calcnu_lux_classes_kernel<S, A, 16, REAL>), grid, dim3(kWave), lds, stream, p, a, cls,
                           ncls, scales);
    return hipGetLastError();
}

hipError_t launch_nu_x_classes(Prec prec, bool real, int cmax, int lds_elems, int nblocks, void *const *psis,
                               const void *args, const XClassDesc *cls, int ncls, const double *scales,
                               hipStream_t stream)
{
    if (real && (prec == PREC_R64 || prec == PREC_R32)) return hipErrorInvalidValue;  // real storage is imaginary time only
    if (nblocks <= 0 || ncls <= 0) return hipSuccess;
    if (cmax < 1 || cmax > 16 || lds_elems < 1) return hipErrorInvalidValue;
    const size_t lds = (size_t)lds_elems * storage_bytes(prec);
    if (lds > 65536) return hipErrorInvalidValue;
#define GP_XCP(S, A)                                                                                          \
    return real ? launch_classes_x<S, A, true>(cmax, nblocks, lds, stream, psis, args, cls, ncls, scales)     \
                : launch_classes_x<S, A, false>(cmax, nblocks, lds, stream, psis, args, cls, ncls, scales);
    switch (prec) {
    case PREC_C64: GP_XCP(float2, float)
    case PREC_C64_F64: GP_XCP(float2, double)
    case PREC_C128: GP_XCP(double2, double)
    case PREC_R64:
        return launch_classes_x<double, double, false>(cmax, nblocks, lds, stream, psis, args, cls, ncls, scales);
    case PREC_R32:
        return launch_classes_x<float, float, false>(cmax, nblocks, lds, stream, psis, args, cls, ncls, scales);
    }
#undef GP_XCP
    return hipErrorInvalidValue;
}

// Launch the L-line form with chunk C (L at most x_max_lines_per_wave(C)).
template <typename S, typename A, int C, bool REAL>
static void launch_batch_l(int L, dim3 grid, hipStream_t stream, S *const *p, const XBatchArgs<A> *a,
                           const int *active, int nlines, int total, const double *scales)
{
    constexpr int LM = x_max_lines_per_wave(C);
    if (LM >= 4 && L == 4)
        hipLaunchKernelGGL((calcnu_lux_batch_kernel<S, A, C, (LM >= 4 ? 4 : 1), REAL>), grid, dim3(kWave), 0,
                           stream, p, a, active, nlines, total, scales);
    else if (LM >= 2 && L == 2)
        hipLaunchKernelGGL((calcnu_lux_batch_kernel<S, A, C, (LM >= 2 ? 2 : 1), REAL>), grid, dim3(kWave), 0,
                           stream, p, a, active, nlines, total, scales);
    else
        hipLaunchKernelGGL((calcnu_lux_batch_kernel<S, A, C, 1, REAL>), grid, dim3(kWave), 0, stream,
                           p, a, active, nlines, total, scales);
}

template <typename S, typename A, bool REAL>
static hipError_t launch_batch_c(int chunk, int lines, int nact, int nlines, void *const *psis, const void *args,
                                 const int *active, const double *scales, hipStream_t stream)
{
    const int64_t total = (int64_t)nact * nlines;
    if (total > INT32_MAX) return hipErrorInvalidValue;
    if (lines < 0 || lines > x_max_lines_per_wave(chunk) || (lines & (lines - 1))) return hipErrorInvalidValue;
    const int L = lines ? lines : x_lines_per_wave(chunk, total);
    const dim3 grid((unsigned)((total + L - 1) / L));
    S *const *p = reinterpret_cast<S *const *>(psis);
    const XBatchArgs<A> *a = static_cast<const XBatchArgs<A> *>(args);
#define GP_XB_CASE(CC)                                                                    \
    case CC:                                                                              \
        launch_batch_l<S, A, CC, REAL>(L, grid, stream, p, a, active, nlines, (int)total, scales); \
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
                             hipStream_t stream, int lines)
{
    if (real && (prec == PREC_R64 || prec == PREC_R32)) return hipErrorInvalidValue;  // real storage is imaginary time only
    if (nact <= 0) return hipSuccess;
#define GP_XB_PREC(S, A)                                                                                   \
    return real ? launch_batch_c<S, A, true>(chunk, lines, nact, nlines, psis, args, active, scales, stream) \
                : launch_batch_c<S, A, false>(chunk, lines, nact, nlines, psis, args, active, scales, stream);
    switch (prec) {
    case PREC_C64: GP_XB_PREC(float2, float)
    case PREC_C64_F64: GP_XB_PREC(float2, double)
    case PREC_C128: GP_XB_PREC(double2, double)
    // real storage: imaginary time only (real time was refused above)
    case PREC_R64:
        return launch_batch_c<double, double, false>(chunk, lines, nact, nlines, psis, args, active, scales, stream);
    case PREC_R32:
        return launch_batch_c<float, float, false>(chunk, lines, nact, nlines, psis, args, active, scales, stream);
    }
#undef GP_XB_PREC
    return hipErrorInvalidValue;
}

// Launch the L-line form (chunk <= 4) or the one-line kernel (chunk >= 5).
template <typename S, typename A, int C, bool REAL>
static void launch_plain_l(int L, dim3 grid, hipStream_t stream, S *p, const XArgs<A> &a, const cx<A> *z,
                           const double *scale, double *partials)
{
    constexpr int LM = x_max_lines_per_wave(C);
    if constexpr (LM == 1) {
        hipLaunchKernelGGL((calcnu_lux_kernel<S, A, C, REAL>), grid, dim3(kWave), 0, stream,
                           p, a, z, scale, partials);
    } else {
        if (LM >= 4 && L == 4)
            hipLaunchKernelGGL((calcnu_lux_lines_kernel<S, A, C, (LM >= 4 ? 4 : 1), REAL>), grid, dim3(kWave), 0,
                               stream, p, a, z, scale, partials);
        else if (L == 2)
            hipLaunchKernelGGL((calcnu_lux_lines_kernel<S, A, C, 2, REAL>), grid, dim3(kWave), 0, stream,
                               p, a, z, scale, partials);
        else
            hipLaunchKernelGGL((calcnu_lux_lines_kernel<S, A, C, 1, REAL>), grid, dim3(kWave), 0, stream,
                               p, a, z, scale, partials);
    }
}

template <typename S, typename A, bool REAL>
static hipError_t launch_c(int chunk, void *psi, const void *args, const void *zt,
                           const double *scale, double *partials, hipStream_t stream)
{
    const XArgs<A> &a = *static_cast<const XArgs<A> *>(args);
    const int nlines = a.ny * a.nz;
    const int L = x_lines_per_wave(chunk, nlines);
    const dim3 grid((unsigned)((nlines + L - 1) / L));
    S *p = static_cast<S *>(psi);
    const cx<A> *z = static_cast<const cx<A> *>(zt);
#define GP_X_CASE(CC)                                                                   \
    case CC:                                                                            \
        launch_plain_l<S, A, CC, REAL>(L, grid, stream, p, a, z, scale, partials);       \
        break;
    static_assert(x_max_lines_per_wave(4) == 2 && x_max_lines_per_wave(5) == 1,
                  "several-line kernels up to chunk 4, the one-line kernel from chunk 5 on");
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
                       const void *zt, const double *scale, double *partials, hipStream_t stream)
{
    if (real && (prec == PREC_R64 || prec == PREC_R32)) return hipErrorInvalidValue;  // real storage is imaginary time only
#define GP_X_PREC(S, A)                                                                   \
    return real ? launch_c<S, A, true>(chunk, psi, args, zt, scale, partials, stream)  \
                : launch_c<S, A, false>(chunk, psi, args, zt, scale, partials, stream);
    switch (prec) {
    case PREC_C64: GP_X_PREC(float2, float)
    case PREC_C64_F64: GP_X_PREC(float2, double)
    case PREC_C128: GP_X_PREC(double2, double)
    // real storage: imaginary time only (real time was refused above)
    case PREC_R64: return launch_c<double, double, false>(chunk, psi, args, zt, scale, partials, stream);
    case PREC_R32: return launch_c<float, float, false>(chunk, psi, args, zt, scale, partials, stream);
    }
#undef GP_X_PREC
    return hipErrorInvalidValue;
}

}  // namespace gpssc
