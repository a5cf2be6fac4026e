// gp_internal.h -- types shared by the host plan and the gfx950 kernels of the
// split-step Crank-Nicolson step.  Internal to libgpssc; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace gpssc {

// Chunked Thomas layout limits.  A line of n points is cut into `lanes`
// contiguous chunks of `chunk` points; the last chunks are padded with zeros.
constexpr int kWave = 64;          // wavefront width on gfx950
constexpr int kMaxChunkX = 16;     // x: 64 lanes x 16 points = 1024
constexpr int kMaxLanesYZ = 64;    // y/z: at most 64 chunks per line
constexpr int kMaxChunkYZ = 16;    // y/z: 64 x 16 = 1024 points per line
constexpr int kMaxStages = 6;      // log2(64) Kogge-Stone stages
constexpr int kMaxBlockYZ = 1024;  // threads per y/z block

// Complex number in the arithmetic type A (double or float).
template <typename A>
struct cx {
    A re, im;
};

template <typename A>
__host__ __device__ __forceinline__ cx<A> mk(A re, A im) { return cx<A>{re, im}; }

template <typename A>
__device__ __forceinline__ cx<A> cadd(cx<A> a, cx<A> b) { return cx<A>{a.re + b.re, a.im + b.im}; }

template <typename A>
__device__ __forceinline__ cx<A> cmul(cx<A> a, cx<A> b)
{
    return cx<A>{fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}

// a*b + c
template <typename A>
__device__ __forceinline__ cx<A> cfma(cx<A> a, cx<A> b, cx<A> c)
{
    return cx<A>{fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}

template <typename A>
__device__ __forceinline__ A cabs2(cx<A> a) { return fma(a.re, a.re, a.im * a.im); }

// Storage <-> arithmetic conversion.  psi is stored as double2 (complex128),
// float2 (complex64), or -- for imaginary-time states, which stay real when
// they start real -- as double or float holding the real part only.  Values
// are always handled as cx<A> in registers; a real element loads with a zero
// imaginary part and stores its real part, so a real state runs exactly the
// arithmetic of the complex state with zero imaginary parts.
template <typename S> struct storage_traits;
template <> struct storage_traits<double2> { using real = double; static constexpr bool complex = true; };
template <> struct storage_traits<float2> { using real = float; static constexpr bool complex = true; };
template <> struct storage_traits<double> { using real = double; static constexpr bool complex = false; };
template <> struct storage_traits<float> { using real = float; static constexpr bool complex = false; };

template <typename A, typename S>
__device__ __forceinline__ cx<A> ld(S v)
{
    if constexpr (storage_traits<S>::complex)
        return cx<A>{(A)v.x, (A)v.y};
    else
        return cx<A>{(A)v, (A)0};
}

template <typename S, typename A>
__device__ __forceinline__ S st(cx<A> v)
{
    using R = typename storage_traits<S>::real;
    if constexpr (storage_traits<S>::complex) {
        S r;
        r.x = (R)v.re;
        r.y = (R)v.im;
        return r;
    } else {
        return (R)v.re;
    }
}

// Register value of a storage type: cx<A> for complex storage, A itself for
// real storage (imaginary-time states, whose imaginary parts are zero).
template <typename S, typename A>
using value_t = typename std::conditional<storage_traits<S>::complex, cx<A>, A>::type;

template <typename V, typename S>
__device__ __forceinline__ V ldv(S v)
{
    if constexpr (storage_traits<S>::complex)
        return V{(decltype(V::re))v.x, (decltype(V::re))v.y};
    else
        return (V)v;
}

template <typename S, typename A>
__device__ __forceinline__ S stv(A v)
{
    return (typename storage_traits<S>::real)v;
}

template <typename S, typename A>
__device__ __forceinline__ S stv(cx<A> v)
{
    return st<S>(v);
}

template <typename S>
__device__ __forceinline__ S szero()
{
    if constexpr (storage_traits<S>::complex) {
        S r;
        r.x = 0;
        r.y = 0;
        return r;
    } else {
        return (S)0;
    }
}

// Real and imaginary part of a stored element, in FP64.
template <typename S>
__device__ __forceinline__ double sre(S v)
{
    if constexpr (storage_traits<S>::complex)
        return (double)v.x;
    else
        return (double)v;
}

template <typename S>
__device__ __forceinline__ double sim(S v)
{
    if constexpr (storage_traits<S>::complex)
        return (double)v.y;
    else
        return 0.0;
}

// v * s componentwise in the storage precision (s rounded to it).  For a
// float state this leaves the norm within about one float ulp of 1: a factor
// that close to 1 rounds most elements back to themselves.  That is also what
// lets a converged float state become an exact fixed point of the step, which
// the imaginary-time stopping rule relies on.
template <typename S>
__device__ __forceinline__ S sscale(S v, typename storage_traits<S>::real s)
{
    if constexpr (storage_traits<S>::complex) {
        v.x *= s;
        v.y *= s;
        return v;
    } else {
        return v * s;
    }
}

// Constant-coefficient factorisation of one axis.  The Crank-Nicolson
// matrix tridiag(o, b, o) (b = 1 + kappa, o = -kappa/2) is Toeplitz, so with
// c the root of o c^2 - b c + o = 0 inside the unit circle and beta = o / c,
//     A = beta (I + c S)(I + c S^T) + beta c^2 e_0 e_0^T
// (S the down-shift).  Solving (I + c S) w = m r (m = 1/beta), then
// (I + c S^T) y = w, gives y = M^-1 r for M = beta (I + c S)(I + c S^T); the
// rank-one term is restored by Sherman-Morrison: x = y + y_0 zt with
// zt = -beta c^2 M^-1 e_0 / (1 + beta c^2 (M^-1 e_0)_0), which decays like c^i
// from the first node.  Both recurrences have the single coefficient a = -c.
template <typename A>
struct SweepCoef {
    A kap;                     // |kappa| = dt/(2 dx^2): kappa = kap (imag) or i kap (real time)
    cx<A> m;                   // 1/beta
    cx<A> a;                   // -c
    cx<A> stage[kMaxStages];   // a^(chunk 2^s): Kogge-Stone stage multipliers
    int nst;                   // stages with a nonzero multiplier
    int nzc;                   // zt is nonzero only at positions < nzc
};

// Streaming loads and stores of psi.  Every sweep reads each element once
// and writes it once, so the accesses are marked nontemporal: the data are
// not kept in the caches for reuse that never comes.
#ifndef GPSSC_NT_LOAD
#define GPSSC_NT_LOAD 1
#endif
#ifndef GPSSC_NT_STORE
#define GPSSC_NT_STORE 1
#endif
template <typename S> struct vec2_of;
template <> struct vec2_of<double2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct vec2_of<float2> { typedef float type __attribute__((ext_vector_type(2))); };

template <typename S>
__device__ __forceinline__ S stream_load(const S *p)
{
    if constexpr (storage_traits<S>::complex) {
        typedef typename vec2_of<S>::type V;
        V v;
        if (GPSSC_NT_LOAD)
            v = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
        else
            v = *reinterpret_cast<const V *>(p);
        S r;
        r.x = v.x;
        r.y = v.y;
        return r;
    } else {
        if (GPSSC_NT_LOAD) return __builtin_nontemporal_load(p);
        return *p;
    }
}

template <typename S>
__device__ __forceinline__ void stream_store(S *p, S val)
{
    if constexpr (storage_traits<S>::complex) {
        typedef typename vec2_of<S>::type V;
        V v;
        v.x = val.x;
        v.y = val.y;
        if (GPSSC_NT_STORE)
            __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
        else
            *reinterpret_cast<V *>(p) = v;
    } else {
        if (GPSSC_NT_STORE)
            __builtin_nontemporal_store(val, p);
        else
            *p = val;
    }
}

// Two neighbouring complex64 columns handled by one thread of the y/z
// sweeps: one 16-byte access per row, as complex128 takes, for the FP32
// arithmetic of complex64.  The two columns never mix; every operation acts
// on each of them exactly as on a column of its own.
template <typename A>
struct cx2 {
    cx<A> p, q;
};

typedef float pair4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ cx2<float> stream_load_pair(const float2 *at)
{
    pair4_t v;
    if (GPSSC_NT_LOAD)
        v = __builtin_nontemporal_load(reinterpret_cast<const pair4_t *>(at));
    else
        v = *reinterpret_cast<const pair4_t *>(at);
    return cx2<float>{cx<float>{v.x, v.y}, cx<float>{v.z, v.w}};
}

__device__ __forceinline__ void stream_store_pair(float2 *at, cx2<float> u)
{
    pair4_t v;
    v.x = u.p.re;
    v.y = u.p.im;
    v.z = u.q.re;
    v.w = u.q.im;
    if (GPSSC_NT_STORE)
        __builtin_nontemporal_store(v, reinterpret_cast<pair4_t *>(at));
    else
        *reinterpret_cast<pair4_t *>(at) = v;
}

// Launch arguments of the calcnu + calclux kernel.
template <typename A>
struct XArgs {
    int nx, ny, nz;
    A c0x, c0y, c0z;     // (N-1)/2 per axis: node i sits at (i - c0) * d
    A dx, dy, dz;
    A hgx, hgy, hgz;     // gamma^2/2, nu^2/2, lambda^2/2
    A dt, g;
    SweepCoef<A> k;
};

// Launch arguments of the strided (y or z) sweep kernel.
template <typename A>
struct SArgs {
    int nx;                // columns across a block (x extent)
    int n;                 // line length
    int lanes;             // chunks per line (blockDim.y)
    int64_t stride;        // element stride along the line
    int64_t outer_stride;  // element stride per blockIdx.y
    SweepCoef<A> k;
};

// Per-solve arguments of the batched kernels (device arrays indexed by solve).
template <typename A>
struct XBatchArgs {
    XArgs<A> x;
    const cx<A> *zt;       // this solve's x correction
};

template <typename A>
struct SBatchArgs {
    SArgs<A> s;
    const cx<A> *zt;       // this solve's y or z correction
};

// Radial Crank-Nicolson (symmetric traps): x holds the grid, coordinates
// (c0x = -1/2: node i at (i + 1/2) dx), trap, dt and g; tab the per-position
// coefficients, six arrays of npad entries: rd, rl, ru (right side
// rd_i u_i + rl_i u_{i-1} + ru_i u_{i+1}), m, a (forward d_i = m_i q_i +
// a_i d_{i-1}) and b (backward x_i = d_i + b_i x_{i+1}), zero past the line.
template <typename A>
struct RadialArgs {
    XArgs<A> x;
    const cx<A> *tab;
    int npad;
};

// Physical quantities of the symmetric traps: nr radial nodes at
// (i + 1/2) dr with cell weights v and face weights s (device arrays), nz
// rows (z nodes of the axial trap at (k - c0z) dz; 1 otherwise).
struct RadialObsArgs {
    int nr, nz;
    double dr, dz, c0z;
    double hgr, hgz;          // gamma^2/2 (radial), lambda^2/2 (z)
    const double *v, *s;
};

// Sums of the observables pass, FP64.
enum {
    OBS_DENS = 0, OBS_POT, OBS_QUART,
    OBS_LINKX, OBS_LINKY, OBS_LINKZ,
    OBS_M1X, OBS_M1Y, OBS_M1Z,
    OBS_M2X, OBS_M2Y, OBS_M2Z,
    OBS_NSUMS
};

template <typename A>
struct ObsArgs {
    int nx, ny, nz;
    double c0x, c0y, c0z, dx, dy, dz;
    double hgx, hgy, hgz;
};

// ---- host-side launchers (one translation unit per kernel family) ----

// Precision of a launch: storage and arithmetic types (double2/double,
// float2/float, float2/double, double/double, float/float).  The values
// equal gp_dtype's.
enum Prec { PREC_C128 = 0, PREC_C64 = 1, PREC_C64_F64 = 2, PREC_R64 = 3, PREC_R32 = 4 };

// x lines one wavefront solves together.  A short line (chunks of a few
// points) leaves its wavefront waiting on latency, so a wavefront interleaves
// up to 4 (chunks of 1-2 points) or 2 (3-4 points) of them -- but only while
// at least 4096 wavefronts (about four per SIMD) remain for the nlines lines,
// since small grids need the wavefronts more than the overlap.
constexpr int x_max_lines_per_wave(int chunk) { return chunk <= 2 ? 4 : chunk <= 4 ? 2 : 1; }
constexpr int x_lines_per_wave(int chunk, int64_t nlines)
{
    int l = 1;
    while (l < x_max_lines_per_wave(chunk) && nlines >= (int64_t)2 * l * 4096) l *= 2;
    return l;
}

// calcnu + calclux.  zt: boundary correction by position (complex, the
// arithmetic type).  scale: NULL or device double (pending 1/sqrt(N)).
// partials: NULL or one double per x line (sum |psi|^2 of its output).
// One one-wavefront block per x_lines_per_wave(chunk, ny nz) lines.
hipError_t launch_nu_x(Prec prec, bool real, int chunk, void *psi, const void *args,
                       const void *zt, const double *scale, double *partials, hipStream_t stream);

// calcluy / calcluz over ceil(nx/(xt cols)) x nouter tiles.  cols: columns
// per thread, 1, or 2 for complex64 with FP32 arithmetic (then nx and both
// strides must be even and psi 16-byte aligned); one block per tile.  zt:
// boundary correction by position.  partials: NULL, or nx * nouter doubles:
// sum |psi|^2 of each line's output, at outer * nx + column.
// xcd_ranges: hand each XCD a contiguous range of tiles (the y sweep; see
// calclu_strided_kernel).
hipError_t launch_strided(Prec prec, bool real, int chunk, int xt, int cols, int nouter,
                          void *psi, const void *args, const void *zt, double *partials, bool xcd_ranges,
                          hipStream_t stream);

// calcluy / calcluz streamed along the lines (sweep_stream.hip): one lane per
// column (cols = 1) or column pair (cols = 2: complex64 with FP32 arithmetic,
// nx and both strides even, psi 16-byte aligned), blocks of blk points (8,
// 12 or 16), nouter * nx columns.  partials as in launch_strided.
hipError_t launch_stream(Prec prec, bool real, int blk, int cols, int nouter, void *psi, const void *args,
                         const void *zt, double *partials, hipStream_t stream);

// calcnorm: sums `n` partials (each times weights[b] when weights is not
// NULL) in a fixed order, writes 1/sqrt(dv*sum) to *scale and raises *flag
// if the norm is not finite and positive.
hipError_t launch_norm_finalize(const double *partials, int n, double dv, double *scale,
                                int *flag, hipStream_t stream, const double *weights = nullptr);

// calcnu + Crank-Nicolson along a radial axis, one wavefront per line
// (nlines lines of args.x.nx points).  dens: NULL or |psi|^2 per stored
// point (one-line states: the norm partials).
hipError_t launch_nu_r(Prec prec, bool real, int chunk, int nlines, void *psi, const void *args,
                       const double *scale, double *dens, hipStream_t stream);

// Density profiles into out[nx + ny + nz]: per node of x, then y, then z,
// the sum of |psi|^2 over the other two axes times w[axis].
hipError_t launch_profiles(Prec prec, const void *psi, int nx, int ny, int nz, const double w[3], double *out,
                           hipStream_t stream);

// Sums of the symmetric-trap quantities into sums[OBS_NSUMS] (partials:
// OBS_NSUMS per row of scratch).
hipError_t launch_radial_observables(Prec prec, const void *psi, const RadialObsArgs &args, double *partials,
                                     double *sums, hipStream_t stream);

// psi <- psi * (*scale)
hipError_t launch_scale(Prec prec, void *psi, int64_t elems, const double *scale,
                        hipStream_t stream);

// psi between storage types: float <-> double of one kind ((C128, C64),
// (R64, R32); exact upwards, rounded to nearest downwards) or complex <->
// real of one precision ((C64, R32), (C128, R64); the real part, or a zero
// imaginary part).
hipError_t launch_convert(Prec to, Prec from, void *dst, const void *src, int64_t elems, hipStream_t stream);

// calcmuen + calcrms raw sums: partials [nblocks][OBS_NSUMS] then a fixed
// order final sum into sums[OBS_NSUMS].
int obs_num_blocks(int nx, int ny);
hipError_t launch_observables(Prec prec, const void *psi, const ObsArgs<double> &args,
                              double *partials, double *sums, hipStream_t stream);

// ---- batched launchers: one launch covers every active solve of one grid
// shape.  psis[i], args[i]: solve i's psi and arguments (device arrays);
// active[0..nact): the solves to advance.  lines (x): lines per wavefront,
// 1, 2 or 4 up to x_max_lines_per_wave(chunk), or 0 for x_lines_per_wave's
// rule; it does not enter the rounding. ----

hipError_t launch_nu_x_batch(Prec prec, bool real, int chunk, int nact, int nlines, void *const *psis,
                             const void *args, const int *active, const double *scales,
                             hipStream_t stream, int lines = 0);

// ---- one launch per sweep over every class of a batch.  The classes'
// blocks follow one another in the grid, class k's from block0 on (block0
// increasing, the first 0); each block finds its class and runs exactly the
// per-class kernel's code for it, so every solve's result is bitwise that
// of the per-class launches. ----

// Bytes of one element of psi in the storage of prec.
inline size_t storage_bytes(Prec prec)
{
    switch (prec) {
    case PREC_C128: return 16;
    case PREC_C64: case PREC_C64_F64: case PREC_R64: return 8;
    case PREC_R32: return 4;
    }
    return 0;
}

// Index of the class that owns block b: the last k with cls[k].block0 <= b.
template <typename D>
__device__ __forceinline__ int class_of_block(const D *__restrict__ cls, int ncls, int b)
{
    int lo = 0, hi = ncls - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (cls[mid].block0 <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

struct XClassDesc {
    int block0;          // first block of the class
    int nlines;          // x lines per solve
    int total;           // nact * nlines
    int chunk, lines;    // points per lane, lines per wavefront
    const int *active;   // the class's active solves (device)
};

// x sweep of every class: nblocks in all; cmax >= every class's chunk;
// lds_elems = the largest lines * (64 chunk + 64) over the classes (LDS of
// at most 64 KiB).
hipError_t launch_nu_x_classes(Prec prec, bool real, int cmax, int lds_elems, int nblocks, void *const *psis,
                               const void *args, const XClassDesc *cls, int ncls, const double *scales,
                               hipStream_t stream);

struct YZClassDesc {
    int block0;          // first block of the class
    int ntiles, ncol;    // tiles per solve, column tiles per outer index
    int xt, lanes;       // threads across, chunks along (xt * lanes <= the block size)
    int chunk, cols;     // points per chunk, columns per thread (2: complex64 pairs)
    const int *active;   // the class's active solves (device)
};

// y or z sweep of every class: nblocks in all, blocks of `threads` threads
// (>= every class's xt * lanes); cmax >= every chunk; lds_bytes = the
// largest 2 xt lanes (16 or 8 bytes per value) over the classes.
hipError_t launch_strided_classes(Prec prec, bool real, int cmax, int threads, size_t lds_bytes, int nblocks,
                                  void *const *psis, const void *args, const YZClassDesc *cls, int ncls,
                                  double *partials, const int64_t *part_off, hipStream_t stream);

struct NormClassDesc {
    int block0;          // first block of the class: one block per active solve
    int npart;           // norm partials per solve
    const int *active;
};

// calcnorm of every class: one block per active solve, as
// launch_norm_finalize_batch.
hipError_t launch_norm_finalize_classes(int nblocks, const NormClassDesc *cls, int ncls, const double *partials,
                                        const int64_t *part_off, const double *dv, double *scales, int *flags,
                                        hipStream_t stream);

// partials + part_off[i]: solve i's per-line norm partials (NULL: none).
// cols: columns per thread as in launch_strided (2: every active solve's psi
// 16-byte aligned, nx even).
hipError_t launch_strided_batch(Prec prec, bool real, int chunk, int xt, int cols, int lanes, int nact,
                                int ncol, int ntiles, void *const *psis, const void *args,
                                const int *active, double *partials, const int64_t *part_off,
                                hipStream_t stream);

// Per solve: 1/sqrt(dv_i * sum of its npart partials) -> scales[i]; flags[i]
// raised for a non-finite or zero norm.
hipError_t launch_norm_finalize_batch(int nact, const int *active, const double *partials,
                                      const int64_t *part_off, int npart, const double *dv,
                                      double *scales, int *flags, hipStream_t stream);

// psi_i <- psi_i * scales[i] for the active solves, then scales[i] <- 1.
hipError_t launch_scale_batch(Prec prec, int nact, const int *active, void *const *psis,
                              int64_t elems, double *scales, hipStream_t stream);

// Observables sums per solve: sums[i * OBS_NSUMS + q].  partials + obs_off[i]:
// solve i's obs_num_blocks(nx, ny) * OBS_NSUMS doubles of scratch.
hipError_t launch_observables_batch(Prec prec, int nact, const int *active, void *const *psis,
                                    const ObsArgs<double> *args, int nx, int ny, double *partials,
                                    const int64_t *obs_off, double *sums, hipStream_t stream);

}  // namespace gpssc
