// host_common.h -- host-side pieces shared by the single-solve plan
// (plan.hip) and the batch (batch.hip): error reporting, argument checks,
// launch-shape policy and the constant Crank-Nicolson coefficients of an
// axis.  Internal to libgpssc.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "gp_internal.h"
#include "gpssc.h"

namespace gpssc_host {

using gpssc::cx;
using cplx = std::complex<double>;

// Message of the last failure on this host thread (defined in plan.hip).
extern thread_local std::string g_last_error;

inline gp_status fail(gp_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

inline gp_status fail_hip(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return GP_ERR_DEVICE;
}


inline const int kChunksX[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16};
inline const int kChunksYZ[] = {1, 2, 4, 8, 16};

// FP32 arithmetic: complex64 and real float storage.
inline bool arith_f32(gp_dtype d) { return d == GP_C64 || d == GP_R32; }
// Real storage (imaginary time only).
inline bool real_storage(gp_dtype d) { return d == GP_R64 || d == GP_R32; }
// Bytes of one stored element.
inline size_t storage_bytes(gp_dtype d)
{
    return d == GP_C128 ? 16 : (d == GP_R32 ? 4 : 8);
}

// Most chunks per y/z line.  A short line holds a few points per thread and
// spends its time in the scan's barriers, one per stage, so lines of up to
// 128 points take at most 8 chunks and lines of up to 256 at most 16 (on
// batches of 48- to 160-point grids: 14% less time in FP32, 6% in FP64, and
// the 32^3 solve 20% faster than at 32 chunks of 1 point).  Longer lines:
// real float32 storage affords 16-point chunks, so 32 chunks cover 512
// points.  16-byte values per thread -- complex128, and complex64 taken as
// column pairs -- keep chunks of at most 8 points (about 73 registers, so
// two blocks of up to 768 threads share a compute unit) while that needs at
// most 48 chunks; longer lines would need blocks too large for two to fit,
// so they take 16-point chunks at 32 chunks per line, which lets a block hold
// twice the columns (wider rows per load) at the same occupancy.
inline int max_lanes_for(gp_dtype dtype, int64_t n)
{
    if (n <= 128) return 8;
    if (n <= 256) return 16;
    if (dtype == GP_R32) return 32;
    if (n > 8 * 48) return 32;
    return gpssc::kMaxLanesYZ;
}

// Chunking of a line of n points along `axis`: chunk points per lane, lanes
// per line.  Returns false when the line is longer than the kernels handle.
// y/z: the fewest points per thread that keep the chunks of a line within
// max_lanes; FP32 arithmetic affords 16-point chunks at 32 chunks per line
// (fewer scan stages, wider blocks), FP64 keeps 64 chunks of at most 8
// points for lines up to 512 so two 1024-thread blocks fit on a compute unit.
inline bool sweep_shape(int64_t n, int axis, int *chunk, int *lanes, int max_lanes = gpssc::kMaxLanesYZ)
{
    if (n < 1) return false;
    if (axis == 0) {
        for (int c : kChunksX)
            if ((int64_t)c * gpssc::kWave >= n) {
                *chunk = c;
                *lanes = gpssc::kWave;
                return true;
            }
        return false;
    }
    for (int c : kChunksYZ) {
        const int64_t p = (n + c - 1) / c;
        if (p <= max_lanes || (c == kChunksYZ[4] && p <= gpssc::kMaxLanesYZ)) {
            *chunk = c;
            *lanes = (int)p;
            return true;
        }
    }
    return false;
}

// Columns per y/z block: as wide as 64 (one full wavefront of contiguous
// x), narrowed so the block holds at most 1024 threads and not far wider
// than the grid.
#ifndef GPSSC_YZ_COLS
#define GPSSC_YZ_COLS 64
#endif

// FP64 arithmetic with 16-point chunks needs about 114 registers, so a
// compute unit holds 16 of its waves: blocks of at most 512 threads let two
// of them share it (measured faster than one block of 1024 with twice the
// row width).
inline int strided_columns(int64_t nx, int lanes, int chunk, gp_dtype dtype)
{
    const int max_threads = (!arith_f32(dtype) && chunk >= 16) ? gpssc::kMaxBlockYZ / 2 : gpssc::kMaxBlockYZ;
    int xt = GPSSC_YZ_COLS;
    while (xt > 1 && xt * lanes > max_threads) xt /= 2;
    while (xt > 16 && xt / 2 >= nx) xt /= 2;
    return xt;
}

// Whether the y (ax = 1) or z (ax = 2) sweep of a grid takes complex64 column
// pairs by default: an even nx, and lines of more than 256 points, where the
// 16-byte rows were measured faster (512x512x384: y 333 -> 318 us, z 351 ->
// 303 us).  On shorter lines the pairs' doubled registers cost more than the
// wider rows bring (a served mix of 64- to 160-point grids handled 5% fewer
// requests per second with pairs on every axis).
inline bool pair_axis(gp_dtype dtype, const int64_t grid[3], int ax)
{
    return dtype == GP_C64 && grid[0] % 2 == 0 && grid[ax] > 256;
}

// Threads across a y/z block when each takes a pair of complex64 columns: a
// thread then holds 16 bytes per row, as in complex128, and the block is
// shaped as complex128's (its register count is about the same).
inline int strided_pair_columns(int64_t nx, int lanes, int chunk)
{
    return strided_columns((nx + 1) / 2, lanes, chunk, GP_C128);
}

// Constant coefficients of one axis, FP64.  Crank-Nicolson along the axis:
// (1 + tau/2 T) psi' = (1 - tau/2 T) psi, T psi_i = -(psi_{i+1} - 2 psi_i +
// psi_{i-1})/(2 dx^2), tau = dt or i dt.  With kappa = tau/(2 dx^2) the left
// matrix is tridiag(o, b, o), b = 1 + kappa, o = -kappa/2, and the right side
// is (1 - kappa) psi_i + kappa/2 (psi_{i-1} + psi_{i+1}).
struct AxisTables {
    int64_t n = 0;
    int chunk = 0, lanes = 0;
    cplx kappa, b, o;
    cplx c, beta, m, a;          // A = beta (I + c S)(I + c S^T) + beta c^2 e0 e0^T; m = 1/beta, a = -c
    std::vector<cplx> zt;        // boundary correction x = y + y_0 zt, by position
    cplx stage[gpssc::kMaxStages];  // a^(chunk 2^s)
};

// The factorisation: c is the root of o c^2 - b c + o = 0 inside the unit
// circle (the two roots multiply to 1), taken as 2o / (b + sqrt(b^2 - 4o^2))
// with the square root that makes |c| < 1, so nothing cancels.  beta = o/c,
// so beta (1 + c^2) = b and beta c = o.  Fills t's coefficients and the
// boundary correction zt[0..n) into caller-provided arrays (w and z: n
// entries of work space each), allocating nothing.
inline void build_axis_into(int64_t n, double dx, double dt, bool real, int chunk, int lanes, AxisTables &t,
                            cplx *zt, cplx *w, cplx *z)
{
    const cplx tau = real ? cplx(0.0, dt) : cplx(dt, 0.0);
    t.n = n;
    t.chunk = chunk;
    t.lanes = lanes;
    t.kappa = tau / (2.0 * dx * dx);
    t.b = 1.0 + t.kappa;
    t.o = -0.5 * t.kappa;
    const cplx disc = std::sqrt(t.b * t.b - 4.0 * t.o * t.o);
    const cplx den = std::abs(t.b + disc) >= std::abs(t.b - disc) ? t.b + disc : t.b - disc;
    t.c = 2.0 * t.o / den;
    t.beta = t.o / t.c;
    t.m = 1.0 / t.beta;
    t.a = -t.c;
    // z = M^-1 e_0 for M = beta (I + c S)(I + c S^T): forward w_i = a^i / beta,
    // then back substitution y_i = w_i + a y_{i+1} from the last node.
    w[0] = t.m;
    for (int64_t i = 1; i < n; ++i) w[i] = t.a * w[i - 1];
    z[n - 1] = w[n - 1];
    for (int64_t i = n - 2; i >= 0; --i) z[i] = w[i] + t.a * z[i + 1];
    // A = M + u e_0^T, u = beta c^2 e_0:  x = y - (beta c^2 y_0 / (1 + beta c^2 z_0)) z
    const cplx bc2 = t.beta * t.c * t.c;
    const cplx gam = -bc2 / (1.0 + bc2 * z[0]);
    for (int64_t i = 0; i < n; ++i) zt[i] = gam * z[i];
    cplx p(1.0, 0.0);
    for (int q = 0; q < chunk; ++q) p *= t.a;
    for (int s = 0; s < gpssc::kMaxStages; ++s) {
        t.stage[s] = p;
        p *= p;
    }
}

// build_axis_into with the correction kept in t.zt.
inline void build_axis(int64_t n, double dx, double dt, bool real, int chunk, int lanes, AxisTables &t)
{
    std::vector<cplx> w((size_t)n), z((size_t)n);
    t.zt.resize((size_t)n);
    build_axis_into(n, dx, dt, real, chunk, lanes, t, t.zt.data(), w.data(), z.data());
}

// Streaming y/z sweep (sweep_stream.hip): the backward recurrence of a
// block of B points starts B - 1 points past the block's end from zero, which
// leaves an error of |a|^B times the line's values at the block's last point.
// Block length of an axis: the smallest B in {8, 12, 16} with |a|^B at most
// 2^-60 (FP64 arithmetic) or 2^-30 (FP32), far below the rounding of the
// result; 0 when even 16 is not enough (only the chunked scan is exact then).
inline int stream_block_len(const AxisTables &t, bool f32)
{
    const double lim = std::ldexp(1.0, f32 ? -30 : -60);
    const double r = std::abs(t.a);
    for (int b : {8, 12, 16})
        if (std::pow(r, (double)b) <= lim) return b;
    return 0;
}

// Whether a y/z axis is streamed by default: never, so far.  On the
// 512x512x384 grid the streamed sweeps measured no faster than the chunked
// scan (complex128 y 0.583 vs 0.583 ms, z 0.704 vs 0.608 ms; complex64 y
// 0.309 vs 0.302, z 0.324 vs 0.301), and a build of both with the arithmetic
// removed showed the same order, so their access patterns, not the
// arithmetic, set the limit.
inline bool stream_by_default(int blk, gp_dtype dtype)
{
    (void)blk;
    (void)dtype;
    return false;
}

template <typename A>
inline cx<A> to_cx(cplx v) { return cx<A>{(A)v.real(), (A)v.imag()}; }

template <typename A>
inline bool is_zero(cplx v) { return (A)v.real() == (A)0 && (A)v.imag() == (A)0; }

// Coefficients of one axis in the arithmetic type.  Stages whose multiplier
// rounds to zero are dropped (every later one is zero too: it is the square
// of the previous); stages that would reach past the last lane are dropped
// because no lane has a partner there.  The correction is kept up to its last
// position that does not round to zero.
template <typename A>
inline gpssc::SweepCoef<A> sweep_coef(const AxisTables &t, const cplx *zt, double dt, double dx)
{
    gpssc::SweepCoef<A> k;
    k.kap = (A)(dt / (2.0 * dx * dx));
    k.m = to_cx<A>(t.m);
    k.a = to_cx<A>(t.a);
    k.nst = 0;
    for (int s = 0; s < gpssc::kMaxStages; ++s) {
        k.stage[s] = to_cx<A>(t.stage[s]);
        if ((1 << s) < t.lanes && !is_zero<A>(t.stage[s]) && k.nst == s) k.nst = s + 1;
    }
    int nz = (int)t.n;
    while (nz > 0 && is_zero<A>(zt[nz - 1])) --nz;
    k.nzc = nz;
    return k;
}

template <typename A>
inline gpssc::SweepCoef<A> sweep_coef(const AxisTables &t, double dt, double dx)
{
    return sweep_coef<A>(t, t.zt.data(), dt, dx);
}

// Device image of the correction vectors of the three axes, in the
// arithmetic type, each padded to chunk * lanes positions.
template <typename A>
inline std::vector<unsigned char> pack_tables(const AxisTables ax[3], size_t off[3])
{
    std::vector<cx<A>> v;
    for (int a = 0; a < 3; ++a) {
        off[a] = v.size();
        for (const cplx &z : ax[a].zt) v.push_back(to_cx<A>(z));
        const size_t npad = (size_t)ax[a].chunk * ax[a].lanes;
        while (v.size() - off[a] < npad) v.push_back(cx<A>{0, 0});
    }
    std::vector<unsigned char> bytes(v.size() * sizeof(cx<A>));
    std::memcpy(bytes.data(), v.data(), bytes.size());
    for (int q = 0; q < 3; ++q) off[q] *= sizeof(cx<A>);
    return bytes;
}

inline bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

inline bool valid_dtype(gp_dtype d)
{
    return d == GP_C128 || d == GP_C64 || d == GP_C64_F64 || d == GP_R64 || d == GP_R32;
}

inline bool valid_grid(const int64_t grid[3])
{
    if (!grid) return false;
    for (int a = 0; a < 3; ++a)
        if (grid[a] < 1) return false;
    return true;
}

class DeviceGuard {
  public:
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
        if (prev_ != dev) (void)hipSetDevice(dev);
        dev_ = dev;
    }
    ~DeviceGuard()
    {
        if (prev_ >= 0 && prev_ != dev_) (void)hipSetDevice(prev_);
    }

  private:
    int prev_ = -1, dev_ = 0;
};

}  // namespace gpssc_host
