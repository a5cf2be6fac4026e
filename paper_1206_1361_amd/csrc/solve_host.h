// solve_host.h -- host-side description of one solve inside a batched
// launch, shared by the fixed batch (batch.hip) and the request server
// (server.hip): its parameters and Crank-Nicolson tables, the launch shape
// of its grid-shape class, the per-solve kernel arguments, and the
// observables built from the kernels' FP64 sums.  Internal to libgpssc.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gp_internal.h"
#include "gpssc.h"
#include "host_common.h"

namespace gpssc_host {

struct SolveDesc {
    int64_t grid[3];
    double dx[3], dt, omega[3], g;
    bool real;
    AxisTables ax[3];
    int64_t elems;
};

// Launch shape shared by every solve of one grid shape.
struct ClassShape {
    int64_t grid[3];
    int chunk[3], lanes[3];
    bool pairs_ok;           // complex64 with an even nx: y/z may take column pairs
    int xt_y, xt_z;          // threads across a y/z block
    int cols_y, cols_z;      // columns per thread (1, or 2 = pairs)
    int nlines, ncol_y, ntiles_y, ncol_z, ntiles_z, obs_blocks;
};

inline void class_tiles(ClassShape &c)
{
    c.nlines = (int)(c.grid[1] * c.grid[2]);
    const int64_t wy = (int64_t)c.xt_y * c.cols_y, wz = (int64_t)c.xt_z * c.cols_z;
    c.ncol_y = (int)((c.grid[0] + wy - 1) / wy);
    c.ntiles_y = c.ncol_y * (int)c.grid[2];
    c.ncol_z = (int)((c.grid[0] + wz - 1) / wz);
    c.ntiles_z = c.ncol_z * (int)c.grid[1];
    c.obs_blocks = gpssc::obs_num_blocks((int)c.grid[0], (int)c.grid[1]);
}

// y/z block width of a class axis (1 = y, 2 = z) at `cols` columns per
// thread.
inline int class_columns(const ClassShape &c, int ax, int cols, gp_dtype dtype)
{
    return cols == 2 ? strided_pair_columns(c.grid[0], c.lanes[ax], c.chunk[ax])
                     : strided_columns(c.grid[0], c.lanes[ax], c.chunk[ax], dtype);
}

// Chunking, lanes and default y/z block shapes of a grid (the grid must
// have passed sweep_shape on every axis): column pairs as pair_axis says.
inline ClassShape class_shape(const int64_t grid[3], gp_dtype dtype)
{
    ClassShape c;
    for (int a = 0; a < 3; ++a) {
        c.grid[a] = grid[a];
        sweep_shape(grid[a], a, &c.chunk[a], &c.lanes[a], max_lanes_for(dtype, grid[a]));
    }
    c.pairs_ok = dtype == GP_C64 && grid[0] % 2 == 0;
    c.cols_y = pair_axis(dtype, grid, 1) ? 2 : 1;
    c.cols_z = pair_axis(dtype, grid, 2) ? 2 : 1;
    c.xt_y = class_columns(c, 1, c.cols_y, dtype);
    c.xt_z = class_columns(c, 2, c.cols_z, dtype);
    class_tiles(c);
    return c;
}

inline bool grid_supported(const int64_t grid[3], gp_dtype dtype)
{
    int c, l;
    for (int a = 0; a < 3; ++a)
        if (!sweep_shape(grid[a], a, &c, &l, max_lanes_for(dtype, grid[a]))) return false;
    return true;
}

inline size_t complex_bytes(gp_dtype dtype) { return arith_f32(dtype) ? sizeof(cx<float>) : sizeof(cx<double>); }

// Bytes of the three correction tables of a solve (chunk * lanes entries per
// axis, in the arithmetic type).
inline size_t table_bytes(const ClassShape &c, gp_dtype dtype)
{
    size_t n = 0;
    for (int a = 0; a < 3; ++a) n += complex_bytes(dtype) * (size_t)c.chunk[a] * (size_t)c.lanes[a];
    return n;
}

inline void build_solve(SolveDesc &x, const ClassShape &c)
{
    for (int a = 0; a < 3; ++a)
        build_axis(x.grid[a], x.dx[a], x.dt, x.real, c.chunk[a], c.lanes[a], x.ax[a]);
    x.elems = x.grid[0] * x.grid[1] * x.grid[2];
}

// Writes the three correction tables of a solve at dst (table_bytes long,
// zero past each axis' length).
inline void pack_solve_tables(const SolveDesc &x, const ClassShape &c, gp_dtype dtype, unsigned char *dst)
{
    std::memset(dst, 0, table_bytes(c, dtype));
    size_t off = 0;
    for (int a = 0; a < 3; ++a) {
        for (int64_t q = 0; q < x.grid[a]; ++q) {
            if (arith_f32(dtype)) {
                const cx<float> v = to_cx<float>(x.ax[a].zt[(size_t)q]);
                std::memcpy(dst + off + (size_t)q * sizeof v, &v, sizeof v);
            } else {
                const cx<double> v = to_cx<double>(x.ax[a].zt[(size_t)q]);
                std::memcpy(dst + off + (size_t)q * sizeof v, &v, sizeof v);
            }
        }
        off += complex_bytes(dtype) * (size_t)c.chunk[a] * (size_t)c.lanes[a];
    }
}

// Kernel arguments of one solve; d_tab: the device address of its packed
// correction tables.
template <typename A>
void fill_solve_args(const SolveDesc &x, const ClassShape &c, const unsigned char *d_tab,
                     gpssc::XBatchArgs<A> &xa, gpssc::SBatchArgs<A> &ya, gpssc::SBatchArgs<A> &za)
{
    gpssc::XArgs<A> &a = xa.x;
    a.nx = (int)x.grid[0];
    a.ny = (int)x.grid[1];
    a.nz = (int)x.grid[2];
    a.c0x = (A)(0.5 * (double)(x.grid[0] - 1));
    a.c0y = (A)(0.5 * (double)(x.grid[1] - 1));
    a.c0z = (A)(0.5 * (double)(x.grid[2] - 1));
    a.dx = (A)x.dx[0];
    a.dy = (A)x.dx[1];
    a.dz = (A)x.dx[2];
    a.hgx = (A)(0.5 * x.omega[0] * x.omega[0]);
    a.hgy = (A)(0.5 * x.omega[1] * x.omega[1]);
    a.hgz = (A)(0.5 * x.omega[2] * x.omega[2]);
    a.dt = (A)x.dt;
    a.g = (A)x.g;
    a.k = sweep_coef<A>(x.ax[0], x.dt, x.dx[0]);
    size_t off = 0;
    xa.zt = reinterpret_cast<const cx<A> *>(d_tab);
    off += sizeof(cx<A>) * (size_t)c.chunk[0] * (size_t)c.lanes[0];
    gpssc::SBatchArgs<A> *yz[2] = {&ya, &za};
    for (int ax = 1; ax < 3; ++ax) {
        gpssc::SArgs<A> &t = yz[ax - 1]->s;
        t.nx = (int)x.grid[0];
        t.n = (int)x.grid[ax];
        t.lanes = c.lanes[ax];
        t.stride = ax == 1 ? x.grid[0] : x.grid[0] * x.grid[1];
        t.outer_stride = ax == 1 ? x.grid[0] * x.grid[1] : x.grid[0];
        t.k = sweep_coef<A>(x.ax[ax], x.dt, x.dx[ax]);
        yz[ax - 1]->zt = reinterpret_cast<const cx<A> *>(d_tab + off);
        off += sizeof(cx<A>) * (size_t)c.chunk[ax] * (size_t)c.lanes[ax];
    }
}

inline gpssc::ObsArgs<double> obs_args(const SolveDesc &x)
{
    gpssc::ObsArgs<double> o;
    o.nx = (int)x.grid[0];
    o.ny = (int)x.grid[1];
    o.nz = (int)x.grid[2];
    o.c0x = 0.5 * (double)(x.grid[0] - 1);
    o.c0y = 0.5 * (double)(x.grid[1] - 1);
    o.c0z = 0.5 * (double)(x.grid[2] - 1);
    o.dx = x.dx[0];
    o.dy = x.dx[1];
    o.dz = x.dx[2];
    o.hgx = 0.5 * x.omega[0] * x.omega[0];
    o.hgy = 0.5 * x.omega[1] * x.omega[1];
    o.hgz = 0.5 * x.omega[2] * x.omega[2];
    return o;
}

// Observables from the FP64 sums of the observables kernels (the
// per-particle definitions of calcmuen / calcrms).
inline gp_status obs_from_sums(const double *S, const SolveDesc &x, gp_obs *out, int64_t steps)
{
    const double dv = x.dx[0] * x.dx[1] * x.dx[2];
    const double norm = dv * S[gpssc::OBS_DENS];
    const double kin = 0.5 * dv *
                       (S[gpssc::OBS_LINKX] / (x.dx[0] * x.dx[0]) + S[gpssc::OBS_LINKY] / (x.dx[1] * x.dx[1]) +
                        S[gpssc::OBS_LINKZ] / (x.dx[2] * x.dx[2]));
    const double pot = dv * S[gpssc::OBS_POT];
    const double inter = x.g * dv * S[gpssc::OBS_QUART];
    out->norm = norm;
    out->kinetic = kin / norm;
    out->potential = pot / norm;
    out->interaction = inter / (norm * norm);
    out->energy = out->kinetic + out->potential + 0.5 * out->interaction;
    out->mu = out->kinetic + out->potential + out->interaction;
    double r2 = 0.0;
    for (int q = 0; q < 3; ++q) {
        const double m2 = dv * S[gpssc::OBS_M2X + q] / norm;
        out->rms[q] = std::sqrt(m2);
        out->mean[q] = dv * S[gpssc::OBS_M1X + q] / norm;
        r2 += m2;
    }
    out->rms_r = std::sqrt(r2);
    out->steps_done = steps;
    bool ok = norm > 0.0 && std::isfinite(out->mu) && std::isfinite(out->energy) && std::isfinite(out->rms_r);
    return ok ? GP_OK : GP_ERR_NONFINITE;
}

inline bool valid_params(const double dx[3], double dt, const double trap[3], double g)
{
    for (int a = 0; a < 3; ++a) {
        if (!finite_pos(dx[a])) return false;
        if (!std::isfinite(trap[a]) || trap[a] < 0.0) return false;
    }
    return finite_pos(dt) && std::isfinite(g);
}

}  // namespace gpssc_host
