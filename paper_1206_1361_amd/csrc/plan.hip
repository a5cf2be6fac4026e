// plan.hip -- host side of libgpssc: argument checks, the constant
// Crank-Nicolson / Thomas tables, device scratch, and the launch sequence of
// one split-step Crank-Nicolson step.  Implements include/gpssc.h.
//
// Paper: "Method of solution" of program summaries (v) and (xiv) (split-step
// Crank-Nicolson propagation in imaginary or real time over small steps) and
// "Summary of revisions" (the routines calcnu, calclux, calcluy, calcluz,
// calcnorm, calcmuen, calcrms that make up a step and its diagnostics).
#include "gpssc.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <algorithm>
#include <vector>

#include "gp_internal.h"
#include "host_common.h"

namespace gpssc_host {
thread_local std::string g_last_error;
}  // namespace gpssc_host

using namespace gpssc_host;

namespace {

struct ProfRec {
    int cls;
    hipEvent_t a, b;
};

}  // namespace

// A gp_step call's key for replay, and one recorded call.
struct StepKey {
    const void *psi;
    int64_t nsteps;
    bool operator==(const StepKey &o) const { return psi == o.psi && nsteps == o.nsteps; }
};
struct StepGraph {
    StepKey key;
    hipGraph_t graph;
    hipGraphExec_t exec;
    uint64_t used;   // call counter of its last launch
};
constexpr size_t kStepKeys = 4, kStepGraphs = 4;

struct gp_plan {
    int ndim = 3;        // space variables: x (1), x and y (2), or all three
    int64_t n[3];
    double dx[3];
    double dt, omega[3], g;
    gp_mode mode;
    gp_dtype dtype;
    hipStream_t stream;
    int device;

    AxisTables ax[3];
    int xt_y, xt_z;
    int x_blocks, y_blocks, z_blocks;   // blocks launched per sweep
    // complex64 with an even nx and long lines: the y/z threads take column
    // pairs (16-byte rows per thread) whenever psi is 16-byte aligned
    bool pairs_y = false, pairs_z = false;
    int xt2_y = 0, xt2_z = 0, y2_blocks = 0, z2_blocks = 0;
    // y/z strategy: block length of the streaming sweep, or 0 for the
    // chunked scan; stream_ok: the longest admissible block (0: none)
    int blk_y = 0, blk_z = 0, blk_ok_y = 0, blk_ok_z = 0;

    unsigned char *d_tables = nullptr;
    size_t tab_off[3];
    double *d_partials = nullptr;   // z-sweep norm partials, one per z line
    int n_zblocks = 0;
    double *d_obs_partials = nullptr;
    int n_obs_blocks = 0;
    double *d_scale = nullptr;
    int *d_flag = nullptr;
    double *d_sums = nullptr;
    double *h_sums = nullptr;   // pinned
    int *h_flag = nullptr;      // pinned

    int64_t steps_done = 0;
    hipEvent_t ev_switch = nullptr;   // orders a new stream after the old one (gp_set_stream)
    // gp_step replay: a call that repeats one of the last kStepKeys calls
    // (same psi, same step count) has its launches captured once, on
    // cap_stream, into a graph that later identical calls replay on the
    // plan's stream (at most kStepGraphs graphs, the least recently used
    // dropped first).  Any change of the launches' arguments (g, trap, sweep
    // strategy) drops them all.
    hipStream_t cap_stream = nullptr;
    std::vector<StepGraph> graphs;
    std::vector<StepKey> recent;      // the last calls' keys, oldest first
    uint64_t calls = 0;
    bool graph_off = false;           // a capture failed: launch eagerly from then on
    bool profiling = false;
    std::vector<ProfRec> prof;
    std::vector<hipEvent_t> pool;

    gpssc::XArgs<double> xd;
    gpssc::XArgs<float> xf;
    gpssc::SArgs<double> sd[2];
    gpssc::SArgs<float> sf[2];

    // symmetric traps (gp_plan_create_radial): 0 = Cartesian, else a gp_geom;
    // x is the radial axis, y the z axis of the axial trap
    int geom = 0;
    unsigned char *d_rtab = nullptr;   // six coefficient arrays (arithmetic type)
    double *d_rv = nullptr, *d_rs = nullptr;   // cell and face weights
    gpssc::RadialArgs<double> rd;
    gpssc::RadialArgs<float> rf;
};

namespace {

// zt[a]: the boundary correction of axis a (its last nonzero position sets
// how far the kernels apply it).
template <typename A>
void fill_args(gp_plan *p, const cplx *const zt[3], gpssc::XArgs<A> &x, gpssc::SArgs<A> s[2])
{
    x.nx = (int)p->n[0];
    x.ny = (int)p->n[1];
    x.nz = (int)p->n[2];
    x.c0x = (A)(0.5 * (double)(p->n[0] - 1));
    x.c0y = (A)(0.5 * (double)(p->n[1] - 1));
    x.c0z = (A)(0.5 * (double)(p->n[2] - 1));
    x.dx = (A)p->dx[0];
    x.dy = (A)p->dx[1];
    x.dz = (A)p->dx[2];
    x.hgx = (A)(0.5 * p->omega[0] * p->omega[0]);
    x.hgy = (A)(0.5 * p->omega[1] * p->omega[1]);
    x.hgz = (A)(0.5 * p->omega[2] * p->omega[2]);
    x.dt = (A)p->dt;
    x.g = (A)p->g;
    x.k = sweep_coef<A>(p->ax[0], zt[0], p->dt, p->dx[0]);
    for (int a = 1; a < 3; ++a) {
        gpssc::SArgs<A> &t = s[a - 1];
        t.nx = (int)p->n[0];
        t.n = (int)p->n[a];
        t.lanes = p->ax[a].lanes;
        t.stride = a == 1 ? p->n[0] : p->n[0] * p->n[1];
        t.outer_stride = a == 1 ? p->n[0] * p->n[1] : p->n[0];
        t.k = sweep_coef<A>(p->ax[a], zt[a], p->dt, p->dx[a]);
    }
}

hipEvent_t take_event(gp_plan *p)
{
    if (!p->pool.empty()) {
        hipEvent_t e = p->pool.back();
        p->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Runs one launcher, bracketed by events while profiling.
template <typename F>
hipError_t timed(gp_plan *p, int cls, F &&launch)
{
    if (!p->profiling) return launch();
    hipEvent_t a = take_event(p), b = take_event(p);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, p->stream);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, p->stream);
    p->prof.push_back(ProfRec{cls, a, b});
    return e;
}

size_t footprint(const int64_t grid[3], gp_dtype dtype, int *xt_y, int *xt_z)
{
    int c[3], l[3];
    for (int a = 0; a < 3; ++a)
        if (!sweep_shape(grid[a], a, &c[a], &l[a], max_lanes_for(dtype, grid[a]))) return 0;
    const size_t cs = arith_f32(dtype) ? 8 : 16;   // table entries: complex<float> or <double>
    size_t tab = 0;
    for (int a = 0; a < 3; ++a) tab += (size_t)c[a] * l[a];
    tab *= cs;
    const int xy = strided_columns(grid[0], l[1], c[1], dtype);
    const int xz = strided_columns(grid[0], l[2], c[2], dtype);
    if (xt_y) *xt_y = xy;
    if (xt_z) *xt_z = xz;
    const size_t zblocks = (size_t)grid[0] * (size_t)grid[1];   // norm partials, one per z line
    const size_t oblocks = (size_t)gpssc::obs_num_blocks((int)grid[0], (int)grid[1]);
    return tab + zblocks * 8 + oblocks * gpssc::OBS_NSUMS * 8 + 8 + 8 + gpssc::OBS_NSUMS * 8;
}

void release(gp_plan *p)
{
    if (!p) return;
    for (ProfRec &r : p->prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
    if (p->ev_switch) (void)hipEventDestroy(p->ev_switch);
    for (StepGraph &g : p->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->d_tables) (void)hipFree(p->d_tables);
    if (p->d_partials) (void)hipFree(p->d_partials);
    if (p->d_obs_partials) (void)hipFree(p->d_obs_partials);
    if (p->d_scale) (void)hipFree(p->d_scale);
    if (p->d_flag) (void)hipFree(p->d_flag);
    if (p->d_sums) (void)hipFree(p->d_sums);
    if (p->h_sums) (void)hipHostFree(p->h_sums);
    if (p->h_flag) (void)hipHostFree(p->h_flag);
    if (p->d_rtab) (void)hipFree(p->d_rtab);
    if (p->d_rv) (void)hipFree(p->d_rv);
    if (p->d_rs) (void)hipFree(p->d_rs);
    delete p;
}

constexpr double kPi = 3.14159265358979323846;

// Dimension and solid angle of a symmetric trap's radial axis.
int radial_dim(int geom) { return geom == GP_GEOM_SPHERICAL ? 3 : 2; }
double radial_solid_angle(int geom) { return geom == GP_GEOM_SPHERICAL ? 4.0 * kPi : 2.0 * kPi; }

// Volume factor of a grid cell: S_D h (times dz for the axial trap); the
// cell weights v_i carry the rest.
double radial_cell(const gp_plan *p)
{
    const double c = radial_solid_angle(p->geom) * p->dx[0];
    return p->geom == GP_GEOM_AXIAL ? c * p->dx[1] : c;
}

// Radial weights and Crank-Nicolson coefficients, FP64.  Face weights
// s_i = ((i+1) h)^(D-1) (the face at (i + 1) h), cell weights
// v_i = ((i+1)^D - i^D) h^(D-1) / D, and with T = -1/2 L,
// L the finite-volume Laplacian [s_i (u_{i+1} - u_i) - s_{i-1} (u_i - u_{i-1})] / (h^2 v_i)
// (s_{-1} = 0: no flux through the origin):
//   right side (1 - tau/2 T) u, left matrix 1 + tau/2 T, the latter
//   factorised by the Thomas recursion into m_i, a_i (forward) and b_i
//   (backward).  Positions past the line keep zero coefficients.
void radial_tables(int dim, int64_t n, double h, double dt, bool real, int npad, std::vector<cplx> &tab,
                   std::vector<double> &v, std::vector<double> &sf)
{
    const cplx tau = real ? cplx(0.0, dt) : cplx(dt, 0.0);
    v.assign((size_t)n, 0.0);
    sf.assign((size_t)n, 0.0);
    for (int64_t i = 0; i < n; ++i) {
        sf[(size_t)i] = std::pow((double)(i + 1) * h, dim - 1);
        v[(size_t)i] = (std::pow((double)(i + 1), dim) - std::pow((double)i, dim)) * std::pow(h, dim - 1) / dim;
    }
    tab.assign(6 * (size_t)npad, cplx(0.0, 0.0));
    cplx cprev(0.0, 0.0);
    for (int64_t i = 0; i < n; ++i) {
        const double below = i > 0 ? sf[(size_t)i - 1] : 0.0, above = sf[(size_t)i];
        const double c = 1.0 / (2.0 * h * h * v[(size_t)i]);
        const cplx t_ii = (below + above) * c, t_lo = -below * c, t_up = -above * c;
        const cplx half = 0.5 * tau;
        const cplx l_lo = half * t_lo, l_ii = 1.0 + half * t_ii, l_up = half * t_up;   // left matrix row
        const cplx den = l_ii - l_lo * cprev;
        const cplx cur = l_up / den;
        tab[0 * (size_t)npad + i] = 1.0 - half * t_ii;   // rd
        tab[1 * (size_t)npad + i] = -half * t_lo;        // rl
        tab[2 * (size_t)npad + i] = -half * t_up;        // ru
        tab[3 * (size_t)npad + i] = 1.0 / den;           // m
        tab[4 * (size_t)npad + i] = -l_lo / den;         // a
        tab[5 * (size_t)npad + i] = -cur;                // b
        cprev = cur;
    }
}

// Arguments of a plan (gp_plan_create_nd), checked before any device call;
// on success chunk and lanes hold the chunking of every axis.
gp_status check_plan_args(int ndim, const int64_t grid[3], const double dx[3], double dt, const double om[3],
                          double g, gp_mode mode, gp_dtype dtype, int chunk[3], int lanes[3])
{
    if (!valid_grid(grid)) return fail(GP_ERR_INVALID, "grid sizes must be >= 1");
    if (ndim < 1 || ndim > 3) return fail(GP_ERR_INVALID, "ndim must be 1, 2 or 3");
    for (int a = ndim; a < 3; ++a)
        if (grid[a] != 1) return fail(GP_ERR_INVALID, "axes beyond ndim must have one node");
    if (!dx || !finite_pos(dx[0]) || !finite_pos(dx[1]) || !finite_pos(dx[2]))
        return fail(GP_ERR_INVALID, "dx must be finite and > 0");
    if (!finite_pos(dt)) return fail(GP_ERR_INVALID, "dt must be finite and > 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(om[a]) || om[a] < 0.0)
            return fail(GP_ERR_INVALID, "trap frequencies must be finite and >= 0");
    if (!std::isfinite(g)) return fail(GP_ERR_INVALID, "g must be finite");
    if (mode != GP_MODE_IMAG && mode != GP_MODE_REAL) return fail(GP_ERR_INVALID, "unknown mode");
    if (!valid_dtype(dtype)) return fail(GP_ERR_INVALID, "unknown dtype");
    if (real_storage(dtype) && mode != GP_MODE_IMAG)
        return fail(GP_ERR_INVALID, "real storage (GP_R64, GP_R32) holds imaginary-time states only");
    for (int a = 0; a < 3; ++a)
        if (!sweep_shape(grid[a], a, &chunk[a], &lanes[a], max_lanes_for(dtype, grid[a])))
            return fail(GP_ERR_UNSUPPORTED, "grid line too long (Nx <= 1024, Ny, Nz <= 1024)");
    if (grid[1] * grid[2] > 0x7fffffffLL || grid[1] > 65535 || grid[2] > 65535)
        return fail(GP_ERR_UNSUPPORTED, "too many grid lines for one launch");
    return GP_OK;
}

// y/z strategy of a plan (the radial plans keep the chunked scan on their
// Cartesian z axis).
void set_sweep(gp_plan *p, gp_sweep s)
{
    const int ok[2] = {p->blk_ok_y, p->blk_ok_z};
    int *blk[2] = {&p->blk_y, &p->blk_z};
    for (int a = 0; a < 2; ++a) {
        if (s == GP_SWEEP_CHUNKED)
            *blk[a] = 0;
        else if (s == GP_SWEEP_STREAM)
            *blk[a] = ok[a];
        else
            *blk[a] = stream_by_default(ok[a], p->dtype) ? ok[a] : 0;
    }
}

// Blocks per sweep and the complex64 column pairs, from the grid, the dtype
// and the chunking (p->ax, p->xt_y, p->xt_z set).  One block per line (x)
// or tile (y, z): blocks that finish early make room for the next ones, so
// the blocks on a compute unit drift out of step and their load, compute and
// store phases overlap.  (A grid of resident blocks looping over the work
// keeps them in lockstep and was measured slower.)
void set_launch_shapes(gp_plan *p)
{
    const int64_t *grid = p->n;
    const int64_t xl = gpssc::x_lines_per_wave(p->ax[0].chunk, grid[1] * grid[2]);
    p->x_blocks = (int)((grid[1] * grid[2] + xl - 1) / xl);
    p->y_blocks = (int)(((grid[0] + p->xt_y - 1) / p->xt_y) * grid[2]);
    p->z_blocks = (int)(((grid[0] + p->xt_z - 1) / p->xt_z) * grid[1]);
    p->pairs_y = pair_axis(p->dtype, grid, 1);
    p->pairs_z = pair_axis(p->dtype, grid, 2);
    if (p->pairs_y) {
        p->xt2_y = strided_pair_columns(grid[0], p->ax[1].lanes, p->ax[1].chunk);
        p->y2_blocks = (int)(((grid[0] + 2 * p->xt2_y - 1) / (2 * p->xt2_y)) * grid[2]);
    }
    if (p->pairs_z) {
        p->xt2_z = strided_pair_columns(grid[0], p->ax[2].lanes, p->ax[2].chunk);
        p->z2_blocks = (int)(((grid[0] + 2 * p->xt2_z - 1) / (2 * p->xt2_z)) * grid[1]);
    }
    const bool f32 = arith_f32(p->dtype);
    p->blk_ok_y = p->ndim >= 2 ? stream_block_len(p->ax[1], f32) : 0;
    p->blk_ok_z = p->ndim >= 3 ? stream_block_len(p->ax[2], f32) : 0;
    set_sweep(p, GP_SWEEP_AUTO);
}

gp_status check_psi(const gp_plan *p, const void *psi, int64_t elems)
{
    if (!psi) return fail(GP_ERR_INVALID, "psi is NULL");
    const int64_t want = p->n[0] * p->n[1] * p->n[2];
    if (elems != want)
        return fail(GP_ERR_INVALID, "psi holds " + std::to_string(elems) + " elements, the grid needs " +
                                        std::to_string(want));
    const uintptr_t align = storage_bytes(p->dtype);
    if ((uintptr_t)psi % align != 0) return fail(GP_ERR_INVALID, "psi is misaligned");
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, psi);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(GP_ERR_INVALID, "psi is not a device pointer");
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return fail(GP_ERR_INVALID, "psi is not device memory");
    if (attr.device != p->device) return fail(GP_ERR_INVALID, "psi lives on another device than the plan");
    return GP_OK;
}

gp_status read_flag(gp_plan *p)
{
    hipError_t e = hipMemcpyAsync(p->h_flag, p->d_flag, sizeof(int), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return fail_hip(e, "synchronising the plan's stream");
    if (*p->h_flag) {
        *p->h_flag = 0;
        e = hipMemcpyAsync(p->d_flag, p->h_flag, sizeof(int), hipMemcpyHostToDevice, p->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) return fail_hip(e, "clearing the error flag");
        return fail(GP_ERR_NONFINITE, "the norm became zero or non-finite during imaginary-time steps");
    }
    return GP_OK;
}

// Forgets the recorded calls (their launches hold the old arguments), after
// waiting for the plan's stream, where a replay of them may still run.
void drop_step_graph(gp_plan *p)
{
    if (!p->graphs.empty()) (void)hipStreamSynchronize(p->stream);
    for (StepGraph &g : p->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    p->graphs.clear();
    p->recent.clear();
}

void set_g(gp_plan *p, double g)
{
    drop_step_graph(p);
    p->g = g;
    p->xd.g = g;
    p->xf.g = (float)g;
    p->rd.x.g = g;
    p->rf.x.g = (float)g;
}

void set_trap(gp_plan *p, const double om_in[3])
{
    drop_step_graph(p);
    double om[3];
    if (p->geom) {   // radial axis: gamma; the axial trap's z (stored along y): lambda
        om[0] = om_in[0];
        om[1] = p->geom == GP_GEOM_AXIAL ? om_in[2] : 0.0;
        om[2] = 0.0;
    } else {
        for (int a = 0; a < 3; ++a) om[a] = a < p->ndim ? om_in[a] : 0.0;   // no trap along absent axes
    }
    for (int a = 0; a < 3; ++a) p->omega[a] = om[a];
    p->xd.hgx = 0.5 * om[0] * om[0];
    p->xd.hgy = 0.5 * om[1] * om[1];
    p->xd.hgz = 0.5 * om[2] * om[2];
    p->xf.hgx = (float)p->xd.hgx;
    p->xf.hgy = (float)p->xd.hgy;
    p->xf.hgz = (float)p->xd.hgz;
    p->rd.x.hgx = p->xd.hgx;
    p->rd.x.hgy = p->xd.hgy;
    p->rd.x.hgz = p->xd.hgz;
    p->rf.x.hgx = p->xf.hgx;
    p->rf.x.hgy = p->xf.hgy;
    p->rf.x.hgz = p->xf.hgz;
}

// Queues the launches of nsteps steps on the plan's stream (psi checked).
hipError_t enqueue_steps(gp_plan *p, void *psi, int64_t nsteps, const double *g_steps, const double *trap_steps)
{
    const gpssc::Prec prec = static_cast<gpssc::Prec>(p->dtype);
    const bool a32 = arith_f32(p->dtype);   // FP32 arithmetic
    const bool real = p->mode == GP_MODE_REAL;
    const void *xargs = a32 ? (const void *)&p->xf : (const void *)&p->xd;
    const void *yargs = a32 ? (const void *)&p->sf[0] : (const void *)&p->sd[0];
    const void *zargs = a32 ? (const void *)&p->sf[1] : (const void *)&p->sd[1];
    const unsigned char *T = p->d_tables;
    const int nd = p->ndim;
    const bool aligned16 = reinterpret_cast<uintptr_t>(psi) % 16 == 0;
    const bool pair_y = p->pairs_y && aligned16, pair_z = p->pairs_z && aligned16;
    // the streamed sweeps of complex64 (FP32 arithmetic) take column pairs
    // whenever nx is even and psi 16-byte aligned
    const bool spair = p->dtype == GP_C64 && p->n[0] % 2 == 0 && aligned16;
    double dv = 1.0;
    for (int a = 0; a < nd; ++a) dv *= p->dx[a];
    // the last sweep leaves the norm partials, one per line along its axis
    double *parts = real ? nullptr : p->d_partials;
    int nparts = nd == 3 ? (int)(p->n[0] * p->n[1]) : (nd == 2 ? (int)(p->n[0] * p->n[2])
                                                                 : (int)(p->n[1] * p->n[2]));
    const double *weights = nullptr;
    if (p->geom) {   // symmetric traps: one partial per radial node, weighted by its cell
        dv = radial_cell(p);
        nparts = (int)p->n[0];
        weights = p->d_rv;
    }
    hipError_t e = hipSuccess;
    for (int64_t s = 0; s < nsteps && e == hipSuccess; ++s) {
        if (g_steps) set_g(p, g_steps[s]);
        if (trap_steps) set_trap(p, trap_steps + 3 * s);
        const double *scale = (!real && s > 0) ? p->d_scale : nullptr;
        e = timed(p, GP_KERNEL_NU_X, [&] {
            if (p->geom) {
                const void *rargs = a32 ? (const void *)&p->rf : (const void *)&p->rd;
                return gpssc::launch_nu_r(prec, real, p->ax[0].chunk, (int)(p->n[1] * p->n[2]), psi, rargs, scale,
                                          nd == 1 ? parts : nullptr, p->stream);
            }
            return gpssc::launch_nu_x(prec, real, p->ax[0].chunk, psi, xargs,
                                      T + p->tab_off[0], scale, nd == 1 ? parts : nullptr, p->stream);
        });
        if (e != hipSuccess) break;
        if (nd >= 2) {
            e = timed(p, GP_KERNEL_Y, [&] {
                if (p->blk_y)
                    return gpssc::launch_stream(prec, real, p->blk_y, spair ? 2 : 1, (int)p->n[2], psi, yargs,
                                                T + p->tab_off[1], nd == 2 ? parts : nullptr, p->stream);
                return gpssc::launch_strided(prec, real, p->ax[1].chunk, pair_y ? p->xt2_y : p->xt_y,
                                             pair_y ? 2 : 1, (int)p->n[2], psi, yargs, T + p->tab_off[1],
                                             nd == 2 ? parts : nullptr, true, p->stream);
            });
            if (e != hipSuccess) break;
        }
        if (nd == 3) {
            e = timed(p, GP_KERNEL_Z, [&] {
                if (p->blk_z)
                    return gpssc::launch_stream(prec, real, p->blk_z, spair ? 2 : 1, (int)p->n[1], psi, zargs,
                                                T + p->tab_off[2], parts, p->stream);
                return gpssc::launch_strided(prec, real, p->ax[2].chunk, pair_z ? p->xt2_z : p->xt_z,
                                             pair_z ? 2 : 1, (int)p->n[1], psi, zargs, T + p->tab_off[2], parts,
                                             false, p->stream);
            });
        }
        if (e != hipSuccess || real) continue;
        e = timed(p, GP_KERNEL_NORM, [&] {
            return gpssc::launch_norm_finalize(p->d_partials, nparts, dv, p->d_scale, p->d_flag, p->stream,
                                               weights);
        });
    }
    if (e == hipSuccess && !real) {
        const int64_t elems = p->n[0] * p->n[1] * p->n[2];
        e = timed(p, GP_KERNEL_SCALE,
                  [&] { return gpssc::launch_scale(prec, psi, elems, p->d_scale, p->stream); });
    }
    return e;
}

// The launches of nsteps steps on psi captured on the plan's capture stream
// into a new graph (nothing runs), which replaces the least recently used
// one when kStepGraphs are kept; on failure nothing is kept.
hipError_t capture_steps(gp_plan *p, void *psi, int64_t nsteps, StepGraph **out)
{
    hipError_t e = hipSuccess;
    if (!p->cap_stream) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    const hipStream_t user = p->stream;
    p->stream = p->cap_stream;   // the launchers queue on p->stream
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t le = enqueue_steps(p, psi, nsteps, nullptr, nullptr);
        e = hipStreamEndCapture(p->cap_stream, &g);
        if (le != hipSuccess) e = le;
        if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    }
    p->stream = user;
    if (e != hipSuccess) {
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
        return e;
    }
    if (p->graphs.size() >= kStepGraphs) {   // the least recently used one goes
        auto lru = std::min_element(p->graphs.begin(), p->graphs.end(),
                                    [](const StepGraph &a, const StepGraph &b) { return a.used < b.used; });
        (void)hipStreamSynchronize(user);   // a replay of it may still run
        (void)hipGraphExecDestroy(lru->exec);
        (void)hipGraphDestroy(lru->graph);
        p->graphs.erase(lru);
    }
    p->graphs.push_back(StepGraph{StepKey{psi, nsteps}, g, x, p->calls});
    *out = &p->graphs.back();
    return hipSuccess;
}

// Queues nsteps steps.  With schedules, step s uses g_steps[s] and the trap
// trap_steps[3s .. 3s+2]; the plan keeps the last step's values.  A call
// that repeats one of the last few (same psi and step count, no schedule,
// no profiling) is captured once and replayed from then on: the same
// launches with the same arguments, so the same results.
gp_status run_steps(gp_plan *p, void *psi, int64_t psi_elems, int64_t nsteps, const double *g_steps,
                    const double *trap_steps)
{
    DeviceGuard guard(p->device);
    gp_status st = check_psi(p, psi, psi_elems);
    if (st != GP_OK) return st;
    if (nsteps == 0) return GP_OK;
    // a caller capturing the plan's stream into a graph of its own gets the
    // launches themselves
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    bool capturing = false;
    if (hipStreamIsCapturing(p->stream, &cs) != hipSuccess) {
        (void)hipGetLastError();
        capturing = true;
    } else {
        capturing = cs != hipStreamCaptureStatusNone;
    }
    const bool plain = !g_steps && !trap_steps && !p->profiling && !p->graph_off && !capturing;
    hipError_t e = hipSuccess;
    const StepKey key{psi, nsteps};
    ++p->calls;
    StepGraph *hit = nullptr;
    if (plain)
        for (StepGraph &g : p->graphs)
            if (g.key == key) hit = &g;
    if (!hit && plain && std::find(p->recent.begin(), p->recent.end(), key) != p->recent.end()) {
        e = capture_steps(p, psi, nsteps, &hit);
        if (e != hipSuccess) {   // not capturable here: launch eagerly, now and later
            (void)hipGetLastError();
            p->graph_off = true;
            hit = nullptr;
        }
    }
    if (hit) {
        hit->used = p->calls;
        e = hipGraphLaunch(hit->exec, p->stream);
    } else {
        e = enqueue_steps(p, psi, nsteps, g_steps, trap_steps);
    }
    if (plain) {
        p->recent.erase(std::remove(p->recent.begin(), p->recent.end(), key), p->recent.end());
        p->recent.push_back(key);
        if (p->recent.size() > kStepKeys) p->recent.erase(p->recent.begin());
    }
    if (e != hipSuccess) return fail_hip(e, "launching a step kernel");
    p->steps_done += nsteps;
    return GP_OK;
}

// calcmuen / calcrms of a symmetric trap from the weighted sums of the
// radial observables kernel: dV = S_D h (dz) times the cell weights; the
// radial kinetic term summed by parts over the faces, S_D (dz) / (2h) sum
// s_i |u_{i+1} - u_i|^2; the z links of the axial trap as in Cartesian
// space.  rms and mean: slot 0 the radial variable, slot 1 z (axial).
gp_status radial_observables(gp_plan *p, const void *psi, gp_obs *out, gp_status earlier)
{
    gpssc::RadialObsArgs a;
    a.nr = (int)p->n[0];
    a.nz = (int)p->n[1];
    a.dr = p->dx[0];
    a.dz = p->geom == GP_GEOM_AXIAL ? p->dx[1] : 1.0;
    a.c0z = 0.5 * (double)(p->n[1] - 1);
    a.hgr = 0.5 * p->omega[0] * p->omega[0];
    a.hgz = 0.5 * p->omega[1] * p->omega[1];
    a.v = p->d_rv;
    a.s = p->d_rs;
    hipError_t e = timed(p, GP_KERNEL_OBS, [&] {
        return gpssc::launch_radial_observables(static_cast<gpssc::Prec>(p->dtype), psi, a, p->d_obs_partials,
                                                p->d_sums, p->stream);
    });
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->h_sums, p->d_sums, sizeof(double) * gpssc::OBS_NSUMS, hipMemcpyDeviceToHost,
                           p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return fail_hip(e, "computing observables");
    const double *S = p->h_sums;
    const double dv = radial_cell(p);
    const double hz = a.dz;
    const double norm = dv * S[gpssc::OBS_DENS];
    double kin = radial_solid_angle(p->geom) * (p->geom == GP_GEOM_AXIAL ? hz : 1.0) / (2.0 * p->dx[0]) *
                 S[gpssc::OBS_LINKX];
    if (p->geom == GP_GEOM_AXIAL) kin += 0.5 * dv * S[gpssc::OBS_LINKY] / (hz * hz);
    out->norm = norm;
    out->kinetic = kin / norm;
    out->potential = dv * S[gpssc::OBS_POT] / norm;
    out->interaction = p->g * dv * S[gpssc::OBS_QUART] / (norm * norm);
    out->energy = out->kinetic + out->potential + 0.5 * out->interaction;
    out->mu = out->kinetic + out->potential + out->interaction;
    out->rms[0] = std::sqrt(dv * S[gpssc::OBS_M2X] / norm);
    out->mean[0] = dv * S[gpssc::OBS_M1X] / norm;
    out->rms[1] = p->geom == GP_GEOM_AXIAL ? std::sqrt(dv * S[gpssc::OBS_M2Y] / norm) : 0.0;
    out->mean[1] = p->geom == GP_GEOM_AXIAL ? dv * S[gpssc::OBS_M1Y] / norm : 0.0;
    out->rms[2] = 0.0;
    out->mean[2] = 0.0;
    out->rms_r = std::sqrt(dv * (S[gpssc::OBS_M2X] + S[gpssc::OBS_M2Y]) / norm);
    out->steps_done = p->steps_done;
    if (earlier != GP_OK) return earlier;
    const double all[] = {out->norm, out->mu, out->energy, out->rms[0], out->rms[1], out->rms_r, out->mean[0],
                          out->mean[1], out->kinetic, out->potential, out->interaction};
    bool ok = norm > 0.0;
    for (double v : all) ok = ok && std::isfinite(v);
    if (!ok) return fail(GP_ERR_NONFINITE, "psi has a zero or non-finite norm or observable");
    return GP_OK;
}

}  // namespace

extern "C" {

const char *gp_status_string(gp_status s)
{
    switch (s) {
    case GP_OK: return "ok";
    case GP_ERR_INVALID: return "invalid argument";
    case GP_ERR_NOMEM: return "out of device memory";
    case GP_ERR_DEVICE: return "device error";
    case GP_ERR_NONFINITE: return "non-finite or zero norm";
    case GP_ERR_UNSUPPORTED: return "unsupported size";
    }
    return "unknown status";
}

const char *gp_last_error(void) { return g_last_error.c_str(); }

gp_status gp_sweep_shape(int64_t n, int axis, gp_dtype dtype, int *chunk, int *lanes)
{
    if (!chunk || !lanes || axis < 0 || axis > 2 || !valid_dtype(dtype))
        return fail(GP_ERR_INVALID, "bad gp_sweep_shape arguments");
    if (n < 1) return fail(GP_ERR_INVALID, "line length must be >= 1");
    if (!sweep_shape(n, axis, chunk, lanes, max_lanes_for(dtype, n))) return fail(GP_ERR_UNSUPPORTED, "line too long");
    return GP_OK;
}

gp_status gp_sweep_tables(int64_t n, double dx, double dt, gp_mode mode, int chunk, int lanes,
                          double *coef, size_t coef_len, double *stage, size_t stage_len,
                          double *zt, size_t zt_len)
{
    if (n < 1 || !finite_pos(dx) || !finite_pos(dt) || (mode != GP_MODE_IMAG && mode != GP_MODE_REAL) ||
        chunk < 1 || lanes < 1 || (int64_t)chunk * lanes < n || lanes > gpssc::kWave)
        return fail(GP_ERR_INVALID, "bad gp_sweep_tables arguments");
    if (!coef || coef_len < 14 || !stage || stage_len < 2 * (size_t)gpssc::kMaxStages || !zt ||
        zt_len < 2 * (size_t)n)
        return fail(GP_ERR_INVALID, "gp_sweep_tables output buffer too short");
    AxisTables t;
    build_axis(n, dx, dt, mode == GP_MODE_REAL, chunk, lanes, t);
    const cplx c7[7] = {t.kappa, t.b, t.o, t.c, t.beta, t.m, t.a};
    for (int q = 0; q < 7; ++q) {
        coef[2 * q] = c7[q].real();
        coef[2 * q + 1] = c7[q].imag();
    }
    for (int s = 0; s < gpssc::kMaxStages; ++s) {
        stage[2 * s] = t.stage[s].real();
        stage[2 * s + 1] = t.stage[s].imag();
    }
    for (int64_t i = 0; i < n; ++i) {
        zt[2 * i] = t.zt[(size_t)i].real();
        zt[2 * i + 1] = t.zt[(size_t)i].imag();
    }
    return GP_OK;
}

size_t gp_plan_footprint_bytes(const int64_t grid[3], gp_dtype dtype)
{
    if (!valid_grid(grid) || !valid_dtype(dtype)) return 0;
    return footprint(grid, dtype, nullptr, nullptr);
}

gp_status gp_plan_create(const int64_t grid[3], const double dx[3], double dt, double gamma,
                         double nu, double lambda, double g, gp_mode mode, gp_dtype dtype,
                         void *hip_stream, gp_plan **out)
{
    return gp_plan_create_nd(3, grid, dx, dt, gamma, nu, lambda, g, mode, dtype, hip_stream, out);
}

gp_status gp_plan_create_nd(int ndim, const int64_t grid[3], const double dx[3], double dt, double gamma,
                            double nu, double lambda, double g, gp_mode mode, gp_dtype dtype,
                            void *hip_stream, gp_plan **out)
{
    if (!out) return fail(GP_ERR_INVALID, "out is NULL");
    *out = nullptr;
    const double om[3] = {gamma, nu, lambda};
    int chunk[3], lanes[3];
    gp_status st = check_plan_args(ndim, grid, dx, dt, om, g, mode, dtype, chunk, lanes);
    if (st != GP_OK) return st;

    gp_plan *p = new (std::nothrow) gp_plan();
    if (!p) return fail(GP_ERR_NOMEM, "host allocation failed");
    p->ndim = ndim;
    for (int a = 0; a < 3; ++a) {
        p->n[a] = grid[a];
        p->dx[a] = dx[a];
        p->omega[a] = a < ndim ? om[a] : 0.0;   // no trap along absent axes
    }
    p->dt = dt;
    p->g = g;
    p->mode = mode;
    p->dtype = dtype;
    p->stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        release(p);
        return fail_hip(e, "hipGetDevice");
    }

    const bool real = mode == GP_MODE_REAL;
    for (int a = 0; a < 3; ++a) build_axis(grid[a], dx[a], dt, real, chunk[a], lanes[a], p->ax[a]);
    footprint(grid, dtype, &p->xt_y, &p->xt_z);
    std::vector<unsigned char> tab = arith_f32(dtype) ? pack_tables<float>(p->ax, p->tab_off)
                                                     : pack_tables<double>(p->ax, p->tab_off);
    p->n_zblocks = (int)(grid[0] * grid[1]);   // one norm partial per z line
    p->n_obs_blocks = gpssc::obs_num_blocks((int)grid[0], (int)grid[1]);

#define GP_ALLOC(ptr, bytes)                                                    \
    do {                                                                        \
        e = hipMalloc((void **)&(ptr), (bytes));                                \
        if (e != hipSuccess) {                                                  \
            (void)hipGetLastError();                                            \
            release(p);                                                         \
            return e == hipErrorOutOfMemory ? fail(GP_ERR_NOMEM, "hipMalloc failed") \
                                            : fail_hip(e, "hipMalloc");         \
        }                                                                       \
    } while (0)
    GP_ALLOC(p->d_tables, tab.size());
    GP_ALLOC(p->d_partials, sizeof(double) * (size_t)p->n_zblocks);
    GP_ALLOC(p->d_obs_partials, sizeof(double) * gpssc::OBS_NSUMS * (size_t)p->n_obs_blocks);
    GP_ALLOC(p->d_scale, sizeof(double));
    GP_ALLOC(p->d_flag, sizeof(int));
    GP_ALLOC(p->d_sums, sizeof(double) * gpssc::OBS_NSUMS);
#undef GP_ALLOC
    e = hipHostMalloc((void **)&p->h_sums, sizeof(double) * gpssc::OBS_NSUMS, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&p->h_flag, sizeof(int), hipHostMallocDefault);
    if (e != hipSuccess) {
        release(p);
        return fail_hip(e, "hipHostMalloc");
    }
    *p->h_flag = 0;
    e = hipMemcpyAsync(p->d_tables, tab.data(), tab.size(), hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(p->d_flag, p->h_flag, sizeof(int), hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) {
        release(p);
        return fail_hip(e, "uploading the tables");
    }
    const cplx *zt[3] = {p->ax[0].zt.data(), p->ax[1].zt.data(), p->ax[2].zt.data()};
    fill_args<double>(p, zt, p->xd, p->sd);
    fill_args<float>(p, zt, p->xf, p->sf);
    set_launch_shapes(p);
    *out = p;
    return GP_OK;
}

gp_status gp_plan_create_radial(gp_geom geom, const int64_t grid[3], const double dx[3], double dt,
                                double gamma, double nu, double lambda, double g, gp_mode mode, gp_dtype dtype,
                                void *hip_stream, gp_plan **out)
{
    if (!out) return fail(GP_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (geom != GP_GEOM_CIRCULAR && geom != GP_GEOM_SPHERICAL && geom != GP_GEOM_AXIAL)
        return fail(GP_ERR_INVALID, "unknown geometry");
    if (!std::isfinite(nu) || nu < 0.0 || !std::isfinite(lambda) || lambda < 0.0)
        return fail(GP_ERR_INVALID, "trap frequencies must be finite and >= 0");
    const int nd = geom == GP_GEOM_AXIAL ? 2 : 1;
    // gamma along the radial axis (x), lambda along z (stored along y) for the axial trap
    gp_status st = gp_plan_create_nd(nd, grid, dx, dt, gamma, geom == GP_GEOM_AXIAL ? lambda : 0.0, 0.0, g, mode,
                                     dtype, hip_stream, out);
    if (st != GP_OK) return st;
    gp_plan *p = *out;
    *out = nullptr;
    p->geom = geom;
    p->blk_ok_y = p->blk_ok_z = 0;   // the radial plans keep the chunked scan
    set_sweep(p, GP_SWEEP_AUTO);
    const int chunk = p->ax[0].chunk;
    const int npad = gpssc::kWave * chunk;
    std::vector<cplx> tab;
    std::vector<double> v, sf;
    radial_tables(radial_dim(geom), grid[0], dx[0], dt, mode == GP_MODE_REAL, npad, tab, v, sf);
    std::vector<unsigned char> bytes;
    if (arith_f32(dtype)) {
        std::vector<cx<float>> t(tab.size());
        for (size_t i = 0; i < tab.size(); ++i) t[i] = to_cx<float>(tab[i]);
        bytes.assign(reinterpret_cast<unsigned char *>(t.data()), reinterpret_cast<unsigned char *>(t.data() + t.size()));
    } else {
        std::vector<cx<double>> t(tab.size());
        for (size_t i = 0; i < tab.size(); ++i) t[i] = to_cx<double>(tab[i]);
        bytes.assign(reinterpret_cast<unsigned char *>(t.data()), reinterpret_cast<unsigned char *>(t.data() + t.size()));
    }
    DeviceGuard guard(p->device);
    hipError_t e = hipMalloc((void **)&p->d_rtab, bytes.size());
    if (e == hipSuccess) e = hipMalloc((void **)&p->d_rv, sizeof(double) * v.size());
    if (e == hipSuccess) e = hipMalloc((void **)&p->d_rs, sizeof(double) * sf.size());
    // the observables kernel keeps one partial row per z node
    if (e == hipSuccess && p->n_obs_blocks < (int)grid[1]) {
        (void)hipFree(p->d_obs_partials);
        p->d_obs_partials = nullptr;
        e = hipMalloc((void **)&p->d_obs_partials, sizeof(double) * gpssc::OBS_NSUMS * (size_t)grid[1]);
        p->n_obs_blocks = (int)grid[1];
    }
    if (e == hipSuccess) e = hipMemcpyAsync(p->d_rtab, bytes.data(), bytes.size(), hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->d_rv, v.data(), sizeof(double) * v.size(), hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->d_rs, sf.data(), sizeof(double) * sf.size(), hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        release(p);
        return e == hipErrorOutOfMemory ? fail(GP_ERR_NOMEM, "hipMalloc failed") : fail_hip(e, "radial tables");
    }
    p->rd.x = p->xd;
    p->rf.x = p->xf;
    p->rd.x.c0x = -0.5;    // node i at (i + 1/2) h
    p->rf.x.c0x = -0.5f;
    p->rd.tab = reinterpret_cast<const cx<double> *>(p->d_rtab);
    p->rf.tab = reinterpret_cast<const cx<float> *>(p->d_rtab);
    p->rd.npad = p->rf.npad = npad;
    *out = p;
    return GP_OK;
}

gp_status gp_plan_destroy(gp_plan *plan)
{
    if (!plan) return GP_OK;
    {
        DeviceGuard guard(plan->device);
        (void)hipStreamSynchronize(plan->stream);
        release(plan);
    }
    return GP_OK;
}

gp_status gp_set_g(gp_plan *plan, double g)
{
    if (!plan) return fail(GP_ERR_INVALID, "plan is NULL");
    if (!std::isfinite(g)) return fail(GP_ERR_INVALID, "g must be finite");
    DeviceGuard guard(plan->device);
    set_g(plan, g);
    return GP_OK;
}

gp_status gp_set_stream(gp_plan *plan, void *hip_stream)
{
    if (!plan) return fail(GP_ERR_INVALID, "plan is NULL");
    hipStream_t next = static_cast<hipStream_t>(hip_stream);
    if (next == plan->stream) return GP_OK;
    // work queued later on the new stream starts after everything already
    // queued on the old one: both use the plan's scratch (the pending
    // 1/sqrt(N), the partial sums, the error flag)
    DeviceGuard guard(plan->device);
    hipError_t e = hipSuccess;
    if (!plan->ev_switch) e = hipEventCreateWithFlags(&plan->ev_switch, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(plan->ev_switch, plan->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(next, plan->ev_switch, 0);
    if (e != hipSuccess) return fail_hip(e, "ordering the new stream after the old one");
    plan->stream = next;
    return GP_OK;
}

gp_status gp_set_trap(gp_plan *plan, double gamma, double nu, double lambda)
{
    if (!plan) return fail(GP_ERR_INVALID, "plan is NULL");
    const double om[3] = {gamma, nu, lambda};
    for (double w : om)
        if (!std::isfinite(w) || w < 0.0) return fail(GP_ERR_INVALID, "trap frequencies must be finite and >= 0");
    DeviceGuard guard(plan->device);
    set_trap(plan, om);
    return GP_OK;
}

gp_status gp_step(gp_plan *p, void *psi, int64_t psi_elems, int64_t nsteps)
{
    if (!p) return fail(GP_ERR_INVALID, "plan is NULL");
    if (nsteps < 0) return fail(GP_ERR_INVALID, "nsteps must be >= 0");
    return run_steps(p, psi, psi_elems, nsteps, nullptr, nullptr);
}

gp_status gp_step_schedule(gp_plan *p, void *psi, int64_t psi_elems, int64_t nsteps,
                           const double *g_steps, const double *trap_steps)
{
    if (!p) return fail(GP_ERR_INVALID, "plan is NULL");
    if (nsteps < 0) return fail(GP_ERR_INVALID, "nsteps must be >= 0");
    for (int64_t s = 0; s < nsteps; ++s) {
        if (g_steps && !std::isfinite(g_steps[s])) return fail(GP_ERR_INVALID, "g schedule holds a non-finite value");
        if (trap_steps)
            for (int a = 0; a < 3; ++a)
                if (!std::isfinite(trap_steps[3 * s + a]) || trap_steps[3 * s + a] < 0.0)
                    return fail(GP_ERR_INVALID, "trap schedule holds a negative or non-finite value");
    }
    return run_steps(p, psi, psi_elems, nsteps, g_steps, trap_steps);
}

gp_status gp_sync(gp_plan *p)
{
    if (!p) return fail(GP_ERR_INVALID, "plan is NULL");
    DeviceGuard guard(p->device);
    return read_flag(p);
}

gp_status gp_observables(gp_plan *p, const void *psi, int64_t psi_elems, gp_obs *out)
{
    if (!p) return fail(GP_ERR_INVALID, "plan is NULL");
    if (!out) return fail(GP_ERR_INVALID, "out is NULL");
    DeviceGuard guard(p->device);
    gp_status st = check_psi(p, psi, psi_elems);
    if (st != GP_OK) return st;
    const gp_status earlier = read_flag(p);
    if (earlier == GP_ERR_DEVICE) return earlier;

    if (p->geom) return radial_observables(p, psi, out, earlier);
    gpssc::ObsArgs<double> a;
    a.nx = (int)p->n[0];
    a.ny = (int)p->n[1];
    a.nz = (int)p->n[2];
    a.c0x = 0.5 * (double)(p->n[0] - 1);
    a.c0y = 0.5 * (double)(p->n[1] - 1);
    a.c0z = 0.5 * (double)(p->n[2] - 1);
    a.dx = p->dx[0];
    a.dy = p->dx[1];
    a.dz = p->dx[2];
    a.hgx = 0.5 * p->omega[0] * p->omega[0];
    a.hgy = 0.5 * p->omega[1] * p->omega[1];
    a.hgz = 0.5 * p->omega[2] * p->omega[2];
    hipError_t e = timed(p, GP_KERNEL_OBS, [&] {
        return gpssc::launch_observables(static_cast<gpssc::Prec>(p->dtype), psi, a, p->d_obs_partials, p->d_sums,
                                         p->stream);
    });
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->h_sums, p->d_sums, sizeof(double) * gpssc::OBS_NSUMS,
                           hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return fail_hip(e, "computing observables");

    const double *S = p->h_sums;
    // present axes only: their cell volume and their kinetic links
    double dv = 1.0, links = 0.0;
    for (int q = 0; q < p->ndim; ++q) {
        dv *= p->dx[q];
        links += S[gpssc::OBS_LINKX + q] / (p->dx[q] * p->dx[q]);
    }
    const double norm = dv * S[gpssc::OBS_DENS];
    const double kin = 0.5 * dv * links;
    const double pot = dv * S[gpssc::OBS_POT];
    const double inter = p->g * dv * S[gpssc::OBS_QUART];
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
    out->steps_done = p->steps_done;
    if (earlier != GP_OK) return earlier;
    const double all[] = {out->norm, out->mu, out->energy, out->rms[0], out->rms[1], out->rms[2],
                          out->rms_r, out->mean[0], out->mean[1], out->mean[2], out->kinetic,
                          out->potential, out->interaction};
    bool ok = norm > 0.0;
    for (double v : all) ok = ok && std::isfinite(v);
    if (!ok) return fail(GP_ERR_NONFINITE, "psi has a zero or non-finite norm or observable");
    return GP_OK;
}

gp_status gp_density_profiles(gp_plan *p, const void *psi, int64_t psi_elems, double *px, double *py, double *pz)
{
    if (!p) return fail(GP_ERR_INVALID, "plan is NULL");
    if (!px || !py || !pz) return fail(GP_ERR_INVALID, "px, py and pz are required");
    if (p->geom) return fail(GP_ERR_UNSUPPORTED, "density profiles are for Cartesian plans");
    DeviceGuard guard(p->device);
    gp_status st = check_psi(p, psi, psi_elems);
    if (st != GP_OK) return st;
    const int64_t total = p->n[0] + p->n[1] + p->n[2];
    // profile weights: the spacings of the other present axes
    double w[3];
    for (int a = 0; a < 3; ++a) {
        w[a] = 1.0;
        for (int b = 0; b < p->ndim; ++b)
            if (b != a) w[a] *= p->dx[b];
    }
    double *d = nullptr, *h = nullptr;
    hipError_t e = hipMalloc((void **)&d, sizeof(double) * (size_t)total);
    if (e == hipSuccess) e = hipHostMalloc((void **)&h, sizeof(double) * (size_t)total, hipHostMallocDefault);
    if (e == hipSuccess)
        e = gpssc::launch_profiles(static_cast<gpssc::Prec>(p->dtype), psi, (int)p->n[0], (int)p->n[1], (int)p->n[2],
                                   w, d, p->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h, d, sizeof(double) * (size_t)total, hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e == hipSuccess) {
        std::memcpy(px, h, sizeof(double) * (size_t)p->n[0]);
        std::memcpy(py, h + p->n[0], sizeof(double) * (size_t)p->n[1]);
        std::memcpy(pz, h + p->n[0] + p->n[1], sizeof(double) * (size_t)p->n[2]);
    }
    if (d) (void)hipFree(d);
    if (h) (void)hipHostFree(h);
    if (e != hipSuccess) return fail_hip(e, "computing density profiles");
    return GP_OK;
}

gp_status gp_plan_describe(const gp_plan *p, char *buf, size_t len)
{
    if (!p || !buf || len == 0) return fail(GP_ERR_INVALID, "bad gp_plan_describe arguments");
    const bool a32 = arith_f32(p->dtype);
    int nst[3], nzc[3];
    const gpssc::SweepCoef<double> *kd[3] = {&p->xd.k, &p->sd[0].k, &p->sd[1].k};
    const gpssc::SweepCoef<float> *kf[3] = {&p->xf.k, &p->sf[0].k, &p->sf[1].k};
    for (int a = 0; a < 3; ++a) {
        nst[a] = a32 ? kf[a]->nst : kd[a]->nst;
        nzc[a] = a32 ? kf[a]->nzc : kd[a]->nzc;
    }
    const char *names[] = {"c128", "c64", "c64/f64", "r64", "r32"};
    const char *geoms[] = {"", " circular", " spherical", " axial"};
    const char *dt = names[(int)p->dtype];
    // y/z columns per block: with column pairs (16-byte aligned psi), 2 per
    // thread; otherwise one
    char cols[2][64];
    for (int a = 0; a < 2; ++a) {
        const int xt = a ? p->xt_z : p->xt_y, blocks = a ? p->z_blocks : p->y_blocks;
        const int blk = a ? p->blk_z : p->blk_y;
        if (blk)
            std::snprintf(cols[a], sizeof cols[a], "streamed in blocks of %d%s", blk,
                          p->dtype == GP_C64 && p->n[0] % 2 == 0 ? ", column pairs when 16-byte aligned" : "");
        else if (a ? p->pairs_z : p->pairs_y)
            std::snprintf(cols[a], sizeof cols[a], "%d cols in pairs, %d blocks", 2 * (a ? p->xt2_z : p->xt2_y),
                          a ? p->z2_blocks : p->y2_blocks);
        else
            std::snprintf(cols[a], sizeof cols[a], "%d cols, %d blocks", xt, blocks);
    }
    std::snprintf(buf, len,
                  "grid %lldx%lldx%lld %dD%s %s %s | x: chunk %d x 64 lanes, %d stages, correction %d, "
                  "%d blocks | y: chunk %d x %d lanes, %d stages, correction %d, %s | "
                  "z: chunk %d x %d lanes, %d stages, correction %d, %s",
                  (long long)p->n[0], (long long)p->n[1], (long long)p->n[2], p->ndim, geoms[p->geom],
                  p->mode == GP_MODE_REAL ? "real" : "imag", dt, p->ax[0].chunk, nst[0], nzc[0],
                  p->x_blocks, p->ax[1].chunk, p->ax[1].lanes, nst[1], nzc[1], cols[0],
                  p->ax[2].chunk, p->ax[2].lanes, nst[2], nzc[2], cols[1]);
    return GP_OK;
}

gp_status gp_plan_set_sweep(gp_plan *p, gp_sweep strategy)
{
    if (!p) return fail(GP_ERR_INVALID, "plan is NULL");
    if (strategy != GP_SWEEP_AUTO && strategy != GP_SWEEP_CHUNKED && strategy != GP_SWEEP_STREAM)
        return fail(GP_ERR_INVALID, "unknown sweep strategy");
    DeviceGuard guard(p->device);
    drop_step_graph(p);
    set_sweep(p, strategy);
    return GP_OK;
}

gp_status gp_profile_enable(gp_plan *p, int on)
{
    if (!p) return fail(GP_ERR_INVALID, "plan is NULL");
    p->profiling = on != 0;
    return GP_OK;
}

gp_status gp_profile_read(gp_plan *p, double *ms, int64_t *launches)
{
    if (!p || !ms || !launches) return fail(GP_ERR_INVALID, "bad gp_profile_read arguments");
    DeviceGuard guard(p->device);
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return fail_hip(e, "synchronising the plan's stream");
    for (int k = 0; k < GP_KERNEL_COUNT; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (ProfRec &r : p->prof) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
            ms[r.cls] += t;
            launches[r.cls] += 1;
        }
        p->pool.push_back(r.a);
        p->pool.push_back(r.b);
    }
    p->prof.clear();
    return GP_OK;
}

}  // extern "C"

// ---- gp_step_noalloc: the step with its device memory in a static array ----
//
// For callers that cannot allocate device memory.  The correction tables of
// the three axes, one norm partial per z line, the 1/sqrt(N) slot and the
// error flag live in `scratch`, a fixed array that each device holds until
// the process ends.  Layout (bytes):
//   [0, 48 Ki)                   tables, each axis padded to chunk * lanes entries
//   [48 Ki, 48 Ki + 2 Mi)        norm partials, at most kNoallocMaxLines doubles
//   then 256 B                   1/sqrt(N) (double)
//   then 256 B                   error flag (int)
namespace {
constexpr int64_t kNoallocMaxLines = int64_t(1) << 18;   // Nx * Ny
constexpr size_t kNoallocTableBytes = 3 * 1024 * sizeof(cx<double>);
constexpr size_t kNoallocPartialOff = kNoallocTableBytes;
constexpr size_t kNoallocScaleOff = kNoallocPartialOff + (size_t)kNoallocMaxLines * sizeof(double);
constexpr size_t kNoallocFlagOff = kNoallocScaleOff + 256;
constexpr size_t kNoallocBytes = kNoallocFlagOff + 256;
constexpr int kNoallocMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {

// Table words written by one install launch; they travel as a kernel
// argument (copied at launch), so no host buffer has to outlive the call.
constexpr int kInstallWords = 256;
struct InstallWords {
    uint64_t w[kInstallWords];
};

__global__ void noalloc_install_kernel(uint64_t *dst, InstallWords src, int nwords, int *flag)
{
    const int t = threadIdx.x;
    if (t < nwords) dst[t] = src.w[t];
    if (flag && t == 0) *flag = 0;
}

// Guards the per-device addresses and the host staging of the tables.
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kNoallocMaxDevices];

struct NoallocHost {
    cplx zt[3][1024];
    cplx w[1024], z[1024];
};
NoallocHost g_noalloc_host;

// Device address of `scratch` on device dev (current), looked up once per
// device.  The array's name is only a host-side handle: kernels and copies
// take this address.  Call with g_noalloc_mu held.
void *noalloc_scratch(int dev, hipError_t *err)
{
    *err = hipSuccess;
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) return nullptr;
        g_noalloc_ptr[dev] = ptr;
    }
    return g_noalloc_ptr[dev];
}

// Writes the first nzc correction entries of every axis (the only ones the
// kernels read) into the device tables, in the arithmetic type A, and clears
// the error flag.
template <typename A>
hipError_t noalloc_install(gp_plan *p, const int nzc[3])
{
    InstallWords words;
    hipError_t e = hipSuccess;
    bool flag_cleared = false;
    constexpr int per = sizeof(cx<A>) / sizeof(uint64_t) > 0 ? (int)(sizeof(cx<A>) / sizeof(uint64_t)) : 1;
    for (int a = 0; a < 3 && e == hipSuccess; ++a) {
        const int nwords = nzc[a] * per;
        uint64_t *dst = reinterpret_cast<uint64_t *>(p->d_tables + p->tab_off[a]);
        for (int w0 = 0; w0 < nwords && e == hipSuccess; w0 += kInstallWords) {
            const int nw = nwords - w0 < kInstallWords ? nwords - w0 : kInstallWords;
            for (int q = 0; q < nw; q += per) {
                const cx<A> v = to_cx<A>(g_noalloc_host.zt[a][(w0 + q) / per]);
                std::memcpy(&words.w[q], &v, sizeof v);
            }
            hipLaunchKernelGGL(noalloc_install_kernel, dim3(1), dim3(kInstallWords), 0, p->stream, dst + w0, words,
                               nw, flag_cleared ? nullptr : p->d_flag);
            flag_cleared = true;
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess && !flag_cleared) {
        hipLaunchKernelGGL(noalloc_install_kernel, dim3(1), dim3(kInstallWords), 0, p->stream, nullptr, words, 0,
                           p->d_flag);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace

extern "C" {

gp_status gp_step_noalloc(const int64_t grid[3], const double dx[3], double dt, double gamma, double nu,
                          double lambda, double g, gp_mode mode, gp_dtype dtype, void *hip_stream, void *psi,
                          int64_t psi_elems, int64_t nsteps)
{
    const double om[3] = {gamma, nu, lambda};
    int chunk[3], lanes[3];
    gp_status st = check_plan_args(3, grid, dx, dt, om, g, mode, dtype, chunk, lanes);
    if (st != GP_OK) return st;
    if (nsteps < 0) return fail(GP_ERR_INVALID, "nsteps must be >= 0");
    if (grid[0] * grid[1] > kNoallocMaxLines)
        return fail(GP_ERR_UNSUPPORTED, "gp_step_noalloc: Nx*Ny = " + std::to_string(grid[0] * grid[1]) +
                                            " exceeds its scratch maximum of " + std::to_string(kNoallocMaxLines) +
                                            " z lines");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev < 0 || dev >= kNoallocMaxDevices) return fail(GP_ERR_UNSUPPORTED, "gp_step_noalloc: device index too high");

    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    unsigned char *base = static_cast<unsigned char *>(noalloc_scratch(dev, &e));
    if (!base) return fail_hip(e, "hipGetSymbolAddress of the static scratch array");

    // a plan on the stack whose device memory is the static array
    gp_plan p;
    for (int a = 0; a < 3; ++a) {
        p.n[a] = grid[a];
        p.dx[a] = dx[a];
        p.omega[a] = om[a];
    }
    p.dt = dt;
    p.g = g;
    p.mode = mode;
    p.dtype = dtype;
    p.stream = static_cast<hipStream_t>(hip_stream);
    p.device = dev;
    p.graph_off = true;   // no step replay: it would record call keys and graphs
    const bool real = mode == GP_MODE_REAL;
    const cplx *zt[3];
    size_t elem_off = 0;
    const size_t cs = arith_f32(dtype) ? sizeof(cx<float>) : sizeof(cx<double>);
    for (int a = 0; a < 3; ++a) {
        build_axis_into(grid[a], dx[a], dt, real, chunk[a], lanes[a], p.ax[a], g_noalloc_host.zt[a],
                        g_noalloc_host.w, g_noalloc_host.z);
        zt[a] = g_noalloc_host.zt[a];
        p.tab_off[a] = elem_off * cs;   // the padded layout of pack_tables
        elem_off += (size_t)chunk[a] * lanes[a];
    }
    footprint(grid, dtype, &p.xt_y, &p.xt_z);
    p.n_zblocks = (int)(grid[0] * grid[1]);
    p.d_tables = base;
    p.d_partials = reinterpret_cast<double *>(base + kNoallocPartialOff);
    p.d_scale = reinterpret_cast<double *>(base + kNoallocScaleOff);
    p.d_flag = reinterpret_cast<int *>(base + kNoallocFlagOff);
    fill_args<double>(&p, zt, p.xd, p.sd);
    fill_args<float>(&p, zt, p.xf, p.sf);
    set_launch_shapes(&p);

    st = check_psi(&p, psi, psi_elems);
    if (st != GP_OK) return st;
    if (nsteps == 0) return GP_OK;
    DeviceGuard guard(dev);
    const bool a32 = arith_f32(dtype);
    const int nzc[3] = {a32 ? p.xf.k.nzc : p.xd.k.nzc, a32 ? p.sf[0].k.nzc : p.sd[0].k.nzc,
                        a32 ? p.sf[1].k.nzc : p.sd[1].k.nzc};
    e = a32 ? noalloc_install<float>(&p, nzc) : noalloc_install<double>(&p, nzc);
    if (e != hipSuccess) return fail_hip(e, "installing the tables");
    return run_steps(&p, psi, psi_elems, nsteps, nullptr, nullptr);
}

}  // extern "C"
