// batch.hip -- many independent solves advanced together (gp_batch_*).
//
// Solves with the same grid shape form a class; one launch per class and
// sweep covers every active solve of the class, reading each solve's psi
// pointer, coefficients and trap from device arrays.  A step of all classes
// is captured once into a HIP graph and replayed.  Every per-solve number
// comes from the same device functions as a single plan (gp_plan_*), so a
// solve gives bitwise the same result alone and inside a batch.
//
// Paper: the split-step Crank-Nicolson step of program summaries (v) and
// (xiv) ("Method of solution"), with calcnu, calclux/y/z, calcnorm and
// calcmuen/calcrms as named in "Summary of revisions".
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "gp_internal.h"
#include "gpssc.h"
#include "host_common.h"
#include "solve_host.h"

using namespace gpssc_host;

namespace {

struct Solve : SolveDesc {
    int cls;
    int64_t part_off;        // into the per-line norm partials
    int64_t obs_off;         // into the observables partials
    size_t tab_off;          // bytes into the correction tables
    void *psi = nullptr;
};

struct Class : ClassShape {
    std::vector<int> members;
    int nact = 0;
    int *d_active = nullptr;     // active solve indices
    int x_lines = 0;             // x lines per wavefront (0: the library's rule; GP_BATCH_TUNE times them)
};

}  // namespace

struct gp_batch {
    int n = 0;
    gp_mode mode;
    gp_dtype dtype;
    int flags = 0;
    int device = 0;
    hipStream_t caller = nullptr;   // ordering with the caller's work
    hipStream_t own = nullptr;      // the batch's queue (capturable)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<Solve> s;
    std::vector<Class> cls;
    std::vector<unsigned char> active;

    unsigned char *d_tables = nullptr;
    unsigned char *d_xargs = nullptr, *d_yargs = nullptr, *d_zargs = nullptr;
    void **d_psis = nullptr;
    double *d_partials = nullptr;
    int64_t *d_part_off = nullptr;
    int64_t *d_obs_off = nullptr;
    double *d_dv = nullptr;
    double *d_scales = nullptr;
    int *d_flags = nullptr;
    gpssc::ObsArgs<double> *d_obsargs = nullptr;
    double *d_obs_partials = nullptr;
    double *d_sums = nullptr;
    double *h_sums = nullptr;   // pinned
    int *h_flags = nullptr;     // pinned
    void **h_psis = nullptr;    // pinned
    int *h_active = nullptr;    // pinned, staging for the class lists

    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_ok = false;
    int64_t steps_done = 0;
    // the captured step runs each class on a branch of its own (fork from
    // and join back to `own`), so the classes' launches overlap on the device
    std::vector<hipStream_t> branch;
    std::vector<hipEvent_t> ev_join;
    hipEvent_t ev_fork = nullptr;

    // GP_BATCH_FINISH_F64: the same solves in FP64 storage (complex128 for
    // complex64, float64 for float32), on buffers of the batch's own
    gp_batch *fin = nullptr;
    unsigned char *d_shadow = nullptr;
    std::vector<void *> shadow;

    // GP_BATCH_ONE_LAUNCH: each sweep of a step is one launch over every
    // class with active solves, described by these arrays (device, with a
    // pinned staging copy); rebuilt whenever the active lists or the class
    // shapes change
    gpssc::XClassDesc *d_xcls = nullptr;
    gpssc::YZClassDesc *d_ycls = nullptr, *d_zcls = nullptr;
    gpssc::NormClassDesc *d_ncls = nullptr;
    unsigned char *h_cls = nullptr;
    struct {
        int ncls = 0;
        int xblocks = 0, yblocks = 0, zblocks = 0, nblocks = 0;
        int cmax_x = 1, cmax_y = 1, cmax_z = 1;
        int lds_x = 0;
        int thr_y = 0, thr_z = 0;
        size_t lds_y = 0, lds_z = 0;
    } one;
};

namespace {

bool bound(const gp_batch *b)
{
    for (const Solve &x : b->s)
        if (!x.psi) return false;
    return true;
}

void release(gp_batch *b)
{
    if (!b) return;
    if (b->fin) {
        (void)hipStreamSynchronize(b->fin->own);
        release(b->fin);
    }
    if (b->d_shadow) (void)hipFree(b->d_shadow);
    void *cls_dev[] = {b->d_xcls, b->d_ycls, b->d_zcls, b->d_ncls};
    for (void *p : cls_dev)
        if (p) (void)hipFree(p);
    if (b->h_cls) (void)hipHostFree(b->h_cls);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (Class &c : b->cls)
        if (c.d_active) (void)hipFree(c.d_active);
    void *dev[] = {b->d_tables, b->d_xargs, b->d_yargs, b->d_zargs, b->d_psis, b->d_partials,
                   b->d_part_off, b->d_obs_off, b->d_dv, b->d_scales, b->d_flags, b->d_obsargs,
                   b->d_obs_partials, b->d_sums};
    for (void *p : dev)
        if (p) (void)hipFree(p);
    void *host[] = {b->h_sums, b->h_flags, b->h_psis, b->h_active};
    for (void *p : host)
        if (p) (void)hipHostFree(p);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    for (hipEvent_t e : b->ev_join) (void)hipEventDestroy(e);
    for (hipStream_t st : b->branch) (void)hipStreamDestroy(st);
    if (b->own) (void)hipStreamDestroy(b->own);
    delete b;
}

template <typename A>
std::vector<unsigned char> pack_batch_args(const gp_batch *b, int which)
{
    std::vector<unsigned char> out;
    for (const Solve &x : b->s) {
        gpssc::XBatchArgs<A> xa;
        gpssc::SBatchArgs<A> ya, za;
        fill_solve_args<A>(x, b->cls[(size_t)x.cls], b->d_tables + x.tab_off, xa, ya, za);
        const unsigned char *p;
        size_t len;
        if (which == 0) {
            p = reinterpret_cast<const unsigned char *>(&xa);
            len = sizeof xa;
        } else if (which == 1) {
            p = reinterpret_cast<const unsigned char *>(&ya);
            len = sizeof ya;
        } else {
            p = reinterpret_cast<const unsigned char *>(&za);
            len = sizeof za;
        }
        out.insert(out.end(), p, p + len);
    }
    return out;
}

// Bytes of one value a y/z thread holds per row (LDS per thread = 2 of
// them): the arithmetic's complex (or real) value, or a complex64 pair.
size_t yz_value_bytes(gp_dtype dtype, int cols)
{
    if (cols == 2) return 16;
    if (dtype == GP_R32) return 4;
    if (dtype == GP_R64 || dtype == GP_C64) return 8;
    return 16;
}

// The class descriptors of GP_BATCH_ONE_LAUNCH from the classes' active
// counts and shapes (classes without active solves are left out), uploaded
// on the batch's own queue.
hipError_t upload_classes(gp_batch *b)
{
    if (!(b->flags & GP_BATCH_ONE_LAUNCH)) return hipSuccess;
    const size_t nc = b->cls.size();
    gpssc::XClassDesc *hx = reinterpret_cast<gpssc::XClassDesc *>(b->h_cls);
    gpssc::YZClassDesc *hy = reinterpret_cast<gpssc::YZClassDesc *>(hx + nc);
    gpssc::YZClassDesc *hz = hy + nc;
    gpssc::NormClassDesc *hn = reinterpret_cast<gpssc::NormClassDesc *>(hz + nc);
    auto &o = b->one;
    o = {};
    int k = 0;
    for (const Class &c : b->cls) {
        if (!c.nact) continue;
        if ((int64_t)c.nact * c.nlines > INT32_MAX || (int64_t)c.nact * std::max(c.ntiles_y, c.ntiles_z) > INT32_MAX)
            return hipErrorInvalidValue;
        const int total = c.nact * c.nlines;
        const int L = c.x_lines ? c.x_lines : gpssc::x_lines_per_wave(c.chunk[0], total);
        hx[k] = gpssc::XClassDesc{o.xblocks, c.nlines, total, c.chunk[0], L, c.d_active};
        o.xblocks += (total + L - 1) / L;
        o.cmax_x = std::max(o.cmax_x, c.chunk[0]);
        o.lds_x = std::max(o.lds_x, L * (gpssc::kWave * c.chunk[0] + gpssc::kWave));
        hy[k] = gpssc::YZClassDesc{o.yblocks, c.ntiles_y, c.ncol_y, c.xt_y, c.lanes[1], c.chunk[1], c.cols_y,
                                   c.d_active};
        o.yblocks += c.nact * c.ntiles_y;
        o.cmax_y = std::max(o.cmax_y, c.chunk[1]);
        o.thr_y = std::max(o.thr_y, c.xt_y * c.lanes[1]);
        o.lds_y = std::max(o.lds_y, 2 * (size_t)c.xt_y * c.lanes[1] * yz_value_bytes(b->dtype, c.cols_y));
        hz[k] = gpssc::YZClassDesc{o.zblocks, c.ntiles_z, c.ncol_z, c.xt_z, c.lanes[2], c.chunk[2], c.cols_z,
                                   c.d_active};
        o.zblocks += c.nact * c.ntiles_z;
        o.cmax_z = std::max(o.cmax_z, c.chunk[2]);
        o.thr_z = std::max(o.thr_z, c.xt_z * c.lanes[2]);
        o.lds_z = std::max(o.lds_z, 2 * (size_t)c.xt_z * c.lanes[2] * yz_value_bytes(b->dtype, c.cols_z));
        hn[k] = gpssc::NormClassDesc{o.nblocks, (int)(c.grid[0] * c.grid[1]), c.d_active};
        o.nblocks += c.nact;
        ++k;
    }
    o.ncls = k;
    if (!k) return hipSuccess;
    hipError_t e = hipMemcpyAsync(b->d_xcls, hx, sizeof(*hx) * (size_t)k, hipMemcpyHostToDevice, b->own);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_ycls, hy, sizeof(*hy) * (size_t)k, hipMemcpyHostToDevice, b->own);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_zcls, hz, sizeof(*hz) * (size_t)k, hipMemcpyHostToDevice, b->own);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_ncls, hn, sizeof(*hn) * (size_t)k, hipMemcpyHostToDevice, b->own);
    if (e == hipSuccess) e = hipStreamSynchronize(b->own);
    return e;
}

// Uploads the active list of every class (pinned staging, stream-ordered on
// the batch's own queue, then waits so the staging can be reused).
hipError_t upload_active(gp_batch *b)
{
    int off = 0;
    for (Class &c : b->cls) {
        c.nact = 0;
        for (int m : c.members)
            if (b->active[(size_t)m]) b->h_active[off + c.nact++] = m;
        off += (int)c.members.size();
    }
    off = 0;
    for (Class &c : b->cls) {
        if (c.nact) {
            hipError_t e = hipMemcpyAsync(c.d_active, b->h_active + off, sizeof(int) * (size_t)c.nact,
                                          hipMemcpyHostToDevice, b->own);
            if (e != hipSuccess) return e;
        }
        off += (int)c.members.size();
    }
    hipError_t e = hipStreamSynchronize(b->own);
    if (e == hipSuccess) e = upload_classes(b);
    return e;
}

// One step of the active solves of one class, queued on `st`.
hipError_t enqueue_class(gp_batch *b, const Class &c, hipStream_t st)
{
    const gpssc::Prec prec = static_cast<gpssc::Prec>(b->dtype);
    const bool real = b->mode == GP_MODE_REAL;
    hipError_t e = gpssc::launch_nu_x_batch(prec, real, c.chunk[0], c.nact, c.nlines, b->d_psis, b->d_xargs,
                                            c.d_active, real ? nullptr : b->d_scales, st, c.x_lines);
    if (e != hipSuccess) return e;
    e = gpssc::launch_strided_batch(prec, real, c.chunk[1], c.xt_y, c.cols_y, c.lanes[1], c.nact, c.ncol_y,
                                    c.ntiles_y, b->d_psis, b->d_yargs, c.d_active, nullptr, nullptr, st);
    if (e != hipSuccess) return e;
    e = gpssc::launch_strided_batch(prec, real, c.chunk[2], c.xt_z, c.cols_z, c.lanes[2], c.nact, c.ncol_z,
                                    c.ntiles_z, b->d_psis, b->d_zargs, c.d_active,
                                    real ? nullptr : b->d_partials, b->d_part_off, st);
    if (e != hipSuccess || real) return e;
    return gpssc::launch_norm_finalize_batch(c.nact, c.d_active, b->d_partials, b->d_part_off,
                                             (int)(c.grid[0] * c.grid[1]), b->d_dv, b->d_scales, b->d_flags, st);
}

// GP_BATCH_ONE_LAUNCH: one step of every active solve in four launches
// (three in real time) over all classes, queued on `st`.
hipError_t enqueue_classes(gp_batch *b, hipStream_t st)
{
    const auto &o = b->one;
    if (!o.ncls) return hipSuccess;
    const gpssc::Prec prec = static_cast<gpssc::Prec>(b->dtype);
    const bool real = b->mode == GP_MODE_REAL;
    hipError_t e = gpssc::launch_nu_x_classes(prec, real, o.cmax_x, o.lds_x, o.xblocks, b->d_psis, b->d_xargs,
                                              b->d_xcls, o.ncls, real ? nullptr : b->d_scales, st);
    if (e == hipSuccess)
        e = gpssc::launch_strided_classes(prec, real, o.cmax_y, o.thr_y, o.lds_y, o.yblocks, b->d_psis,
                                          b->d_yargs, b->d_ycls, o.ncls, nullptr, nullptr, st);
    if (e == hipSuccess)
        e = gpssc::launch_strided_classes(prec, real, o.cmax_z, o.thr_z, o.lds_z, o.zblocks, b->d_psis,
                                          b->d_zargs, b->d_zcls, o.ncls, real ? nullptr : b->d_partials,
                                          b->d_part_off, st);
    if (e != hipSuccess || real) return e;
    return gpssc::launch_norm_finalize_classes(o.nblocks, b->d_ncls, o.ncls, b->d_partials, b->d_part_off,
                                               b->d_dv, b->d_scales, b->d_flags, st);
}

// One step of every active solve, queued on the batch's own stream.
hipError_t enqueue_step(gp_batch *b)
{
    if (b->flags & GP_BATCH_ONE_LAUNCH) return enqueue_classes(b, b->own);
    for (const Class &c : b->cls) {
        if (!c.nact) continue;
        hipError_t e = enqueue_class(b, c, b->own);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The same step as a fork/join over the classes: class k on branch[k],
// started after everything before it on `own` and joined back before
// anything after it.  The classes touch disjoint memory (each solve's psi,
// partials, scale and flag belong to one class), so only the order within
// a class matters, and every solve's result is unchanged.
// The branch streams and events, one per class (created before a capture
// begins).
hipError_t make_branches(gp_batch *b)
{
    hipError_t e = hipSuccess;
    if (!b->ev_fork) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
    while (e == hipSuccess && b->branch.size() < b->cls.size()) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (st) b->branch.push_back(st);
        if (ev) b->ev_join.push_back(ev);
    }
    return e;
}

hipError_t enqueue_step_branches(gp_batch *b)
{
    if (!b->ev_fork || b->branch.size() < b->cls.size()) return hipErrorInvalidValue;
    hipError_t e = hipEventRecord(b->ev_fork, b->own);
    for (size_t k = 0; k < b->cls.size() && e == hipSuccess; ++k) {
        const Class &c = b->cls[k];
        if (!c.nact) continue;
        e = hipStreamWaitEvent(b->branch[k], b->ev_fork, 0);
        if (e == hipSuccess) e = enqueue_class(b, c, b->branch[k]);
        if (e == hipSuccess) e = hipEventRecord(b->ev_join[k], b->branch[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->own, b->ev_join[k], 0);
    }
    return e;
}

hipError_t build_graph(gp_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_ok = false;
    const bool one = (b->flags & GP_BATCH_ONE_LAUNCH) != 0;
    hipError_t e = one ? hipSuccess : make_branches(b);
    if (e == hipSuccess) e = hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = one ? enqueue_classes(b, b->own) : enqueue_step_branches(b);
    e = hipStreamEndCapture(b->own, &b->graph);
    if (le != hipSuccess) return le;
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return e;
    b->graph_ok = true;
    return hipSuccess;
}

// Launch shapes of the y/z sweeps per class: the number of columns per
// block that runs fastest on this device, timed on scratch memory of one
// solve's size (the choice does not change any result: each column's
// arithmetic and its norm partial are independent of it).
hipError_t tune_class(gp_batch *b, Class &c)
{
    const Solve &x = b->s[(size_t)c.members[0]];
    void *scratch = nullptr;
    const size_t bytes = storage_bytes(b->dtype) * (size_t)x.elems;
    hipError_t e = hipMalloc(&scratch, bytes);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(scratch, 0, bytes, b->own);
    int *d_one = nullptr;
    void **d_ptr = nullptr;
    const int zero = 0;
    if (e == hipSuccess) e = hipMalloc(&d_one, sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&d_ptr, sizeof(void *) * (size_t)b->n);
    if (e == hipSuccess) e = hipMemcpyAsync(d_one, &zero, sizeof(int), hipMemcpyHostToDevice, b->own);
    // a pointer table whose entry for the first member is the scratch
    std::vector<void *> tab((size_t)b->n, scratch);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_ptr, tab.data(), sizeof(void *) * tab.size(), hipMemcpyHostToDevice, b->own);
    int m0 = c.members[0];
    int *d_m0 = nullptr;
    if (e == hipSuccess) e = hipMalloc(&d_m0, sizeof(int));
    if (e == hipSuccess) e = hipMemcpyAsync(d_m0, &m0, sizeof(int), hipMemcpyHostToDevice, b->own);
    if (e == hipSuccess) e = hipStreamSynchronize(b->own);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    const gpssc::Prec prec = static_cast<gpssc::Prec>(b->dtype);
    const bool real = b->mode == GP_MODE_REAL;
    for (int ax = 1; ax < 3 && e == hipSuccess; ++ax) {
        const int lanes = c.lanes[ax];
        const int nouter = (int)(ax == 1 ? c.grid[2] : c.grid[1]);
        int best = ax == 1 ? c.xt_y : c.xt_z;
        int best_cols = ax == 1 ? c.cols_y : c.cols_z;
        float best_ms = 1e30f;
        for (int cols = 1; cols <= (c.pairs_ok ? 2 : 1) && e == hipSuccess; ++cols)
        for (int xt : {16, 32, 64}) {
            if (xt * lanes > gpssc::kMaxBlockYZ) continue;
            if (xt > 16 && xt * cols / 2 >= c.grid[0]) continue;
            const int ncol = (int)((c.grid[0] + xt * cols - 1) / (xt * cols));
            const void *args = ax == 1 ? (const void *)b->d_yargs : (const void *)b->d_zargs;
            double *parts = (ax == 2 && !real) ? b->d_partials : nullptr;
            auto run = [&] {
                return gpssc::launch_strided_batch(prec, real, c.chunk[ax], xt, cols, lanes, 1, ncol,
                                                   ncol * nouter, d_ptr, args, d_m0, parts, b->d_part_off,
                                                   b->own);
            };
            e = run();  // warm
            if (e != hipSuccess) break;
            e = hipEventRecord(t0, b->own);
            for (int r = 0; r < 3 && e == hipSuccess; ++r) e = run();
            if (e == hipSuccess) e = hipEventRecord(t1, b->own);
            if (e == hipSuccess) e = hipEventSynchronize(t1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
            if (e == hipSuccess && ms < best_ms) {
                best_ms = ms;
                best = xt;
                best_cols = cols;
            }
        }
        if (ax == 1) {
            c.xt_y = best;
            c.cols_y = best_cols;
        } else {
            c.xt_z = best;
            c.cols_z = best_cols;
        }
    }
    // x: lines per wavefront, with every member of the class in the launch
    // (all aliased to the scratch: only the launch shape is timed)
    int *d_all = nullptr;
    const int nm = (int)c.members.size();
    if (e == hipSuccess) e = hipMalloc(&d_all, sizeof(int) * (size_t)nm);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_all, c.members.data(), sizeof(int) * (size_t)nm, hipMemcpyHostToDevice, b->own);
    if (e == hipSuccess) e = hipStreamSynchronize(b->own);
    float best_x = 1e30f;
    for (int L = 1; L <= gpssc::x_max_lines_per_wave(c.chunk[0]) && e == hipSuccess; L *= 2) {
        auto run = [&] {
            return gpssc::launch_nu_x_batch(prec, real, c.chunk[0], nm, c.nlines, d_ptr, b->d_xargs, d_all, nullptr,
                                            b->own, L);
        };
        e = run();  // warm
        if (e == hipSuccess) e = hipEventRecord(t0, b->own);
        for (int r = 0; r < 3 && e == hipSuccess; ++r) e = run();
        if (e == hipSuccess) e = hipEventRecord(t1, b->own);
        if (e == hipSuccess) e = hipEventSynchronize(t1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
        if (e == hipSuccess && ms < best_x) {
            best_x = ms;
            c.x_lines = L;
        }
    }
    if (d_all) (void)hipFree(d_all);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (d_m0) (void)hipFree(d_m0);
    if (d_ptr) (void)hipFree(d_ptr);
    if (d_one) (void)hipFree(d_one);
    (void)hipFree(scratch);
    return e;
}

hipError_t sync_in(gp_batch *b)
{
    hipError_t e = hipEventRecord(b->ev_in, b->caller);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->own, b->ev_in, 0);
    return e;
}

hipError_t sync_out(gp_batch *b)
{
    hipError_t e = hipEventRecord(b->ev_out, b->own);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->caller, b->ev_out, 0);
    return e;
}

gp_status solve_imag_finished(gp_batch *b, double tol, int64_t check_every, int64_t max_steps, gp_obs *out,
                              int64_t *steps, unsigned char *converged);

}  // namespace

extern "C" {

gp_status gp_batch_create(int nsolves, const int64_t *grids, const double *dx, const double *dt,
                          const double *traps, const double *g, gp_mode mode, gp_dtype dtype, int flags,
                          void *hip_stream, gp_batch **out)
{
    if (!out) return fail(GP_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (nsolves < 1 || !grids || !dx || !dt || !traps || !g)
        return fail(GP_ERR_INVALID, "need nsolves >= 1 and every parameter array");
    if (mode != GP_MODE_IMAG && mode != GP_MODE_REAL) return fail(GP_ERR_INVALID, "unknown mode");
    if (!valid_dtype(dtype)) return fail(GP_ERR_INVALID, "unknown dtype");
    if (real_storage(dtype) && mode != GP_MODE_IMAG)
        return fail(GP_ERR_INVALID, "real storage (GP_R64, GP_R32) holds imaginary-time states only");
    if (flags & ~(GP_BATCH_GRAPH | GP_BATCH_TUNE | GP_BATCH_FINISH_F64 | GP_BATCH_ONE_LAUNCH))
        return fail(GP_ERR_INVALID, "unknown flags");
    // The launch over every class is switched off: its first GPU test (the
    // complex64 case of test_one_launch_matches_per_class_launches_bitwise)
    // ended in a device fault whose cause is not found; a CPU emulation of
    // its kernels under AddressSanitizer shows every access in bounds and
    // its results bitwise equal to the per-class launches.
    if (flags & GP_BATCH_ONE_LAUNCH)
        return fail(GP_ERR_UNSUPPORTED, "GP_BATCH_ONE_LAUNCH is switched off (an unexplained device fault in its test)");
    if ((flags & GP_BATCH_FINISH_F64) && (mode != GP_MODE_IMAG || (dtype != GP_C64 && dtype != GP_R32)))
        return fail(GP_ERR_INVALID, "GP_BATCH_FINISH_F64 is for imaginary-time batches in GP_C64 or GP_R32");
    for (int i = 0; i < nsolves; ++i) {
        if (!valid_grid(grids + 3 * i)) return fail(GP_ERR_INVALID, "grid sizes must be >= 1");
        if (!valid_params(dx + 3 * i, dt[i], traps + 3 * i, g[i]))
            return fail(GP_ERR_INVALID, "dx and dt must be finite and > 0, traps finite and >= 0, g finite");
        if (!grid_supported(grids + 3 * i, dtype)) return fail(GP_ERR_UNSUPPORTED, "grid line too long (each <= 1024)");
    }
    gp_batch *b = new (std::nothrow) gp_batch();
    if (!b) return fail(GP_ERR_NOMEM, "host allocation failed");
    b->n = nsolves;
    b->mode = mode;
    b->dtype = dtype;
    b->flags = flags;
    b->caller = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
    if (e != hipSuccess) {
        release(b);
        return fail_hip(e, "creating the batch's stream");
    }
    const bool real = mode == GP_MODE_REAL;
    // classes by grid shape
    std::map<std::tuple<int64_t, int64_t, int64_t>, int> index;
    b->s.resize((size_t)nsolves);
    int64_t part = 0, obs = 0;
    size_t tab_bytes = 0;
    for (int i = 0; i < nsolves; ++i) {
        Solve &x = b->s[(size_t)i];
        for (int a = 0; a < 3; ++a) {
            x.grid[a] = grids[3 * i + a];
            x.dx[a] = dx[3 * i + a];
            x.omega[a] = traps[3 * i + a];
        }
        x.dt = dt[i];
        x.g = g[i];
        x.real = real;
        auto key = std::make_tuple(x.grid[0], x.grid[1], x.grid[2]);
        auto it = index.find(key);
        if (it == index.end()) {
            Class c;
            static_cast<ClassShape &>(c) = class_shape(x.grid, dtype);
            it = index.emplace(key, (int)b->cls.size()).first;
            b->cls.push_back(c);
        }
        x.cls = it->second;
        Class &c = b->cls[(size_t)x.cls];
        c.members.push_back(i);
        build_solve(x, c);
        x.tab_off = tab_bytes;
        tab_bytes += table_bytes(c, dtype);
        x.part_off = part;
        part += x.grid[0] * x.grid[1];
        x.obs_off = obs;
        obs += (int64_t)c.obs_blocks * gpssc::OBS_NSUMS;
    }
    b->active.assign((size_t)nsolves, 1);
    // tables
    std::vector<unsigned char> tab(tab_bytes, 0);
    for (const Solve &x : b->s) pack_solve_tables(x, b->cls[(size_t)x.cls], dtype, tab.data() + x.tab_off);
#define GB_ALLOC(ptr, bytes)                                                          \
    do {                                                                              \
        e = hipMalloc((void **)&(ptr), (bytes));                                      \
        if (e != hipSuccess) {                                                        \
            (void)hipGetLastError();                                                  \
            release(b);                                                               \
            return e == hipErrorOutOfMemory ? fail(GP_ERR_NOMEM, "hipMalloc failed")  \
                                            : fail_hip(e, "hipMalloc");               \
        }                                                                             \
    } while (0)
    GB_ALLOC(b->d_tables, std::max<size_t>(tab_bytes, 16));
    const size_t xs = arith_f32(dtype) ? sizeof(gpssc::XBatchArgs<float>) : sizeof(gpssc::XBatchArgs<double>);
    const size_t ss = arith_f32(dtype) ? sizeof(gpssc::SBatchArgs<float>) : sizeof(gpssc::SBatchArgs<double>);
    GB_ALLOC(b->d_xargs, xs * (size_t)nsolves);
    GB_ALLOC(b->d_yargs, ss * (size_t)nsolves);
    GB_ALLOC(b->d_zargs, ss * (size_t)nsolves);
    GB_ALLOC(b->d_psis, sizeof(void *) * (size_t)nsolves);
    GB_ALLOC(b->d_partials, sizeof(double) * (size_t)std::max<int64_t>(part, 1));
    GB_ALLOC(b->d_part_off, sizeof(int64_t) * (size_t)nsolves);
    GB_ALLOC(b->d_obs_off, sizeof(int64_t) * (size_t)nsolves);
    GB_ALLOC(b->d_dv, sizeof(double) * (size_t)nsolves);
    GB_ALLOC(b->d_scales, sizeof(double) * (size_t)nsolves);
    GB_ALLOC(b->d_flags, sizeof(int) * (size_t)nsolves);
    GB_ALLOC(b->d_obsargs, sizeof(gpssc::ObsArgs<double>) * (size_t)nsolves);
    GB_ALLOC(b->d_obs_partials, sizeof(double) * (size_t)obs);
    GB_ALLOC(b->d_sums, sizeof(double) * gpssc::OBS_NSUMS * (size_t)nsolves);
    for (Class &c : b->cls) GB_ALLOC(c.d_active, sizeof(int) * c.members.size());
    if (flags & GP_BATCH_ONE_LAUNCH) {
        const size_t nc = b->cls.size();
        GB_ALLOC(b->d_xcls, sizeof(gpssc::XClassDesc) * nc);
        GB_ALLOC(b->d_ycls, sizeof(gpssc::YZClassDesc) * nc);
        GB_ALLOC(b->d_zcls, sizeof(gpssc::YZClassDesc) * nc);
        GB_ALLOC(b->d_ncls, sizeof(gpssc::NormClassDesc) * nc);
    }
#undef GB_ALLOC
    e = hipHostMalloc((void **)&b->h_sums, sizeof(double) * gpssc::OBS_NSUMS * (size_t)nsolves, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_flags, sizeof(int) * (size_t)nsolves, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_psis, sizeof(void *) * (size_t)nsolves, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_active, sizeof(int) * (size_t)nsolves, hipHostMallocDefault);
    if (e == hipSuccess && (flags & GP_BATCH_ONE_LAUNCH))
        e = hipHostMalloc((void **)&b->h_cls,
                          b->cls.size() * (sizeof(gpssc::XClassDesc) + 2 * sizeof(gpssc::YZClassDesc) +
                                           sizeof(gpssc::NormClassDesc)),
                          hipHostMallocDefault);
    if (e != hipSuccess) {
        release(b);
        return fail_hip(e, "hipHostMalloc");
    }
    // per-solve constants
    std::vector<int64_t> offs((size_t)nsolves), ooffs((size_t)nsolves);
    std::vector<double> dvs((size_t)nsolves), ones((size_t)nsolves, 1.0);
    std::vector<int> zeros((size_t)nsolves, 0);
    std::vector<gpssc::ObsArgs<double>> oa((size_t)nsolves);
    for (int i = 0; i < nsolves; ++i) {
        const Solve &x = b->s[(size_t)i];
        offs[(size_t)i] = x.part_off;
        ooffs[(size_t)i] = x.obs_off;
        dvs[(size_t)i] = x.dx[0] * x.dx[1] * x.dx[2];
        oa[(size_t)i] = obs_args(x);
    }
    std::vector<unsigned char> xa = arith_f32(dtype) ? pack_batch_args<float>(b, 0) : pack_batch_args<double>(b, 0);
    std::vector<unsigned char> ya = arith_f32(dtype) ? pack_batch_args<float>(b, 1) : pack_batch_args<double>(b, 1);
    std::vector<unsigned char> za = arith_f32(dtype) ? pack_batch_args<float>(b, 2) : pack_batch_args<double>(b, 2);
    struct Up {
        void *dst;
        const void *src;
        size_t n;
    } ups[] = {
        {b->d_tables, tab.data(), tab.size()},
        {b->d_xargs, xa.data(), xa.size()},
        {b->d_yargs, ya.data(), ya.size()},
        {b->d_zargs, za.data(), za.size()},
        {b->d_part_off, offs.data(), sizeof(int64_t) * offs.size()},
        {b->d_obs_off, ooffs.data(), sizeof(int64_t) * ooffs.size()},
        {b->d_dv, dvs.data(), sizeof(double) * dvs.size()},
        {b->d_scales, ones.data(), sizeof(double) * ones.size()},
        {b->d_flags, zeros.data(), sizeof(int) * zeros.size()},
        {b->d_obsargs, oa.data(), sizeof(gpssc::ObsArgs<double>) * oa.size()},
    };
    for (const Up &u : ups)
        if (e == hipSuccess && u.n) e = hipMemcpyAsync(u.dst, u.src, u.n, hipMemcpyHostToDevice, b->own);
    if (e == hipSuccess) e = hipStreamSynchronize(b->own);
    if (e == hipSuccess && (flags & GP_BATCH_TUNE)) {
        for (Class &c : b->cls) {
            e = tune_class(b, c);
            if (e != hipSuccess) break;
            class_tiles(c);
        }
        // the tuned shapes change the per-solve y/z arguments only through
        // the block shape, which the kernels read from blockDim
    }
    if (e == hipSuccess) e = upload_active(b);
    if (e != hipSuccess) {
        release(b);
        return fail_hip(e, "setting up the batch");
    }
    if (flags & GP_BATCH_FINISH_F64) {
        const gp_dtype fd = dtype == GP_C64 ? GP_C128 : GP_R64;
        gp_status st = gp_batch_create(nsolves, grids, dx, dt, traps, g, mode, fd, flags & ~GP_BATCH_FINISH_F64,
                                       hip_stream, &b->fin);
        if (st != GP_OK) {
            release(b);
            return st;
        }
        std::vector<size_t> off((size_t)nsolves);
        std::vector<int64_t> elems((size_t)nsolves);
        size_t total = 0;
        for (int i = 0; i < nsolves; ++i) {
            off[(size_t)i] = total;
            elems[(size_t)i] = b->s[(size_t)i].elems;
            total += ((size_t)elems[(size_t)i] * storage_bytes(fd) + 255) / 256 * 256;
        }
        e = hipMalloc((void **)&b->d_shadow, total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            release(b);
            return e == hipErrorOutOfMemory ? fail(GP_ERR_NOMEM, "hipMalloc of the FP64 states failed")
                                            : fail_hip(e, "hipMalloc");
        }
        b->shadow.resize((size_t)nsolves);
        for (int i = 0; i < nsolves; ++i) b->shadow[(size_t)i] = b->d_shadow + off[(size_t)i];
        st = gp_batch_set_psi(b->fin, b->shadow.data(), elems.data());
        if (st == GP_OK) {
            std::vector<unsigned char> none((size_t)nsolves, 0);
            st = gp_batch_set_active(b->fin, none.data());
        }
        if (st != GP_OK) {
            release(b);
            return st;
        }
    }
    *out = b;
    return GP_OK;
}

gp_status gp_batch_destroy(gp_batch *b)
{
    if (!b) return GP_OK;
    DeviceGuard guard(b->device);
    (void)hipStreamSynchronize(b->own);
    release(b);
    return GP_OK;
}

gp_status gp_batch_set_psi(gp_batch *b, void *const *psi, const int64_t *elems)
{
    if (!b) return fail(GP_ERR_INVALID, "batch is NULL");
    if (!psi || !elems) return fail(GP_ERR_INVALID, "psi and elems arrays are required");
    DeviceGuard guard(b->device);
    const uintptr_t align = storage_bytes(b->dtype);
    for (int i = 0; i < b->n; ++i) {
        if (!psi[i]) return fail(GP_ERR_INVALID, "psi[" + std::to_string(i) + "] is NULL");
        if (elems[i] != b->s[(size_t)i].elems)
            return fail(GP_ERR_INVALID, "psi[" + std::to_string(i) + "] holds " + std::to_string(elems[i]) +
                                            " elements, its grid needs " + std::to_string(b->s[(size_t)i].elems));
        if ((uintptr_t)psi[i] % align) return fail(GP_ERR_INVALID, "psi[" + std::to_string(i) + "] is misaligned");
        hipPointerAttribute_t attr;
        if (hipPointerGetAttributes(&attr, psi[i]) != hipSuccess) {
            (void)hipGetLastError();
            return fail(GP_ERR_INVALID, "psi[" + std::to_string(i) + "] is not a device pointer");
        }
        if ((attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) || attr.device != b->device)
            return fail(GP_ERR_INVALID, "psi[" + std::to_string(i) + "] is not device memory of the batch's device");
    }
    hipError_t e = sync_in(b);
    if (e == hipSuccess) e = hipStreamSynchronize(b->own);   // the staging below is reused
    for (int i = 0; i < b->n; ++i) {
        b->s[(size_t)i].psi = psi[i];
        b->h_psis[i] = psi[i];
    }
    // column pairs need every member's psi 16-byte aligned; a class with a
    // member that is not goes back to one column per thread
    for (Class &c : b->cls) {
        if (c.cols_y == 1 && c.cols_z == 1) continue;
        bool aligned = true;
        for (int m : c.members) aligned = aligned && (uintptr_t)psi[m] % 16 == 0;
        if (aligned) continue;
        c.cols_y = c.cols_z = 1;
        c.xt_y = class_columns(c, 1, 1, b->dtype);
        c.xt_z = class_columns(c, 2, 1, b->dtype);
        class_tiles(c);
        b->graph_ok = false;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_psis, b->h_psis, sizeof(void *) * (size_t)b->n, hipMemcpyHostToDevice, b->own);
    if (e == hipSuccess) e = hipStreamSynchronize(b->own);
    if (e == hipSuccess && !b->graph_ok) e = upload_classes(b);   // the shapes may have changed
    if (e != hipSuccess) return fail_hip(e, "binding psi");
    return GP_OK;
}

gp_status gp_batch_set_active(gp_batch *b, const unsigned char *mask)
{
    if (!b) return fail(GP_ERR_INVALID, "batch is NULL");
    DeviceGuard guard(b->device);
    hipError_t e = hipStreamSynchronize(b->own);
    if (e != hipSuccess) return fail_hip(e, "synchronising the batch");
    for (int i = 0; i < b->n; ++i) b->active[(size_t)i] = mask ? (mask[i] ? 1 : 0) : 1;
    e = upload_active(b);
    if (e != hipSuccess) return fail_hip(e, "uploading the active lists");
    b->graph_ok = false;
    return GP_OK;
}

gp_status gp_batch_step(gp_batch *b, int64_t nsteps)
{
    if (!b) return fail(GP_ERR_INVALID, "batch is NULL");
    if (nsteps < 0) return fail(GP_ERR_INVALID, "nsteps must be >= 0");
    if (!bound(b)) return fail(GP_ERR_INVALID, "bind psi with gp_batch_set_psi first");
    if (nsteps == 0) return GP_OK;
    DeviceGuard guard(b->device);
    hipError_t e = sync_in(b);
    const bool use_graph = (b->flags & GP_BATCH_GRAPH) != 0;
    if (e == hipSuccess && use_graph && !b->graph_ok) e = build_graph(b);
    for (int64_t s = 0; s < nsteps && e == hipSuccess; ++s)
        e = use_graph ? hipGraphLaunch(b->exec, b->own) : enqueue_step(b);
    if (e == hipSuccess && b->mode == GP_MODE_IMAG) {
        for (const Class &c : b->cls) {
            if (!c.nact) continue;
            e = gpssc::launch_scale_batch(static_cast<gpssc::Prec>(b->dtype), c.nact, c.d_active, b->d_psis, c.grid[0] * c.grid[1] * c.grid[2],
                                          b->d_scales, b->own);
            if (e != hipSuccess) break;
        }
    }
    if (e == hipSuccess) e = sync_out(b);
    if (e != hipSuccess) return fail_hip(e, "queueing batch steps");
    b->steps_done += nsteps;
    return GP_OK;
}

gp_status gp_batch_observables(gp_batch *b, gp_obs *out)
{
    if (!b || !out) return fail(GP_ERR_INVALID, "batch and out are required");
    if (!bound(b)) return fail(GP_ERR_INVALID, "bind psi with gp_batch_set_psi first");
    DeviceGuard guard(b->device);
    hipError_t e = sync_in(b);
    for (const Class &c : b->cls) {
        if (!c.nact || e != hipSuccess) continue;
        e = gpssc::launch_observables_batch(static_cast<gpssc::Prec>(b->dtype), c.nact, c.d_active, b->d_psis, b->d_obsargs, (int)c.grid[0],
                                            (int)c.grid[1], b->d_obs_partials, b->d_obs_off, b->d_sums, b->own);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->h_sums, b->d_sums, sizeof(double) * gpssc::OBS_NSUMS * (size_t)b->n,
                           hipMemcpyDeviceToHost, b->own);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->h_flags, b->d_flags, sizeof(int) * (size_t)b->n, hipMemcpyDeviceToHost, b->own);
    if (e == hipSuccess) e = hipStreamSynchronize(b->own);
    if (e == hipSuccess) e = sync_out(b);
    if (e != hipSuccess) return fail_hip(e, "computing batch observables");
    bool flagged = false;
    for (int i = 0; i < b->n; ++i) flagged = flagged || b->h_flags[i] != 0;
    if (flagged) {   // report once, then clear
        std::vector<int> zeros((size_t)b->n, 0);
        e = hipMemcpyAsync(b->d_flags, zeros.data(), sizeof(int) * zeros.size(), hipMemcpyHostToDevice, b->own);
        if (e == hipSuccess) e = hipStreamSynchronize(b->own);
        if (e != hipSuccess) return fail_hip(e, "clearing the batch's error flags");
    }
    gp_status worst = GP_OK;
    for (int i = 0; i < b->n; ++i) {
        if (!b->active[(size_t)i]) continue;
        gp_status st = obs_from_sums(b->h_sums + (size_t)i * gpssc::OBS_NSUMS, b->s[(size_t)i], &out[i],
                                     b->steps_done);
        if (b->h_flags[i]) st = GP_ERR_NONFINITE;
        if (st != GP_OK) worst = st;
    }
    if (worst != GP_OK) return fail(worst, "a solve has a zero or non-finite norm or observable");
    return GP_OK;
}

gp_status gp_batch_solve_imag(gp_batch *b, double tol, int64_t check_every, int64_t max_steps, gp_obs *out,
                              int64_t *steps, unsigned char *converged)
{
    if (!b || !out || !steps || !converged) return fail(GP_ERR_INVALID, "batch and output arrays are required");
    if (b->mode != GP_MODE_IMAG) return fail(GP_ERR_INVALID, "gp_batch_solve_imag needs an imaginary-time batch");
    if (!(tol > 0.0) || check_every < 1 || max_steps < 1)
        return fail(GP_ERR_INVALID, "need tol > 0, check_every >= 1, max_steps >= 1");
    if (b->fin) return solve_imag_finished(b, tol, check_every, max_steps, out, steps, converged);
    std::vector<unsigned char> act((size_t)b->n, 1);
    std::vector<double> last((size_t)b->n, NAN);
    for (int i = 0; i < b->n; ++i) {
        steps[i] = 0;
        converged[i] = 0;
    }
    gp_status st = gp_batch_set_active(b, act.data());
    if (st != GP_OK) return st;
    st = gp_batch_observables(b, out);
    if (st != GP_OK) return st;
    for (int i = 0; i < b->n; ++i) last[(size_t)i] = out[i].mu;
    int64_t done = 0;
    int left = b->n;
    while (left > 0 && done < max_steps) {
        const int64_t k = std::min(check_every, max_steps - done);
        st = gp_batch_step(b, k);
        if (st == GP_OK) st = gp_batch_observables(b, out);
        if (st != GP_OK) return st;
        done += k;
        bool changed = false;
        for (int i = 0; i < b->n; ++i) {
            if (!act[(size_t)i]) continue;
            steps[i] = done;
            if (std::fabs(out[i].mu - last[(size_t)i]) < tol) {
                converged[i] = 1;
                act[(size_t)i] = 0;
                --left;
                changed = true;
            }
            last[(size_t)i] = out[i].mu;
        }
        if (changed && left > 0) {
            st = gp_batch_set_active(b, act.data());
            if (st != GP_OK) return st;
        }
    }
    // leave every solve active again
    return gp_batch_set_active(b, nullptr);
}

gp_status gp_batch_describe(const gp_batch *b, char *buf, size_t len)
{
    if (!b || !buf || len == 0) return fail(GP_ERR_INVALID, "bad gp_batch_describe arguments");
    std::string d = std::to_string(b->n) + " solves, " + std::to_string(b->cls.size()) + " classes";
    for (const Class &c : b->cls) {
        char t[256];
        std::snprintf(t, sizeof t,
                      " | %lldx%lldx%lld: %zu solves, x chunk %d (%s lines per wave), y chunk %d x %d (%d cols%s), "
                      "z chunk %d x %d (%d cols%s)",
                      (long long)c.grid[0], (long long)c.grid[1], (long long)c.grid[2], c.members.size(), c.chunk[0],
                      c.x_lines ? std::to_string(c.x_lines).c_str() : "auto",
                      c.chunk[1], c.lanes[1], c.xt_y * c.cols_y, c.cols_y == 2 ? " in pairs" : "", c.chunk[2],
                      c.lanes[2], c.xt_z * c.cols_z, c.cols_z == 2 ? " in pairs" : "");
        d += t;
    }
    std::snprintf(buf, len, "%s", d.c_str());
    return GP_OK;
}

}  // extern "C"

namespace {

// gp_batch_solve_imag with GP_BATCH_FINISH_F64.  A solve runs in the batch's
// float storage until its chemical potential moves by less than
// kSwitchFactor * tol between two evaluations; its state is then copied
// (exactly) to double storage and it continues in the FP64 batch, where the
// stopping rule |delta mu| < tol applies to FP64 evaluations only.  At the
// end each state is rounded back into the caller's float buffer; out[i]
// holds the last evaluation (of the FP64 state for the solves that reached
// it).
constexpr double kSwitchFactor = 100.0;

gp_status solve_imag_finished(gp_batch *b, double tol, int64_t check_every, int64_t max_steps, gp_obs *out,
                              int64_t *steps, unsigned char *converged)
{
    const int n = b->n;
    gp_batch *f = b->fin;
    const gpssc::Prec p32 = static_cast<gpssc::Prec>(b->dtype), p64 = static_cast<gpssc::Prec>(f->dtype);
    std::vector<unsigned char> act32((size_t)n, 1), act64((size_t)n, 0);
    std::vector<int> phase((size_t)n, 0);   // 0 float, 1 double, 2 done
    std::vector<double> last((size_t)n, NAN);
    std::vector<gp_obs> o64((size_t)n);
    for (int i = 0; i < n; ++i) {
        steps[i] = 0;
        converged[i] = 0;
    }
    gp_status st = gp_batch_set_active(b, act32.data());
    if (st == GP_OK) st = gp_batch_set_active(f, act64.data());
    if (st == GP_OK) st = gp_batch_observables(b, out);
    if (st != GP_OK) return st;
    for (int i = 0; i < n; ++i) last[(size_t)i] = out[i].mu;
    DeviceGuard guard(b->device);
    auto to_f64 = [&](int i) {
        return gpssc::launch_convert(p64, p32, b->shadow[(size_t)i], b->s[(size_t)i].psi, b->s[(size_t)i].elems,
                                     b->caller);
    };
    auto to_f32 = [&](int i) {
        return gpssc::launch_convert(p32, p64, b->s[(size_t)i].psi, b->shadow[(size_t)i], b->s[(size_t)i].elems,
                                     b->caller);
    };
    int64_t done = 0;
    int left = n;
    while (left > 0 && done < max_steps) {
        const int64_t k = std::min(check_every, max_steps - done);
        int n32 = 0, n64 = 0;
        for (int i = 0; i < n; ++i) {
            n32 += act32[(size_t)i];
            n64 += act64[(size_t)i];
        }
        if (n32) st = gp_batch_step(b, k);
        if (st == GP_OK && n64) st = gp_batch_step(f, k);
        if (st == GP_OK && n32) st = gp_batch_observables(b, out);
        if (st == GP_OK && n64) st = gp_batch_observables(f, o64.data());
        if (st != GP_OK) return st;
        done += k;
        bool changed = false;
        hipError_t e = hipSuccess;
        for (int i = 0; i < n && e == hipSuccess; ++i) {
            if (phase[(size_t)i] == 2) continue;
            steps[i] = done;
            if (phase[(size_t)i] == 1) out[i] = o64[(size_t)i];
            const double mu = out[i].mu;
            if (phase[(size_t)i] == 0 && std::fabs(mu - last[(size_t)i]) < kSwitchFactor * tol) {
                e = to_f64(i);
                phase[(size_t)i] = 1;
                act32[(size_t)i] = 0;
                act64[(size_t)i] = 1;
                changed = true;
                last[(size_t)i] = NAN;   // two FP64 evaluations before the rule applies
                continue;
            }
            if (phase[(size_t)i] == 1 && std::fabs(mu - last[(size_t)i]) < tol) {
                converged[i] = 1;
                phase[(size_t)i] = 2;
                act64[(size_t)i] = 0;
                --left;
                changed = true;
                e = to_f32(i);
            }
            last[(size_t)i] = mu;
        }
        if (e != hipSuccess) return fail_hip(e, "moving a state between float and double storage");
        if (changed && left > 0) {
            st = gp_batch_set_active(b, act32.data());
            if (st == GP_OK) st = gp_batch_set_active(f, act64.data());
            if (st != GP_OK) return st;
        }
    }
    // the solves stopped by the step cap in FP64 storage go back too
    hipError_t e = hipSuccess;
    for (int i = 0; i < n && e == hipSuccess; ++i)
        if (phase[(size_t)i] == 1) e = to_f32(i);
    if (e == hipSuccess) e = hipStreamSynchronize(b->caller);
    if (e != hipSuccess) return fail_hip(e, "moving the states back to float storage");
    std::vector<unsigned char> none((size_t)n, 0);
    st = gp_batch_set_active(f, none.data());
    if (st != GP_OK) return st;
    return gp_batch_set_active(b, nullptr);
}

}  // namespace
