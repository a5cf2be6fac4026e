// server.hip -- continuous batching of solve requests (gp_server_*).
//
// An engine thread owns the device work.  Each round it (1) admits queued
// requests whose footprint fits the arena and a free slot, copying their
// initial state in, (2) advances every resident solve by the same number of
// steps with one launch per sweep per (grid shape, mode) class -- the
// batched kernels of gp_batch -- and (3) handles the solves whose event
// (a chemical-potential check, the end of a run) falls at the round's end:
// it evaluates their observables, stops the converged or finished ones,
// copies their state out and frees their memory.  Rounds are at most
// check_every steps and requests are admitted only at multiples of
// check_every engine steps, so every solve's events stay at multiples of
// check_every of its own steps whatever else is resident.
//
// Paper: the split-step Crank-Nicolson step of program summaries (v) and
// (xiv) ("Method of solution"), with calcnu, calclux/y/z, calcnorm and
// calcmuen/calcrms as named in "Summary of revisions".
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "gp_internal.h"
#include "gpssc.h"
#include "host_common.h"
#include "solve_host.h"

using namespace gpssc_host;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxSlots = 4096;
constexpr int kMaxPass = 64;   // times later requests may pass the head of the queue

size_t round_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// Per-request device memory, in this order inside its arena block.
struct Footprint {
    size_t psi, tables, norm, obs, total;
};

Footprint footprint(const ClassShape &c, gp_dtype dtype, bool real)
{
    Footprint f;
    f.psi = round_up(storage_bytes(dtype) * (size_t)(c.grid[0] * c.grid[1] * c.grid[2]));
    f.tables = round_up(table_bytes(c, dtype));
    f.norm = real ? 0 : round_up(sizeof(double) * (size_t)(c.grid[0] * c.grid[1]));
    f.obs = round_up(sizeof(double) * gpssc::OBS_NSUMS * (size_t)c.obs_blocks);
    f.total = f.psi + f.tables + f.norm + f.obs;
    return f;
}

// First-fit allocator over one device allocation; offsets and lengths are
// multiples of kAlign; neighbouring free blocks are merged.
struct Arena {
    unsigned char *base = nullptr;
    size_t size = 0, in_use = 0, peak = 0;
    std::map<size_t, size_t> free_;   // offset -> length

    void reset(unsigned char *b, size_t n)
    {
        base = b;
        size = n / kAlign * kAlign;
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t n, size_t *off)
    {
        n = round_up(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, start = it->first + n;
            free_.erase(it);
            if (rest) free_[start] = rest;
            in_use += n;
            peak = std::max(peak, in_use);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = round_up(n);
        in_use -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Pending {
    uint64_t id;
    gp_request r;
    double t_submit;
    int passed = 0;
    bool auto_real = false;   // complex host buffers, real storage (GP_SERVER_REAL_AUTO)
};

struct Live {
    uint64_t id;
    gp_request r;
    double t_submit, t_admit;
    SolveDesc d;
    gp_dtype dt = GP_C128;        // storage
    int cls = -1, slot = -1;
    size_t off = 0, bytes = 0;
    int64_t steps = 0, next_event = 0;
    double last_mu = 0.0;
    bool fresh = true;     // its step-0 observables are pending (imaginary time)
    bool due = false;      // an event at the end of this round
    bool done = false;
    bool auto_real = false;
};

struct SClass : ClassShape {
    bool real = false;
    gp_dtype dt = GP_C128;        // storage of its solves
    std::vector<int> slots;       // resident slots
    int *d_list = nullptr;        // device: the resident slots
    int *d_due = nullptr;         // device: slots with an event this round
    int *d_fresh = nullptr;       // device: slots needing their step-0 observables
    int *h_stage = nullptr;       // pinned staging, 3 * max_slots
    int ndue = 0, nfresh = 0;
};

double now_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

bool same_key(const SClass &c, const int64_t g[3], bool real, gp_dtype dt)
{
    return c.real == real && c.dt == dt && c.grid[0] == g[0] && c.grid[1] == g[1] && c.grid[2] == g[2];
}

// Storage of one request: the server's dtype, or its real counterpart for a
// real imaginary-time state (same arithmetic type).
gp_dtype request_dtype(gp_dtype server, const gp_request &r)
{
    if (!r.real_state) return server;
    return server == GP_C128 ? GP_R64 : (server == GP_C64 ? GP_R32 : server);
}

}  // namespace

struct gp_server {
    gp_dtype dtype;
    int device = 0;
    int max_slots = 0;
    int64_t K = 1;
    int flags = 0;
    std::chrono::steady_clock::time_point t0;
    hipStream_t stream = nullptr;
    unsigned char *d_arena = nullptr;
    unsigned char *d_stage = nullptr;   // engine thread: complex staging of GP_SERVER_REAL_AUTO requests
    size_t stage_bytes = 0;
    // engine thread: the captured step's per-class branches
    std::vector<hipStream_t> branch;
    std::vector<hipEvent_t> ev_join;
    hipEvent_t ev_fork = nullptr;

    // guarded by mu
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    bool idle = true;
    gp_status failed = GP_OK;
    std::string fail_msg;
    std::deque<Pending> queue;
    std::deque<gp_result> results;
    uint64_t next_id = 1;
    gp_server_counters st{};
    std::thread worker;

    // engine thread only
    Arena arena;
    std::vector<Live> live;
    std::vector<SClass> cls;
    std::vector<int> free_slots;
    int64_t engine_step = 0;
    bool lists_dirty = true;
    double acc_in = 0.0, acc_out = 0.0, acc_rounds = 0.0;   // published in st at the end of a round
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    // per-slot device arrays and pinned staging
    unsigned char *d_xargs = nullptr, *d_yargs = nullptr, *d_zargs = nullptr;
    unsigned char *h_xargs = nullptr, *h_yargs = nullptr, *h_zargs = nullptr;
    size_t xsz = 0, ssz = 0;
    void **d_psis = nullptr, **h_psis = nullptr;
    int64_t *d_part_off = nullptr, *h_part_off = nullptr;
    int64_t *d_obs_off = nullptr, *h_obs_off = nullptr;
    double *d_dv = nullptr, *h_dv = nullptr;
    double *d_scales = nullptr, *h_one = nullptr;
    int *d_flags = nullptr, *h_flags = nullptr, *h_zero = nullptr;
    gpssc::ObsArgs<double> *d_obsargs = nullptr, *h_obsargs = nullptr;
    double *d_sums = nullptr, *h_sums = nullptr;     // observables at events
    double *d_sums0 = nullptr, *h_sums0 = nullptr;   // step-0 observables of new solves
};

namespace {

void free_graph(gp_server *S)
{
    if (S->exec) (void)hipGraphExecDestroy(S->exec);
    if (S->graph) (void)hipGraphDestroy(S->graph);
    S->exec = nullptr;
    S->graph = nullptr;
}

void release(gp_server *S)
{
    free_graph(S);
    if (S->d_stage) (void)hipFree(S->d_stage);
    if (S->ev_fork) (void)hipEventDestroy(S->ev_fork);
    for (hipEvent_t e : S->ev_join) (void)hipEventDestroy(e);
    for (hipStream_t st : S->branch) (void)hipStreamDestroy(st);
    for (SClass &c : S->cls) {
        if (c.d_list) (void)hipFree(c.d_list);
        if (c.d_due) (void)hipFree(c.d_due);
        if (c.d_fresh) (void)hipFree(c.d_fresh);
        if (c.h_stage) (void)hipHostFree(c.h_stage);
    }
    void *dev[] = {S->d_arena, S->d_xargs, S->d_yargs, S->d_zargs, S->d_psis, S->d_part_off, S->d_obs_off,
                   S->d_dv, S->d_scales, S->d_flags, S->d_obsargs, S->d_sums, S->d_sums0};
    for (void *p : dev)
        if (p) (void)hipFree(p);
    void *host[] = {S->h_xargs, S->h_yargs, S->h_zargs, S->h_psis, S->h_part_off, S->h_obs_off, S->h_dv,
                    S->h_one, S->h_flags, S->h_zero, S->h_obsargs, S->h_sums, S->h_sums0};
    for (void *p : host)
        if (p) (void)hipHostFree(p);
    if (S->stream) (void)hipStreamDestroy(S->stream);
    delete S;
}

// Finds or creates the class of a grid and mode (engine thread).
hipError_t class_of(gp_server *S, const int64_t grid[3], bool real, gp_dtype dt, int *out)
{
    for (size_t i = 0; i < S->cls.size(); ++i)
        if (same_key(S->cls[i], grid, real, dt)) {
            *out = (int)i;
            return hipSuccess;
        }
    // reuse an empty class slot before growing
    int idx = -1;
    for (size_t i = 0; i < S->cls.size(); ++i)
        if (S->cls[i].slots.empty()) {
            idx = (int)i;
            break;
        }
    if (idx < 0) {
        SClass c;
        const size_t n = sizeof(int) * (size_t)S->max_slots;
        hipError_t e = hipMalloc((void **)&c.d_list, n);
        if (e == hipSuccess) e = hipMalloc((void **)&c.d_due, n);
        if (e == hipSuccess) e = hipMalloc((void **)&c.d_fresh, n);
        if (e == hipSuccess) e = hipHostMalloc((void **)&c.h_stage, 3 * n, hipHostMallocDefault);
        if (e != hipSuccess) {
            if (c.d_list) (void)hipFree(c.d_list);
            if (c.d_due) (void)hipFree(c.d_due);
            if (c.d_fresh) (void)hipFree(c.d_fresh);
            if (c.h_stage) (void)hipHostFree(c.h_stage);
            return e;
        }
        idx = (int)S->cls.size();
        S->cls.push_back(c);
    }
    SClass &c = S->cls[(size_t)idx];
    static_cast<ClassShape &>(c) = class_shape(grid, dt);
    c.real = real;
    c.dt = dt;
    c.slots.clear();
    c.ndue = c.nfresh = 0;
    *out = idx;
    return hipSuccess;
}

// Copies a request in: tables, kernel arguments and psi (engine thread).
// Grows the complex staging buffer to at least n bytes (engine thread; the
// stream has no pending use of it: every use ends with a synchronisation).
hipError_t ensure_stage(gp_server *S, size_t n)
{
    if (S->stage_bytes >= n) return hipSuccess;
    if (S->d_stage) (void)hipFree(S->d_stage);
    S->d_stage = nullptr;
    S->stage_bytes = 0;
    hipError_t e = hipMalloc((void **)&S->d_stage, n);
    if (e == hipSuccess) S->stage_bytes = n;
    return e;
}

template <typename A>
hipError_t stage_solve(gp_server *S, Live &L, const SClass &c, const Footprint &f)
{
    unsigned char *blk = S->d_arena + L.off;
    std::vector<unsigned char> tab(f.tables, 0);
    pack_solve_tables(L.d, c, L.dt, tab.data());
    const int s = L.slot;
    auto *xa = reinterpret_cast<gpssc::XBatchArgs<A> *>(S->h_xargs + S->xsz * (size_t)s);
    auto *ya = reinterpret_cast<gpssc::SBatchArgs<A> *>(S->h_yargs + S->ssz * (size_t)s);
    auto *za = reinterpret_cast<gpssc::SBatchArgs<A> *>(S->h_zargs + S->ssz * (size_t)s);
    fill_solve_args<A>(L.d, c, blk + f.psi, *xa, *ya, *za);
    S->h_psis[s] = blk;
    S->h_part_off[s] = (int64_t)((L.off + f.psi + f.tables) / sizeof(double));
    S->h_obs_off[s] = (int64_t)((L.off + f.psi + f.tables + f.norm) / sizeof(double));
    S->h_dv[s] = L.d.dx[0] * L.d.dx[1] * L.d.dx[2];
    S->h_obsargs[s] = obs_args(L.d);
    struct Up {
        void *dst;
        const void *src;
        size_t n;
    } ups[] = {
        {blk + f.psi, tab.data(), tab.size()},
        {S->d_xargs + S->xsz * (size_t)s, xa, S->xsz},
        {S->d_yargs + S->ssz * (size_t)s, ya, S->ssz},
        {S->d_zargs + S->ssz * (size_t)s, za, S->ssz},
        {S->d_psis + s, S->h_psis + s, sizeof(void *)},
        {S->d_part_off + s, S->h_part_off + s, sizeof(int64_t)},
        {S->d_obs_off + s, S->h_obs_off + s, sizeof(int64_t)},
        {S->d_dv + s, S->h_dv + s, sizeof(double)},
        {S->d_scales + s, S->h_one, sizeof(double)},
        {S->d_flags + s, S->h_zero, sizeof(int)},
        {S->d_obsargs + s, S->h_obsargs + s, sizeof(gpssc::ObsArgs<double>)},
        {blk, L.r.psi_in, storage_bytes(L.dt) * (size_t)L.d.elems},
    };
    hipError_t e = hipSuccess;
    for (const Up &u : ups)
        if (e == hipSuccess && !(L.auto_real && u.dst == blk))
            e = hipMemcpyAsync(u.dst, u.src, u.n, hipMemcpyHostToDevice, S->stream);
    if (e == hipSuccess && L.auto_real) {
        // the complex state through the staging buffer, its real part to the slot
        e = ensure_stage(S, storage_bytes(S->dtype) * (size_t)L.d.elems);
        if (e == hipSuccess)
            e = hipMemcpyAsync(S->d_stage, L.r.psi_in, storage_bytes(S->dtype) * (size_t)L.d.elems,
                               hipMemcpyHostToDevice, S->stream);
        if (e == hipSuccess)
            e = gpssc::launch_convert(static_cast<gpssc::Prec>(L.dt), static_cast<gpssc::Prec>(S->dtype), blk,
                                      S->d_stage, L.d.elems, S->stream);
    }
    // the tables vector is pageable and local: finish its copy before it goes
    if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
    return e;
}

hipError_t upload_lists(gp_server *S)
{
    for (SClass &c : S->cls) {
        if (c.slots.empty()) continue;
        std::copy(c.slots.begin(), c.slots.end(), c.h_stage);
        hipError_t e = hipMemcpyAsync(c.d_list, c.h_stage, sizeof(int) * c.slots.size(), hipMemcpyHostToDevice,
                                      S->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The branch streams and events of the captured step, one per class
// (created before a capture begins).
hipError_t make_branches(gp_server *S)
{
    hipError_t e = hipSuccess;
    if (!S->ev_fork) e = hipEventCreateWithFlags(&S->ev_fork, hipEventDisableTiming);
    while (e == hipSuccess && S->branch.size() < S->cls.size()) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (st) S->branch.push_back(st);
        if (ev) S->ev_join.push_back(ev);
    }
    return e;
}

// One step of the resident solves of one class, queued on `st`.
hipError_t enqueue_class(gp_server *S, const SClass &c, hipStream_t st)
{
    double *base = reinterpret_cast<double *>(S->d_arena);
    const int n = (int)c.slots.size();
    const gpssc::Prec prec = static_cast<gpssc::Prec>(c.dt);
    hipError_t e = gpssc::launch_nu_x_batch(prec, c.real, c.chunk[0], n, c.nlines, S->d_psis, S->d_xargs, c.d_list,
                                            c.real ? nullptr : S->d_scales, st);
    if (e != hipSuccess) return e;
    e = gpssc::launch_strided_batch(prec, c.real, c.chunk[1], c.xt_y, c.cols_y, c.lanes[1], n, c.ncol_y, c.ntiles_y,
                                    S->d_psis, S->d_yargs, c.d_list, nullptr, nullptr, st);
    if (e != hipSuccess) return e;
    e = gpssc::launch_strided_batch(prec, c.real, c.chunk[2], c.xt_z, c.cols_z, c.lanes[2], n, c.ncol_z, c.ntiles_z,
                                    S->d_psis, S->d_zargs, c.d_list, c.real ? nullptr : base, S->d_part_off, st);
    if (e != hipSuccess || c.real) return e;
    return gpssc::launch_norm_finalize_batch(n, c.d_list, base, S->d_part_off, (int)(c.grid[0] * c.grid[1]), S->d_dv,
                                             S->d_scales, S->d_flags, st);
}

// One step of every resident solve.  Inside a capture the classes become
// parallel branches (fork from and join back to the server's stream): they
// touch disjoint memory, so only the order within a class matters.
hipError_t enqueue_step(gp_server *S, bool branches = false)
{
    hipError_t e = hipSuccess;
    if (branches) {
        if (!S->ev_fork || S->branch.size() < S->cls.size()) return hipErrorInvalidValue;   // see make_branches
        e = hipEventRecord(S->ev_fork, S->stream);
    }
    for (size_t k = 0; k < S->cls.size() && e == hipSuccess; ++k) {
        const SClass &c = S->cls[k];
        if (c.slots.empty()) continue;
        if (!branches) {
            e = enqueue_class(S, c, S->stream);
            continue;
        }
        e = hipStreamWaitEvent(S->branch[k], S->ev_fork, 0);
        if (e == hipSuccess) e = enqueue_class(S, c, S->branch[k]);
        if (e == hipSuccess) e = hipEventRecord(S->ev_join[k], S->branch[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(S->stream, S->ev_join[k], 0);
    }
    return e;
}

hipError_t capture(gp_server *S)
{
    free_graph(S);
    hipError_t e = make_branches(S);
    if (e == hipSuccess) e = hipStreamBeginCapture(S->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = enqueue_step(S, true);
    e = hipStreamEndCapture(S->stream, &S->graph);
    if (le != hipSuccess) return le;
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&S->exec, S->graph, nullptr, nullptr, 0);
    if (e == hipSuccess) {
        std::lock_guard<std::mutex> lk(S->mu);
        ++S->st.graph_captures;
    }
    return e;
}

// Observables sums of the listed slots of one class into sums (per slot).
hipError_t observe(gp_server *S, const SClass &c, int n, const int *d_slots, double *sums)
{
    return gpssc::launch_observables_batch(static_cast<gpssc::Prec>(c.dt), n, d_slots, S->d_psis, S->d_obsargs,
                                           (int)c.grid[0], (int)c.grid[1], reinterpret_cast<double *>(S->d_arena),
                                           S->d_obs_off, sums, S->stream);
}

void finish(gp_server *S, Live &L, gp_status status, const gp_obs &obs, bool converged)
{
    gp_result r{};
    r.id = L.id;
    r.tag = L.r.tag;
    r.status = status;
    r.converged = converged ? 1 : 0;
    r.steps = L.steps;
    r.obs = obs;
    r.obs.steps_done = L.steps;
    r.t_submit = L.t_submit;
    r.t_admit = L.t_admit;
    L.done = true;
    // psi out, then the memory is free
    const double tc = now_since(S->t0);
    hipError_t e = hipSuccess;
    if (L.auto_real) {   // back to complex through the staging buffer
        e = ensure_stage(S, storage_bytes(S->dtype) * (size_t)L.d.elems);
        if (e == hipSuccess)
            e = gpssc::launch_convert(static_cast<gpssc::Prec>(S->dtype), static_cast<gpssc::Prec>(L.dt),
                                      S->d_stage, S->d_arena + L.off, L.d.elems, S->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(L.r.psi_out, S->d_stage, storage_bytes(S->dtype) * (size_t)L.d.elems,
                               hipMemcpyDeviceToHost, S->stream);
    } else {
        e = hipMemcpyAsync(L.r.psi_out, S->d_arena + L.off, storage_bytes(L.dt) * (size_t)L.d.elems,
                           hipMemcpyDeviceToHost, S->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess && r.status == GP_OK) r.status = GP_ERR_DEVICE;
    S->acc_out += now_since(S->t0) - tc;
    S->arena.release(L.off, L.bytes);
    S->free_slots.push_back(L.slot);
    SClass &c = S->cls[(size_t)L.cls];
    c.slots.erase(std::find(c.slots.begin(), c.slots.end(), L.slot));
    S->lists_dirty = true;
    r.t_done = now_since(S->t0);
    std::lock_guard<std::mutex> lk(S->mu);
    S->results.push_back(r);
    ++S->st.completed;
    --S->st.resident;
    S->st.bytes_in_use = S->arena.in_use;
    S->cv_done.notify_all();
}

// Fails every queued and resident request (engine error).
void fail_all(gp_server *S, hipError_t e, const char *what)
{
    std::lock_guard<std::mutex> lk(S->mu);
    S->failed = GP_ERR_DEVICE;
    S->fail_msg = std::string(what) + ": " + hipGetErrorString(e);
    const double t = now_since(S->t0);
    auto push = [&](uint64_t id, const gp_request &r, double ts, double ta) {
        gp_result x{};
        x.id = id;
        x.tag = r.tag;
        x.status = GP_ERR_DEVICE;
        x.t_submit = ts;
        x.t_admit = ta;
        x.t_done = t;
        S->results.push_back(x);
        ++S->st.completed;
    };
    for (Live &L : S->live)
        if (!L.done) push(L.id, L.r, L.t_submit, L.t_admit);
    for (const Pending &p : S->queue) push(p.id, p.r, p.t_submit, -1.0);
    S->live.clear();
    S->queue.clear();
    S->st.queued = S->st.resident = 0;
    S->stop = true;
    S->cv_done.notify_all();
}

// One engine round; returns false when the engine should stop.
bool round_once(gp_server *S)
{
    double tnow = 0.0;
    struct Admit {
        Pending p;
        size_t off;
    };
    std::vector<Admit> admitted;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        if (S->stop) return false;
        if (S->live.empty()) {
            S->engine_step = 0;
            if (S->queue.empty()) {
                S->idle = true;
                S->cv_done.notify_all();
                S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
                if (S->stop) return false;
            }
            S->idle = false;
        }
        tnow = now_since(S->t0);
        if (S->engine_step % S->K == 0) {
            // arrival order; a request that does not fit may be passed by
            // later ones, until it has waited kMaxPass rounds at the head
            size_t slots_left = S->free_slots.size();
            for (auto it = S->queue.begin(); it != S->queue.end() && slots_left > 0;) {
                const gp_dtype rdt = request_dtype(S->dtype, it->r);
                const ClassShape shp = class_shape(it->r.grid, rdt);
                const size_t need = footprint(shp, rdt, it->r.mode == GP_MODE_REAL).total;
                size_t off = 0;
                if (S->arena.alloc(need, &off)) {
                    admitted.push_back({*it, off});
                    it = S->queue.erase(it);
                    --slots_left;
                    continue;
                }
                if (it == S->queue.begin() && ++it->passed > kMaxPass) break;
                ++it;
            }
            S->st.queued = (int64_t)S->queue.size();
            S->st.bytes_in_use = S->arena.in_use;
            S->st.bytes_peak = S->arena.peak;
        }
    }
    // set up the admitted requests
    for (const Admit &ad : admitted) {
        const Pending &p = ad.p;
        Live L;
        L.id = p.id;
        L.r = p.r;
        L.auto_real = p.auto_real;
        L.t_submit = p.t_submit;
        L.t_admit = tnow;
        L.off = ad.off;
        for (int a = 0; a < 3; ++a) {
            L.d.grid[a] = p.r.grid[a];
            L.d.dx[a] = p.r.dx[a];
            L.d.omega[a] = p.r.trap[a];
        }
        L.d.dt = p.r.dt;
        L.d.g = p.r.g;
        L.d.real = p.r.mode == GP_MODE_REAL;
        L.dt = request_dtype(S->dtype, p.r);
        hipError_t e = class_of(S, L.d.grid, L.d.real, L.dt, &L.cls);
        if (e != hipSuccess) {
            fail_all(S, e, "allocating a class");
            return false;
        }
        SClass &c = S->cls[(size_t)L.cls];
        const Footprint f = footprint(c, L.dt, L.d.real);
        L.bytes = f.total;
        build_solve(L.d, c);
        L.slot = S->free_slots.back();
        S->free_slots.pop_back();
        const double tc = now_since(S->t0);
        e = arith_f32(S->dtype) ? stage_solve<float>(S, L, c, f) : stage_solve<double>(S, L, c, f);
        S->acc_in += now_since(S->t0) - tc;
        if (e != hipSuccess) {
            fail_all(S, e, "copying a request in");
            return false;
        }
        c.slots.push_back(L.slot);
        L.fresh = !L.d.real;
        L.next_event = L.d.real ? L.r.steps : std::min<int64_t>(S->K, L.r.steps);
        S->live.push_back(L);
        S->lists_dirty = true;
        std::lock_guard<std::mutex> lk(S->mu);
        ++S->st.resident;
        S->st.max_resident = std::max(S->st.max_resident, S->st.resident);
    }
    if (S->live.empty()) return true;

    // the round's length: up to the next event of any solve, and never past
    // the next admission point
    int64_t q = S->K - S->engine_step % S->K;
    for (const Live &L : S->live) q = std::min(q, L.next_event - L.steps);
    for (Live &L : S->live) L.due = L.steps + q == L.next_event;
    for (SClass &c : S->cls) c.ndue = c.nfresh = 0;
    const double tr = now_since(S->t0);
    hipError_t e = hipSuccess;
    if (S->lists_dirty) {
        e = upload_lists(S);
        if (e == hipSuccess && (S->flags & GP_SERVER_GRAPH)) e = capture(S);
        if (e != hipSuccess) {
            fail_all(S, e, "updating the resident lists");
            return false;
        }
        S->lists_dirty = false;
    }
    const int ms = S->max_slots;
    for (const Live &L : S->live) {
        SClass &c = S->cls[(size_t)L.cls];
        if (L.fresh) c.h_stage[ms + c.nfresh++] = L.slot;
        if (L.due) c.h_stage[2 * ms + c.ndue++] = L.slot;
    }
    // step-0 observables of new imaginary-time solves
    for (SClass &c : S->cls) {
        if (!c.nfresh || e != hipSuccess) continue;
        e = hipMemcpyAsync(c.d_fresh, c.h_stage + ms, sizeof(int) * (size_t)c.nfresh, hipMemcpyHostToDevice,
                           S->stream);
        if (e == hipSuccess) e = observe(S, c, c.nfresh, c.d_fresh, S->d_sums0);
    }
    for (int64_t k = 0; k < q && e == hipSuccess; ++k)
        e = (S->flags & GP_SERVER_GRAPH) ? hipGraphLaunch(S->exec, S->stream) : enqueue_step(S);
    // events: imaginary-time solves end the round normalised (as a gp_step
    // call ends), then every due solve is measured
    for (SClass &c : S->cls) {
        if (!c.ndue || e != hipSuccess) continue;
        e = hipMemcpyAsync(c.d_due, c.h_stage + 2 * ms, sizeof(int) * (size_t)c.ndue, hipMemcpyHostToDevice,
                           S->stream);
        if (e == hipSuccess && !c.real)
            e = gpssc::launch_scale_batch(static_cast<gpssc::Prec>(c.dt), c.ndue, c.d_due, S->d_psis,
                                          c.grid[0] * c.grid[1] * c.grid[2], S->d_scales, S->stream);
        if (e == hipSuccess) e = observe(S, c, c.ndue, c.d_due, S->d_sums);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(S->h_sums, S->d_sums, sizeof(double) * gpssc::OBS_NSUMS * (size_t)ms,
                           hipMemcpyDeviceToHost, S->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(S->h_sums0, S->d_sums0, sizeof(double) * gpssc::OBS_NSUMS * (size_t)ms,
                           hipMemcpyDeviceToHost, S->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(S->h_flags, S->d_flags, sizeof(int) * (size_t)ms, hipMemcpyDeviceToHost, S->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess) {
        fail_all(S, e, "running a round");
        return false;
    }
    S->acc_rounds += now_since(S->t0) - tr;
    S->engine_step += q;
    int64_t nsteps = 0;
    for (Live &L : S->live) {
        gp_obs o{};
        L.steps += q;
        nsteps += q;
        if (L.fresh) {
            L.fresh = false;
            gp_status s0 = obs_from_sums(S->h_sums0 + (size_t)L.slot * gpssc::OBS_NSUMS, L.d, &o, 0);
            if (s0 != GP_OK) {
                finish(S, L, s0, o, false);
                continue;
            }
            L.last_mu = o.mu;
        }
        if (!L.due) continue;
        gp_status stt = obs_from_sums(S->h_sums + (size_t)L.slot * gpssc::OBS_NSUMS, L.d, &o, L.steps);
        if (S->h_flags[L.slot]) stt = GP_ERR_NONFINITE;
        if (stt != GP_OK) {
            finish(S, L, stt, o, false);
            continue;
        }
        if (L.d.real) {
            finish(S, L, GP_OK, o, false);
            continue;
        }
        const bool conv = L.r.tol > 0.0 && std::fabs(o.mu - L.last_mu) < L.r.tol;
        if (conv || L.steps >= L.r.steps) {
            finish(S, L, GP_OK, o, conv);
            continue;
        }
        L.last_mu = o.mu;
        L.next_event = std::min(L.steps + S->K, L.r.steps);
    }
    S->live.erase(std::remove_if(S->live.begin(), S->live.end(), [](const Live &L) { return L.done; }),
                  S->live.end());
    std::lock_guard<std::mutex> lk(S->mu);
    ++S->st.quanta;
    S->st.solve_steps += nsteps;
    S->st.bytes_in_use = S->arena.in_use;
    S->st.seconds_copy_in = S->acc_in;
    S->st.seconds_copy_out = S->acc_out;
    S->st.seconds_rounds = S->acc_rounds;
    return true;
}

void engine(gp_server *S)
{
    (void)hipSetDevice(S->device);
    while (round_once(S)) {
    }
    std::lock_guard<std::mutex> lk(S->mu);
    S->idle = true;
    S->cv_done.notify_all();
}

}  // namespace

extern "C" {

size_t gp_server_request_bytes(const int64_t grid[3], gp_dtype dtype, gp_mode mode)
{
    if (!grid || !valid_dtype(dtype) || !valid_grid(grid) || !grid_supported(grid, dtype)) return 0;
    return footprint(class_shape(grid, dtype), dtype, mode == GP_MODE_REAL).total;
}

gp_status gp_server_create(gp_dtype dtype, uint64_t hbm_budget, int max_slots, int64_t check_every, int flags,
                           gp_server **out)
{
    if (!out) return fail(GP_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!valid_dtype(dtype)) return fail(GP_ERR_INVALID, "unknown dtype");
    if (max_slots < 1 || max_slots > kMaxSlots) return fail(GP_ERR_INVALID, "max_slots must be in 1..4096");
    if (check_every < 1) return fail(GP_ERR_INVALID, "check_every must be >= 1");
    if (hbm_budget < kAlign) return fail(GP_ERR_INVALID, "hbm_budget is too small");
    if (flags & ~(GP_SERVER_GRAPH | GP_SERVER_REAL_AUTO)) return fail(GP_ERR_INVALID, "unknown flags");
    gp_server *S = new (std::nothrow) gp_server();
    if (!S) return fail(GP_ERR_NOMEM, "host allocation failed");
    S->dtype = dtype;
    S->max_slots = max_slots;
    S->K = check_every;
    S->flags = flags;
    S->t0 = std::chrono::steady_clock::now();
    S->xsz = arith_f32(dtype) ? sizeof(gpssc::XBatchArgs<float>) : sizeof(gpssc::XBatchArgs<double>);
    S->ssz = arith_f32(dtype) ? sizeof(gpssc::SBatchArgs<float>) : sizeof(gpssc::SBatchArgs<double>);
    const size_t m = (size_t)max_slots;
    hipError_t e = hipGetDevice(&S->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc((void **)&S->d_arena, (size_t)hbm_budget);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        release(S);
        return fail(GP_ERR_NOMEM, "the arena does not fit in device memory");
    }
    struct D {
        void **p;
        size_t n;
    } devs[] = {
        {(void **)&S->d_xargs, S->xsz * m},       {(void **)&S->d_yargs, S->ssz * m},
        {(void **)&S->d_zargs, S->ssz * m},       {(void **)&S->d_psis, sizeof(void *) * m},
        {(void **)&S->d_part_off, 8 * m},         {(void **)&S->d_obs_off, 8 * m},
        {(void **)&S->d_dv, 8 * m},               {(void **)&S->d_scales, 8 * m},
        {(void **)&S->d_flags, sizeof(int) * m},  {(void **)&S->d_obsargs, sizeof(gpssc::ObsArgs<double>) * m},
        {(void **)&S->d_sums, sizeof(double) * gpssc::OBS_NSUMS * m},
        {(void **)&S->d_sums0, sizeof(double) * gpssc::OBS_NSUMS * m},
    };
    for (const D &d : devs)
        if (e == hipSuccess) e = hipMalloc(d.p, d.n);
    D hosts[] = {
        {(void **)&S->h_xargs, S->xsz * m},       {(void **)&S->h_yargs, S->ssz * m},
        {(void **)&S->h_zargs, S->ssz * m},       {(void **)&S->h_psis, sizeof(void *) * m},
        {(void **)&S->h_part_off, 8 * m},         {(void **)&S->h_obs_off, 8 * m},
        {(void **)&S->h_dv, 8 * m},               {(void **)&S->h_one, 8},
        {(void **)&S->h_flags, sizeof(int) * m},  {(void **)&S->h_zero, sizeof(int)},
        {(void **)&S->h_obsargs, sizeof(gpssc::ObsArgs<double>) * m},
        {(void **)&S->h_sums, sizeof(double) * gpssc::OBS_NSUMS * m},
        {(void **)&S->h_sums0, sizeof(double) * gpssc::OBS_NSUMS * m},
    };
    for (const D &d : hosts)
        if (e == hipSuccess) e = hipHostMalloc(d.p, d.n, hipHostMallocDefault);
    if (e == hipSuccess) {
        *S->h_one = 1.0;
        *S->h_zero = 0;
        e = hipMemsetAsync(S->d_sums, 0, sizeof(double) * gpssc::OBS_NSUMS * m, S->stream);
    }
    if (e == hipSuccess) e = hipMemsetAsync(S->d_sums0, 0, sizeof(double) * gpssc::OBS_NSUMS * m, S->stream);
    if (e == hipSuccess) e = hipMemsetAsync(S->d_flags, 0, sizeof(int) * m, S->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        release(S);
        return e == hipErrorOutOfMemory ? fail(GP_ERR_NOMEM, "device allocation failed")
                                        : fail_hip(e, "creating the server");
    }
    S->arena.reset(S->d_arena, (size_t)hbm_budget);
    for (int s = max_slots - 1; s >= 0; --s) S->free_slots.push_back(s);
    S->st.bytes_budget = S->arena.size;
    try {
        S->worker = std::thread(engine, S);
    } catch (...) {
        release(S);
        return fail(GP_ERR_DEVICE, "could not start the engine thread");
    }
    *out = S;
    return GP_OK;
}

gp_status gp_server_destroy(gp_server *S)
{
    if (!S) return GP_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    DeviceGuard guard(S->device);
    (void)hipStreamSynchronize(S->stream);
    release(S);
    return GP_OK;
}

gp_status gp_server_submit(gp_server *S, const gp_request *r, uint64_t *id)
{
    if (!S || !r || !id) return fail(GP_ERR_INVALID, "server, request and id are required");
    if (r->mode != GP_MODE_IMAG && r->mode != GP_MODE_REAL) return fail(GP_ERR_INVALID, "unknown mode");
    if (!valid_grid(r->grid)) return fail(GP_ERR_INVALID, "grid sizes must be >= 1");
    if (!valid_params(r->dx, r->dt, r->trap, r->g))
        return fail(GP_ERR_INVALID, "dx and dt must be finite and > 0, trap finite and >= 0, g finite");
    if (r->steps < 1) return fail(GP_ERR_INVALID, "steps must be >= 1");
    if (!std::isfinite(r->tol) || r->tol < 0.0) return fail(GP_ERR_INVALID, "tol must be finite and >= 0");
    if (!r->psi_in || !r->psi_out) return fail(GP_ERR_INVALID, "psi_in and psi_out are required");
    if (real_storage(S->dtype) && r->mode != GP_MODE_IMAG)
        return fail(GP_ERR_INVALID, "a server with real storage takes imaginary-time requests only");
    if (r->real_state && (r->mode != GP_MODE_IMAG || S->dtype == GP_C64_F64))
        return fail(GP_ERR_INVALID, "real_state needs an imaginary-time request on a GP_C128 or GP_C64 server");
    gp_request rq = *r;
    bool auto_real = false;
    if ((S->flags & GP_SERVER_REAL_AUTO) && r->mode == GP_MODE_IMAG && !r->real_state &&
        (S->dtype == GP_C64 || S->dtype == GP_C128)) {
        // an imaginary-time state with no imaginary part stays real: every
        // imaginary-time operator is real
        const int64_t n = r->grid[0] * r->grid[1] * r->grid[2];
        bool zero = true;
        if (S->dtype == GP_C64) {
            const float *v = static_cast<const float *>(r->psi_in);
            for (int64_t q = 0; q < n && zero; ++q) zero = v[2 * q + 1] == 0.0f;
        } else {
            const double *v = static_cast<const double *>(r->psi_in);
            for (int64_t q = 0; q < n && zero; ++q) zero = v[2 * q + 1] == 0.0;
        }
        if (zero) {
            auto_real = true;
            rq.real_state = 1;
        }
    }
    const gp_dtype rdt = request_dtype(S->dtype, rq);
    if (!grid_supported(r->grid, rdt)) return fail(GP_ERR_UNSUPPORTED, "grid line too long (each <= 1024)");
    const size_t need = gp_server_request_bytes(r->grid, rdt, r->mode);
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->failed != GP_OK) return fail(S->failed, "the server's engine failed: " + S->fail_msg);
    if (S->stop) return fail(GP_ERR_INVALID, "the server is stopping");
    if (round_up(need) > S->arena.size)
        return fail(GP_ERR_NOMEM, "the request needs " + std::to_string(need) + " bytes, the arena holds " +
                                      std::to_string(S->arena.size));
    Pending p;
    p.id = S->next_id++;
    p.r = rq;
    p.auto_real = auto_real;
    p.t_submit = now_since(S->t0);
    S->queue.push_back(p);
    ++S->st.submitted;
    S->st.queued = (int64_t)S->queue.size();
    S->idle = false;
    *id = p.id;
    S->cv_work.notify_all();
    return GP_OK;
}

gp_status gp_server_poll(gp_server *S, gp_result *out, int max, double wait_seconds, int *n)
{
    if (!S || !n || (max > 0 && !out)) return fail(GP_ERR_INVALID, "server, out and n are required");
    if (!std::isfinite(wait_seconds) || wait_seconds < 0.0) return fail(GP_ERR_INVALID, "wait_seconds must be >= 0");
    *n = 0;
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->results.empty() && wait_seconds > 0.0)
        S->cv_done.wait_for(lk, std::chrono::duration<double>(wait_seconds),
                            [&] { return !S->results.empty() || S->failed != GP_OK; });
    while (*n < max && !S->results.empty()) {
        out[(*n)++] = S->results.front();
        S->results.pop_front();
    }
    return GP_OK;
}

gp_status gp_server_drain(gp_server *S, double wait_seconds, int *idle)
{
    if (!S || !idle) return fail(GP_ERR_INVALID, "server and idle are required");
    if (!std::isfinite(wait_seconds) || wait_seconds < 0.0) return fail(GP_ERR_INVALID, "wait_seconds must be >= 0");
    std::unique_lock<std::mutex> lk(S->mu);
    auto quiet = [&] { return S->failed != GP_OK || (S->queue.empty() && S->st.resident == 0 && S->idle); };
    S->cv_done.wait_for(lk, std::chrono::duration<double>(wait_seconds), quiet);
    *idle = quiet() ? 1 : 0;
    if (S->failed != GP_OK) return fail(S->failed, "the server's engine failed: " + S->fail_msg);
    return GP_OK;
}

gp_status gp_server_stats(gp_server *S, gp_server_counters *out)
{
    if (!S || !out) return fail(GP_ERR_INVALID, "server and out are required");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    return GP_OK;
}

}  // extern "C"
