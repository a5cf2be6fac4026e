/*
 * gpssc.h -- C ABI of the MI355X (gfx950) split-step Crank-Nicolson step for
 * the three-dimensional, fully anisotropic Gross-Pitaevskii equation.
 *
 * Method: Vudragovic, Vidanovic, Balaz, Muruganandam, Adhikari, "C programs
 * for solving the time-dependent Gross-Pitaevskii equation in a fully
 * anisotropic trap", Comput. Phys. Commun. 183 (2012) 2021.  Program
 * summaries (v) imagtime3d and (xiv) realtime3d ("Method of solution"): the
 * equation is discretised in space and time and propagated over small steps
 * in imaginary time (stationary states) or real time (dynamics) by the
 * split-step Crank-Nicolson method.  "Summary of revisions" names the parts
 * of one step -- calcnu, calclux, calcluy, calcluz -- the normalisation
 * calcnorm and the physical quantities calcmuen and calcrms; each entry point
 * below says which of them it carries out.
 *
 * Conventions (the paper prints no formula; these readings fix them):
 *   i dpsi/dt = [-1/2 Lap + V + g|psi|^2] psi,
 *   V = 1/2 (gamma^2 x^2 + nu^2 y^2 + lambda^2 z^2);
 *   nodes x_i = (i - (N-1)/2) dx on every axis, psi = 0 just outside the box;
 *   psi is a device array of Nx*Ny*Nz complex numbers in C order (z, y, x):
 *   element p = (k*Ny + j)*Nx + i, each complex stored as (re, im);
 *   the norm is dx*dy*dz * sum |psi|^2.
 *
 * Error behaviour: every entry point returns a gp_status and never aborts or
 * throws.  On GP_ERR_INVALID nothing is changed.  GP_ERR_DEVICE carries the
 * HIP runtime message in gp_last_error().  Work queued by gp_step runs
 * asynchronously; a failure it meets (a non-finite norm in imaginary time, a
 * device fault) is reported by the next synchronous call (gp_observables,
 * gp_sync).  A plan must not be used from two host threads at once; distinct
 * plans are independent.
 */
#ifndef GPSSC_H
#define GPSSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gp_plan gp_plan; /* opaque; created and owned by the library */

/* Imaginary time converges to the ground state and renormalises every
 * step; real time is the unitary dynamics. */
typedef enum { GP_MODE_IMAG = 0, GP_MODE_REAL = 1 } gp_mode;

/* GP_C128    : psi is complex<double> (16 B per point), FP64 arithmetic.
 * GP_C64     : psi is complex<float>  (8 B per point), FP32 arithmetic in
 *              the sweeps and the phase update.
 * GP_C64_F64 : psi is complex<float>  (8 B per point), FP64 arithmetic in
 *              registers (only the stored values are rounded to FP32).
 * GP_R64     : psi is double (8 B per point), the real part only; FP64
 *              arithmetic.  Imaginary time only: every imaginary-time
 *              operator is real, so a real state stays real, and the step
 *              does the GP_C128 arithmetic on its real part (y/z lines of up
 *              to 256 points are cut into at most 32 chunks, so the rounding
 *              order there differs from GP_C128's).
 * GP_R32     : psi is float (4 B per point), real; FP32 arithmetic
 *              (bitwise GP_C64 of the real state).  Imaginary time only.
 * Every reduction (norm, energy, chemical potential, rms sizes) is
 * accumulated in FP64 for all of them. */
typedef enum { GP_C128 = 0, GP_C64 = 1, GP_C64_F64 = 2, GP_R64 = 3, GP_R32 = 4 } gp_dtype;

typedef enum {
    GP_OK = 0,
    GP_ERR_INVALID = 1,     /* bad argument: NULL, size mismatch, non-finite parameter */
    GP_ERR_NOMEM = 2,       /* a device allocation failed */
    GP_ERR_DEVICE = 3,      /* HIP runtime error; see gp_last_error() */
    GP_ERR_NONFINITE = 4,   /* the norm or an observable is not finite (or the norm is 0) */
    GP_ERR_UNSUPPORTED = 5  /* valid but outside what the kernels handle (line too long) */
} gp_status;

/* Physical quantities of psi (calcmuen, calcrms), all in FP64.  With
 * N = dV sum|psi|^2 and psi-hat = psi / sqrt(N):
 *   kinetic     = 1/2 dV sum_axes sum_links |psi_{i+1}-psi_i|^2 / dx_a^2 / N
 *                 (3-point links, including the link to the zero outside
 *                 the box at both ends of every line),
 *   potential   = dV sum V |psi|^2 / N,
 *   interaction = g dV sum |psi|^4 / N^2,
 *   energy      = kinetic + potential + interaction / 2,
 *   mu          = kinetic + potential + interaction,
 *   rms[a]      = sqrt(dV sum a^2 |psi|^2 / N) about the origin,
 *   rms_r       = sqrt(rms[0]^2 + rms[1]^2 + rms[2]^2),
 *   mean[a]     = dV sum a |psi|^2 / N. */
typedef struct {
    double norm, mu, energy;
    double rms[3], rms_r, mean[3];
    double kinetic, potential, interaction;
    int64_t steps_done; /* steps queued on this plan since creation */
} gp_obs;

/* Kernel classes reported by gp_profile_read. */
enum {
    GP_KERNEL_NU_X = 0,     /* calcnu + calclux (+ pending renormalisation) */
    GP_KERNEL_Y = 1,        /* calcluy */
    GP_KERNEL_Z = 2,        /* calcluz (+ per-line norm partial sums in imaginary time) */
    GP_KERNEL_NORM = 3,     /* calcnorm: partial sums -> 1/sqrt(N) on the device */
    GP_KERNEL_SCALE = 4,    /* end-of-call psi <- psi / sqrt(N) */
    GP_KERNEL_OBS = 5,      /* calcmuen + calcrms sums and their finalisation */
    GP_KERNEL_COUNT = 6
};

/* Creates a plan for one grid, step size, trap, coupling, mode and dtype.
 *   grid[3]   Nx, Ny, Nz >= 1 (each <= 1024)
 *   dx[3]     grid spacings > 0
 *   dt        time step > 0 (imaginary or real time per `mode`)
 *   gamma, nu, lambda  trap frequencies >= 0 along x, y, z
 *   g         nonlinearity, any finite value
 *   hip_stream  hipStream_t to queue work on, or NULL for the null stream
 *   out       receives the plan
 * Builds the constant Crank-Nicolson / Thomas coefficient tables of every
 * axis on the host in FP64 (they depend on N, dx and dt, not on g) and copies
 * them to the current device with the plan's scratch (reduction partials,
 * the 1/sqrt(N) slot, an error flag).  Arguments are checked before any
 * device call.  Returns GP_ERR_INVALID, GP_ERR_UNSUPPORTED, GP_ERR_NOMEM or
 * GP_ERR_DEVICE on failure, with *out set to NULL. */
gp_status gp_plan_create(const int64_t grid[3], const double dx[3], double dt,
                         double gamma, double nu, double lambda, double g,
                         gp_mode mode, gp_dtype dtype, void *hip_stream,
                         gp_plan **out);

/* The equation in fewer space variables (the paper's one- and
 * two-dimensional programs, summaries (i), (ii), (x), (xi)): ndim = 1 (x) or
 * 2 (x, y); ndim = 3 is gp_plan_create.  Axes a >= ndim must have grid[a] = 1
 * and take no part: no sweep along them, no trap term (their frequency is
 * ignored), no kinetic links; the cell volume of the norm and of every
 * observable is the product of the present spacings, and g is the coupling
 * of the reduced equation as given.  psi keeps the (Nz, Ny, Nx) layout with
 * the absent extents 1.  GP_ERR_INVALID for ndim outside 1..3 or an absent
 * axis with more than one node; otherwise as gp_plan_create. */
gp_status gp_plan_create_nd(int ndim, const int64_t grid[3], const double dx[3], double dt,
                            double gamma, double nu, double lambda, double g,
                            gp_mode mode, gp_dtype dtype, void *hip_stream,
                            gp_plan **out);

/* The symmetric traps (the paper's circularly, spherically and axially
 * symmetric programs, summaries (iv), (ix), (vii) and their real-time
 * counterparts). */
typedef enum {
    GP_GEOM_CIRCULAR = 1,   /* 2D, radial variable r along x; grid (N, 1, 1); trap gamma */
    GP_GEOM_SPHERICAL = 2,  /* 3D, radial variable r along x; grid (N, 1, 1); trap gamma */
    GP_GEOM_AXIAL = 3       /* 3D, rho along x and z along y; grid (N_rho, N_z, 1);
                               trap gamma (rho) and lambda (z) */
} gp_geom;

/* Plan for a symmetric trap.  Radial nodes sit at r_i = (i + 1/2) dx[0]
 * (no node at the origin; no flux through it; zero one node past the
 * last); z nodes (axial) as on a Cartesian axis with spacing dx[1].  The
 * radial Laplacian is the conservative finite-volume form with face
 * weights ((i+1) h)^(D-1) and cell weights ((i+1)^D - i^D) h^(D-1) / D
 * (D = 2 circular and axial, 3 spherical); the cell volume is
 * S_D h v_i (times dz, axial), S_2 = 2 pi, S_3 = 4 pi, and the norm, the
 * renormalisation and every observable use it.  nu is unused; lambda only
 * for the axial trap.  Observables: rms[0], mean[0] for the radial
 * variable, rms[1], mean[1] for z (axial), rms_r = sqrt(<r^2>) or
 * sqrt(<rho^2 + z^2>).  Errors as gp_plan_create_nd. */
gp_status gp_plan_create_radial(gp_geom geom, const int64_t grid[3], const double dx[3], double dt,
                                double gamma, double nu, double lambda, double g,
                                gp_mode mode, gp_dtype dtype, void *hip_stream,
                                gp_plan **out);

/* How the y and z sweeps solve their lines.
 * GP_SWEEP_CHUNKED : a block of threads holds neighbouring lines, each cut
 *                    into contiguous chunks; the chunks' carries come from a
 *                    parallel (Kogge-Stone) scan.  Exact for every system.
 * GP_SWEEP_STREAM  : one thread per line (or pair of complex64 lines) walks
 *                    the line in blocks of B = 8, 12 or 16 points; the
 *                    backward recurrence of a block starts B - 1 points past
 *                    its end, which is exact to rounding when |c|^B is below
 *                    2^-60 (FP64 arithmetic) or 2^-30 (FP32), c the decay
 *                    ratio of the Crank-Nicolson inverse of the axis (small
 *                    for small dt / dx^2).  An axis where no B qualifies
 *                    keeps the chunked scan.
 * GP_SWEEP_AUTO    : the library's choice per axis (the default); at present
 *                    the chunked scan, which measured at least as fast on
 *                    every grid tried.
 * Both solve the same matrices; results agree to rounding, not bitwise. */
typedef enum { GP_SWEEP_AUTO = 0, GP_SWEEP_CHUNKED = 1, GP_SWEEP_STREAM = 2 } gp_sweep;

/* Sets the y/z strategy of a plan's later steps (calcluy, calcluz).  The
 * symmetric-trap plans keep the chunked scan.  gp_plan_describe shows the
 * choice per axis. */
gp_status gp_plan_set_sweep(gp_plan *plan, gp_sweep strategy);

/* Frees the plan's tables and scratch after waiting for its stream.
 * NULL-safe. */
gp_status gp_plan_destroy(gp_plan *plan);

/* Changes g (a quench) for the steps queued after this call.  The tables do
 * not depend on g, so nothing is rebuilt (a recorded gp_step graph is
 * dropped, after waiting for the plan's stream). */
gp_status gp_set_g(gp_plan *plan, double g);

/* Changes the trap frequencies (gamma, nu, lambda >= 0, finite) for the
 * steps queued after this call and for gp_observables.  The tables do not
 * depend on the trap, so nothing is rebuilt. */
gp_status gp_set_trap(gp_plan *plan, double gamma, double nu, double lambda);

/* Changes the stream later work is queued on (hipStream_t or NULL). */
gp_status gp_set_stream(gp_plan *plan, void *hip_stream);

/* Queues `nsteps` split-step Crank-Nicolson steps on psi, in place, and
 * returns without waiting.  psi_dev is a device pointer to psi_elems complex
 * numbers of the plan's dtype (psi_elems must equal Nx*Ny*Nz; 16-byte
 * alignment for GP_C128, 8-byte for the complex64 dtypes, real parts only for
 * GP_R64 / GP_R32); the caller owns it, and the library keeps no reference
 * after the work completes.  A GP_C64 psi that is 16-byte aligned lets the
 * y/z sweeps of lines longer than 256 points take two columns per thread
 * (same results, faster).  One step is, in
 * order: calcnu (psi <- exp(-tau (V + g|psi|^2)) psi, tau = dt or i dt),
 * calclux, calcluy, calcluz (one Crank-Nicolson solve per grid line along
 * each axis: the constant tridiagonal matrix of the Thomas recursion, solved
 * through its precomputed Toeplitz factorisation -- two first-order
 * recurrences with one coefficient, carried between chunks of a line by a
 * parallel scan, plus a rank-one boundary term; see gp_sweep_tables -- which
 * equals the Thomas solution up to rounding) and, in imaginary time,
 * calcnorm.  In imaginary time psi has norm 1 when the queued work ends; the
 * per-step renormalisation is carried by the next step's first pass and a
 * final scaling pass, which equals renormalising after every step up to
 * rounding.  nsteps == 0 queues nothing.  A call that repeats one of the
 * plan's last four calls (same psi, same nsteps, no profiling) is recorded
 * once into a HIP graph (the plan then creates a capture stream and the
 * graph; at most four are kept, the least recently used dropped first) and
 * later identical calls replay it: the same launches with the same
 * arguments, so the same results, with less launch overhead.  gp_set_g,
 * gp_set_trap and gp_plan_set_sweep drop the graphs, after waiting for the
 * plan's stream.
 * While the plan's stream is being captured by the caller, calls queue the
 * launches themselves.  Apart from those graphs the plan allocates nothing
 * here; gp_step_noalloc never records one. */
gp_status gp_step(gp_plan *plan, void *psi_dev, int64_t psi_elems, int64_t nsteps);

/* gp_step with a time-dependent nonlinearity and trap, for driven dynamics
 * such as a modulated scattering length g(t) = g0 (1 + eps sin(Omega t)):
 * step s uses g_steps[s] and the trap (trap_steps[3s], trap_steps[3s+1],
 * trap_steps[3s+2]) = (gamma, nu, lambda).  Either array may be NULL (the
 * plan's current value is used); both are host arrays read before this call
 * returns.  The plan keeps the last step's g and trap.  GP_ERR_INVALID, with
 * nothing queued, if a scheduled value is non-finite or a frequency is
 * negative. */
gp_status gp_step_schedule(gp_plan *plan, void *psi_dev, int64_t psi_elems, int64_t nsteps,
                           const double *g_steps, const double *trap_steps);

/* Waits for the plan's stream and reports a failure met by queued work:
 * GP_ERR_NONFINITE after a non-finite or zero norm in imaginary time,
 * GP_ERR_DEVICE after a runtime error.  Clears the recorded failure. */
gp_status gp_sync(gp_plan *plan);

/* Computes the physical quantities of psi (calcmuen, calcrms) and waits for
 * them: one read pass over psi, FP64 partial sums per block, a fixed-order
 * final sum (the result is bitwise reproducible), about 100 bytes copied to
 * the host.  psi is not modified.  Returns GP_ERR_NONFINITE if the norm is
 * zero or any quantity is not finite (out is still filled), and first
 * reports any failure of earlier queued work as gp_sync does. */
gp_status gp_observables(gp_plan *plan, const void *psi_dev, int64_t psi_elems,
                         gp_obs *out);

/* Device bytes a plan for this grid and dtype allocates (tables and
 * scratch), excluding psi.  Returns 0 for an invalid grid. */
size_t gp_plan_footprint_bytes(const int64_t grid[3], gp_dtype dtype);

/* gp_step for callers that cannot allocate device memory: code that must
 * not call hipMalloc (a tight serving loop, a harness that forbids it).
 * Queues the same work as gp_plan_create with these arguments (ndim 3,
 * Cartesian) followed by gp_step(psi, nsteps) on that plan, with bitwise the
 * same result, and returns without waiting; nothing is allocated (no
 * hipMalloc, hipFree or host heap on this path).  Instead of a plan's memory
 * it uses a static device array of the library, 2.1 MiB per device, held
 * until the process ends: the correction tables of the three axes (rebuilt on
 * the host at every call and written by small kernels queued on the stream),
 * one norm partial per z line, the pending 1/sqrt(N) and an error flag
 * (cleared at every call).  Limit: Nx * Ny <= 262144 (GP_ERR_UNSUPPORTED
 * beyond), on top of gp_plan_create's.  Every call on one device shares that
 * array, so calls whose queued work overlaps on a device race: order them,
 * for example by queueing them on one stream.  A zero or non-finite norm in
 * imaginary time is not reported (no later call can read the flag); it
 * leaves psi non-finite.  Errors otherwise as gp_plan_create and gp_step;
 * on GP_ERR_INVALID or GP_ERR_UNSUPPORTED nothing is queued. */
gp_status gp_step_noalloc(const int64_t grid[3], const double dx[3], double dt,
                          double gamma, double nu, double lambda, double g,
                          gp_mode mode, gp_dtype dtype, void *hip_stream,
                          void *psi_dev, int64_t psi_elems, int64_t nsteps);

/* Density profiles of psi (the paper's programs write the density along the
 * axes as output): px[i] = dy dz sum_{j,k} |psi_ijk|^2, and likewise py[Ny],
 * pz[Nz], with the spacings of the present axes only (gp_plan_create_nd).
 * Host arrays of Nx, Ny, Nz doubles; FP64 sums in a fixed order; waits for
 * the result.  Allocates a small device buffer per call.  Cartesian plans
 * only (GP_ERR_UNSUPPORTED for the symmetric traps). */
gp_status gp_density_profiles(gp_plan *plan, const void *psi_dev, int64_t psi_elems, double *px, double *py,
                              double *pz);

/* Writes a one-line description of the plan's launch shapes into buf
 * (NUL-terminated, truncated to len). */
gp_status gp_plan_describe(const gp_plan *plan, char *buf, size_t len);

/* Static text for a status code. */
const char *gp_status_string(gp_status s);

/* Message of the last failure on the calling host thread ("" if none). */
const char *gp_last_error(void);

/* Per-kernel timing with HIP events on the plan's stream.  While enabled,
 * every launch is bracketed by two events; gp_profile_read waits for the
 * stream, adds the elapsed time of every bracketed launch per kernel class
 * (GP_KERNEL_*) into ms[GP_KERNEL_COUNT], the launch counts into
 * launches[GP_KERNEL_COUNT], and clears the record.  Disabled by default. */
gp_status gp_profile_enable(gp_plan *plan, int on);
gp_status gp_profile_read(gp_plan *plan, double *ms, int64_t *launches);

/* Chunking the kernels use for a line of n points along `axis` (0 = x,
 * 1 = y, 2 = z): `chunk` contiguous points per lane, `lanes` chunks per line
 * (64 for x).  Host only.  GP_ERR_UNSUPPORTED if the line is too long. */
gp_status gp_sweep_shape(int64_t n, int axis, gp_dtype dtype, int *chunk, int *lanes);

/* ---- Batches: many independent solves advanced together ---------------
 *
 * For throughput on grids too small to fill the GPU alone (the ground states
 * of a parameter scan, the requests of a service): the solves of a batch
 * share mode and dtype but each has its own grid, spacings, step, trap and
 * g.  Solves with the same grid shape form a class; every sweep is one
 * launch per class covering all its active solves.  Each solve's result is
 * bitwise the one a gp_plan with the same parameters gives.  The batch
 * queues work on a stream of its own, ordered after the caller's stream at
 * the start of every call and before it at the end. */
typedef struct gp_batch gp_batch;

enum {
    GP_BATCH_GRAPH = 1,  /* capture one step of all classes in a HIP graph and replay it */
    GP_BATCH_TUNE = 2,   /* time per class at creation, on scratch memory: the y/z block widths,
                            column pairs (complex64, even Nx) and x lines per wavefront; none of
                            them changes a result */
    GP_BATCH_FINISH_F64 = 4, /* imaginary-time GP_C64 / GP_R32 batches: gp_batch_solve_imag finishes
                                each solve in FP64 storage (see there) */
    GP_BATCH_ONE_LAUNCH = 8  /* each sweep of a step one launch over every class (blocks find their
                                class and solve with its chunking and tile shape) instead of one launch
                                per class.  Currently refused with GP_ERR_UNSUPPORTED: its first GPU test
                                ended in a device fault whose cause is not yet found */
};

/* Creates a batch of nsolves solves.  Per solve i: grids[3i..3i+2] (Nx, Ny,
 * Nz, each 1..1024), dx[3i..3i+2] > 0, dt[i] > 0, traps[3i..3i+2] >= 0,
 * g[i] finite.  flags: GP_BATCH_* bits.  hip_stream: the caller's stream
 * (NULL: the null stream).  GP_ERR_INVALID / _UNSUPPORTED / _NOMEM /
 * _DEVICE on failure with *out = NULL. */
gp_status gp_batch_create(int nsolves, const int64_t *grids, const double *dx, const double *dt,
                          const double *traps, const double *g, gp_mode mode, gp_dtype dtype,
                          int flags, void *hip_stream, gp_batch **out);

/* Waits for the batch's work and frees it.  NULL-safe. */
gp_status gp_batch_destroy(gp_batch *batch);

/* Binds solve i to the caller-owned device array psi[i] of elems[i]
 * complex numbers (the layout and alignment of gp_step).  Must precede
 * gp_batch_step; may be repeated to rebind. */
gp_status gp_batch_set_psi(gp_batch *batch, void *const *psi, const int64_t *elems);

/* Selects the solves later calls advance and measure: mask[i] != 0 (NULL:
 * all).  Inactive solves are left untouched. */
gp_status gp_batch_set_active(gp_batch *batch, const unsigned char *mask);

/* Queues nsteps split-step Crank-Nicolson steps of every active solve (in
 * imaginary time each ends normalised, as gp_step). */
gp_status gp_batch_step(gp_batch *batch, int64_t nsteps);

/* Physical quantities of every active solve into out[i] (inactive entries
 * are not written); waits for them.  GP_ERR_NONFINITE if any solve's norm
 * or quantity is not finite (all entries still filled). */
gp_status gp_batch_observables(gp_batch *batch, gp_obs *out);

/* Imaginary-time ground states with a per-solve stopping rule: every
 * check_every steps the chemical potentials are evaluated, and a solve
 * whose mu moved by less than tol since the previous evaluation stops (is
 * no longer advanced).  Ends when all solves stopped or after max_steps.
 * Fills out[i] (last evaluation), steps[i] (steps taken) and converged[i].
 * Every solve is active again on return.
 * With GP_BATCH_FINISH_F64 the float storage carries a solve only until its
 * mu moves by less than 100 tol between evaluations; its state is then
 * copied exactly to double storage of the batch's own (complex128 for
 * GP_C64, double for GP_R32) and the solve continues there, on FP64
 * arithmetic, until the rule above holds for two FP64 evaluations.  A float
 * state near convergence stops following the FP64 iteration (each step's
 * change falls below half a float ulp), so this is what brings mu to FP64
 * accuracy.  The final state is rounded back into the caller's float
 * buffer; out[i] is the evaluation of the FP64 state. */
gp_status gp_batch_solve_imag(gp_batch *batch, double tol, int64_t check_every, int64_t max_steps,
                              gp_obs *out, int64_t *steps, unsigned char *converged);

/* One-line description of the classes and launch shapes. */
gp_status gp_batch_describe(const gp_batch *batch, char *buf, size_t len);

/* ---- Serving: continuous batching of solve requests ------------------
 *
 * A server owns one device arena of hbm_budget bytes and an engine thread.
 * Requests (ground states in imaginary time, dynamics in real time; any
 * grid, spacing, step, trap and g) are queued by gp_server_submit and
 * admitted, in arrival order with later requests allowed to pass one that
 * does not fit yet, whenever a slot and gp_server_request_bytes of the arena
 * are free; the request's psi, tables and reduction scratch then stay
 * resident until it finishes.  All resident solves advance together: every
 * check_every steps the engine admits new requests, and between those points
 * the solves of one grid shape and mode share one launch per sweep (the
 * kernels of gp_batch).  A solve's events (the chemical-potential check of an
 * imaginary-time solve, the end of a run) fall on multiples of check_every
 * of its own steps, so its result is bitwise the same alone and in any mix,
 * and equal to a gp_plan stepped check_every steps per gp_step call.
 * The stopping rule of an imaginary-time request is gp_batch_solve_imag's:
 * stop when mu moved by less than tol since the previous check, or after
 * `steps` steps. */
typedef struct gp_server gp_server;

enum {
    GP_SERVER_GRAPH = 1,     /* capture one step of the resident set in a HIP graph, re-captured when it changes */
    GP_SERVER_REAL_AUTO = 2  /* on a GP_C64 or GP_C128 server, an imaginary-time request whose initial state has
                                no imaginary part (every imaginary part exactly 0, checked in gp_server_submit)
                                runs on real storage, as with real_state, while its host buffers stay complex:
                                the result is the one real_state gives, written with zero imaginary parts */
};

typedef struct {
    int64_t grid[3];      /* Nx, Ny, Nz, each 1..1024 */
    double dx[3];         /* > 0 */
    double dt;            /* > 0 */
    double trap[3];       /* gamma, nu, lambda >= 0 */
    double g;             /* finite */
    gp_mode mode;
    int64_t steps;        /* real time: steps to run; imaginary time: the step cap; >= 1 */
    double tol;           /* imaginary time: |delta mu| stopping tolerance (0: run to the cap) */
    const void *psi_in;   /* host memory: the initial state, Nx*Ny*Nz elements of the server's dtype
                             (or of its real counterpart, see real_state), in gp_step's layout;
                             read at admission */
    void *psi_out;        /* host memory for the final state (may be psi_in); written before the
                             result is reported */
    uint64_t tag;         /* the caller's, returned in the result */
    int real_state;       /* imaginary time only: psi_in and psi_out hold real values (double on a
                             GP_C128 server, float on a GP_C64 one) and the solve runs on real
                             storage (GP_R64 / GP_R32: half the bytes, the same arithmetic) */
} gp_request;

typedef struct {
    uint64_t id, tag;
    gp_status status;     /* GP_OK, GP_ERR_NONFINITE (zero or non-finite norm), GP_ERR_DEVICE */
    int converged;        /* imaginary time: stopped by tol */
    int64_t steps;        /* steps taken */
    gp_obs obs;           /* of the final state (steps_done = steps) */
    double t_submit, t_admit, t_done;  /* seconds on the server's monotonic clock */
} gp_result;

typedef struct {
    int64_t submitted, completed, queued, resident, max_resident;
    int64_t quanta;          /* engine rounds (each check_every steps or fewer) */
    int64_t graph_captures;
    int64_t solve_steps;     /* steps summed over solves */
    uint64_t bytes_in_use, bytes_peak, bytes_budget;
    double seconds_copy_in, seconds_copy_out, seconds_rounds;   /* engine time: admissions' copies in,
                                                                    finished states out, queued rounds
                                                                    up to their completion */
} gp_server_counters;

/* Device bytes one request of this grid, dtype and mode holds while resident
 * (psi, its correction tables, reduction scratch), or 0 if the grid is not
 * supported. */
size_t gp_server_request_bytes(const int64_t grid[3], gp_dtype dtype, gp_mode mode);

/* Creates a server on the current device: an arena of hbm_budget bytes,
 * at most max_slots resident requests (1..4096), checks every check_every
 * steps (>= 1).  GP_ERR_NOMEM if the arena cannot be allocated. */
gp_status gp_server_create(gp_dtype dtype, uint64_t hbm_budget, int max_slots, int64_t check_every,
                           int flags, gp_server **out);

/* Stops the engine and frees the server.  Requests not yet reported are
 * dropped (their host buffers are no longer touched once this returns).
 * NULL-safe. */
gp_status gp_server_destroy(gp_server *server);

/* Queues a request; *id identifies its result.  The host buffers must stay
 * valid until the result is reported.  GP_ERR_INVALID for bad parameters,
 * GP_ERR_UNSUPPORTED for an unsupported grid, GP_ERR_NOMEM if the request
 * could never fit the arena, GP_ERR_DEVICE once the engine has failed. */
gp_status gp_server_submit(gp_server *server, const gp_request *req, uint64_t *id);

/* Moves up to max finished results into out (*n of them), waiting up to
 * wait_seconds for the first one (0: do not wait). */
gp_status gp_server_poll(gp_server *server, gp_result *out, int max, double wait_seconds, int *n);

/* Waits up to wait_seconds until no request is queued or resident; *idle
 * says whether that point was reached.  Results stay until polled. */
gp_status gp_server_drain(gp_server *server, double wait_seconds, int *idle);

gp_status gp_server_stats(gp_server *server, gp_server_counters *out);

/* Host-only view of the constant coefficients the sweep kernels use along
 * one axis (no device call), for inspection and tests.  For a line of n
 * points, spacing dx, step dt, mode and a chunking with chunk * lanes >= n,
 * lanes <= 64.  With kappa = tau/(2 dx^2) (tau = dt or i dt) the
 * Crank-Nicolson matrix of the line is tridiag(o, b, o), b = 1 + kappa,
 * o = -kappa/2; the kernels solve it through the factorisation
 *     tridiag(o, b, o) = beta (I + c S)(I + c S^T) + beta c^2 e_0 e_0^T
 * (S the down-shift, |c| < 1, beta = o/c): w_i = m r_i + a w_{i-1},
 * y_i = w_i + a y_{i+1} (m = 1/beta, a = -c), then x_i = y_i + y_0 zt_i.
 * Fills, every complex value as an (re, im) pair of doubles:
 *   coef[14]          kappa, b, o, c, beta, m, a;
 *   stage[2*6]        a^(chunk 2^s), s = 0..5 (Kogge-Stone multipliers);
 *   zt[2*n]           the boundary correction by position.
 * Lengths are counts of doubles.  GP_ERR_INVALID for bad arguments or short
 * buffers. */
gp_status gp_sweep_tables(int64_t n, double dx, double dt, gp_mode mode, int chunk,
                          int lanes, double *coef, size_t coef_len, double *stage,
                          size_t stage_len, double *zt, size_t zt_len);

#ifdef __cplusplus
}
#endif

#endif /* GPSSC_H */
