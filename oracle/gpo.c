/*
 * gpo.c -- CPU FP64 oracle for the split-step Crank-Nicolson (SSCN) step of
 * the three-dimensional, fully anisotropic Gross-Pitaevskii (GP) equation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no source,
 * header, table or helper with the GPU library, and the GPU library never
 * calls it.
 *
 * What is computed (Vudragovic et al., Comput. Phys. Commun. 183 (2012) 2021,
 * program summaries (v) imagtime3d and (xiv) realtime3d, "Method of solution";
 * "Summary of revisions" names the routines calcnu, calclux, calcluy, calcluz,
 * calcnorm, calcmuen and calcrms that carry the time evolution, the
 * normalisation and the physical quantities).  The paper prints no formula;
 * the readings used here are:
 *
 *   equation   i dpsi/dt = [ -1/2 Lap + V + g|psi|^2 ] psi,
 *              V = 1/2 (gamma^2 x^2 + nu^2 y^2 + lambda^2 z^2);
 *              imaginary time replaces t by -i t and renormalises.
 *   grid       x_i = (i - (N-1)/2) dx, i = 0..N-1 per axis; Dirichlet ghost
 *              values psi_{-1} = psi_N = 0.  Storage is C order (z, y, x):
 *              p = (k*Ny + j)*Nx + i, complex<double> interleaved (re, im).
 *   one step   (Lie splitting, in the order the routines are named)
 *              1. calcnu : psi <- exp(-tau theta) psi, theta = V + g|psi|^2
 *                          taken from psi before the sub-step;
 *                          tau = dt (imaginary time) or i dt (real time).
 *              2. calclux, calcluy, calcluz : for every grid line along the
 *                 axis, Crank-Nicolson
 *                     (1 + tau/2 T) psi' = (1 - tau/2 T) psi,
 *                 T psi_i = -(psi_{i+1} - 2 psi_i + psi_{i-1}) / (2 dx^2),
 *                 i.e. with kappa = tau/(2 dx^2):
 *                     A = tridiag(-kappa/2, 1 + kappa, -kappa/2)
 *                     q_i = (1 - kappa) psi_i + kappa/2 (psi_{i-1} + psi_{i+1})
 *                 solved by the Thomas recursion whose coefficients depend
 *                 only on (N, kappa) and are computed once per sweep.
 *              3. calcnorm (imaginary time only): N = dV sum |psi|^2,
 *                 psi <- psi / sqrt(N).
 *   physical quantities (calcmuen, calcrms), on psi-hat = psi / sqrt(N):
 *              K = 1/2 dV sum_axes sum_links |psi_{i+1} - psi_i|^2 / dx_a^2
 *                  (links include the two ghost links of every line),
 *              P = dV sum V |psi|^2,  I = g dV sum |psi|^4,
 *              E  = K/N + P/N + I/(2 N^2),
 *              mu = K/N + P/N + I/N^2,
 *              rms_a = sqrt(dV sum a^2 |psi|^2 / N), rms_r = |(rms_a)|,
 *              mean_a = dV sum a |psi|^2 / N.
 *
 * Fewer space variables (program summaries (i) imagtime1d, (ii) imagtime2d,
 * (x) realtime1d and (xi) realtime2d; "Nature of problem": one, two or three
 * space dimensions).  The _nd entry points take ndim = 1 (x) or 2 (x, y);
 * the absent axes have one node and no part in the equation: no sweep along
 * them, no trap term or kinetic links for them, and the cell volume dV is
 * the product of the present spacings only.  So the ndim-dimensional
 * equation is the one above with the Laplacian, V and the sums restricted
 * to the present variables (reading: g is the coupling of that equation as
 * given, no conversion from three dimensions).
 *
 * Sums over the grid are formed per z plane in index order and then over the
 * planes in index order, so the result does not depend on the thread count.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define GPO_IMAG 0
#define GPO_REAL 1

#define GPO_OK 0
#define GPO_ERR_INVALID 1
#define GPO_ERR_NOMEM 2
#define GPO_ERR_NONFINITE 4

/* Observable slots written by gpo_observables. */
enum {
    GPO_OBS_NORM = 0, GPO_OBS_MU, GPO_OBS_ENERGY,
    GPO_OBS_RMS_X, GPO_OBS_RMS_Y, GPO_OBS_RMS_Z, GPO_OBS_RMS_R,
    GPO_OBS_MEAN_X, GPO_OBS_MEAN_Y, GPO_OBS_MEAN_Z,
    GPO_OBS_KIN, GPO_OBS_POT, GPO_OBS_INT,
    GPO_OBS_COUNT
};

/* ------------------------------------------------------------------ */
/* parameters                                                          */
/* ------------------------------------------------------------------ */

static int valid_params(const int64_t n[3], const double dx[3], double dt,
                        const double omega[3], double g, int mode)
{
    if (!n || !dx || !omega) return 0;
    for (int a = 0; a < 3; ++a) {
        if (n[a] < 1) return 0;
        if (!(dx[a] > 0.0) || !isfinite(dx[a])) return 0;
        if (!(omega[a] >= 0.0) || !isfinite(omega[a])) return 0;
    }
    if (!(dt > 0.0) || !isfinite(dt)) return 0;
    if (!isfinite(g)) return 0;
    if (mode != GPO_IMAG && mode != GPO_REAL) return 0;
    return 1;
}

int gpo_validate(const int64_t n[3], const double dx[3], double dt,
                 const double omega[3], double g, int mode)
{
    return valid_params(n, dx, dt, omega, g, mode) ? GPO_OK : GPO_ERR_INVALID;
}

/* ndim in 1..3, and one node along every absent axis. */
static int valid_ndim(int ndim, const int64_t n[3])
{
    if (ndim < 1 || ndim > 3 || !n) return 0;
    for (int a = ndim; a < 3; ++a)
        if (n[a] != 1) return 0;
    return 1;
}

/* Cell volume of the present axes. */
static double cell_volume(int ndim, const double dx[3])
{
    double v = 1.0;
    for (int a = 0; a < ndim; ++a) v *= dx[a];
    return v;
}

/* Grid node coordinate along one axis: symmetric about the origin. */
double gpo_coord(int64_t n, double dx, int64_t i)
{
    return ((double)i - 0.5 * (double)(n - 1)) * dx;
}

/* Harmonic trap V = 1/2 (gamma^2 x^2 + nu^2 y^2 + lambda^2 z^2). */
static double potential(const double omega[3], double x, double y, double z)
{
    return 0.5 * (omega[0] * omega[0] * x * x + omega[1] * omega[1] * y * y
                  + omega[2] * omega[2] * z * z);
}

/* tau = dt in imaginary time, i*dt in real time. */
static cplx tau_of(double dt, int mode)
{
    return mode == GPO_REAL ? I * dt : (cplx)dt;
}

static int max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void gpo_set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int gpo_get_threads(void) { return max_threads(); }

/* ------------------------------------------------------------------ */
/* Thomas recursion for the constant-coefficient tridiagonal system    */
/*   diag * x_i + off * (x_{i-1} + x_{i+1}) = r_i,  x_{-1} = x_N = 0    */
/* ------------------------------------------------------------------ */

/* Coefficients that depend on (n, diag, off) only:
 *   m_0 = 1/diag,                 cp_0 = off * m_0,
 *   m_i = 1/(diag - off*cp_{i-1}), cp_i = off * m_i.                  */
static void thomas_tables(int64_t n, cplx diag, cplx off, cplx *m, cplx *cp)
{
    m[0] = 1.0 / diag;
    cp[0] = off * m[0];
    for (int64_t i = 1; i < n; ++i) {
        m[i] = 1.0 / (diag - off * cp[i - 1]);
        cp[i] = off * m[i];
    }
}

/* Forward elimination then back substitution, in place on r. */
static void thomas_apply(int64_t n, cplx off, const cplx *m, const cplx *cp,
                         cplx *r)
{
    r[0] = r[0] * m[0];
    for (int64_t i = 1; i < n; ++i)
        r[i] = (r[i] - off * r[i - 1]) * m[i];
    for (int64_t i = n - 2; i >= 0; --i)
        r[i] = r[i] - cp[i] * r[i + 1];
}

/* Exposed for the dense-solve check: solves the system above. */
int gpo_thomas(int64_t n, double diag_re, double diag_im, double off_re,
               double off_im, const double *rhs, double *x)
{
    if (n < 1 || !rhs || !x) return GPO_ERR_INVALID;
    cplx diag = diag_re + I * diag_im, off = off_re + I * off_im;
    cplx *m = malloc(sizeof(cplx) * (size_t)n);
    cplx *cp = malloc(sizeof(cplx) * (size_t)n);
    cplx *r = malloc(sizeof(cplx) * (size_t)n);
    if (!m || !cp || !r) { free(m); free(cp); free(r); return GPO_ERR_NOMEM; }
    thomas_tables(n, diag, off, m, cp);
    memcpy(r, rhs, sizeof(cplx) * (size_t)n);
    thomas_apply(n, off, m, cp, r);
    memcpy(x, r, sizeof(cplx) * (size_t)n);
    free(m); free(cp); free(r);
    return GPO_OK;
}

/* ------------------------------------------------------------------ */
/* calcnu: pointwise potential + nonlinear sub-step                    */
/* ------------------------------------------------------------------ */

static void calcnu(const int64_t n[3], const double dx[3], double dt,
                   const double omega[3], double g, int mode, cplx *psi)
{
    const int64_t nx = n[0], ny = n[1], nz = n[2];
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k) {
        double z = gpo_coord(nz, dx[2], k);
        for (int64_t j = 0; j < ny; ++j) {
            double y = gpo_coord(ny, dx[1], j);
            for (int64_t i = 0; i < nx; ++i) {
                double x = gpo_coord(nx, dx[0], i);
                int64_t p = (k * ny + j) * nx + i;
                double dens = creal(psi[p]) * creal(psi[p])
                            + cimag(psi[p]) * cimag(psi[p]);
                double theta = potential(omega, x, y, z) + g * dens;
                if (mode == GPO_REAL)
                    psi[p] *= cos(dt * theta) - I * sin(dt * theta);
                else
                    psi[p] *= exp(-dt * theta);
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* calclux / calcluy / calcluz: Crank-Nicolson along one axis          */
/* ------------------------------------------------------------------ */

/* Solves every line along `axis` (0 = x, 1 = y, 2 = z). */
static int calclu(const int64_t n[3], const double dx[3], double dt, int mode,
                  int axis, cplx *psi)
{
    const int64_t nx = n[0], ny = n[1];
    const int64_t len = n[axis];
    const int64_t stride = axis == 0 ? 1 : (axis == 1 ? nx : nx * ny);
    const int64_t nlines = (n[0] * n[1] * n[2]) / len;
    const cplx kappa = tau_of(dt, mode) / (2.0 * dx[axis] * dx[axis]);
    const cplx diag = 1.0 + kappa, off = -0.5 * kappa;      /* left side  */
    const cplx rdiag = 1.0 - kappa, roff = 0.5 * kappa;     /* right side */

    cplx *m = malloc(sizeof(cplx) * (size_t)len);
    cplx *cp = malloc(sizeof(cplx) * (size_t)len);
    if (!m || !cp) { free(m); free(cp); return GPO_ERR_NOMEM; }
    thomas_tables(len, diag, off, m, cp);

    int failed = 0;
#pragma omp parallel
    {
        cplx *line = malloc(sizeof(cplx) * (size_t)len);
        cplx *r = malloc(sizeof(cplx) * (size_t)len);
        if (!line || !r) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(static)
        for (int64_t l = 0; l < nlines; ++l) {
            if (!line || !r) continue;
            /* first element of line l */
            int64_t base;
            if (axis == 0) {
                base = l * nx;
            } else if (axis == 1) {
                int64_t i = l % nx, k = l / nx;
                base = k * nx * ny + i;
            } else {
                base = l;   /* l = j*nx + i */
            }
            for (int64_t t = 0; t < len; ++t) line[t] = psi[base + t * stride];
            for (int64_t t = 0; t < len; ++t) {
                cplx left = t > 0 ? line[t - 1] : 0.0;
                cplx right = t + 1 < len ? line[t + 1] : 0.0;
                r[t] = rdiag * line[t] + roff * (left + right);
            }
            thomas_apply(len, off, m, cp, r);
            for (int64_t t = 0; t < len; ++t) psi[base + t * stride] = r[t];
        }
        free(line);
        free(r);
    }
    free(m);
    free(cp);
    return failed ? GPO_ERR_NOMEM : GPO_OK;
}

/* ------------------------------------------------------------------ */
/* calcnorm                                                            */
/* ------------------------------------------------------------------ */

/* sum |psi|^2, per plane then over planes (thread-count independent). */
static double sum_density(const int64_t n[3], const cplx *psi, double *plane)
{
    const int64_t nxy = n[0] * n[1], nz = n[2];
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k) {
        double s = 0.0;
        for (int64_t q = 0; q < nxy; ++q) {
            cplx v = psi[k * nxy + q];
            s += creal(v) * creal(v) + cimag(v) * cimag(v);
        }
        plane[k] = s;
    }
    double s = 0.0;
    for (int64_t k = 0; k < nz; ++k) s += plane[k];
    return s;
}

int gpo_norm_nd(int ndim, const int64_t n[3], const double dx[3], const double *psi_ri,
                double *norm_out)
{
    if (!valid_ndim(ndim, n) || !dx || !psi_ri || !norm_out) return GPO_ERR_INVALID;
    double *plane = malloc(sizeof(double) * (size_t)n[2]);
    if (!plane) return GPO_ERR_NOMEM;
    *norm_out = cell_volume(ndim, dx) * sum_density(n, (const cplx *)psi_ri, plane);
    free(plane);
    return GPO_OK;
}

int gpo_norm(const int64_t n[3], const double dx[3], const double *psi_ri,
             double *norm_out)
{
    return gpo_norm_nd(3, n, dx, psi_ri, norm_out);
}

static int calcnorm(const int64_t n[3], double dv, cplx *psi, double *plane)
{
    const int64_t total = n[0] * n[1] * n[2];
    double norm = dv * sum_density(n, psi, plane);
    if (!(norm > 0.0) || !isfinite(norm)) return GPO_ERR_NONFINITE;
    double s = 1.0 / sqrt(norm);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < total; ++p) psi[p] *= s;
    return GPO_OK;
}

/* ------------------------------------------------------------------ */
/* one SSCN step, repeated                                             */
/* ------------------------------------------------------------------ */

int gpo_step_nd(int ndim, const int64_t n[3], const double dx[3], double dt,
                const double omega[3], double g, int mode, double *psi_ri,
                int64_t nsteps)
{
    if (!valid_params(n, dx, dt, omega, g, mode) || !valid_ndim(ndim, n) || !psi_ri || nsteps < 0)
        return GPO_ERR_INVALID;
    cplx *psi = (cplx *)psi_ri;
    double om[3];
    for (int a = 0; a < 3; ++a) om[a] = a < ndim ? omega[a] : 0.0;   /* no trap along absent axes */
    const double dv = cell_volume(ndim, dx);
    double *plane = malloc(sizeof(double) * (size_t)n[2]);
    if (!plane) return GPO_ERR_NOMEM;
    int st = GPO_OK;
    for (int64_t s = 0; s < nsteps && st == GPO_OK; ++s) {
        calcnu(n, dx, dt, om, g, mode, psi);
        for (int a = 0; a < ndim && st == GPO_OK; ++a) st = calclu(n, dx, dt, mode, a, psi);
        if (st == GPO_OK && mode == GPO_IMAG) st = calcnorm(n, dv, psi, plane);
    }
    free(plane);
    return st;
}

int gpo_step(const int64_t n[3], const double dx[3], double dt,
             const double omega[3], double g, int mode, double *psi_ri,
             int64_t nsteps)
{
    return gpo_step_nd(3, n, dx, dt, omega, g, mode, psi_ri, nsteps);
}

/* Single sub-steps, so that tests can check each against an independent
 * formulation.  which: 0 = calcnu, 1..3 = calclux/y/z, 4 = calcnorm. */
int gpo_substep(const int64_t n[3], const double dx[3], double dt,
                const double omega[3], double g, int mode, double *psi_ri,
                int which)
{
    if (!valid_params(n, dx, dt, omega, g, mode) || !psi_ri)
        return GPO_ERR_INVALID;
    cplx *psi = (cplx *)psi_ri;
    switch (which) {
    case 0: calcnu(n, dx, dt, omega, g, mode, psi); return GPO_OK;
    case 1: case 2: case 3: return calclu(n, dx, dt, mode, which - 1, psi);
    case 4: {
        double *plane = malloc(sizeof(double) * (size_t)n[2]);
        if (!plane) return GPO_ERR_NOMEM;
        int st = calcnorm(n, dx[0] * dx[1] * dx[2], psi, plane);
        free(plane);
        return st;
    }
    default: return GPO_ERR_INVALID;
    }
}

/* ------------------------------------------------------------------ */
/* calcmuen / calcrms: physical quantities                             */
/* ------------------------------------------------------------------ */

/* Raw sums of one z plane, in index order. */
typedef struct {
    double dens, pot, quart, link[3], m1[3], m2[3];
} plane_sums;

int gpo_observables_nd(int ndim, const int64_t n[3], const double dx[3],
                       const double omega[3], double g, const double *psi_ri,
                       double *out)
{
    if (!n || !dx || !omega || !psi_ri || !out || !valid_ndim(ndim, n)) return GPO_ERR_INVALID;
    double om[3];
    for (int a = 0; a < 3; ++a) om[a] = a < ndim ? omega[a] : 0.0;
    for (int a = 0; a < 3; ++a)
        if (n[a] < 1 || !(dx[a] > 0.0)) return GPO_ERR_INVALID;
    const cplx *psi = (const cplx *)psi_ri;
    const int64_t nx = n[0], ny = n[1], nz = n[2];
    plane_sums *ps = calloc((size_t)nz, sizeof(plane_sums));
    if (!ps) return GPO_ERR_NOMEM;

#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k) {
        plane_sums s;
        memset(&s, 0, sizeof s);
        double z = gpo_coord(nz, dx[2], k);
        for (int64_t j = 0; j < ny; ++j) {
            double y = gpo_coord(ny, dx[1], j);
            for (int64_t i = 0; i < nx; ++i) {
                double x = gpo_coord(nx, dx[0], i);
                int64_t p = (k * ny + j) * nx + i;
                cplx v = psi[p];
                double w = creal(v) * creal(v) + cimag(v) * cimag(v);
                s.dens += w;
                s.pot += potential(om, x, y, z) * w;
                s.quart += w * w;
                s.m1[0] += x * w; s.m1[1] += y * w; s.m1[2] += z * w;
                s.m2[0] += x * x * w; s.m2[1] += y * y * w; s.m2[2] += z * z * w;
                /* link to the next node along each axis; the ghost beyond the
                 * last node is zero, the link before the first node is added
                 * at the first node. */
                cplx nxt[3];
                nxt[0] = i + 1 < nx ? psi[p + 1] : 0.0;
                nxt[1] = j + 1 < ny ? psi[p + nx] : 0.0;
                nxt[2] = k + 1 < nz ? psi[p + nx * ny] : 0.0;
                int first[3] = { i == 0, j == 0, k == 0 };
                for (int a = 0; a < 3; ++a) {
                    cplx d = nxt[a] - v;
                    s.link[a] += creal(d) * creal(d) + cimag(d) * cimag(d);
                    if (first[a]) s.link[a] += w;
                }
            }
        }
        ps[k] = s;
    }
    plane_sums t;
    memset(&t, 0, sizeof t);
    for (int64_t k = 0; k < nz; ++k) {
        t.dens += ps[k].dens; t.pot += ps[k].pot; t.quart += ps[k].quart;
        for (int a = 0; a < 3; ++a) {
            t.link[a] += ps[k].link[a];
            t.m1[a] += ps[k].m1[a];
            t.m2[a] += ps[k].m2[a];
        }
    }
    free(ps);

    const double dv = cell_volume(ndim, dx);
    const double norm = dv * t.dens;
    for (int q = 0; q < GPO_OBS_COUNT; ++q) out[q] = NAN;
    out[GPO_OBS_NORM] = norm;
    if (!(norm > 0.0) || !isfinite(norm)) return GPO_ERR_NONFINITE;
    double kin = 0.0;
    for (int a = 0; a < ndim; ++a) kin += t.link[a] / (dx[a] * dx[a]);
    kin *= 0.5 * dv;
    const double pot = dv * t.pot;
    const double inter = g * dv * t.quart;
    out[GPO_OBS_KIN] = kin / norm;
    out[GPO_OBS_POT] = pot / norm;
    out[GPO_OBS_INT] = inter / (norm * norm);
    out[GPO_OBS_ENERGY] = kin / norm + pot / norm + 0.5 * inter / (norm * norm);
    out[GPO_OBS_MU] = kin / norm + pot / norm + inter / (norm * norm);
    double r2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double m2 = dv * t.m2[a] / norm;
        out[GPO_OBS_RMS_X + a] = sqrt(m2);
        out[GPO_OBS_MEAN_X + a] = dv * t.m1[a] / norm;
        r2 += m2;
    }
    out[GPO_OBS_RMS_R] = sqrt(r2);
    for (int q = 0; q < GPO_OBS_COUNT; ++q)
        if (!isfinite(out[q])) return GPO_ERR_NONFINITE;
    return GPO_OK;
}

int gpo_observables(const int64_t n[3], const double dx[3],
                    const double omega[3], double g, const double *psi_ri,
                    double *out)
{
    return gpo_observables_nd(3, n, dx, omega, g, psi_ri, out);
}
