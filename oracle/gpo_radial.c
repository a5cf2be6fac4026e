/*
 * gpo_radial.c -- CPU FP64 oracle for the symmetric forms of the
 * Gross-Pitaevskii equation: the two-dimensional circularly symmetric and
 * the three-dimensional spherically symmetric trap (one radial variable),
 * and the three-dimensional axially symmetric trap (variables rho, z).
 *
 * TEST INFRASTRUCTURE ONLY, like gpo.c: loaded by the test suite, the smoke
 * check and the benchmark's CPU leg; shares nothing with the GPU library.
 *
 * Paper: program summaries (iv) imagtimecir, (ix) imagtimesph, (vii)
 * imagtimeaxial and their real-time counterparts (xiii), (xvi), and the
 * abstract's list of trap geometries (circularly and spherically symmetric
 * traps in one space variable, the axially symmetric trap in two).  The
 * paper names the split-step Crank-Nicolson method but prints no radial
 * discretisation, so the one below is a reading of this oracle:
 *
 *   radial grid    r_i = (i + 1/2) h, i = 0..N-1; no flux through r = 0;
 *                  Dirichlet psi_N = 0 one node beyond the last.
 *   weights        in D dimensions (D = 2 circular and axial, 3 spherical)
 *                  s_{i+1/2} = ((i+1) h)^(D-1)   (face areas per solid angle)
 *                  v_i = ((i+1)^D - i^D) h^(D-1) / D  (so h sum v_i f_i
 *                                                    ~ int f r^(D-1) dr)
 *   Laplacian      conservative finite volume:
 *                  (L psi)_i = [s_{i+1/2}(psi_{i+1} - psi_i)
 *                              - s_{i-1/2}(psi_i - psi_{i-1})] / (h^2 v_i),
 *                  s_{-1/2} = 0; along z (axial) the usual 3-point form on
 *                  the symmetric node grid of gpo.c.
 *   equation       i dpsi/dt = [-1/2 L + V + g|psi|^2] psi with
 *                  V = 1/2 w^2 r^2 (circular, spherical; w = omega[0]) or
 *                  V = 1/2 (gamma^2 rho^2 + lambda^2 z^2) (axial; gamma =
 *                  omega[0], lambda = omega[2]).
 *   volume         dV_i = S_D h v_i (x dz, axial), S_2 = 2 pi, S_3 = 4 pi;
 *                  the norm is N = sum dV |psi|^2.
 *   one step       calcnu, then Crank-Nicolson along r (a tridiagonal system
 *                  with position-dependent, time-constant coefficients,
 *                  solved by the Thomas recursion), then along z (axial),
 *                  then calcnorm in imaginary time.
 *   quantities     K = 1/2 <psi, -L psi> summed by parts:
 *                    radial part (S_D / (2h)) sum_i s_{i+1/2} |psi_{i+1} - psi_i|^2
 *                    (x dz, axial; the last link goes to the zero ghost),
 *                    z part 1/2 sum dV |psi_{k+1} - psi_k|^2 / dz^2 with both
 *                    ghost links (axial);
 *                  P, I, E, mu as in gpo.c with these volumes;
 *                  rms slot 0 = sqrt(<r^2>) (or <rho^2>), slot 1 (axial) =
 *                  sqrt(<z^2>), rms_r = sqrt(<r^2>) (or <rho^2 + z^2>);
 *                  mean slot 0 = <r> (or <rho>), slot 1 (axial) = <z>.
 *
 * Layout: psi is complex<double> with x = the radial index fastest; the
 * circular and spherical forms use a grid (N, 1, 1), the axial form
 * (N_rho, N_z, 1) with z along the second axis.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define GPO_IMAG 0
#define GPO_REAL 1
#define GPO_OK 0
#define GPO_ERR_INVALID 1
#define GPO_ERR_NOMEM 2
#define GPO_ERR_NONFINITE 4

enum { GEOM_CIRCULAR = 1, GEOM_SPHERICAL = 2, GEOM_AXIAL = 3 };

enum {
    OBS_NORM = 0, OBS_MU, OBS_ENERGY,
    OBS_RMS_X, OBS_RMS_Y, OBS_RMS_Z, OBS_RMS_R,
    OBS_MEAN_X, OBS_MEAN_Y, OBS_MEAN_Z,
    OBS_KIN, OBS_POT, OBS_INT,
    OBS_COUNT
};

static const double PI = 3.14159265358979323846;

static int dim_of(int geom) { return geom == GEOM_SPHERICAL ? 3 : 2; }

static double solid_angle(int geom) { return geom == GEOM_SPHERICAL ? 4.0 * PI : 2.0 * PI; }

static int valid(int geom, const int64_t n[3], const double dx[3], double dt,
                 const double omega[3], double g, int mode)
{
    if (geom != GEOM_CIRCULAR && geom != GEOM_SPHERICAL && geom != GEOM_AXIAL) return 0;
    if (!n || !dx || !omega) return 0;
    if (n[0] < 1 || n[1] < 1 || n[2] != 1) return 0;
    if (geom != GEOM_AXIAL && n[1] != 1) return 0;
    for (int a = 0; a < 2; ++a)
        if (!(dx[a] > 0.0) || !isfinite(dx[a])) return 0;
    for (int a = 0; a < 3; ++a)
        if (!(omega[a] >= 0.0) || !isfinite(omega[a])) return 0;
    if (!(dt > 0.0) || !isfinite(dt) || !isfinite(g)) return 0;
    return mode == GPO_IMAG || mode == GPO_REAL;
}

/* r_i, s_{i+1/2} and v_i of the radial axis. */
static void radial_weights(int d, int64_t n, double h, double *r, double *s, double *v)
{
    for (int64_t i = 0; i < n; ++i) {
        r[i] = ((double)i + 0.5) * h;
        s[i] = pow((double)(i + 1) * h, d - 1);
        v[i] = (pow((double)(i + 1), d) - pow((double)i, d)) * pow(h, d - 1) / d;
    }
}

static double zcoord(int64_t n, double dz, int64_t k) { return ((double)k - 0.5 * (double)(n - 1)) * dz; }

/* General tridiagonal system lo_i x_{i-1} + di_i x_i + up_i x_{i+1} = r_i
 * (x_{-1} = x_n = 0) by the Thomas recursion, in place on r. */
static int thomas_general(int64_t n, const cplx *lo, const cplx *di, const cplx *up, cplx *r)
{
    cplx *cp = malloc(sizeof(cplx) * (size_t)n);
    if (!cp) return GPO_ERR_NOMEM;
    cplx den = di[0];
    cp[0] = up[0] / den;
    r[0] = r[0] / den;
    for (int64_t i = 1; i < n; ++i) {
        den = di[i] - lo[i] * cp[i - 1];
        cp[i] = up[i] / den;
        r[i] = (r[i] - lo[i] * r[i - 1]) / den;
    }
    for (int64_t i = n - 2; i >= 0; --i) r[i] -= cp[i] * r[i + 1];
    free(cp);
    return GPO_OK;
}

/* Coefficients of the radial Crank-Nicolson system, which depend on the grid
 * and the step only: with T = -1/2 L,
 *   T_ii = (s_{i-1/2} + s_{i+1/2}) / (2 h^2 v_i),
 *   T_{i,i-1} = -s_{i-1/2} / (2 h^2 v_i),  T_{i,i+1} = -s_{i+1/2} / (2 h^2 v_i),
 * the right side is (1 - tau/2 T) psi and the left matrix 1 + tau/2 T. */
typedef struct {
    cplx *tii, *tlo, *tup;   /* T by row */
} radial_op;

static int radial_op_make(int64_t nr, double h, const double *s, const double *v, radial_op *op)
{
    op->tii = malloc(sizeof(cplx) * (size_t)nr);
    op->tlo = malloc(sizeof(cplx) * (size_t)nr);
    op->tup = malloc(sizeof(cplx) * (size_t)nr);
    if (!op->tii || !op->tlo || !op->tup) return GPO_ERR_NOMEM;
    for (int64_t i = 0; i < nr; ++i) {
        const double sm = i > 0 ? s[i - 1] : 0.0, sp = s[i];
        const double c = 1.0 / (2.0 * h * h * v[i]);
        op->tii[i] = (sm + sp) * c;
        op->tlo[i] = -sm * c;
        op->tup[i] = -sp * c;
    }
    return GPO_OK;
}

static void radial_op_free(radial_op *op)
{
    free(op->tii);
    free(op->tlo);
    free(op->tup);
}

/* Crank-Nicolson along the radial axis of every z row. */
static int radial_sweep(const radial_op *op, const int64_t n[3], double dt, int mode, cplx *psi)
{
    const int64_t nr = n[0], rows = n[1];
    const cplx tau = mode == GPO_REAL ? I * dt : (cplx)dt;
    cplx *lo = malloc(sizeof(cplx) * (size_t)nr), *di = malloc(sizeof(cplx) * (size_t)nr),
         *up = malloc(sizeof(cplx) * (size_t)nr), *q = malloc(sizeof(cplx) * (size_t)nr);
    int st = (!lo || !di || !up || !q) ? GPO_ERR_NOMEM : GPO_OK;
    for (int64_t row = 0; row < rows && st == GPO_OK; ++row) {
        cplx *line = psi + row * nr;
        for (int64_t i = 0; i < nr; ++i) {
            const cplx left = i > 0 ? line[i - 1] : 0.0, right = i + 1 < nr ? line[i + 1] : 0.0;
            q[i] = (1.0 - 0.5 * tau * op->tii[i]) * line[i] - 0.5 * tau * (op->tlo[i] * left + op->tup[i] * right);
            lo[i] = 0.5 * tau * op->tlo[i];
            di[i] = 1.0 + 0.5 * tau * op->tii[i];
            up[i] = 0.5 * tau * op->tup[i];
        }
        st = thomas_general(nr, lo, di, up, q);
        if (st == GPO_OK) memcpy(line, q, sizeof(cplx) * (size_t)nr);
    }
    free(lo); free(di); free(up); free(q);
    return st;
}

/* Crank-Nicolson along z (axial): the constant 3-point form. */
static int z_sweep(const int64_t n[3], const double dx[3], double dt, int mode, cplx *psi)
{
    const int64_t nr = n[0], nz = n[1];
    const cplx tau = mode == GPO_REAL ? I * dt : (cplx)dt;
    const cplx kap = tau / (2.0 * dx[1] * dx[1]);
    cplx *lo = malloc(sizeof(cplx) * (size_t)nz), *di = malloc(sizeof(cplx) * (size_t)nz),
         *up = malloc(sizeof(cplx) * (size_t)nz), *q = malloc(sizeof(cplx) * (size_t)nz);
    int st = (!lo || !di || !up || !q) ? GPO_ERR_NOMEM : GPO_OK;
    for (int64_t i = 0; i < nr && st == GPO_OK; ++i) {
        for (int64_t k = 0; k < nz; ++k) {
            const cplx left = k > 0 ? psi[(k - 1) * nr + i] : 0.0;
            const cplx right = k + 1 < nz ? psi[(k + 1) * nr + i] : 0.0;
            q[k] = (1.0 - kap) * psi[k * nr + i] + 0.5 * kap * (left + right);
            lo[k] = up[k] = -0.5 * kap;
            di[k] = 1.0 + kap;
        }
        st = thomas_general(nz, lo, di, up, q);
        for (int64_t k = 0; k < nz && st == GPO_OK; ++k) psi[k * nr + i] = q[k];
    }
    free(lo); free(di); free(up); free(q);
    return st;
}

/* Volume of cell (i, k). */
static double cell(int geom, const double dx[3], const double *v, int64_t i)
{
    double w = solid_angle(geom) * dx[0] * v[i];
    return geom == GEOM_AXIAL ? w * dx[1] : w;
}

static double potential(int geom, const double omega[3], double r, double z)
{
    if (geom == GEOM_AXIAL) return 0.5 * (omega[0] * omega[0] * r * r + omega[2] * omega[2] * z * z);
    return 0.5 * omega[0] * omega[0] * r * r;
}

int gpo_radial_step(int geom, const int64_t n[3], const double dx[3], double dt, const double omega[3],
                    double g, int mode, double *psi_ri, int64_t nsteps)
{
    if (!valid(geom, n, dx, dt, omega, g, mode) || !psi_ri || nsteps < 0) return GPO_ERR_INVALID;
    cplx *psi = (cplx *)psi_ri;
    const int d = dim_of(geom);
    const int64_t nr = n[0], rows = n[1];
    double *r = malloc(sizeof(double) * (size_t)nr), *s = malloc(sizeof(double) * (size_t)nr),
           *v = malloc(sizeof(double) * (size_t)nr);
    if (!r || !s || !v) { free(r); free(s); free(v); return GPO_ERR_NOMEM; }
    radial_weights(d, nr, dx[0], r, s, v);
    radial_op op;
    int st = radial_op_make(nr, dx[0], s, v, &op);
    for (int64_t step = 0; step < nsteps && st == GPO_OK; ++step) {
        /* calcnu */
        for (int64_t k = 0; k < rows; ++k) {
            const double z = geom == GEOM_AXIAL ? zcoord(rows, dx[1], k) : 0.0;
            for (int64_t i = 0; i < nr; ++i) {
                cplx *p = psi + k * nr + i;
                const double dens = creal(*p) * creal(*p) + cimag(*p) * cimag(*p);
                const double theta = potential(geom, omega, r[i], z) + g * dens;
                if (mode == GPO_REAL)
                    *p *= cos(dt * theta) - I * sin(dt * theta);
                else
                    *p *= exp(-dt * theta);
            }
        }
        st = radial_sweep(&op, n, dt, mode, psi);
        if (st == GPO_OK && geom == GEOM_AXIAL) st = z_sweep(n, dx, dt, mode, psi);
        if (st == GPO_OK && mode == GPO_IMAG) {
            double norm = 0.0;
            for (int64_t k = 0; k < rows; ++k) {
                double row = 0.0;
                for (int64_t i = 0; i < nr; ++i) {
                    const cplx p = psi[k * nr + i];
                    row += cell(geom, dx, v, i) * (creal(p) * creal(p) + cimag(p) * cimag(p));
                }
                norm += row;
            }
            if (!(norm > 0.0) || !isfinite(norm)) {
                st = GPO_ERR_NONFINITE;
                break;
            }
            const double sc = 1.0 / sqrt(norm);
            for (int64_t p = 0; p < nr * rows; ++p) psi[p] *= sc;
        }
    }
    radial_op_free(&op);
    free(r); free(s); free(v);
    return st;
}

int gpo_radial_observables(int geom, const int64_t n[3], const double dx[3], const double omega[3], double g,
                           const double *psi_ri, double *out)
{
    if (!valid(geom, n, dx, 1.0, omega, g, GPO_IMAG) || !psi_ri || !out) return GPO_ERR_INVALID;
    const cplx *psi = (const cplx *)psi_ri;
    const int d = dim_of(geom);
    const int64_t nr = n[0], rows = n[1];
    double *r = malloc(sizeof(double) * (size_t)nr), *s = malloc(sizeof(double) * (size_t)nr),
           *v = malloc(sizeof(double) * (size_t)nr);
    if (!r || !s || !v) { free(r); free(s); free(v); return GPO_ERR_NOMEM; }
    radial_weights(d, nr, dx[0], r, s, v);
    double dens = 0.0, pot = 0.0, quart = 0.0, klink_r = 0.0, klink_z = 0.0;
    double m1r = 0.0, m2r = 0.0, m1z = 0.0, m2z = 0.0;
    const double zfac = geom == GEOM_AXIAL ? dx[1] : 1.0;
    for (int64_t k = 0; k < rows; ++k) {
        const double z = geom == GEOM_AXIAL ? zcoord(rows, dx[1], k) : 0.0;
        for (int64_t i = 0; i < nr; ++i) {
            const cplx p = psi[k * nr + i];
            const double w = creal(p) * creal(p) + cimag(p) * cimag(p);
            const double dv = cell(geom, dx, v, i);
            dens += dv * w;
            pot += dv * potential(geom, omega, r[i], z) * w;
            quart += dv * w * w;
            m1r += dv * r[i] * w;
            m2r += dv * r[i] * r[i] * w;
            m1z += dv * z * w;
            m2z += dv * z * z * w;
            /* radial link to i+1 (zero ghost beyond the last node) */
            const cplx nxt = i + 1 < nr ? psi[k * nr + i + 1] : 0.0;
            const cplx dr = nxt - p;
            klink_r += solid_angle(geom) / (2.0 * dx[0]) * zfac * s[i] *
                       (creal(dr) * creal(dr) + cimag(dr) * cimag(dr));
            if (geom == GEOM_AXIAL) {
                const cplx up = k + 1 < rows ? psi[(k + 1) * nr + i] : 0.0;
                const cplx dz = up - p;
                double links = creal(dz) * creal(dz) + cimag(dz) * cimag(dz);
                if (k == 0) links += w;   /* ghost link below the first node */
                klink_z += 0.5 * dv * links / (dx[1] * dx[1]);
            }
        }
    }
    free(r); free(s); free(v);
    for (int q = 0; q < OBS_COUNT; ++q) out[q] = 0.0;
    out[OBS_NORM] = dens;
    if (!(dens > 0.0) || !isfinite(dens)) return GPO_ERR_NONFINITE;
    const double kin = klink_r + klink_z;
    out[OBS_KIN] = kin / dens;
    out[OBS_POT] = pot / dens;
    out[OBS_INT] = g * quart / (dens * dens);
    out[OBS_ENERGY] = out[OBS_KIN] + out[OBS_POT] + 0.5 * out[OBS_INT];
    out[OBS_MU] = out[OBS_KIN] + out[OBS_POT] + out[OBS_INT];
    out[OBS_RMS_X] = sqrt(m2r / dens);
    out[OBS_MEAN_X] = m1r / dens;
    if (geom == GEOM_AXIAL) {
        out[OBS_RMS_Y] = sqrt(m2z / dens);
        out[OBS_MEAN_Y] = m1z / dens;
    }
    out[OBS_RMS_R] = sqrt((m2r + m2z) / dens);
    for (int q = 0; q < OBS_COUNT; ++q)
        if (!isfinite(out[q])) return GPO_ERR_NONFINITE;
    return GPO_OK;
}
