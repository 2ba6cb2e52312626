/*
 * Plain FP64 CPU oracle of the 3-D form of the accurate interface-capturing
 * lattice Boltzmann scheme (H. Liang, arXiv:2203.05230): the update of
 * Sec. 2.2 (Eq. (9)-(13)) on a D3Q19 lattice, recovering Eq. (8) in three
 * dimensions.  The paper writes the scheme for D2Q9; every equation it uses
 * is dimension-free (sums over the lattice velocities, the isotropic
 * gradient, f_eq and F_i), so the 3-D form only changes the lattice.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it shares no code, header, table or constant generator
 * with the HIP path.
 *
 * Same readings as the 2-D oracle (interface width in the Jain convention,
 * clip of phi only inside psi, explicit Euler d_t(phi u) with zero at the
 * first step, equilibrium initialisation, cell-centred nodes) and the same
 * plain dataflow: separate phi, psi, gradient and flux arrays, collision, then
 * PUSH streaming into a second population array.  OpenMP splits the outer
 * z loop.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* D3Q19: rest; the 6 faces; the 12 edges.  w = 1/3, 1/18, 1/36; c_s^2 = 1/3. */
static const int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static const double W[19] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                             1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0;

enum { VEL3_ZERO = 0, VEL3_DEFORMATION = 1, VEL3_VORTEX_XY = 2, VEL3_UNIFORM = 3 };

enum {
    MUT3_NONE = 0,
    MUT3_EDGE_WEIGHT = 1,   /* edge weight 1/36 replaced by 1/18 in the collision */
    MUT3_GRAD_ZX = 2,       /* gradient components x and z exchanged */
    MUT3_STREAM_BACK = 3,   /* streaming to x - c_i instead of x + c_i */
    MUT3_DROP_GZ = 4        /* z component of the bracket of Eq. (11) dropped */
};

typedef struct {
    int32_t nx, ny, nz;
    double eps, tau, delta;
    int32_t vel_kind;
    double U, period_T;   /* amplitude and period (steps) of the deformation and vortex fields */
    double ux, uy, uz;    /* uniform velocity */
    int32_t mutation;     /* 0 in every real use; nonzero plants one known mistake (MUT3_*) */
} orc3_params;

void orc3_lattice(int* cx, int* cy, int* cz, double* w) {
    for (int i = 0; i < 19; ++i) {
        cx[i] = CX[i];
        cy[i] = CY[i];
        cz[i] = CZ[i];
        w[i] = W[i];
    }
}

/* Prescribed velocity at cell-centre coordinates X, Y, Z (lattice units) and
 * step t.  DEFORMATION is the classic three-dimensional deformation field
 * (divergence-free on a cube): u = 2U sin^2(pi x) sin(2 pi y) sin(2 pi z),
 * v = -U sin(2 pi x) sin^2(pi y) sin(2 pi z), w = -U sin(2 pi x) sin(2 pi y)
 * sin^2(pi z), all times cos(pi t / T), with x = X / nx etc.  VORTEX_XY is the
 * 2-D single vortex of the benchmark workloads in every z plane (w = 0). */
void orc3_velocity(const orc3_params* p, double X, double Y, double Z, double t, double* u, double* v, double* w) {
    const double PI = 3.14159265358979323846;
    const double x = X / p->nx, y = Y / p->ny, z = Z / p->nz;
    switch (p->vel_kind) {
    case VEL3_DEFORMATION: {
        const double tm = cos(PI * t / p->period_T);
        const double sx = sin(PI * x), sy = sin(PI * y), sz = sin(PI * z);
        *u = 2.0 * p->U * sx * sx * sin(2.0 * PI * y) * sin(2.0 * PI * z) * tm;
        *v = -p->U * sin(2.0 * PI * x) * sy * sy * sin(2.0 * PI * z) * tm;
        *w = -p->U * sin(2.0 * PI * x) * sin(2.0 * PI * y) * sz * sz * tm;
        break;
    }
    case VEL3_VORTEX_XY: {
        const double tm = cos(PI * t / p->period_T);
        const double sx = sin(PI * x), sy = sin(PI * y);
        *u = -p->U * sx * sx * sin(2.0 * PI * y) * tm;
        *v = p->U * sy * sy * sin(2.0 * PI * x) * tm;
        *w = 0.0;
        break;
    }
    case VEL3_UNIFORM:
        *u = p->ux;
        *v = p->uy;
        *w = p->uz;
        break;
    default:
        *u = *v = *w = 0.0;
    }
}

/* Eq. (10) */
void orc3_feq(double phi, double u, double v, double w, double* out) {
    for (int i = 0; i < 19; ++i) {
        const double cu = CX[i] * u + CY[i] * v + CZ[i] * w;
        out[i] = W[i] * phi * (1.0 + cu / CS2);
    }
}

/* Eq. (11): F_i = w_i c_i . G / c_s^2 */
void orc3_forcing(double gx, double gy, double gz, double* out) {
    for (int i = 0; i < 19; ++i) out[i] = W[i] * (CX[i] * gx + CY[i] * gy + CZ[i] * gz) / CS2;
}

static inline int wrap(int a, int n) {
    const int r = a % n;
    return r < 0 ? r + n : r;
}

/* Second-order isotropic gradient sum_i w_i c_i chi(x + c_i) / c_s^2, periodic. */
void orc3_gradient(const double* chi, int nx, int ny, int nz, double* gx, double* gy, double* gz) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double sx = 0.0, sy = 0.0, sz = 0.0;
                for (int q = 0; q < 19; ++q) {
                    const double c =
                        chi[((size_t)wrap(k + CZ[q], nz) * ny + wrap(j + CY[q], ny)) * nx + wrap(i + CX[q], nx)];
                    sx += W[q] * CX[q] * c;
                    sy += W[q] * CY[q] * c;
                    sz += W[q] * CZ[q] * c;
                }
                const size_t m = ((size_t)k * ny + j) * nx + i;
                gx[m] = sx / CS2;
                gy[m] = sy / CS2;
                gz[m] = sz / CS2;
            }
}

/* Full run: phi0 and phi_out are nz*ny*nx, x fastest.  mass (optional) gets
 * sum phi at t = 0..nsteps.  Returns 0, -1 for bad parameters, -2 without memory. */
int orc3_run(const orc3_params* p, const double* phi0, long nsteps, double* phi_out, double* mass) {
    if (p->nx < 1 || p->ny < 1 || p->nz < 1 || !(p->tau > 0.5) || !(p->eps > 0.0) || nsteps < 0) return -1;
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const size_t n = (size_t)nx * ny * nz;
    double* f = (double*)malloc(19 * n * sizeof(double));
    double* fn = (double*)malloc(19 * n * sizeof(double));
    double* phi = (double*)malloc(n * sizeof(double));
    double* psi = (double*)malloc(n * sizeof(double));
    double* gx = (double*)malloc(n * sizeof(double));
    double* gy = (double*)malloc(n * sizeof(double));
    double* gz = (double*)malloc(n * sizeof(double));
    double* pu = (double*)malloc(3 * n * sizeof(double));
    if (!f || !fn || !phi || !psi || !gx || !gy || !gz || !pu) {
        free(f); free(fn); free(phi); free(psi); free(gx); free(gy); free(gz); free(pu);
        return -2;
    }
    /* initial state: equilibrium populations, (phi u) at t = 0 */
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t m = ((size_t)k * ny + j) * nx + i;
                double u, v, w, fe[19];
                orc3_velocity(p, i + 0.5, j + 0.5, k + 0.5, 0.0, &u, &v, &w);
                orc3_feq(phi0[m], u, v, w, fe);
                for (int q = 0; q < 19; ++q) f[q * n + m] = fe[q];
                pu[3 * m] = phi0[m] * u;
                pu[3 * m + 1] = phi0[m] * v;
                pu[3 * m + 2] = phi0[m] * w;
            }

    const double tau = p->tau, kf = 1.0 - 0.5 / tau;
    const int sdir = p->mutation == MUT3_STREAM_BACK ? -1 : 1;
    for (long step = 0; step <= nsteps; ++step) {
        /* Eq. (12) */
#pragma omp parallel for schedule(static)
        for (size_t m = 0; m < n; ++m) {
            double s = 0.0;
            for (int q = 0; q < 19; ++q) s += f[q * n + m];
            phi[m] = s;
        }
        if (mass) {
            double s = 0.0;
            for (size_t m = 0; m < n; ++m) s += phi[m];
            mass[step] = s;
        }
        if (step == nsteps) break;

        /* Eq. (13) with the clip of phi described after it */
#pragma omp parallel for schedule(static)
        for (size_t m = 0; m < n; ++m) {
            const double pc = phi[m] < 0.0 ? 0.0 : (phi[m] > 1.0 ? 1.0 : phi[m]);
            psi[m] = p->eps * log((pc + p->delta) / (1.0 - pc + p->delta));
        }
        if (p->mutation == MUT3_GRAD_ZX)
            orc3_gradient(psi, nx, ny, nz, gz, gy, gx);
        else
            orc3_gradient(psi, nx, ny, nz, gx, gy, gz);

#pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    const size_t m = ((size_t)k * ny + j) * nx + i;
                    double u, v, w;
                    orc3_velocity(p, i + 0.5, j + 0.5, k + 0.5, (double)step, &u, &v, &w);
                    /* n = grad psi / (|grad psi| + delta), Eq. (13); S: the tanh form of
                     * Eq. (6) written in psi, (1 - tanh^2(psi / (2 eps))) / (4 eps) */
                    const double mag = sqrt(gx[m] * gx[m] + gy[m] * gy[m] + gz[m] * gz[m]);
                    const double th = tanh(psi[m] / (2.0 * p->eps));
                    const double S = (1.0 - th * th) / (4.0 * p->eps);
                    const double nxv = gx[m] / (mag + p->delta), nyv = gy[m] / (mag + p->delta),
                                 nzv = gz[m] / (mag + p->delta);
                    const double phu = phi[m] * u, phv = phi[m] * v, phw = phi[m] * w;
                    /* bracket of Eq. (11): d_t(phi u) by explicit Euler + c_s^2 S n */
                    const double Gx = (phu - pu[3 * m]) + CS2 * S * nxv;
                    const double Gy = (phv - pu[3 * m + 1]) + CS2 * S * nyv;
                    const double Gz = p->mutation == MUT3_DROP_GZ ? 0.0 : (phw - pu[3 * m + 2]) + CS2 * S * nzv;
                    double fe[19], F[19];
                    orc3_feq(phi[m], u, v, w, fe);
                    orc3_forcing(Gx, Gy, Gz, F);
                    if (p->mutation == MUT3_EDGE_WEIGHT)
                        for (int q = 7; q < 19; ++q) {
                            fe[q] *= 2.0;
                            F[q] *= 2.0;
                        }
                    for (int q = 0; q < 19; ++q) {
                        const double fi = f[q * n + m];
                        /* Eq. (9): collision, then push to x + c_q */
                        const double post = fi - (fi - fe[q]) / tau + kf * F[q];
                        const int ti = wrap(i + sdir * CX[q], nx), tj = wrap(j + sdir * CY[q], ny),
                                  tk = wrap(k + sdir * CZ[q], nz);
                        fn[q * n + ((size_t)tk * ny + tj) * nx + ti] = post;
                    }
                    pu[3 * m] = phu;
                    pu[3 * m + 1] = phv;
                    pu[3 * m + 2] = phw;
                }
        double* t = f;
        f = fn;
        fn = t;
    }
    if (phi_out) memcpy(phi_out, phi, n * sizeof(double));
    free(f); free(fn); free(phi); free(psi); free(gx); free(gy); free(gz); free(pu);
    return 0;
}
