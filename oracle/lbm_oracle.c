/*
 * Plain FP64 CPU oracle for the accurate interface-capturing lattice
 * Boltzmann scheme (H. Liang, "An accurate lattice Boltzmann method for
 * interface capturing", arXiv:2203.05230): D2Q9 BGK with a forcing term that
 * recovers the improved conservative Allen-Cahn equation (Sec. 2.1, Eq. (8)).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the HIP library against a slow,
 * obviously correct implementation.  It shares no code, header, table or
 * constant generator with the HIP path.
 *
 * Dataflow is deliberately the plainest one: separate arrays for phi, psi,
 * grad psi and the forcing, collision into a temporary, then PUSH streaming
 * into a second population array, one time step at a time.  OpenMP only
 * splits the outer row loop.
 *
 * Readings of the paper used here (all selectable so tests can compare them):
 *  - interface-width convention (reading "Jain", default): psi = eps ln(..)
 *    as in Eq. (13) and the sharpening magnitude (1/(4 eps)) (1 - tanh^2(psi/(2 eps))),
 *    which is the tanh form of Eq. (6) rewritten so that it is consistent
 *    with the psi of Eq. (13); "literal" keeps Eq. (6)/(11) as printed with
 *    the psi of Eq. (13); "liang" uses psi = (eps/4) ln(..) so that Eq. (2)-(6)
 *    are consistent with the printed tanh(2 psi / eps).
 *  - clip of phi to [0,1] only inside psi (end of Sec. 2.2).
 *  - gradient: the second-order isotropic lattice stencil
 *    grad chi = sum_i w_i c_i chi(x + c_i) / c_s^2 (Sec. 2.2, text after Eq. (12)).
 *  - d_t(phi u) by explicit Euler with (phi u) at the previous step; at the
 *    first step the previous value is phi0 u(x, 0).
 *  - populations initialised at equilibrium f_eq(phi0, u(x, 0)).
 *  - node (i, j) sits at the cell centre X = i + 1/2, Y = j + 1/2.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

/* D2Q9 lattice, Sec. 2.2 after Eq. (10): w_0 = 4/9, w_1..4 = 1/9,
 * w_5..8 = 1/36, c_s^2 = 1/3.  Velocity order: rest, E, N, W, S, NE, NW, SW, SE. */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0;

enum { VEL_ZERO = 0, VEL_VORTEX = 1, VEL_ROTATION = 2, VEL_UNIFORM = 3, VEL_VORTEX_PAPER = 4 };
enum { READ_JAIN = 0, READ_LITERAL = 1, READ_LIANG = 2 };
enum { MODEL_IMPROVED = 0, MODEL_CONVENTIONAL = 1 };

#define MLP_IN 25
#define MLP_H 64
#define MLP_OUT 2
#define MLP_NPARAM (MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_OUT * MLP_H + MLP_OUT)

typedef struct {
    int32_t nx, ny;
    double eps, tau, delta;
    int32_t vel_kind;
    double U, period_T;   /* single vortex amplitude and period (steps) */
    double omega, cx, cy; /* solid-body rotation rate and centre (lattice units) */
    double ux, uy;        /* uniform velocity */
    int32_t reading;
    int32_t model;
    const double* mlp; /* NULL: no learned closure; else MLP_NPARAM weights */
    double theta;      /* closure band: applied where theta < phi_clip < 1 - theta */
    int32_t mutation;  /* 0 in every real use; nonzero plants one known mistake
                          (MUT_*) so tests can show that the pins catch it */
    double noise;      /* 0 in every real use; > 0 perturbs the post-collision
                          populations (noise_kind) by relative errors noise xi,
                          xi uniform in [-1, 1), to measure how the iteration
                          amplifies rounding-sized errors */
    uint64_t noise_seed;
    int32_t noise_kind;  /* NOISE_POPULATIONS: every f*_i times (1 + noise xi).
                            NOISE_SHIFTED: the shifted populations g_i = f*_i - w_i phi*
                            (i >= 1, phi* = sum_i f*_i at the node) times (1 + noise xi)
                            and f*_0 the remainder, so the node's sum is kept: the
                            error pattern of storing g_i in a format of unit
                            roundoff `noise` */
    int32_t noise_every; /* perturb after the steps s with (s + 1) % noise_every == 0
                            and after the last step (<= 1: after every step) */
} orc_params;

enum { NOISE_POPULATIONS = 0, NOISE_SHIFTED = 1 };

/* splitmix64 (Steele, Lea, Flood 2014): counter-based stream for the noise option */
static uint64_t splitmix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static double unit_noise(uint64_t seed, uint64_t counter) {
    return (double)(splitmix64(seed ^ splitmix64(counter)) >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

enum {
    MUT_NONE = 0,
    MUT_DROP_DT_PHIU = 1,   /* d_t(phi u) left out of Eq. (11) */
    MUT_NO_FORCE_FACTOR = 2, /* (1 - 1/(2 tau)) of Eq. (9) replaced by 1 */
    MUT_FLUX_SIGN = 3,       /* sharpening flux with the wrong sign */
    MUT_GRAD_SWAP = 4,       /* gradient components transposed */
    MUT_STREAM_BACK = 5,     /* streaming to x - c_i instead of x + c_i */
    MUT_NO_CLIP = 6,         /* psi from the unclipped phi (|.| inside the log) */
    MUT_VEL_SWAP = 7,        /* u and v exchanged */
    MUT_FEQ_NO_U = 8,        /* velocity term dropped from Eq. (10) */
    MUT_DIAG_WEIGHT = 9,     /* diagonal weight 1/36 replaced by 1/18 in the collision */
    MUT_CONV_WIDTH4 = 10,    /* conventional model: 4 phi (1 - phi) / eps, the paper's width, under the Jain width */
    MUT_CONV_NORMAL_PSI = 11, /* conventional model: normal taken from grad psi instead of grad phi */
    MUT_CLOSURE_NO_CS2 = 12, /* closure correction added to the bracket of Eq. (11) without the c_s^2 factor */
    MUT_CLOSURE_STENCIL_T = 13 /* closure input neighbourhood transposed (dx outer, dy inner) */
};

int orc_nparam(void) { return MLP_NPARAM; }

void orc_lattice(int* cx, int* cy, double* w) {
    for (int i = 0; i < 9; ++i) {
        cx[i] = CX[i];
        cy[i] = CY[i];
        w[i] = W[i];
    }
}

/* Prescribed velocity.  X, Y are cell-centre coordinates in lattice units on
 * an nx-by-ny periodic grid; t is the step count.
 * VORTEX_PAPER is Eq. (14) as printed; VORTEX is the same field with the
 * opposite rotation sense (u negative, v positive in the first quadrant). */
void orc_velocity(const orc_params* p, double X, double Y, double t, double* u, double* v) {
    const double PI = 3.14159265358979323846;
    double x = X / p->nx, y = Y / p->ny;
    switch (p->vel_kind) {
    case VEL_VORTEX:
    case VEL_VORTEX_PAPER: {
        double sx = sin(PI * x), sy = sin(PI * y);
        double tm = cos(PI * t / p->period_T);
        double a = p->U * sx * sx * sin(2.0 * PI * y) * tm;
        double b = p->U * sy * sy * sin(2.0 * PI * x) * tm;
        if (p->vel_kind == VEL_VORTEX) {
            *u = -a;
            *v = b;
        } else {
            *u = a;
            *v = -b;
        }
        break;
    }
    case VEL_ROTATION:
        *u = -p->omega * (Y - p->cy);
        *v = p->omega * (X - p->cx);
        break;
    case VEL_UNIFORM:
        *u = p->ux;
        *v = p->uy;
        break;
    default:
        *u = 0.0;
        *v = 0.0;
    }
}

/* Eq. (13) with the clip of phi to [0,1] described after it. */
double orc_psi(double phi, double eps, double delta, int reading) {
    double pc = phi < 0.0 ? 0.0 : (phi > 1.0 ? 1.0 : phi);
    double r = log((pc + delta) / (1.0 - pc + delta));
    if (reading == READ_LIANG) return 0.25 * eps * r;
    return eps * r;
}

/* Sharpening magnitude, the bracket of Eq. (6) written in psi (see the
 * reading notes at the top of this file). */
double orc_sharpen(double psi, double eps, int reading) {
    if (reading == READ_JAIN) {
        double th = tanh(psi / (2.0 * eps));
        return (1.0 - th * th) / (4.0 * eps);
    }
    double th = tanh(2.0 * psi / eps);
    return (1.0 - th * th) / eps;
}

/* Sharpening magnitude of the conventional conservative ACE, Eq. (1):
 * 4 phi (1 - phi) / eps in the paper's width; in the Jain width this is
 * phi (1 - phi) / eps. */
double orc_sharpen_conventional(double phi, double eps, int reading) {
    if (reading == READ_JAIN) return phi * (1.0 - phi) / eps;
    return 4.0 * phi * (1.0 - phi) / eps;
}

/* Eq. (10). */
void orc_feq(double phi, double u, double v, double* out) {
    for (int i = 0; i < 9; ++i) {
        double cu = CX[i] * u + CY[i] * v;
        out[i] = W[i] * phi * (1.0 + cu / CS2);
    }
}

/* Eq. (11): F_i = w_i c_i . G / c_s^2, where G is the bracket of Eq. (11). */
void orc_forcing(double gx, double gy, double* out) {
    for (int i = 0; i < 9; ++i) out[i] = W[i] * (CX[i] * gx + CY[i] * gy) / CS2;
}

static inline int wrap(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

/* Second-order isotropic gradient on a periodic grid. */
void orc_gradient(const double* chi, int nx, int ny, double* gx, double* gy) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            double sx = 0.0, sy = 0.0;
            for (int k = 0; k < 9; ++k) {
                double c = chi[(size_t)wrap(j + CY[k], ny) * nx + wrap(i + CX[k], nx)];
                sx += W[k] * CX[k] * c;
                sy += W[k] * CY[k] * c;
            }
            gx[(size_t)j * nx + i] = sx / CS2;
            gy[(size_t)j * nx + i] = sy / CS2;
        }
    }
}

static double gelu(double x) {
    const double k = 0.79788456080286535588; /* sqrt(2/pi) */
    return 0.5 * x * (1.0 + tanh(k * (x + 0.044715 * x * x * x)));
}

/* Learned closure: 25 -> 64 -> 64 -> 2 MLP with tanh-GELU.  Weight layout:
 * W1[64][25], b1[64], W2[64][64], b2[64], W3[2][64], b3[2]. */
void orc_mlp(const double* w, const double* in, double* out) {
    const double* W1 = w;
    const double* b1 = W1 + MLP_H * MLP_IN;
    const double* W2 = b1 + MLP_H;
    const double* b2 = W2 + MLP_H * MLP_H;
    const double* W3 = b2 + MLP_H;
    const double* b3 = W3 + MLP_OUT * MLP_H;
    double h1[MLP_H], h2[MLP_H];
    for (int o = 0; o < MLP_H; ++o) {
        double s = b1[o];
        for (int k = 0; k < MLP_IN; ++k) s += W1[o * MLP_IN + k] * in[k];
        h1[o] = gelu(s);
    }
    for (int o = 0; o < MLP_H; ++o) {
        double s = b2[o];
        for (int k = 0; k < MLP_H; ++k) s += W2[o * MLP_H + k] * h1[k];
        h2[o] = gelu(s);
    }
    for (int o = 0; o < MLP_OUT; ++o) {
        double s = b3[o];
        for (int k = 0; k < MLP_H; ++k) s += W3[o * MLP_H + k] * h2[k];
        out[o] = s;
    }
}

/* Sharpening flux S n at every node of a periodic phi field (Eq. (6), (7),
 * (13) for the improved model, Eq. (1) for the conventional one). */
void orc_flux(const orc_params* p, const double* phi, int nx, int ny, double* fx, double* fy) {
    size_t n = (size_t)nx * ny;
    double* src = (double*)calloc(n ? n : 1, sizeof(double));
    double* gx = (double*)malloc(n * sizeof(double));
    double* gy = (double*)malloc(n * sizeof(double));
    if (!src || !gx || !gy) {
        free(src);
        free(gx);
        free(gy);
        for (size_t k = 0; k < n; ++k) fx[k] = fy[k] = NAN;
        return;
    }
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < n; ++k) {
        if (p->model == MODEL_CONVENTIONAL && p->mutation != MUT_CONV_NORMAL_PSI)
            src[k] = phi[k];
        else if (p->mutation == MUT_NO_CLIP)
            src[k] = p->eps * log((phi[k] + p->delta) / (1.0 - phi[k] + p->delta));
        else
            src[k] = orc_psi(phi[k], p->eps, p->delta, p->reading);
    }
    orc_gradient(src, nx, ny, gx, gy);
    if (p->mutation == MUT_GRAD_SWAP) {
        double* t = gx;
        gx = gy;
        gy = t;
    }
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < n; ++k) {
        double mag = sqrt(gx[k] * gx[k] + gy[k] * gy[k]);
        double nxv = gx[k] / (mag + p->delta), nyv = gy[k] / (mag + p->delta);
        double S = p->model == MODEL_CONVENTIONAL ? orc_sharpen_conventional(phi[k], p->eps, p->reading)
                                                  : orc_sharpen(src[k], p->eps, p->reading);
        if (p->model == MODEL_CONVENTIONAL && p->mutation == MUT_CONV_WIDTH4) S *= 4.0;
        fx[k] = S * nxv;
        fy[k] = S * nyv;
    }
    free(src);
    free(gx);
    free(gy);
}

/* Learned-closure correction on a periodic phi field: input is the 5x5
 * neighbourhood of phi (row-major, dy = -2..2 outer, dx = -2..2 inner); the
 * correction is zero outside the interface band. */
void orc_closure_field(const orc_params* p, const double* phi, int nx, int ny, double* cxo, double* cyo) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            size_t k = (size_t)j * nx + i;
            double pc = phi[k] < 0.0 ? 0.0 : (phi[k] > 1.0 ? 1.0 : phi[k]);
            cxo[k] = 0.0;
            cyo[k] = 0.0;
            if (!p->mlp || !(pc > p->theta && pc < 1.0 - p->theta)) continue;
            double in[MLP_IN], out[MLP_OUT];
            int m = 0;
            for (int dy = -2; dy <= 2; ++dy)
                for (int dx = -2; dx <= 2; ++dx) {
                    if (p->mutation == MUT_CLOSURE_STENCIL_T)
                        in[m++] = phi[(size_t)wrap(j + dx, ny) * nx + wrap(i + dy, nx)];
                    else
                        in[m++] = phi[(size_t)wrap(j + dy, ny) * nx + wrap(i + dx, nx)];
                }
            orc_mlp(p->mlp, in, out);
            cxo[k] = out[0];
            cyo[k] = out[1];
        }
    }
}

/* The iteration on an lnx-by-lny periodic patch whose node (i, j) is global
 * node ((ox + i) mod p->nx, (oy + j) mod p->ny) for the velocity field.
 * With ox = oy = 0 and the patch equal to the grid this is the plain run. */
static int run_core(const orc_params* p, int ox, int oy, int lnx, int lny, const double* phi0, long nsteps,
                    double* phi_out, double* mass) {
    size_t n = (size_t)lnx * lny;
    double* f = (double*)malloc(9 * n * sizeof(double));
    double* fn = (double*)malloc(9 * n * sizeof(double));
    double* phi = (double*)malloc(n * sizeof(double));
    double* fxs = (double*)malloc(n * sizeof(double));
    double* fys = (double*)malloc(n * sizeof(double));
    double* ccx = (double*)malloc(n * sizeof(double));
    double* ccy = (double*)malloc(n * sizeof(double));
    double* pux = (double*)malloc(n * sizeof(double));
    double* puy = (double*)malloc(n * sizeof(double));
    double* Xg = (double*)malloc(lnx * sizeof(double));
    double* Yg = (double*)malloc(lny * sizeof(double));
    if (!f || !fn || !phi || !fxs || !fys || !ccx || !ccy || !pux || !puy || !Xg || !Yg) {
        free(f); free(fn); free(phi); free(fxs); free(fys); free(ccx); free(ccy);
        free(pux); free(puy); free(Xg); free(Yg);
        return -2;
    }
    for (int i = 0; i < lnx; ++i) Xg[i] = wrap(ox + i, p->nx) + 0.5;
    for (int j = 0; j < lny; ++j) Yg[j] = wrap(oy + j, p->ny) + 0.5;

    /* initial state: equilibrium populations, (phi u) at t = 0 */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < lny; ++j)
        for (int i = 0; i < lnx; ++i) {
            size_t k = (size_t)j * lnx + i;
            double u, v, fe[9];
            orc_velocity(p, Xg[i], Yg[j], 0.0, &u, &v);
            orc_feq(phi0[k], u, v, fe);
            for (int q = 0; q < 9; ++q) f[q * n + k] = fe[q];
            pux[k] = phi0[k] * u;
            puy[k] = phi0[k] * v;
        }

    for (long step = 0; step <= nsteps; ++step) {
        /* Eq. (12) */
#pragma omp parallel for schedule(static)
        for (size_t k = 0; k < n; ++k) {
            double s = 0.0;
            for (int q = 0; q < 9; ++q) s += f[q * n + k];
            phi[k] = s;
        }
        if (mass) {
            double m = 0.0;
            for (size_t k = 0; k < n; ++k) m += phi[k];
            mass[step] = m;
        }
        if (step == nsteps) break;

        /* Eq. (13), (7), (6): sharpening flux S n */
        orc_flux(p, phi, lnx, lny, fxs, fys);
        /* learned closure (zero without weights) */
        orc_closure_field(p, phi, lnx, lny, ccx, ccy);

        const double tau = p->tau;
        const double kf = p->mutation == MUT_NO_FORCE_FACTOR ? 1.0 : 1.0 - 0.5 / tau;
        const double sgn = p->mutation == MUT_FLUX_SIGN ? -1.0 : 1.0;
        const double dtw = p->mutation == MUT_DROP_DT_PHIU ? 0.0 : 1.0;
        const int sdir = p->mutation == MUT_STREAM_BACK ? -1 : 1;
#pragma omp parallel for schedule(static)
        for (int j = 0; j < lny; ++j) {
            for (int i = 0; i < lnx; ++i) {
                size_t k = (size_t)j * lnx + i;
                double u, v;
                orc_velocity(p, Xg[i], Yg[j], (double)step, &u, &v);
                if (p->mutation == MUT_VEL_SWAP) {
                    double t = u;
                    u = v;
                    v = t;
                }
                double phu = phi[k] * u, phv = phi[k] * v;
                /* bracket of Eq. (11): d_t(phi u) (explicit Euler) + c_s^2 (S n + c) */
                double gx = dtw * (phu - pux[k]) + CS2 * (sgn * fxs[k] + ccx[k]);
                double gy = dtw * (phv - puy[k]) + CS2 * (sgn * fys[k] + ccy[k]);
                if (p->mutation == MUT_CLOSURE_NO_CS2) {
                    gx += (1.0 - CS2) * ccx[k];
                    gy += (1.0 - CS2) * ccy[k];
                }
                double fe[9], F[9], post[9];
                orc_feq(phi[k], p->mutation == MUT_FEQ_NO_U ? 0.0 : u, p->mutation == MUT_FEQ_NO_U ? 0.0 : v, fe);
                orc_forcing(gx, gy, F);
                if (p->mutation == MUT_DIAG_WEIGHT)
                    for (int q = 5; q < 9; ++q) {
                        fe[q] *= 2.0;
                        F[q] *= 2.0;
                    }
                /* Eq. (9): collision */
                for (int q = 0; q < 9; ++q) {
                    double fi = f[q * n + k];
                    post[q] = fi - (fi - fe[q]) / tau + kf * F[q];
                }
                if (p->noise > 0.0 && (p->noise_every <= 1 || (step + 1) % p->noise_every == 0 || step + 1 == nsteps)) {
                    uint64_t ctr = ((uint64_t)step * n + k) * 9u;
                    if (p->noise_kind == NOISE_SHIFTED) {
                        double ps = 0.0, moving = 0.0;
                        for (int q = 0; q < 9; ++q) ps += post[q];
                        for (int q = 1; q < 9; ++q) {
                            double g = post[q] - W[q] * ps;
                            post[q] = W[q] * ps + g * (1.0 + p->noise * unit_noise(p->noise_seed, ctr + (uint64_t)q));
                            moving += post[q];
                        }
                        post[0] = ps - moving;
                    } else {
                        for (int q = 0; q < 9; ++q)
                            post[q] *= 1.0 + p->noise * unit_noise(p->noise_seed, ctr + (uint64_t)q);
                    }
                }
                /* Eq. (9): push to x + c_q */
                for (int q = 0; q < 9; ++q) {
                    int ti = wrap(i + sdir * CX[q], lnx), tj = wrap(j + sdir * CY[q], lny);
                    fn[q * n + (size_t)tj * lnx + ti] = post[q];
                }
                pux[k] = phu;
                puy[k] = phv;
            }
        }
        double* tmp = f;
        f = fn;
        fn = tmp;
    }
    if (phi_out) memcpy(phi_out, phi, n * sizeof(double));
    free(f); free(fn); free(phi); free(fxs); free(fys); free(ccx); free(ccy);
    free(pux); free(puy); free(Xg); free(Yg);
    return 0;
}

/* Full run: phi0 and phi_out are ny*nx, x fastest.  mass (optional) gets
 * sum phi at t = 0..nsteps (nsteps + 1 values). */
int orc_run(const orc_params* p, const double* phi0, long nsteps, double* phi_out, double* mass) {
    if (p->nx < 1 || p->ny < 1 || !(p->tau > 0.5) || !(p->eps > 0.0) || nsteps < 0) return -1;
    return run_core(p, 0, 0, p->nx, p->ny, phi0, nsteps, phi_out, mass);
}

/* phi after nsteps on the wy-by-wx window with lower-left node (x0, y0) of
 * the full periodic run, computed on a padded patch only.  Each step reads
 * at most 2 nodes away (3 with the closure stencil), so a pad of that many
 * nodes per step leaves the window exact.  phi0 is the whole grid. */
int orc_run_window(const orc_params* p, const double* phi0, int x0, int y0, int wx, int wy, long nsteps,
                   double* phi_out) {
    if (p->nx < 1 || p->ny < 1 || !(p->tau > 0.5) || !(p->eps > 0.0) || nsteps < 0 || wx < 1 || wy < 1) return -1;
    long reach = p->mlp ? 3 : 2;
    long pad = reach * nsteps + 1;
    long lnx = wx + 2 * pad, lny = wy + 2 * pad;
    if (lnx > 1L << 20 || lny > 1L << 20) return -1;
    size_t n = (size_t)lnx * lny;
    double* loc0 = (double*)malloc(n * sizeof(double));
    double* locT = (double*)malloc(n * sizeof(double));
    if (!loc0 || !locT) {
        free(loc0);
        free(locT);
        return -2;
    }
    int ox = (int)(x0 - pad), oy = (int)(y0 - pad);
    for (long j = 0; j < lny; ++j)
        for (long i = 0; i < lnx; ++i)
            loc0[(size_t)j * lnx + i] = phi0[(size_t)wrap((int)(oy + j), p->ny) * p->nx + wrap((int)(ox + i), p->nx)];
    int rc = run_core(p, ox, oy, (int)lnx, (int)lny, loc0, nsteps, locT, NULL);
    if (rc == 0)
        for (int j = 0; j < wy; ++j)
            for (int i = 0; i < wx; ++i)
                phi_out[(size_t)j * wx + i] = locT[(size_t)(j + pad) * lnx + (i + pad)];
    free(loc0);
    free(locT);
    return rc;
}
