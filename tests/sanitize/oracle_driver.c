/* Driver for the AddressSanitizer/UndefinedBehaviorSanitizer build of the
 * D2Q9 oracle (test infrastructure checking test infrastructure).  The oracle
 * source is compiled into this translation unit; every reading, both
 * models, every velocity kind, the closure hook, every planted mistake and
 * the padded-window mode run a few steps on small ragged grids, including
 * the degenerate 1 x n and n x 1 ones.  Exit status 0 when every run
 * returned 0 and every value of the unplanted runs is finite. */
#include <math.h>
#include <stdio.h>

#include "lbm_oracle.c"

static int failures = 0;

static void check_run(const orc_params* p, const char* what, int need_finite) {
    size_t n = (size_t)p->nx * p->ny;
    double* phi0 = (double*)malloc(n * sizeof(double));
    double* out = (double*)malloc(n * sizeof(double));
    double* mass = (double*)malloc(8 * sizeof(double));
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            double dx = i + 0.5 - 0.5 * p->nx, dy = j + 0.5 - 0.6 * p->ny;
            double r = sqrt(dx * dx + dy * dy);
            phi0[(size_t)j * p->nx + i] = 0.5 * (1.0 + tanh((0.3 * (p->nx < p->ny ? p->nx : p->ny) - r) / (2.0 * p->eps)));
        }
    int rc = orc_run(p, phi0, 7, out, mass);
    int bad = rc != 0;
    for (size_t k = 0; k < n && !bad && need_finite; ++k) bad = !isfinite(out[k]);
    for (int k = 0; k < 8 && !bad && need_finite; ++k) bad = !isfinite(mass[k]);
    if (!bad && p->nx >= 6 && p->ny >= 6) {
        double win[12];
        rc = orc_run_window(p, phi0, p->nx - 2, 1, 4, 3, 2, win);
        bad = rc != 0;
        for (int k = 0; k < 12 && !bad && need_finite; ++k) bad = !isfinite(win[k]);
    }
    if (bad) {
        fprintf(stderr, "oracle run failed: %s, mutation %d (%d x %d)\n", what, p->mutation, p->nx, p->ny);
        ++failures;
    }
    free(phi0);
    free(out);
    free(mass);
}

int main(void) {
    double* w = (double*)malloc(MLP_NPARAM * sizeof(double));
    uint64_t s = 99;
    for (int k = 0; k < MLP_NPARAM; ++k) w[k] = 0.2 * unit_noise(s, (uint64_t)k);
    const int dims[][2] = {{24, 17}, {1, 12}, {12, 1}, {3, 5}, {33, 40}};
    for (int d = 0; d < 5; ++d)
        for (int vel = VEL_ZERO; vel <= VEL_VORTEX_PAPER; ++vel)
            for (int reading = READ_JAIN; reading <= READ_LIANG; ++reading)
                for (int model = MODEL_IMPROVED; model <= MODEL_CONVENTIONAL; ++model)
                    for (int closure = 0; closure <= 1; ++closure) {
                        orc_params p;
                        memset(&p, 0, sizeof p);
                        p.nx = dims[d][0];
                        p.ny = dims[d][1];
                        p.eps = 1.0;
                        p.tau = 0.8;
                        p.delta = 1e-10;
                        p.vel_kind = vel;
                        p.U = 0.02;
                        p.period_T = 50.0;
                        p.omega = 0.002;
                        p.cx = 0.5 * p.nx;
                        p.cy = 0.5 * p.ny;
                        p.ux = 0.03;
                        p.uy = -0.02;
                        p.reading = reading;
                        p.model = model;
                        p.mlp = closure ? w : NULL;
                        p.theta = 0.02;
                        check_run(&p, "switches", 1);
                    }
    for (int mut = 1; mut <= MUT_CLOSURE_STENCIL_T; ++mut) {
        orc_params p;
        memset(&p, 0, sizeof p);
        p.nx = 20;
        p.ny = 14;
        p.eps = 0.5;
        p.tau = 0.7;
        p.delta = 1e-10;
        p.vel_kind = VEL_VORTEX;
        p.U = 0.02;
        p.period_T = 40.0;
        p.model = (mut == MUT_CONV_WIDTH4 || mut == MUT_CONV_NORMAL_PSI) ? MODEL_CONVENTIONAL : MODEL_IMPROVED;
        p.mlp = (mut >= MUT_CLOSURE_NO_CS2) ? w : NULL;
        p.theta = 0.02;
        p.mutation = mut;
        p.noise = mut == 1 ? 1e-7 : 0.0;
        p.noise_seed = 5;
        /* a planted mistake may drive the field out of range (the unclipped
         * logarithm does): only the sanitizers and the return code judge it */
        check_run(&p, "planted mistake", 0);
    }
    free(w);
    printf("oracle_driver: %d failures\n", failures);
    return failures ? 1 : 0;
}
