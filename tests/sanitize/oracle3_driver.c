/* Driver for the AddressSanitizer/UndefinedBehaviorSanitizer build of the
 * D3Q19 oracle (test infrastructure).  Every velocity kind and planted
 * mistake runs a few steps on small ragged and degenerate grids.  Exit
 * status 0 when every run returned 0 and every value is finite. */
#include <math.h>
#include <stdio.h>

#include "lbm_oracle3.c"

int main(void) {
    int failures = 0;
    const int dims[][3] = {{9, 7, 5}, {1, 1, 8}, {8, 1, 1}, {3, 5, 4}};
    for (int d = 0; d < 4; ++d)
        for (int vel = 0; vel <= 3; ++vel)
            for (int mut = 0; mut <= 4; ++mut) {
                orc3_params p;
                memset(&p, 0, sizeof p);
                p.nx = dims[d][0];
                p.ny = dims[d][1];
                p.nz = dims[d][2];
                p.eps = 1.0;
                p.tau = 0.8;
                p.delta = 1e-10;
                p.vel_kind = vel;
                p.U = 0.02;
                p.period_T = 30.0;
                p.ux = 0.02;
                p.uy = 0.01;
                p.uz = -0.01;
                p.mutation = mut;
                size_t n = (size_t)p.nx * p.ny * p.nz;
                double* phi0 = (double*)malloc(n * sizeof(double));
                double* out = (double*)malloc(n * sizeof(double));
                double mass[6];
                for (size_t k = 0; k < n; ++k) phi0[k] = 0.5 + 0.4 * sin(0.7 * (double)k);
                int rc = orc3_run(&p, phi0, 5, out, mass);
                int bad = rc != 0;
                for (size_t k = 0; k < n && !bad; ++k) bad = !isfinite(out[k]);
                if (bad) {
                    fprintf(stderr, "oracle3 run failed: vel %d mutation %d (%d x %d x %d)\n", vel, mut, p.nx, p.ny, p.nz);
                    ++failures;
                }
                free(phi0);
                free(out);
            }
    printf("oracle3_driver: %d failures\n", failures);
    return failures ? 1 : 0;
}
