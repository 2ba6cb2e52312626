/* Host-side driver for the AddressSanitizer/UndefinedBehaviorSanitizer build
 * of the library (host code only; no GPU is touched).  It walks the
 * parameter-validation paths of every entry point, the status strings and
 * the batched form's host-only schedule check, which builds the items,
 * neighbour lists and slot tables with the library's own host code.  Exit
 * status 0 when every call returned what the header promises; a sanitizer
 * report aborts the process with a nonzero status. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbac.h"
#include "lbac3.h"

static int failures = 0;

#define EXPECT(cond)                                                           \
    do {                                                                       \
        if (!(cond)) {                                                         \
            fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                        \
        }                                                                      \
    } while (0)

static int init_with(const lbac_params* p, const double* phi0) {
    lbac_ctx* h = NULL;
    int rc = lbac_init(p, phi0, &h);
    if (rc == LBAC_OK) lbac_free(h);
    return rc;
}

static void validation_2d(void) {
    double* phi0 = (double*)malloc(16 * 16 * sizeof(double));
    for (int k = 0; k < 256; ++k) phi0[k] = 0.5;
    lbac_params p;
    lbac_default_params(&p, 16, 16);

    lbac_params q = p;
    q.tau = 0.5;
    EXPECT(init_with(&q, phi0) == LBAC_EINVAL);
    q = p;
    q.tau = NAN;
    EXPECT(init_with(&q, phi0) == LBAC_EINVAL);
    q = p;
    q.eps = 0.0;
    EXPECT(init_with(&q, phi0) == LBAC_EINVAL);
    q = p;
    q.delta = -1e-3;
    EXPECT(init_with(&q, phi0) == LBAC_EINVAL);
    q = p;
    q.precision = 7;
    EXPECT(init_with(&q, phi0) == LBAC_EINVAL);
    q = p;
    q.model = 5;
    EXPECT(init_with(&q, phi0) == LBAC_EINVAL);
    q = p;
    q.vel_kind = LBAC_VEL_UNIFORM;
    q.ux = 0.3;
    q.uy = 0.1;
    EXPECT(init_with(&q, phi0) == LBAC_EINVAL);
    q = p;
    q.vel_kind = LBAC_VEL_VORTEX;
    q.period_T = 0.0;
    EXPECT(init_with(&q, phi0) == LBAC_EINVAL);

    const int sizes[][2] = {{0, 16}, {16, 0}, {-3, 4}, {70000, 4}, {65536, 4096}};
    for (int s = 0; s < 5; ++s) {
        q = p;
        q.nx = sizes[s][0];
        q.ny = sizes[s][1];
        EXPECT(init_with(&q, phi0) == LBAC_EINVAL);
    }
    phi0[37] = NAN;
    EXPECT(init_with(&p, phi0) == LBAC_EINVAL);
    phi0[37] = INFINITY;
    EXPECT(init_with(&p, phi0) == LBAC_EINVAL);
    phi0[37] = 0.5;

    lbac_ctx* h = NULL;
    EXPECT(lbac_init(&p, NULL, &h) == LBAC_EINVAL);
    EXPECT(lbac_init(NULL, phi0, &h) == LBAC_EINVAL);
    EXPECT(lbac_step(NULL, 1) == LBAC_EINVAL);
    EXPECT(lbac_mass(NULL, NULL) == LBAC_EINVAL);
    EXPECT(lbac_free(NULL) == LBAC_OK);
    for (int code = 1; code >= -8; --code) EXPECT(lbac_strerror(code) != NULL);
    EXPECT(strcmp(lbac_strerror(0), "ok") == 0);
    EXPECT(lbac_last_error(NULL) != NULL);

    /* the batched form: invalid counts and precisions are rejected on the host */
    lbac_batch* b = NULL;
    const double* phis[2] = {phi0, phi0};
    lbac_params ps[2] = {p, p};
    EXPECT(lbac_batch_init(ps, phis, 0, &b) == LBAC_EINVAL);
    EXPECT(lbac_batch_init(NULL, phis, 2, &b) == LBAC_EINVAL);
    ps[1].precision = LBAC_F64;
    EXPECT(lbac_batch_init(ps, phis, 2, &b) == LBAC_EINVAL);
    EXPECT(lbac_batch_free(NULL) == LBAC_EINVAL || lbac_batch_free(NULL) == LBAC_OK);

    /* closure workspace sizes: positive for valid shapes, an error for bad ones */
    EXPECT(lbac_closure_workspace_bytes(512, 512, 4) > 0);
    EXPECT(lbac_closure_workspace_bytes(0, 512, 4) < 0);
    EXPECT(lbac_closure_workspace_bytes(2, 512, 4) < 0);
    EXPECT(lbac_closure_workspace_bytes(512, 512, 0) < 0);
    free(phi0);
}

static void validation_3d(void) {
    double* phi0 = (double*)malloc(512 * sizeof(double));
    for (int k = 0; k < 512; ++k) phi0[k] = 0.5;
    lbac3_params p;
    lbac3_default_params(&p, 8, 8, 8);
    lbac3_ctx* h = NULL;
    lbac3_params q = p;
    q.tau = 0.5;
    EXPECT(lbac3_init(&q, phi0, &h) == LBAC_EINVAL);
    q = p;
    q.eps = 0.0;
    EXPECT(lbac3_init(&q, phi0, &h) == LBAC_EINVAL);
    const int dims[][3] = {{0, 4, 4}, {4, 4, 0}, {5000, 2, 2}, {1024, 1024, 256}};
    for (int s = 0; s < 4; ++s) {
        q = p;
        q.nx = dims[s][0];
        q.ny = dims[s][1];
        q.nz = dims[s][2];
        EXPECT(lbac3_init(&q, phi0, &h) == LBAC_EINVAL);
    }
    EXPECT(lbac3_init(NULL, NULL, &h) == LBAC_EINVAL);
    EXPECT(lbac3_step(NULL, 1) == LBAC_EINVAL);
    EXPECT(lbac3_last_error(NULL) != NULL);
    free(phi0);
}

/* the host-only schedule check over a seeded list of ragged instances, every
 * protocol, several residencies */
static void schedule(void) {
    enum { COUNT = 24 };
    int32_t nx[COUNT], ny[COUNT];
    int64_t ns[COUNT];
    unsigned s = 12345u;
    for (int k = 0; k < COUNT; ++k) {
        s = s * 1103515245u + 12345u;
        nx[k] = 3 + (int32_t)((s >> 8) % 300);
        s = s * 1103515245u + 12345u;
        ny[k] = 3 + (int32_t)((s >> 8) % 300);
        s = s * 1103515245u + 12345u;
        ns[k] = (int64_t)((s >> 8) % 40);
    }
    nx[0] = 1;
    ny[1] = 1;
    ns[2] = 0;
    const int strips[] = {8, 13, 40};
    const int workers[] = {1, 3, 40};
    for (int a = 0; a < 3; ++a)
        for (int w = 0; w < 3; ++w) {
            int32_t verdict = -1;
            int64_t ran = -1;
            EXPECT(lbac_batch_schedule_check(nx, ny, ns, COUNT, strips[a], workers[w], 0, 7u + (uint64_t)w, &verdict,
                                             &ran) == LBAC_OK);
            EXPECT(verdict == 0);
            EXPECT(ran > 0);
        }
    /* the two protocols that exist to be caught */
    int32_t verdict = -1;
    const int32_t one_nx[1] = {64}, one_ny[1] = {64};
    const int64_t one_ns[1] = {30};
    EXPECT(lbac_batch_schedule_check(one_nx, one_ny, one_ns, 1, 16, 8, 1, 1u, &verdict, NULL) == LBAC_OK);
    EXPECT(verdict == 2);
    EXPECT(lbac_batch_schedule_check(nx, ny, ns, COUNT, 8, 2, 2, 1u, &verdict, NULL) == LBAC_OK);
    EXPECT(verdict == 1);
    EXPECT(lbac_batch_schedule_check(nx, ny, ns, 0, 8, 2, 0, 1u, &verdict, NULL) == LBAC_EINVAL);
    EXPECT(lbac_batch_schedule_check(nx, ny, ns, COUNT, 4, 2, 0, 1u, &verdict, NULL) == LBAC_EINVAL);
}

int main(void) {
    validation_2d();
    validation_3d();
    schedule();
    printf("abi_driver: %d failures\n", failures);
    return failures ? 1 : 0;
}
