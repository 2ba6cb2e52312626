/*
 * lbac3 — the 3-D form of the accurate interface-capturing lattice Boltzmann
 * step (H. Liang, arXiv:2203.05230, Sec. 2.2, Eq. (9)-(13)) on a D3Q19
 * lattice, MI355X (gfx950) HIP implementation behind a C ABI.
 *
 * The paper writes the scheme for D2Q9; every equation it uses is free of the
 * dimension (sums over the lattice velocities, the isotropic gradient
 * grad chi = sum_i w_i c_i chi(x + c_i) / c_s^2, f_eq and F_i of Eq. (10)-(11)),
 * so this form changes only the lattice: D3Q19 with w = 1/3 (rest), 1/18
 * (the 6 faces), 1/36 (the 12 edges), c_s^2 = 1/3.  Interface width, clip,
 * regulariser, time derivative and initial state follow the same readings as
 * lbac.h.  Status codes and the precision constants are those of lbac.h.
 *
 * Layout: phi arrays are nz * ny * nx doubles in host memory, x fastest,
 * then y, then z; node (i, j, k) sits at the cell centre (i + 1/2, j + 1/2,
 * k + 1/2).  The lattice is periodic in every direction.
 */
#ifndef LBAC3_H
#define LBAC3_H

#include <stdint.h>

#include "lbac.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Prescribed velocity u(x, t), x = X / nx, y = Y / ny, z = Z / nz:
 * DEFORMATION: u = 2U sin^2(pi x) sin(2 pi y) sin(2 pi z), v = -U sin(2 pi x)
 *   sin^2(pi y) sin(2 pi z), w = -U sin(2 pi x) sin(2 pi y) sin^2(pi z), all
 *   times cos(pi t / period_T) (divergence-free on a cube);
 * VORTEX_XY: the single vortex of LBAC_VEL_VORTEX in every z plane, w = 0;
 * UNIFORM: (ux, uy, uz); ZERO: none. */
#define LBAC3_VEL_ZERO 0
#define LBAC3_VEL_DEFORMATION 1
#define LBAC3_VEL_VORTEX_XY 2
#define LBAC3_VEL_UNIFORM 3

typedef struct lbac3_params {
    int32_t nx, ny, nz;  /* lattice size, 1 <= nx, ny, nz <= 4096, nx * ny * nz <= 2^27 */
    double eps;          /* interface width (> 0), width convention of lbac.h */
    double tau;          /* relaxation time (> 1/2); M = (tau - 1/2) / 3 */
    double delta;        /* regulariser of Eq. (13) (>= 0) */
    int32_t vel_kind;    /* LBAC3_VEL_* */
    double U, period_T;  /* amplitude and period (steps) of DEFORMATION and VORTEX_XY */
    double ux, uy, uz;   /* UNIFORM velocity */
    int32_t precision;   /* LBAC_F64 or LBAC_F32 (collision and storage) */
    void* stream;        /* hipStream_t to work on, or NULL for a stream of the context's own */
} lbac3_params;

typedef struct lbac3_ctx lbac3_ctx;

/* Fills p with a 3-D deformation run on nx x ny x nz: eps 1, tau 0.8,
 * delta 1e-10, U 0.02, period 3 nx / U steps, FP32, own stream. */
void lbac3_default_params(lbac3_params* p, int32_t nx, int32_t ny, int32_t nz);

/* Creates a context on the current device: populations at equilibrium
 * f_eq(phi0, u(x, 0)), t = 0.  phi0: host, nz*ny*nx finite doubles (copied).
 * *out is owned by the caller until lbac3_free.  LBAC_EINVAL for bad
 * parameters (including |u| + |v| + |w| >= 1/3 anywhere), LBAC_ENOMEM,
 * LBAC_EDEVICE. */
int lbac3_init(const lbac3_params* p, const double* phi0, lbac3_ctx** out);

/* Advances n >= 0 steps (one fused kernel launch per step) on the context's
 * stream; returns when they are queued. */
int lbac3_step(lbac3_ctx* h, int64_t n);

/* phi(x, t) = sum_i f_i(x, t) (the pulled sum, Eq. (12)) into host memory
 * (nz*ny*nx doubles).  Synchronises. */
int lbac3_phi(lbac3_ctx* h, double* out);

/* Sum of phi over the lattice, accumulated in FP64 in a fixed order.
 * Synchronises; LBAC_ENONFINITE if the sum is not finite. */
int lbac3_mass(lbac3_ctx* h, double* out);

/* Relative L1 (e1) and L2 (e2) distance of phi from ref (host, nz*ny*nx). */
int lbac3_shape_error(lbac3_ctx* h, const double* ref, double* e1, double* e2);

/* Steps taken since lbac3_init. */
int lbac3_time(lbac3_ctx* h, int64_t* t);

/* Launch shape.  Every block updates a tile of tile_x x tile_y columns, one
 * thread per column, and marches strip_z >= 1 planes; the one-column rim
 * around the tile is pulled again by the block for its psi.  Tile shapes:
 * 32 x 8, 32 x 16, 64 x 4, 64 x 8, 128 x 4, and with LBAC_F32 also 32 x 32,
 * 64 x 16, 128 x 8.  variant LBAC3_KEEP (0): the update keeps its node's 19
 * pulled values in registers; LBAC3_REPULL (1): it re-reads them (cache
 * hits), issued with the next plane's loads; LBAC3_PREFETCH (2): the next
 * plane's loads are in flight during the update.  z_major 0: blocks take the
 * tiles with x fastest, then y, then the strip; 1: the strip index fastest.
 * Even strips march up and odd strips down, so two neighbouring strips read
 * the planes they share at the same time.  Results do not depend on the
 * launch shape (bitwise).  LBAC_EINVAL for other values. */
#define LBAC3_KEEP 0
#define LBAC3_REPULL 1
#define LBAC3_PREFETCH 2
int lbac3_set_launch(lbac3_ctx* h, int32_t tile_x, int32_t tile_y, int32_t variant, int32_t strip_z,
                     int32_t z_major);
int lbac3_get_launch(lbac3_ctx* h, int32_t* tile_x, int32_t* tile_y, int32_t* variant, int32_t* strip_z,
                     int32_t* z_major);

/* Times every launch shape (tile, variant, strip_z among the powers of two
 * from 4 to 128 and ceil(nz / k) for k = 1..16, z_major) over
 * `steps` steps each (state unchanged) and keeps the fastest; *us_per_step
 * (may be NULL) gets its time. */
int lbac3_autotune(lbac3_ctx* h, int32_t steps, double* us_per_step);

/* HBM bytes one step moves by design: read and write of the 19 stored
 * populations (FP64 304, FP32 152). */
int lbac3_bytes_per_node(lbac3_ctx* h, double* bytes);

/* Message of the context's last error ("" if none); NULL context: a
 * description of the last failed lbac3_init. */
const char* lbac3_last_error(lbac3_ctx* h);

/* Releases the context and its device memory. */
int lbac3_free(lbac3_ctx* h);

#ifdef __cplusplus
}
#endif

#endif /* LBAC3_H */
