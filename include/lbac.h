/*
 * lbac — accurate interface-capturing lattice Boltzmann step on MI355X.
 *
 * C ABI of the library.  It advances the order parameter phi of the improved
 * conservative Allen-Cahn equation (H. Liang, arXiv:2203.05230, Sec. 2.1,
 * Eq. (8)) with the D2Q9 BGK scheme of Sec. 2.2 (Eq. (9)-(13)) on a periodic
 * nx-by-ny lattice, under a prescribed velocity field u(x, t), interface
 * width eps, mobility M = c_s^2 (tau - 1/2) and regulariser delta.
 *
 * Conventions shared by every entry point:
 *  - Status: 0 (LBAC_OK) on success, a negative LBAC_E* code on failure; no
 *    C++ exception crosses this boundary.  lbac_last_error() gives the text
 *    of the last failure of a context.
 *  - Lattice units: dx = dt = 1, c_s^2 = 1/3.  Node (i, j) sits at the cell
 *    centre X = i + 1/2, Y = j + 1/2; host arrays of nodes are row-major
 *    ny-by-nx doubles, x fastest.
 *  - Host pointers are owned by the caller and only read or written during
 *    the call.  Device pointers (the *_device calls) must be device memory
 *    on the context's device, owned by the caller, and are used in stream
 *    order on the context's stream.
 *  - The width convention is the one under which Eq. (13) and the tanh
 *    profile phi = (1 + tanh(d / (2 eps))) / 2 agree: psi = eps ln(..) is the
 *    signed distance and the sharpening magnitude is
 *    (1 - tanh^2(psi / (2 eps))) / (4 eps).  The paper's own eps (printed in
 *    Eq. (2)-(6) as tanh(2 s / eps)) is four times this eps.
 */
#ifndef LBAC_H
#define LBAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LBAC_OK 0
#define LBAC_EINVAL (-1)     /* invalid argument or parameter */
#define LBAC_ENOMEM (-2)     /* allocation failed (device or allocator callback) */
#define LBAC_EDEVICE (-3)    /* HIP runtime error; text in lbac_last_error() */
#define LBAC_ENONFINITE (-4) /* a reduction produced NaN or Inf */
#define LBAC_ESTATE (-5)     /* call not valid in the context's current state */

/* velocity fields, u(x, t) of the problem statement (Sec. 3, Eq. (14)).
 * With x = X / nx, y = Y / ny:
 *  VORTEX:       u = -U sin^2(pi x) sin(2 pi y) c(t), v = U sin^2(pi y) sin(2 pi x) c(t)
 *  VORTEX_PAPER: the signs printed in Eq. (14) (u = +U.., v = -U..)
 *  with c(t) = cos(pi t / period_T), t the step count since init;
 *  ROTATION:     u = -omega (Y - cy), v = omega (X - cx)   (solid body)
 *  UNIFORM:      u = ux, v = uy                              */
#define LBAC_VEL_ZERO 0
#define LBAC_VEL_VORTEX 1
#define LBAC_VEL_ROTATION 2
#define LBAC_VEL_UNIFORM 3
#define LBAC_VEL_VORTEX_PAPER 4

/* arithmetic and population storage */
#define LBAC_F64 0           /* FP64 collide, FP64 populations */
#define LBAC_F32 1           /* FP32 collide, FP32 populations */
#define LBAC_F32_F16STORE 2  /* FP32 collide; populations stored shifted, f_i - w_i phi, in FP16, plus FP32 phi */
#define LBAC_F32_BF16STORE 3 /* as above with BF16 */

/* interface model */
#define LBAC_MODEL_IMPROVED 0     /* Eq. (8): normal and sharpening from psi (the paper's method) */
#define LBAC_MODEL_CONVENTIONAL 1 /* Eq. (1): normal from grad phi, sharpening phi (1 - phi) / eps */

/* Optional device allocator (for example a framework's caching allocator).
 * alloc returns device memory of at least `bytes` on the current device, or
 * NULL; free releases it.  Both are called on the host thread that calls the
 * library.  When the pointer to this struct is NULL the library uses
 * hipMalloc / hipFree. */
typedef struct lbac_allocator {
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* ptr, void* user);
    void* user;
} lbac_allocator;

typedef struct lbac_params {
    int32_t nx, ny;       /* lattice size, 1 <= nx, ny, nx * ny < 2^31 / 16 */
    double eps;           /* interface width (> 0), width convention above */
    double tau;           /* relaxation time (> 1/2); M = (tau - 1/2) / 3 */
    double delta;         /* regulariser of Eq. (13) (>= 0), same in psi and n */
    int32_t vel_kind;     /* LBAC_VEL_* */
    double U, period_T;   /* vortex amplitude and period in steps (period_T > 0) */
    double omega, cx, cy; /* rotation rate and centre (lattice units) */
    double ux, uy;        /* uniform velocity */
    int32_t precision;    /* LBAC_F64 .. LBAC_F32_BF16STORE */
    int32_t model;        /* LBAC_MODEL_* */
    void* stream;         /* hipStream_t the context works on; NULL = a stream the library creates */
    const lbac_allocator* alloc; /* NULL = hipMalloc */
} lbac_params;

typedef struct lbac_ctx lbac_ctx;

/* Fills *p with the 64x64 single-vortex defaults (eps 1, tau 0.8,
 * delta 1e-10, U 0.02, period 2000, FP64, improved model). */
void lbac_default_params(lbac_params* p, int32_t nx, int32_t ny);

/* Creates a context on the current HIP device and sets the populations to
 * the equilibrium of Eq. (10) for phi0 and u(x, 0); t = 0.
 * phi0: host, ny*nx doubles, copied.  *out: owned by the library until
 * lbac_free.  Errors: LBAC_EINVAL (tau <= 1/2, eps <= 0, delta < 0, bad
 * sizes, non-finite phi0, max |u| + |v| >= 1/3 over the grid, which would
 * make an equilibrium population of Eq. (10) change sign),
 * LBAC_ENOMEM, LBAC_EDEVICE. */
int lbac_init(const lbac_params* p, const double* phi0, lbac_ctx** out);

/* Same, with phi0 a device array of ny*nx doubles (read in stream order). */
int lbac_init_device(const lbac_params* p, const double* phi0_device, lbac_ctx** out);

/* Releases every resource of the context (NULL is allowed). */
int lbac_free(lbac_ctx* h);

/* Advances n >= 0 steps of Eq. (9) (one fused collide-and-stream kernel per
 * step) on the context's stream; t += n.  Asynchronous: a device error may
 * surface here or at the next synchronising call. */
int lbac_step(lbac_ctx* h, int64_t n);

/* phi(x, t) = sum_i f_i (Eq. (12)) at every node, as ny*nx host doubles.
 * Synchronises the context's stream. */
int lbac_phi(lbac_ctx* h, double* out);

/* Same into a device array of ny*nx doubles, in stream order (no sync). */
int lbac_phi_device(lbac_ctx* h, double* out_device);

/* Total mass sum_x phi(x, t), accumulated in FP64 in a fixed order (so the
 * result is reproducible).  Synchronises.  LBAC_ENONFINITE if not finite. */
int lbac_mass(lbac_ctx* h, double* out);

/* Shape errors against a reference field ref (host, ny*nx doubles):
 * e1 = sum|phi - ref| / sum|ref| (the relative L1 norm of Sec. 3) and
 * e2 = ||phi - ref||_2 / ||ref||_2.  Either output may be NULL.  Synchronises. */
int lbac_shape_error(lbac_ctx* h, const double* ref, double* e1, double* e2);

/* Steps taken since init (or since the state was last set). */
int lbac_time(lbac_ctx* h, int64_t* t);

/* Checkpoint: the context's full state (populations and t) as an opaque
 * byte blob.  With buf == NULL, *bytes receives the size needed.  Restoring
 * a blob from a context with the same parameters continues bitwise. */
int lbac_get_state(lbac_ctx* h, void* buf, size_t* bytes);
int lbac_set_state(lbac_ctx* h, const void* buf, size_t bytes);

/* Launch shape of the step kernel: block width bx (64, 128 or 256 lattice
 * columns) and strip height (rows marched per block, >= 1).  Results do not
 * depend on the shape (bitwise).  LBAC_EINVAL for unsupported values. */
int lbac_set_launch(lbac_ctx* h, int32_t bx, int32_t strip_h);
int lbac_get_launch(lbac_ctx* h, int32_t* bx, int32_t* strip_h);

/* Times every supported launch shape over `steps` steps each (state is left
 * unchanged) and keeps the fastest; *us_per_step (may be NULL) gets its time. */
int lbac_autotune(lbac_ctx* h, int32_t steps, double* us_per_step);

/* Graph replay: when chunk > 0 (even), lbac_step replays a captured HIP
 * graph of `chunk` step kernels for every full chunk; 0 launches kernels one
 * by one.  Bitwise identical either way. */
int lbac_set_graph_chunk(lbac_ctx* h, int32_t chunk);

/* HBM bytes one step moves by design (read + write of the stored state). */
int lbac_bytes_per_node(lbac_ctx* h, double* bytes);

/* hipStream_t of the context. */
void* lbac_stream(lbac_ctx* h);

/* Text of a status code, and of the last failure of a context. */
const char* lbac_strerror(int code);
const char* lbac_last_error(lbac_ctx* h);

#ifdef __cplusplus
}
#endif
#endif /* LBAC_H */
