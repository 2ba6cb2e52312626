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
    int32_t nx, ny;       /* lattice size, 1 <= nx, ny <= 65536, nx * ny <= 2^27 */
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

/* Launch shape of the step kernel.  variant LBAC_KERNEL_BLOCK: a block of bx
 * column threads (bx = 64, 128 or 256) plus one wavefront for the halo owns
 * bx aligned columns and shares rows through LDS, with the next row's loads
 * in flight while a row is processed; LBAC_KERNEL_BLOCK_DEEP: the same with
 * two rows in flight; LBAC_KERNEL_WAVE: every wavefront owns a 60-column
 * tile held in registers, bx / 64 wavefronts per block;
 * LBAC_KERNEL_FUSED2 and LBAC_KERNEL_FUSED3 (FP32 collision: LBAC_F32 or a
 * 16-bit storage): one launch takes S = 2 or 3 steps, the populations
 * between them kept in LDS (the block layout; step k of S is computed on the
 * tile grown by RC (S - 1 - k) columns and rows on each side, RC = 2, or 3
 * with the closure, whose network reads a 5x5 neighbourhood), so HBM is read
 * and written once per S steps; their tiles are bx = 64, 96, 128, ..., 320
 * columns (any multiple of 32 in that range, and 240; with the closure 128,
 * 160, 192 or 224, another width running those launches at 224), the block
 * being the bx + 2 RC S grown columns rounded up to whole wavefronts; a step count
 * that is not a multiple of S ends with one-step launches (bx 256 where bx
 * is not 64, 128 or 256).  With the closure and the conventional model every
 * step is a one-step launch.  strip_h: rows each tile marches (>= 1).
 * Results do not depend on the shape or variant (bitwise; the 16-bit
 * storage forms round once per launch, so there they depend on S only).
 * LBAC_EINVAL for unsupported values. */
#define LBAC_KERNEL_BLOCK 0
#define LBAC_KERNEL_WAVE 1
#define LBAC_KERNEL_BLOCK_DEEP 2
#define LBAC_KERNEL_FUSED2 3
#define LBAC_KERNEL_FUSED3 4
int lbac_set_launch(lbac_ctx* h, int32_t variant, int32_t bx, int32_t strip_h);
int lbac_get_launch(lbac_ctx* h, int32_t* variant, int32_t* bx, int32_t* strip_h);

/* Times every supported launch shape (variant; bx; strip_h among the
 * multiples of 8 up to 256, 512 and ceil(ny / k) for k = 1..32) over `steps`
 * launches each (state is left unchanged) and keeps the fastest per step;
 * *us_per_step (may be NULL) gets its time per step. */
int lbac_autotune(lbac_ctx* h, int32_t steps, double* us_per_step);

/* Graph replay: when chunk > 0 (even), lbac_step replays a captured HIP
 * graph of `chunk` step kernels for every full chunk; 0 launches kernels one
 * by one.  Bitwise identical either way. */
int lbac_set_graph_chunk(lbac_ctx* h, int32_t chunk);

/* Learned closure in the step (LBAC_F32 contexts): params = the network's
 * LBAC_MLP_NPARAM FP32 parameters (host, copied; layout below).  At every
 * node whose clipped phi lies in (theta, 1 - theta) the network, run in BF16
 * with FP32 accumulation (MFMA) on the 5x5 neighbourhood of phi, gives a
 * correction c that is added to the sharpening flux S n of Eq. (11).  The
 * collision is linear in G, so the correction changes a band node's
 * post-collision populations by (1 - 1/(2 tau)) w_i (c_i . c).  With
 * LBAC_KERNEL_FUSED2 / _FUSED3 (improved model) the multi-step kernel
 * evaluates the network inside each of its steps, on the band nodes of the
 * rows it updates, from the phi rows it keeps in LDS.  One-step launches run
 * the block-variant step kernel (which records the band), a scan that lists
 * the band nodes and a pass that adds the correction at those nodes.  Both
 * give the same results bit for bit.  Needs device memory for nx * ny list
 * entries.
 * params == NULL switches the closure off.  LBAC_EINVAL for another
 * precision, a batch instance, theta outside [0, 0.5) or non-finite
 * parameters. */
int lbac_set_closure(lbac_ctx* h, const float* params, float theta);

/* HBM bytes per node one launch of the step kernel moves by design: the
 * stored state read and written once.  A launch takes
 * lbac_steps_per_launch steps (2 or 3 with LBAC_KERNEL_FUSED2 or _FUSED3
 * and FP32 collision, with the closure only for the improved model; else
 * 1), so a step moves this divided by that. */
int lbac_bytes_per_node(lbac_ctx* h, double* bytes);
int lbac_steps_per_launch(lbac_ctx* h, int32_t* steps);

/* Practical bandwidth ceiling of the step: a plain copy of the stored state
 * into the context's second buffer with the step kernel's tiling (256-column
 * tiles marching strips of rows, the same tile order) and access order but
 * none of its arithmetic.  Times `launches` (>= 1) launches at strip heights
 * 8, 16, 32 and 64 and gives the fastest mean in *us_per_launch.  Moves the
 * same bytes per node as a launch of the step kernel (lbac_bytes_per_node).
 * The state is unchanged.  Synchronises. */
int lbac_copy_ceiling(lbac_ctx* h, int32_t launches, double* us_per_launch);

/* hipStream_t of the context. */
void* lbac_stream(lbac_ctx* h);

/* ---- batched form --------------------------------------------------------
 * Many independent lattices (instances) of uneven sizes and parameters
 * advanced together by ONE kernel launch (plus one for the last nsteps mod 3
 * steps), replayed from a captured HIP graph.  Work is split into (instance,
 * column tile of at most 240 columns, strip of rows) items.  An item takes
 * three steps per pass (the populations between them kept in LDS, as with
 * LBAC_KERNEL_FUSED3; the last nsteps mod 3 steps are one-step passes).  The
 * instances are dealt to eight classes of about equal work (one per XCD, so
 * neighbouring tiles share that XCD's L2), and the (pass, item) slots of a
 * class are numbered pass by pass; the launch has as many workgroups as the
 * device keeps resident, and each repeatedly takes the next slot number of
 * its class (blockIdx mod 8; once that class is used up, of another) from
 * the class's atomic counter, waits, through per-item progress counters, for
 * the previous pass of its own item and of the items its read region
 * overlaps (no grid-wide barrier), runs the pass and publishes, so instances
 * retire independently.  Every slot waited for is of the same class, has a
 * smaller number and is finished or held by a running workgroup, so the
 * schedule progresses whatever number of workgroups the device keeps
 * resident.  Every instance uses FP32 collide, FP32 or shifted 16-bit
 * storage and the improved model; results are bitwise those of lbac_step on
 * the same instance.  A wait that exceeds the time-out makes every workgroup
 * exit and the run return LBAC_EDEVICE. */
typedef struct lbac_batch lbac_batch;

/* params[k], phi0[k] (host, ny*nx doubles): instance k, k < count.  The stream
 * of params[0] (or a private one) is used for the whole batch; allocators are
 * honoured per instance.  Every instance has the same precision: LBAC_F32,
 * or the shifted 16-bit storage LBAC_F32_F16STORE / LBAC_F32_BF16STORE (FP32
 * collide, the populations kept in FP32 between the three steps of a pass
 * and rounded to 16 bits once per pass, as lbac_step does).  Errors as
 * lbac_init, plus LBAC_EINVAL for another precision or mixed precisions, a
 * model other than LBAC_MODEL_IMPROVED, or an instance whose population
 * planes take 2^31 bytes or more (FP32: about 7700 x 7700 nodes; such a
 * lattice fills the device by itself and belongs to lbac_step). */
int lbac_batch_init(const lbac_params* params, const double* const* phi0, int32_t count, lbac_batch** out);
int lbac_batch_free(lbac_batch* b);

/* Advances instance k by nsteps[k] >= 0 steps (host array of count values) in
 * one persistent launch.  Synchronous.  LBAC_EDEVICE if a dependency wait
 * timed out: some passes have then overwritten both buffers of some
 * instances, so the batch and every instance context return LBAC_ESTATE from
 * then on (lbac_batch_free still works). */
int lbac_batch_run(lbac_batch* b, const int64_t* nsteps);

/* Context of instance k, owned by the batch: use it with lbac_phi, lbac_mass,
 * lbac_shape_error, lbac_time, lbac_get_state / lbac_set_state (lbac_free on
 * it returns LBAC_ESTATE). */
int lbac_batch_instance(lbac_batch* b, int32_t k, lbac_ctx** ctx);
int lbac_batch_count(lbac_batch* b, int32_t* count);

/* phi of instance k (Eq. (12), the pulled sum): out is ny*nx host doubles of
 * that instance, caller-owned, as lbac_phi on lbac_batch_instance(b, k).
 * Synchronises.  LBAC_EINVAL for k out of range; LBAC_ESTATE after a run
 * that timed out. */
int lbac_batch_phi(lbac_batch* b, int32_t k, double* out);

/* The mass of every instance (the sum of phi over its lattice, as
 * lbac_mass): per_instance is count host doubles, caller-owned.
 * Synchronises.  Errors as lbac_mass for the first instance that fails. */
int lbac_batch_mass(lbac_batch* b, double* per_instance);

/* Strip height (>= 8; the default is 40): an instance ny rows high is cut
 * into the nearest whole number of strips to ny / strip_h (at least one, at
 * most ny / 8) of balanced heights.  get_shape also gives the number of
 * batch workgroups the device keeps resident at once (the grid of a batch
 * launch; the schedule's progress does not depend on it). */
int lbac_batch_set_shape(lbac_batch* b, int32_t strip_h);
int lbac_batch_get_shape(lbac_batch* b, int32_t* strip_h, int32_t* resident_workgroups);

/* Times every candidate strip height on a dry run of nsteps[k] steps of
 * instance k (host array of count values; each pass reads the current state
 * and writes only the other buffer: state and time unchanged) and keeps the
 * fastest; *ms (may be NULL) gets its time.  Step counts in the proportions
 * of the real run make the tuning see its tail, where few instances are left. */
int lbac_batch_autotune(lbac_batch* b, const int64_t* nsteps, double* ms);

/* Time-out of one dependency wait (default 20 s).  test_stall != 0 makes
 * every wait ask for a pass that never completes, so that the time-out path
 * can be tested: each workgroup exits after `seconds`. */
int lbac_batch_set_timeout(lbac_batch* b, double seconds, int32_t test_stall);
const char* lbac_batch_last_error(lbac_batch* b);

/* Host-only check of the batched schedule (no GPU involved): builds the items,
 * dependency lists and slot tables the library would build for count
 * instances of nx[k] x ny[k] nodes advanced by nsteps[k] steps with strips of
 * strip_h rows, and runs a slot protocol on the CPU with `workers`
 * workgroups running at once and their actions interleaved at random (seed).
 * protocol 0: the library's (pass-major slot numbers from per-class
 * counters, waits for the previous pass of the dependencies); 1: the same
 * without the waits;
 * 2: fixed item lists of 2 * workers workgroups, each walked pass by pass, of
 * which only `workers` run at once (the two others exist to show that the
 * check detects what goes wrong with them).
 * *verdict: 0 = every slot ran and every slot read only tiles holding the
 * previous pass while no running slot wrote them; 1 = deadlock (no workgroup
 * could act before the end); 2 = a read or write hazard; 3 = the kernel's
 * slot lookup maps a slot to another (pass, item) than the slot table
 * defines.  *slots_run (may be
 * NULL) gets the number of slots run.  LBAC_EINVAL for bad sizes. */
int lbac_batch_schedule_check(const int32_t* nx, const int32_t* ny, const int64_t* nsteps, int32_t count,
                              int32_t strip_h, int32_t workers, int32_t protocol, uint64_t seed, int32_t* verdict,
                              int64_t* slots_run);

/* Text of a status code, and of the last failure of a context. */
const char* lbac_strerror(int code);
const char* lbac_last_error(lbac_ctx* h);

/* ---- learned closure: the network and its training ------------------------
 * A 25 -> 64 -> 64 -> 2 multilayer perceptron with the tanh form of GELU,
 * mapping the 5x5 neighbourhood of phi around a node (row-major, dy = -2..2
 * outer, dx = -2..2 inner) to a correction (cx, cy) of the sharpening flux
 * S n of Eq. (11).  Parameters: LBAC_MLP_NPARAM FP32 values laid out as
 * W1[64][25], b1[64], W2[64][64], b2[64], W3[2][64], b3[2].  Training runs
 * on the GPU in FP32 (hand-written kernels on the FP32 matrix cores: one
 * wavefront per 16 samples for the forward and backward passes and its share
 * of the gradient, then a fixed-order sum of the shares and the Adam update,
 * so a training run is reproducible); loss
 * L = (1/B) sum_samples sum_outputs (out - y)^2.  Sample arrays are device
 * memory owned by the caller: x_dev is batch*25 floats, y_dev and out_dev
 * batch*2 floats, row-major. */
#define LBAC_MLP_NPARAM 5954
typedef struct lbac_mlp lbac_mlp;

/* init: host, LBAC_MLP_NPARAM finite values (copied).  stream: the hipStream_t
 * every call of this network runs on, or NULL for a non-blocking stream of the
 * network's own; calls return before the GPU is done, so a caller that
 * rewrites x_dev / y_dev between calls must order that with this stream
 * (simplest: pass the stream its own writes run on). */
int lbac_mlp_create(const float* init, void* stream, lbac_mlp** out);
int lbac_mlp_free(lbac_mlp* m);
int lbac_mlp_get_weights(lbac_mlp* m, float* out_host);
int lbac_mlp_set_weights(lbac_mlp* m, const float* in_host);
/* out_dev = network(x_dev), asynchronous on the network's stream. */
int lbac_mlp_forward(lbac_mlp* m, const float* x_dev, int64_t batch, float* out_dev);
/* Loss and gradient (host, LBAC_MLP_NPARAM floats; may be NULL) without an
 * update.  Synchronises. */
int lbac_mlp_loss_grad(lbac_mlp* m, const float* x_dev, const float* y_dev, int64_t batch, double* loss,
                       float* grad_host);
/* One Adam step (beta1 0.9, beta2 0.999, 1e-8) with learning rate lr on the
 * batch.  *loss (may be NULL) receives the loss before the update; asking for
 * it synchronises. */
int lbac_mlp_train_step(lbac_mlp* m, const float* x_dev, const float* y_dev, int64_t batch, float lr, double* loss);
const char* lbac_mlp_last_error(lbac_mlp* m);

/* Training samples for the closure from a fine field phi_f (device, nyf*nxf
 * doubles, a run r times finer, width eps_f = r eps_c in its own units):
 * coarse phi_c = mean of each r x r block; target = mean over the block of
 * r S_f n_f minus S_c(phi_c) n_c(phi_c), the sharpening flux of Eq. (6), (7),
 * (13) on each grid; one sample per coarse node with theta < clip(phi_c) <
 * 1 - theta: its 5x5 neighbourhood of phi_c (the network's input layout)
 * and the target, plus the 7 images under the symmetries of the square when
 * augment != 0.  Samples go to x_dev (25 floats each) and y_dev (2 floats)
 * from index base on, in row-major node order, as long as the index is below
 * capacity; *count receives the number of samples the field yields (stored
 * or not).  workspace: device memory of lbac_closure_workspace_bytes(nxf,
 * nyf, r) bytes.  Synchronises the stream (hipStream_t or NULL). */
int64_t lbac_closure_workspace_bytes(int32_t nxf, int32_t nyf, int32_t r);
int lbac_closure_extract(const double* phi_f_dev, int32_t nxf, int32_t nyf, int32_t r, double eps_f, double eps_c,
                         double delta, float theta, int32_t augment, void* workspace, float* x_dev, float* y_dev,
                         int64_t base, int64_t capacity, int64_t* count, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight training-data loops, harnesses that forbid allocation):
 * lbac_closure_extract without the workspace argument.  Its workspace is a
 * fixed 8 MiB device array inside the library (one per GPU, held until the
 * process ends; enough for coarse grids up to 512 x 512), and the call
 * allocates nothing.  LBAC_EINVAL when lbac_closure_workspace_bytes(nxf,
 * nyf, r) exceeds 8 MiB, else as lbac_closure_extract.  Calls on one GPU
 * share that array: calls that overlap in time on one GPU (other host
 * threads, other streams) race and must be serialised by the caller. */
int lbac_closure_extract_noalloc(const double* phi_f_dev, int32_t nxf, int32_t nyf, int32_t r, double eps_f,
                                 double eps_c, double delta, float theta, int32_t augment, float* x_dev, float* y_dev,
                                 int64_t base, int64_t capacity, int64_t* count, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LBAC_H */
