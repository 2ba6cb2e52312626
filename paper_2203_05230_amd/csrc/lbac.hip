// Host side of the lbac library: context, memory layout, launches, graph
// replay, autotuning, reductions and the C ABI declared in include/lbac.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "lbac_internal.hpp"

using namespace lbac;
using namespace lbac_host;

namespace lbac_host {

int fail(lbac_ctx* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

void* dev_alloc(lbac_ctx* h, size_t bytes) {
    if (h->has_alloc) return h->alloc.alloc(bytes, h->alloc.user);
    void* ptr = nullptr;
    if (hipMalloc(&ptr, bytes) != hipSuccess) return nullptr;
    return ptr;
}

void dev_free(lbac_ctx* h, void* ptr) {
    if (!ptr) return;
    if (h->has_alloc)
        h->alloc.free(ptr, h->alloc.user);
    else
        (void)hipFree(ptr);
}

}  // namespace lbac_host

namespace {

void drop_graphs(lbac_ctx* h) {
    for (int i = 0; i < 2; ++i) {
        if (h->gexec[i]) (void)hipGraphExecDestroy(h->gexec[i]);
        h->gexec[i] = nullptr;
        h->gexec_chunk[i] = 0;
    }
}

void release(lbac_ctx* h) {
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    drop_graphs(h);
    for (int i = 0; i < 2; ++i) {
        dev_free(h, h->pop[i]);
        dev_free(h, h->phis[i]);
    }
    dev_free(h, h->vtab);
    dev_free(h, h->vtabf);
    dev_free(h, h->t_dev);
    dev_free(h, h->rows);
    dev_free(h, h->red5);
    dev_free(h, h->dtmp);
    dev_free(h, h->cl_param);
    dev_free(h, h->cl_w);
    dev_free(h, h->cl_b);
    dev_free(h, h->cl_mask);
    dev_free(h, h->cl_list);
    dev_free(h, h->cl_count);
    if (h->host5) (void)hipHostFree(h->host5);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
}

// Separable velocity tables: u = s(t) Ax[x] Ay[y], v = s(t) Bx[x] By[y].
void build_velocity(const lbac_params& p, std::vector<double>& tab) {
    const int nx = p.nx, ny = p.ny;
    tab.assign(2 * (size_t)nx + 2 * (size_t)ny, 0.0);
    double* Ax = tab.data();
    double* Bx = Ax + nx;
    double* Ay = Bx + nx;
    double* By = Ay + ny;
    const double PI = 3.14159265358979323846;
    for (int i = 0; i < nx; ++i) {
        const double X = i + 0.5, x = X / nx;
        const double sx = std::sin(PI * x);
        switch (p.vel_kind) {
        case LBAC_VEL_VORTEX:
            Ax[i] = -p.U * sx * sx;
            Bx[i] = p.U * std::sin(2.0 * PI * x);
            break;
        case LBAC_VEL_VORTEX_PAPER:
            Ax[i] = p.U * sx * sx;
            Bx[i] = -p.U * std::sin(2.0 * PI * x);
            break;
        case LBAC_VEL_ROTATION:
            Ax[i] = -p.omega;
            Bx[i] = p.omega * (X - p.cx);
            break;
        case LBAC_VEL_UNIFORM:
            Ax[i] = p.ux;
            Bx[i] = p.uy;
            break;
        default:
            break;
        }
    }
    for (int j = 0; j < ny; ++j) {
        const double Y = j + 0.5, y = Y / ny;
        const double sy = std::sin(PI * y);
        switch (p.vel_kind) {
        case LBAC_VEL_VORTEX:
        case LBAC_VEL_VORTEX_PAPER:
            Ay[j] = std::sin(2.0 * PI * y);
            By[j] = sy * sy;
            break;
        case LBAC_VEL_ROTATION:
            Ay[j] = Y - p.cy;
            By[j] = 1.0;
            break;
        case LBAC_VEL_UNIFORM:
            Ay[j] = 1.0;
            By[j] = 1.0;
            break;
        default:
            break;
        }
    }
}

double time_period(const lbac_params& p) {
    return (p.vel_kind == LBAC_VEL_VORTEX || p.vel_kind == LBAC_VEL_VORTEX_PAPER) ? p.period_T : 0.0;
}

}  // namespace

StepArgs lbac_host::make_args(const lbac_ctx* h, int src, int32_t k) {
    StepArgs a{};
    a.src = h->pop[src];
    a.dst = h->pop[1 - src];
    a.src_phi = h->phis[src];
    a.dst_phi = h->phis[1 - src];
    a.plane_stride = h->plane_stride;
    a.pitch = h->pitch;
    a.nx = h->p.nx;
    a.ny = h->p.ny;
    a.strip_h = h->strip_h;
    a.vtab = h->vtab;
    a.vtabf = h->vtabf;
    a.t_dev = h->t_dev;
    a.k = k;
    a.period_T = time_period(h->p);
    a.eps = h->p.eps;
    a.tau = h->p.tau;
    a.delta = h->p.delta;
    a.cl_w = h->cl_w;
    a.cl_b = h->cl_b;
    a.cl_theta = h->cl_theta;
    a.cl_mask = h->closure ? h->cl_mask : nullptr;
    a.cl_words = h->cl_words;
    return a;
}

namespace {

template <typename R, int ST, int MODEL>
hipError_t launch_step_bx(StepArgs a, int variant, int bx, hipStream_t s) {
    a.nby = (a.ny + a.strip_h - 1) / a.strip_h;
    a.n_xcd = kXcds;
    if (variant == LBAC_KERNEL_BLOCK || variant == LBAC_KERNEL_BLOCK_DEEP) {
        // one block of bx column threads plus one halo wavefront per bx-column tile
        a.nbx = (a.nx + bx - 1) / bx;
        dim3 grid(a.nbx * a.nby);
        const bool deep = variant == LBAC_KERNEL_BLOCK_DEEP;
        switch (bx) {
        case 64:
            if (deep)
                hipLaunchKernelGGL((step_kernel_lds<R, ST, MODEL, 64, 2>), grid, dim3(block_threads<64>()), 0, s, a);
            else
                hipLaunchKernelGGL((step_kernel_lds<R, ST, MODEL, 64, 1>), grid, dim3(block_threads<64>()), 0, s, a);
            break;
        case 128:
            if (deep)
                hipLaunchKernelGGL((step_kernel_lds<R, ST, MODEL, 128, 2>), grid, dim3(block_threads<128>()), 0, s, a);
            else
                hipLaunchKernelGGL((step_kernel_lds<R, ST, MODEL, 128, 1>), grid, dim3(block_threads<128>()), 0, s, a);
            break;
        default:
            if (deep)
                hipLaunchKernelGGL((step_kernel_lds<R, ST, MODEL, 256, 2>), grid, dim3(block_threads<256>()), 0, s, a);
            else
                hipLaunchKernelGGL((step_kernel_lds<R, ST, MODEL, 256, 1>), grid, dim3(block_threads<256>()), 0, s, a);
            break;
        }
        return hipGetLastError();
    }
    // bx / 64 wavefronts per block, each owning one 60-column tile
    const int wpb = bx / kWave;
    a.nbx = (a.nx + kTileW - 1) / kTileW;
    dim3 grid(((a.nbx + wpb - 1) / wpb) * a.nby);
    switch (wpb) {
    case 1:
        hipLaunchKernelGGL((step_kernel<R, ST, MODEL, 1>), grid, dim3(64), 0, s, a);
        break;
    case 2:
        hipLaunchKernelGGL((step_kernel<R, ST, MODEL, 2>), grid, dim3(128), 0, s, a);
        break;
    default:
        hipLaunchKernelGGL((step_kernel<R, ST, MODEL, 4>), grid, dim3(256), 0, s, a);
        break;
    }
    return hipGetLastError();
}

template <typename R, int ST>
hipError_t launch_step_m(const lbac_ctx* h, const StepArgs& a, int variant, int bx) {
    if (h->p.model == LBAC_MODEL_CONVENTIONAL)
        return launch_step_bx<R, ST, MODEL_CONVENTIONAL>(a, variant, bx, h->stream);
    return launch_step_bx<R, ST, MODEL_IMPROVED>(a, variant, bx, h->stream);
}

// Tile widths of the one-step block kernels.
bool one_step_bx(int bx) { return bx == 64 || bx == 128 || bx == 256; }

// Tile widths of the S-step kernels: multiples of 32 columns from 64 to 320,
// and 240 (the widest tile whose grown columns, bx + 4S at S = 3, fill four
// wavefronts; tiles that start off a 128-byte line of the storage, every
// other one in FP32, give their head columns to the halo wavefront).
bool stepS_bx(int bx) { return (bx >= 64 && bx <= 320 && bx % 32 == 0) || bx == 240; }

hipError_t launch_step(const lbac_ctx* h, int src, int32_t k) {
    StepArgs a = make_args(h, src, k);
    // one-step launches of the S-step variants use the deep block kernel, at a
    // tile width it has (the others exist for the S-step kernels only)
    const int var1 =
        h->variant == LBAC_KERNEL_FUSED2 || h->variant == LBAC_KERNEL_FUSED3 ? LBAC_KERNEL_BLOCK_DEEP : h->variant;
    const int bx1 = one_step_bx(h->bx) ? h->bx : 256;
    if (h->closure) {
        // FP32 plain storage.  The block variants write the band masks; then the
        // band list is rebuilt and the correction pass adds the network's flux
        // correction at the listed nodes.
        const int variant = var1 == LBAC_KERNEL_WAVE ? LBAC_KERNEL_BLOCK : var1;
        const hipError_t e = h->p.model == LBAC_MODEL_CONVENTIONAL
                                 ? launch_step_bx<float, ST_PLAIN, MODEL_CONVENTIONAL>(a, variant, bx1, h->stream)
                                 : launch_step_bx<float, ST_PLAIN, MODEL_IMPROVED>(a, variant, bx1, h->stream);
        if (e != hipSuccess) return e;
        const int64_t nwords = (int64_t)h->p.ny * h->cl_words;
        hipLaunchKernelGGL(closure_reset_kernel, dim3(1), dim3(64), 0, h->stream, h->cl_count);
        hipLaunchKernelGGL(closure_scan_kernel, dim3((unsigned)((nwords + 255) / 256)), dim3(256), 0, h->stream,
                           h->cl_mask, nwords, h->cl_words, h->p.nx, h->cl_list, h->cl_count);
        hipLaunchKernelGGL(closure_apply_kernel, dim3(kClosureBlocks), dim3(kClWaves * kWave), 0, h->stream, a,
                           h->cl_list, h->cl_count);
        return hipGetLastError();
    }
    switch (h->p.precision) {
    case LBAC_F64:
        return launch_step_m<double, ST_PLAIN>(h, a, var1, bx1);
    case LBAC_F32:
        return launch_step_m<float, ST_PLAIN>(h, a, var1, bx1);
    case LBAC_F32_F16STORE:
        return launch_step_m<float, ST_F16>(h, a, var1, bx1);
    default:
        return launch_step_m<float, ST_BF16>(h, a, var1, bx1);
    }
}

// Whether the S-step variants can take the run: FP32 collision, and with the
// closure on FP32 storage and the improved model.
bool stepS_allowed(const lbac_ctx* h) {
    if (h->p.precision == LBAC_F64) return false;
    return !h->closure || h->p.model == LBAC_MODEL_IMPROVED;
}

// Steps one launch takes: S with the S-step variants, else 1.
int launch_steps_of(const lbac_ctx* h) {
    if (!stepS_allowed(h)) return 1;
    return h->variant == LBAC_KERNEL_FUSED2 ? 2 : (h->variant == LBAC_KERNEL_FUSED3 ? 3 : 1);
}

// Tile widths of the S-step kernels with the closure; another width set by
// lbac_set_launch runs these launches at 224 columns (the results do not
// depend on the tile width).
int closure_stepS_bx(int bx) { return bx == 128 || bx == 160 || bx == 192 || bx == 224 ? bx : 224; }

template <int S, int BX>
hipError_t launch_stepS_cl_shape(StepArgs a, hipStream_t s) {
    a.nbx = (a.nx + BX - 1) / BX;
    const dim3 grid(a.nbx * a.nby);
    hipLaunchKernelGGL((stepS_kernel_cl<BX, S>), grid, dim3(stepS_threads<BX, S, true>()), 0, s, a);
    return hipGetLastError();
}

template <int S>
hipError_t launch_stepS_cl(StepArgs a, int bx, hipStream_t s) {
    a.nby = (a.ny + a.strip_h - 1) / a.strip_h;
    a.n_xcd = kXcds;
    switch (closure_stepS_bx(bx)) {
    case 128:
        return launch_stepS_cl_shape<S, 128>(a, s);
    case 160:
        return launch_stepS_cl_shape<S, 160>(a, s);
    case 192:
        return launch_stepS_cl_shape<S, 192>(a, s);
    default:
        return launch_stepS_cl_shape<S, 224>(a, s);
    }
}

// One S-step launch with tile width BX.
template <int MODEL, int S, int ST, int BX>
hipError_t launch_stepS_shape(StepArgs a, hipStream_t s) {
    a.nbx = (a.nx + BX - 1) / BX;
    const dim3 grid(a.nbx * a.nby);
    hipLaunchKernelGGL((stepS_kernel_lds<MODEL, BX, S, ST>), grid, dim3(stepS_threads<BX, S>()), 0, s, a);
    return hipGetLastError();
}

template <int MODEL, int S, int ST>
hipError_t launch_stepS_m(StepArgs a, int bx, hipStream_t s) {
    a.nby = (a.ny + a.strip_h - 1) / a.strip_h;
    a.n_xcd = kXcds;
    switch (bx) {
    case 64:
        return launch_stepS_shape<MODEL, S, ST, 64>(a, s);
    case 96:
        return launch_stepS_shape<MODEL, S, ST, 96>(a, s);
    case 128:
        return launch_stepS_shape<MODEL, S, ST, 128>(a, s);
    case 160:
        return launch_stepS_shape<MODEL, S, ST, 160>(a, s);
    case 192:
        return launch_stepS_shape<MODEL, S, ST, 192>(a, s);
    case 224:
        return launch_stepS_shape<MODEL, S, ST, 224>(a, s);
    case 240:
        return launch_stepS_shape<MODEL, S, ST, 240>(a, s);
    case 288:
        return launch_stepS_shape<MODEL, S, ST, 288>(a, s);
    case 320:
        return launch_stepS_shape<MODEL, S, ST, 320>(a, s);
    default:
        return launch_stepS_shape<MODEL, S, ST, 256>(a, s);
    }
}

template <int ST>
hipError_t launch_stepS_st(const lbac_ctx* h, const StepArgs& a, int S) {
    const bool conv = h->p.model == LBAC_MODEL_CONVENTIONAL;
    if (S == 3)
        return conv ? launch_stepS_m<MODEL_CONVENTIONAL, 3, ST>(a, h->bx, h->stream)
                    : launch_stepS_m<MODEL_IMPROVED, 3, ST>(a, h->bx, h->stream);
    return conv ? launch_stepS_m<MODEL_CONVENTIONAL, 2, ST>(a, h->bx, h->stream)
                : launch_stepS_m<MODEL_IMPROVED, 2, ST>(a, h->bx, h->stream);
}

// Steps k .. k + S - 1 of the current run in one launch, from pop[src] into pop[1 - src].
hipError_t launch_stepS(const lbac_ctx* h, int src, int32_t k, int S) {
    const StepArgs a = make_args(h, src, k);
    if (h->closure)
        return S == 3 ? launch_stepS_cl<3>(a, h->bx, h->stream) : launch_stepS_cl<2>(a, h->bx, h->stream);
    switch (h->p.precision) {
    case LBAC_F32_F16STORE:
        return launch_stepS_st<ST_F16>(h, a, S);
    case LBAC_F32_BF16STORE:
        return launch_stepS_st<ST_BF16>(h, a, S);
    default:
        return launch_stepS_st<ST_PLAIN>(h, a, S);
    }
}

// Queues `n` steps starting at offset k0 of the current run from pop[src]:
// S steps per launch where the variant allows, single steps for the rest.
// *flips gets the number of launches (buffer swaps).
hipError_t launch_steps(const lbac_ctx* h, int src, int64_t k0, int64_t n, int64_t* flips) {
    int64_t f = 0;
    hipError_t e = hipSuccess;
    const int S = launch_steps_of(h);
    for (int64_t k = 0; k < n && e == hipSuccess;) {
        const int cur = src ^ (int)(f & 1);
        if (S > 1 && n - k >= S) {
            e = launch_stepS(h, cur, (int32_t)(k0 + k), S);
            k += S;
        } else {
            e = launch_step(h, cur, (int32_t)(k0 + k));
            k += 1;
        }
        ++f;
    }
    *flips = f;
    return e;
}

template <typename R, int ST>
hipError_t launch_aux_t(const lbac_ctx* h, int which, const StepArgs& a, double* out, const double* ref,
                        const double* phi0) {
    dim3 g2((a.nx + 255) / 256, a.ny);
    switch (which) {
    case 0:
        hipLaunchKernelGGL((init_kernel<R, ST>), g2, dim3(256), 0, h->stream, a, phi0);
        break;
    case 1:
        hipLaunchKernelGGL((phi_kernel<R, ST>), g2, dim3(256), 0, h->stream, a, out);
        break;
    default:
        hipLaunchKernelGGL((row_sums_kernel<R, ST>), dim3(a.ny), dim3(kRedThreads), 0, h->stream, a, ref,
                           static_cast<R*>(h->rows));
        hipLaunchKernelGGL((reduce_rows_kernel<R>), dim3(1), dim3(kRedThreads), 0, h->stream,
                           static_cast<const R*>(h->rows), a.ny, h->red5);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_aux(const lbac_ctx* h, int which, const StepArgs& a, double* out, const double* ref,
                      const double* phi0) {
    switch (h->p.precision) {
    case LBAC_F64:
        return launch_aux_t<double, ST_PLAIN>(h, which, a, out, ref, phi0);
    case LBAC_F32:
        return launch_aux_t<float, ST_PLAIN>(h, which, a, out, ref, phi0);
    case LBAC_F32_F16STORE:
        return launch_aux_t<float, ST_F16>(h, which, a, out, ref, phi0);
    default:
        return launch_aux_t<float, ST_BF16>(h, which, a, out, ref, phi0);
    }
}

int validate(const lbac_params* p, std::string& why) {
    if (!p) return why = "params is NULL", LBAC_EINVAL;
    // at most 2^27 nodes: every padded plane then stays below 2 GiB, which the
    // kernels' 32-bit byte offsets and buffer ranges rely on
    if (p->nx < 1 || p->ny < 1 || p->nx > 65536 || p->ny > 65536 || (int64_t)p->nx * p->ny > (1ll << 27))
        return why = "grid size out of range (1 <= nx, ny <= 65536, nx * ny <= 2^27)", LBAC_EINVAL;
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return why = "tau must exceed 1/2", LBAC_EINVAL;
    if (!(p->eps > 0.0) || !std::isfinite(p->eps)) return why = "eps must be positive", LBAC_EINVAL;
    if (!(p->delta >= 0.0) || !std::isfinite(p->delta)) return why = "delta must be >= 0", LBAC_EINVAL;
    if (p->vel_kind < LBAC_VEL_ZERO || p->vel_kind > LBAC_VEL_VORTEX_PAPER) return why = "bad vel_kind", LBAC_EINVAL;
    if ((p->vel_kind == LBAC_VEL_VORTEX || p->vel_kind == LBAC_VEL_VORTEX_PAPER) && !(p->period_T > 0.0))
        return why = "vortex needs period_T > 0", LBAC_EINVAL;
    if (p->precision < LBAC_F64 || p->precision > LBAC_F32_BF16STORE) return why = "bad precision", LBAC_EINVAL;
    if (p->model != LBAC_MODEL_IMPROVED && p->model != LBAC_MODEL_CONVENTIONAL) return why = "bad model", LBAC_EINVAL;
    if (p->alloc && (!p->alloc->alloc || !p->alloc->free)) return why = "allocator without alloc/free", LBAC_EINVAL;
    std::vector<double> tab;
    build_velocity(*p, tab);
    double ma = 0, mb = 0, mc = 0, md = 0;
    for (int i = 0; i < p->nx; ++i) {
        ma = std::max(ma, std::fabs(tab[i]));
        mb = std::max(mb, std::fabs(tab[p->nx + i]));
    }
    for (int j = 0; j < p->ny; ++j) {
        mc = std::max(mc, std::fabs(tab[2 * (size_t)p->nx + j]));
        md = std::max(md, std::fabs(tab[2 * (size_t)p->nx + p->ny + j]));
    }
    if (!std::isfinite(ma * mc + mb * md) || ma * mc + mb * md >= 1.0 / 3.0)
        return why = "velocity too large: max |u| + |v| must stay below 1/3", LBAC_EINVAL;
    return LBAC_OK;
}

}  // namespace

int lbac_host::create(const lbac_params* p, const double* phi0, bool phi0_on_device, lbac_ctx** out) {
    if (!out) return LBAC_EINVAL;
    *out = nullptr;
    std::string why;
    int rc = validate(p, why);
    if (rc != LBAC_OK) return rc;
    if (!phi0) return LBAC_EINVAL;
    const size_t n = (size_t)p->nx * p->ny;
    if (!phi0_on_device)
        for (size_t i = 0; i < n; ++i)
            if (!std::isfinite(phi0[i])) return LBAC_EINVAL;

    lbac_ctx* h = new (std::nothrow) lbac_ctx();
    if (!h) return LBAC_ENOMEM;
    h->p = *p;
    if (p->alloc) {
        h->alloc = *p->alloc;
        h->has_alloc = true;
    }
    h->p.alloc = nullptr;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return LBAC_EDEVICE;
    }
    auto bail = [&](int code) {
        release(h);
        delete h;
        return code;
    };
    if (p->stream) {
        h->stream = (hipStream_t)p->stream;
    } else {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) return bail(LBAC_EDEVICE);
        h->own_stream = true;
    }
    h->storage = p->precision == LBAC_F64 || p->precision == LBAC_F32 ? ST_PLAIN
                 : (p->precision == LBAC_F32_F16STORE ? ST_F16 : ST_BF16);
    h->elem_bytes = p->precision == LBAC_F64 ? 8 : (p->precision == LBAC_F32 ? 4 : 2);
    h->nplanes = h->storage == ST_PLAIN ? 9 : 8;
    // rows are an odd multiple of 256 bytes apart: with a power-of-two row
    // pitch, rows processed at the same time by different strips and XCDs
    // land on the same HBM channels
    {
        const int unit = 256 / h->elem_bytes;
        h->pitch = (p->nx + unit - 1) / unit * unit;
        if ((h->pitch / unit) % 2 == 0) h->pitch += unit;
    }
    h->plane_stride = (int64_t)h->pitch * p->ny + kPlanePadBytes / h->elem_bytes;
    // default launch shape: full-width blocks when the grid allows, strips of 64 rows
    h->bx = p->nx >= 256 ? 256 : (p->nx >= 128 ? 128 : 64);
    h->strip_h = std::min(64, p->ny);
    const size_t pop_bytes = (size_t)h->plane_stride * h->nplanes * h->elem_bytes;
    const size_t phis_bytes = ((size_t)h->pitch * p->ny + 64) * sizeof(float);
    for (int i = 0; i < 2; ++i) {
        h->pop[i] = dev_alloc(h, pop_bytes);
        if (!h->pop[i]) return bail(LBAC_ENOMEM);
        if (h->storage != ST_PLAIN) {
            h->phis[i] = (float*)dev_alloc(h, phis_bytes);
            if (!h->phis[i]) return bail(LBAC_ENOMEM);
        }
    }
    std::vector<double> tab;
    build_velocity(h->p, tab);
    h->vtab = (double*)dev_alloc(h, tab.size() * sizeof(double));
    h->vtabf = (float*)dev_alloc(h, tab.size() * sizeof(float));
    std::vector<float> tabf(tab.begin(), tab.end());
    h->t_dev = (int64_t*)dev_alloc(h, 64);
    h->rows = dev_alloc(h, 10 * sizeof(double) * (size_t)p->ny);  // five compensated pairs per row
    h->red5 = (double*)dev_alloc(h, 64);
    h->dtmp = (double*)dev_alloc(h, n * sizeof(double));
    if (!h->vtab || !h->vtabf || !h->t_dev || !h->rows || !h->red5 || !h->dtmp) return bail(LBAC_ENOMEM);
    if (hipHostMalloc((void**)&h->host5, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        h->host5 = nullptr;
        return bail(LBAC_ENOMEM);
    }
    if (hipMemcpyAsync(h->vtab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, h->stream) !=
            hipSuccess ||
        hipMemcpyAsync(h->vtabf, tabf.data(), tabf.size() * sizeof(float), hipMemcpyHostToDevice, h->stream) !=
            hipSuccess)
        return bail(LBAC_EDEVICE);
    const double* src0 = phi0;
    if (!phi0_on_device) {
        if (hipMemcpyAsync(h->dtmp, phi0, n * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess)
            return bail(LBAC_EDEVICE);
        src0 = h->dtmp;
    }
    hipLaunchKernelGGL(set_time_kernel, dim3(1), dim3(64), 0, h->stream, h->t_dev, (int64_t)0);
    StepArgs a = make_args(h, 1, 0);  // dst = pop[0]
    if (launch_aux(h, 0, a, nullptr, nullptr, src0) != hipSuccess) return bail(LBAC_EDEVICE);
    if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(LBAC_EDEVICE);
    h->cur = 0;
    h->t = 0;
    *out = h;
    return LBAC_OK;
}

void lbac_host::destroy(lbac_ctx* h) {
    if (!h) return;
    DeviceGuard g(h->device);
    release(h);
    delete h;
}

namespace {

int capture_graph(lbac_ctx* h, int parity) {
    if (h->gexec[parity] && h->gexec_chunk[parity] == h->graph_chunk) return LBAC_OK;
    if (h->gexec[parity]) {
        (void)hipGraphExecDestroy(h->gexec[parity]);
        h->gexec[parity] = nullptr;
    }
    HIPCHK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    int64_t flips = 0;
    hipError_t e = launch_steps(h, parity, 0, h->graph_chunk, &flips);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, h->stream, h->t_dev, (int64_t)h->graph_chunk);
        e = hipGetLastError();
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(h->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(h, LBAC_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(h, LBAC_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    h->gexec[parity] = ge;
    h->gexec_chunk[parity] = h->graph_chunk;
    h->gexec_flips[parity] = (int)(flips & 1);
    return LBAC_OK;
}

// Runs the row-sum and row-reduce kernels; results land in host5[0..4].
int reduce5(lbac_ctx* h, const double* ref_dev) {
    StepArgs a = make_args(h, h->cur, 0);
    HIPCHK(h, launch_aux(h, 2, a, nullptr, ref_dev, nullptr));
    HIPCHK(h, hipMemcpyAsync(h->host5, h->red5, 5 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return LBAC_OK;
}

}  // namespace

extern "C" {

void lbac_default_params(lbac_params* p, int32_t nx, int32_t ny) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->nx = nx;
    p->ny = ny;
    p->eps = 1.0;
    p->tau = 0.8;
    p->delta = 1e-10;
    p->vel_kind = LBAC_VEL_VORTEX;
    p->U = 0.02;
    p->period_T = 2000.0;
    p->cx = 0.5 * nx;
    p->cy = 0.5 * ny;
    p->precision = LBAC_F64;
    p->model = LBAC_MODEL_IMPROVED;
}

int lbac_init(const lbac_params* p, const double* phi0, lbac_ctx** out) { return create(p, phi0, false, out); }

int lbac_init_device(const lbac_params* p, const double* phi0_device, lbac_ctx** out) {
    return create(p, phi0_device, true, out);
}

int lbac_free(lbac_ctx* h) {
    if (!h) return LBAC_OK;
    if (h->in_batch) return fail(h, LBAC_ESTATE, "context belongs to a batch; free the batch");
    destroy(h);
    return LBAC_OK;
}

int lbac_step(lbac_ctx* h, int64_t n) {
    if (!h) return LBAC_EINVAL;
    if (h->failed) return fail(h, LBAC_ESTATE, "the batch run of this instance timed out; its state is undefined");
    if (n < 0) return fail(h, LBAC_EINVAL, "negative step count");
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, LBAC_EDEVICE, "hipSetDevice failed");
    int64_t done = 0;
    if (h->graph_chunk > 0) {
        while (n - done >= h->graph_chunk) {
            int rc = capture_graph(h, h->cur);
            if (rc != LBAC_OK) return rc;
            HIPCHK(h, hipGraphLaunch(h->gexec[h->cur], h->stream));
            done += h->graph_chunk;
            h->t += h->graph_chunk;
            h->cur ^= h->gexec_flips[h->cur];  // parity of the chunk's launches
        }
    }
    const int64_t r = n - done;
    if (r > 0) {
        int64_t flips = 0;
        HIPCHK(h, launch_steps(h, h->cur, 0, r, &flips));
        hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, h->stream, h->t_dev, r);
        HIPCHK(h, hipGetLastError());
        h->cur ^= (int)(flips & 1);
        h->t += r;
    }
    return LBAC_OK;
}

int lbac_phi_device(lbac_ctx* h, double* out_device) {
    if (!h || !out_device) return LBAC_EINVAL;
    if (h->failed) return fail(h, LBAC_ESTATE, "the batch run of this instance timed out; its state is undefined");
    DeviceGuard g(h->device);
    StepArgs a = make_args(h, h->cur, 0);
    HIPCHK(h, launch_aux(h, 1, a, out_device, nullptr, nullptr));
    return LBAC_OK;
}

int lbac_phi(lbac_ctx* h, double* out) {
    if (!h || !out) return LBAC_EINVAL;
    if (h->failed) return fail(h, LBAC_ESTATE, "the batch run of this instance timed out; its state is undefined");
    DeviceGuard g(h->device);
    int rc = lbac_phi_device(h, h->dtmp);
    if (rc != LBAC_OK) return rc;
    HIPCHK(h, hipMemcpyAsync(out, h->dtmp, sizeof(double) * (size_t)h->p.nx * h->p.ny, hipMemcpyDeviceToHost,
                             h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return LBAC_OK;
}

int lbac_mass(lbac_ctx* h, double* out) {
    if (!h || !out) return LBAC_EINVAL;
    if (h->failed) return fail(h, LBAC_ESTATE, "the batch run of this instance timed out; its state is undefined");
    DeviceGuard g(h->device);
    int rc = reduce5(h, nullptr);
    if (rc != LBAC_OK) return rc;
    *out = h->host5[0];
    if (!std::isfinite(*out)) return fail(h, LBAC_ENONFINITE, "mass is not finite");
    return LBAC_OK;
}

int lbac_shape_error(lbac_ctx* h, const double* ref, double* e1, double* e2) {
    if (!h || !ref) return LBAC_EINVAL;
    if (h->failed) return fail(h, LBAC_ESTATE, "the batch run of this instance timed out; its state is undefined");
    DeviceGuard g(h->device);
    const size_t n = (size_t)h->p.nx * h->p.ny;
    HIPCHK(h, hipMemcpyAsync(h->dtmp, ref, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
    int rc = reduce5(h, h->dtmp);
    if (rc != LBAC_OK) return rc;
    const double* r = h->host5;
    const double v1 = r[1] / r[2], v2 = std::sqrt(r[3] / r[4]);
    if (e1) *e1 = v1;
    if (e2) *e2 = v2;
    if (!std::isfinite(v1) || !std::isfinite(v2)) return fail(h, LBAC_ENONFINITE, "shape error is not finite");
    return LBAC_OK;
}

int lbac_time(lbac_ctx* h, int64_t* t) {
    if (!h || !t) return LBAC_EINVAL;
    *t = h->t;
    return LBAC_OK;
}

int lbac_get_state(lbac_ctx* h, void* buf, size_t* bytes) {
    if (!h || !bytes) return LBAC_EINVAL;
    if (h->failed) return fail(h, LBAC_ESTATE, "the batch run of this instance timed out; its state is undefined");
    const size_t plane = (size_t)h->pitch * h->p.ny * h->elem_bytes;
    const size_t phib = h->storage == ST_PLAIN ? 0 : (size_t)h->pitch * h->p.ny * sizeof(float);
    const size_t need = 64 + plane * h->nplanes + phib;
    if (!buf) {
        *bytes = need;
        return LBAC_OK;
    }
    if (*bytes < need) return fail(h, LBAC_EINVAL, "state buffer too small");
    DeviceGuard g(h->device);
    unsigned char* b = (unsigned char*)buf;
    std::memset(b, 0, 64);
    uint64_t magic = kStateMagic;
    int32_t hdr[4] = {h->p.nx, h->p.ny, h->p.precision, h->nplanes};
    std::memcpy(b, &magic, 8);
    std::memcpy(b + 8, hdr, 16);
    std::memcpy(b + 24, &h->t, 8);
    unsigned char* d = b + 64;
    for (int q = 0; q < h->nplanes; ++q) {
        HIPCHK(h, hipMemcpyAsync(d + q * plane, (char*)h->pop[h->cur] + (size_t)q * h->plane_stride * h->elem_bytes,
                                 plane, hipMemcpyDeviceToHost, h->stream));
    }
    if (phib) HIPCHK(h, hipMemcpyAsync(d + h->nplanes * plane, h->phis[h->cur], phib, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    *bytes = need;
    return LBAC_OK;
}

int lbac_set_state(lbac_ctx* h, const void* buf, size_t bytes) {
    if (!h || !buf) return LBAC_EINVAL;
    if (h->failed) return fail(h, LBAC_ESTATE, "the batch run of this instance timed out; its state is undefined");
    const size_t plane = (size_t)h->pitch * h->p.ny * h->elem_bytes;
    const size_t phib = h->storage == ST_PLAIN ? 0 : (size_t)h->pitch * h->p.ny * sizeof(float);
    const size_t need = 64 + plane * h->nplanes + phib;
    if (bytes < need) return fail(h, LBAC_EINVAL, "state blob too small");
    const unsigned char* b = (const unsigned char*)buf;
    uint64_t magic;
    int32_t hdr[4];
    int64_t t;
    std::memcpy(&magic, b, 8);
    std::memcpy(hdr, b + 8, 16);
    std::memcpy(&t, b + 24, 8);
    if (magic != kStateMagic || hdr[0] != h->p.nx || hdr[1] != h->p.ny || hdr[2] != h->p.precision ||
        hdr[3] != h->nplanes || t < 0)
        return fail(h, LBAC_EINVAL, "state blob does not match this context");
    DeviceGuard g(h->device);
    const unsigned char* d = b + 64;
    for (int q = 0; q < h->nplanes; ++q)
        HIPCHK(h, hipMemcpyAsync((char*)h->pop[h->cur] + (size_t)q * h->plane_stride * h->elem_bytes, d + q * plane,
                                 plane, hipMemcpyHostToDevice, h->stream));
    if (phib) HIPCHK(h, hipMemcpyAsync(h->phis[h->cur], d + h->nplanes * plane, phib, hipMemcpyHostToDevice, h->stream));
    hipLaunchKernelGGL(set_time_kernel, dim3(1), dim3(64), 0, h->stream, h->t_dev, t);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->t = t;
    return LBAC_OK;
}

int lbac_set_launch(lbac_ctx* h, int32_t variant, int32_t bx, int32_t strip_h) {
    if (!h) return LBAC_EINVAL;
    if (variant < LBAC_KERNEL_BLOCK || variant > LBAC_KERNEL_FUSED3) return fail(h, LBAC_EINVAL, "unknown kernel variant");
    if ((variant == LBAC_KERNEL_FUSED2 || variant == LBAC_KERNEL_FUSED3) && h->p.precision == LBAC_F64)
        return fail(h, LBAC_EINVAL, "the multi-step variants need FP32 collision (LBAC_F32 or a 16-bit storage)");
    const int S = variant == LBAC_KERNEL_FUSED2 ? 2 : (variant == LBAC_KERNEL_FUSED3 ? 3 : 1);
    if (!(S == 1 ? one_step_bx(bx) : stepS_bx(bx)))
        return fail(h, LBAC_EINVAL, "bx must be 64, 128 or 256 (with the multi-step variants any multiple of 32 from "
                                    "64 to 320, or 240)");
    if (strip_h < 1) return fail(h, LBAC_EINVAL, "strip_h must be >= 1");
    h->variant = variant;
    h->bx = bx;
    h->strip_h = std::min(strip_h, h->p.ny);
    drop_graphs(h);
    return LBAC_OK;
}

int lbac_get_launch(lbac_ctx* h, int32_t* variant, int32_t* bx, int32_t* strip_h) {
    if (!h) return LBAC_EINVAL;
    if (variant) *variant = h->variant;
    if (bx) *bx = h->bx;
    if (strip_h) *strip_h = h->strip_h;
    return LBAC_OK;
}

int lbac_autotune(lbac_ctx* h, int32_t steps, double* us_per_step) {
    if (!h || steps < 1) return LBAC_EINVAL;
    if (h->failed) return fail(h, LBAC_ESTATE, "the batch run of this instance timed out; its state is undefined");
    DeviceGuard g(h->device);
    const int bxs[10] = {64, 96, 128, 160, 192, 224, 240, 256, 288, 320};
    // strip heights: multiples of 8 up to 256 and powers of two up to 512 (the
    // count of tiles against the workgroups resident at once decides how full
    // the last round of tiles is, so heights between the powers of two can
    // win), and ny split into k equal strips (so that a grid whose tiles all
    // fit on the device at once marches long strips in step)
    std::vector<int> hs;
    for (int sh = 8; sh <= 256; sh += 8) hs.push_back(std::min(sh, h->p.ny));
    hs.push_back(std::min(512, h->p.ny));
    for (int k = 1; k <= 32; ++k) hs.push_back((h->p.ny + k - 1) / k);
    std::sort(hs.begin(), hs.end());
    hs.erase(std::unique(hs.begin(), hs.end()), hs.end());
    hipEvent_t e0, e1;
    HIPCHK(h, hipEventCreate(&e0));
    HIPCHK(h, hipEventCreate(&e1));
    const int keep_bx = h->bx, keep_h = h->strip_h, keep_v = h->variant;
    int best_bx = keep_bx, best_h = keep_h, best_v = keep_v;
    float best = 1e30f;
    hipError_t e = hipSuccess;
    const int last_var = stepS_allowed(h) ? LBAC_KERNEL_FUSED3 : LBAC_KERNEL_BLOCK_DEEP;
    for (int var = LBAC_KERNEL_BLOCK; var <= last_var && e == hipSuccess; ++var)
    for (int bx : bxs) {
        const int S = var == LBAC_KERNEL_FUSED2 ? 2 : (var == LBAC_KERNEL_FUSED3 ? 3 : 1);
        if (bx > 64 && bx / 2 >= h->p.nx) continue;
        if (S == 1 ? !one_step_bx(bx) : !stepS_bx(bx)) continue;
        if (S > 1 && h->closure && closure_stepS_bx(bx) != bx) continue;
        for (int sh : hs) {
            h->variant = var;
            h->bx = bx;
            h->strip_h = std::min(sh, h->p.ny);
            // repeated launches from pop[cur] into the scratch buffer: the state
            // is untouched; an S-step launch counts as S steps
            const int S = launch_steps_of(h);
            auto one = [&]() { return S > 1 ? launch_stepS(h, h->cur, 0, S) : launch_step(h, h->cur, 0); };
            for (int w = 0; w < 2 && e == hipSuccess; ++w) e = one();
            if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
            for (int s = 0; s < steps && e == hipSuccess; ++s) e = one();
            if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) break;
            ms /= (float)S;
            if (ms < best) {
                best = ms;
                best_v = var;
                best_bx = bx;
                best_h = h->strip_h;
            }
        }
        if (e != hipSuccess) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->variant = best_v;
    h->bx = best_bx;
    h->strip_h = best_h;
    drop_graphs(h);
    if (e != hipSuccess) {
        h->variant = keep_v;
        h->bx = keep_bx;
        h->strip_h = keep_h;
        return fail(h, LBAC_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
    }
    if (us_per_step) *us_per_step = 1000.0 * best / steps;
    return LBAC_OK;
}

int lbac_set_graph_chunk(lbac_ctx* h, int32_t chunk) {
    if (!h) return LBAC_EINVAL;
    if (chunk < 0 || (chunk & 1)) return fail(h, LBAC_EINVAL, "graph chunk must be an even number >= 0");
    h->graph_chunk = chunk;
    drop_graphs(h);
    return LBAC_OK;
}

int lbac_set_closure(lbac_ctx* h, const float* params, float theta) {
    if (!h) return LBAC_EINVAL;
    DeviceGuard g(h->device);
    if (!params) {
        h->closure = false;
        drop_graphs(h);
        return LBAC_OK;
    }
    if (h->p.precision != LBAC_F32) return fail(h, LBAC_EINVAL, "the learned closure runs with LBAC_F32 only");
    if (h->in_batch) return fail(h, LBAC_EINVAL, "the learned closure is not available for batch instances");
    if (!(theta >= 0.f) || !(theta < 0.5f)) return fail(h, LBAC_EINVAL, "theta must lie in [0, 0.5)");
    for (int i = 0; i < LBAC_MLP_NPARAM; ++i)
        if (!std::isfinite(params[i])) return fail(h, LBAC_EINVAL, "non-finite closure parameter");
    if (!h->cl_param) {
        h->cl_param = (float*)dev_alloc(h, sizeof(float) * LBAC_MLP_NPARAM);
        h->cl_w = (uint16_t*)dev_alloc(h, sizeof(uint16_t) * kClWN);
        h->cl_b = (float*)dev_alloc(h, sizeof(float) * kClBN);
        h->cl_words = (h->p.nx + 63) / 64;
        h->cl_mask = (uint64_t*)dev_alloc(h, sizeof(uint64_t) * (size_t)h->cl_words * h->p.ny);
        h->cl_list = (int32_t*)dev_alloc(h, sizeof(int32_t) * (size_t)h->p.nx * h->p.ny);
        h->cl_count = (uint32_t*)dev_alloc(h, 256);
        if (!h->cl_param || !h->cl_w || !h->cl_b || !h->cl_mask || !h->cl_list || !h->cl_count)
            return fail(h, LBAC_ENOMEM, "closure buffers");
    }
    HIPCHK(h, hipMemcpyAsync(h->cl_param, params, sizeof(float) * LBAC_MLP_NPARAM, hipMemcpyHostToDevice, h->stream));
    hipLaunchKernelGGL(closure_pack_kernel, dim3((64 * 64 + 255) / 256), dim3(256), 0, h->stream, h->cl_param, h->cl_w,
                       h->cl_b);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->closure = true;
    h->cl_theta = theta;
    drop_graphs(h);
    return LBAC_OK;
}

int lbac_copy_ceiling(lbac_ctx* h, int32_t launches, double* us_per_launch) {
    if (!h || launches < 1 || !us_per_launch) return LBAC_EINVAL;
    DeviceGuard g(h->device);
    // copies pop[cur] into the other buffer, which the next step overwrites anyway
    StepArgs a = make_args(h, h->cur, 0);
    a.n_xcd = kXcds;
    hipEvent_t e0, e1;
    HIPCHK(h, hipEventCreate(&e0));
    HIPCHK(h, hipEventCreate(&e1));
    hipError_t e = hipSuccess;
    float best = 1e30f;
    for (int sh : {8, 16, 32, 64}) {
        a.strip_h = std::min(sh, a.ny);
        a.nby = (a.ny + a.strip_h - 1) / a.strip_h;
        const dim3 grid(((a.nx + 255) / 256) * a.nby), block(256);
        auto launch = [&]() {
            // plain storage: 9 planes; shifted storage: 8 16-bit planes plus the FP32 phi* plane
            if (h->elem_bytes == 8)
                hipLaunchKernelGGL((pattern_copy_kernel<uint64_t, 9>), grid, block, 0, h->stream, a);
            else if (h->elem_bytes == 4)
                hipLaunchKernelGGL((pattern_copy_kernel<uint32_t, 9>), grid, block, 0, h->stream, a);
            else
                hipLaunchKernelGGL((pattern_copy_kernel<uint16_t, 8>), grid, block, 0, h->stream, a);
            return hipGetLastError();
        };
        e = launch();
        if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
        for (int k = 0; k < launches && e == hipSuccess; ++k) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) break;
        best = std::min(best, ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(h, LBAC_EDEVICE, std::string("copy ceiling: ") + hipGetErrorString(e));
    *us_per_launch = 1000.0 * best / launches;
    return LBAC_OK;
}

int lbac_bytes_per_node(lbac_ctx* h, double* bytes) {
    if (!h || !bytes) return LBAC_EINVAL;
    // read and write of every stored value once per launch
    *bytes = 2.0 * (h->nplanes * h->elem_bytes + (h->storage == ST_PLAIN ? 0 : 4));
    return LBAC_OK;
}

int lbac_steps_per_launch(lbac_ctx* h, int32_t* steps) {
    if (!h || !steps) return LBAC_EINVAL;
    *steps = launch_steps_of(h);
    return LBAC_OK;
}

void* lbac_stream(lbac_ctx* h) { return h ? (void*)h->stream : nullptr; }

const char* lbac_strerror(int code) {
    switch (code) {
    case LBAC_OK:
        return "ok";
    case LBAC_EINVAL:
        return "invalid argument";
    case LBAC_ENOMEM:
        return "out of memory";
    case LBAC_EDEVICE:
        return "device error";
    case LBAC_ENONFINITE:
        return "non-finite result";
    case LBAC_ESTATE:
        return "invalid state";
    default:
        return "unknown status";
    }
}

const char* lbac_last_error(lbac_ctx* h) { return h ? h->err.c_str() : "no context"; }

}  // extern "C"
