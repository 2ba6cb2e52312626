// Device code of the lbac library: the fused collide-and-stream step of the
// accurate interface-capturing LB scheme (H. Liang, arXiv:2203.05230,
// Sec. 2.2, Eq. (9)-(13)) and the small kernels around it (initialisation,
// phi, reductions).
//
// Storage.  The state between steps is the post-collision population
// f*_i(x, t-1), not yet streamed, in nine planes (SoA, x fastest, rows
// `pitch` elements apart).  A step PULLS: the pre-collision population at x
// is f_i(x, t) = f*_i(x - c_i, t-1).  In the shifted low-precision form the
// planes hold g_i = f*_i - w_i phi* for i = 1..8 in 16 bits plus phi* in FP32,
// with g_0 = -(g_1 + .. + g_8), so the nine populations always sum to phi*.
//
// Step kernel dataflow (one launch per step).  A block owns a strip of bx
// columns and strip_h rows and marches up it one row per iteration.  At
// iteration `it` it loads lattice row r of every plane (own columns plus a
// two-column halo) into a three-row LDS ring, forms phi (Eq. (12)) and psi
// (Eq. (13)) on row r-1 over the strip plus a one-column halo, and updates
// row r-2: the isotropic gradient of psi from the three-row psi ring, the
// normal, the sharpening term, d_t(phi u), the forcing of Eq. (11), the BGK
// collision of Eq. (9), and the store of f*.  Every population row is read
// from HBM once per strip (plus two halo columns and four halo rows); phi at
// t-1, needed by the explicit-Euler d_t(phi u), is the plain sum of the nine
// stored values at x (collision conserves the sum), so no extra plane is
// read or written.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbac {

// ---------------------------------------------------------------------------
// D2Q9 lattice (Sec. 2.2, after Eq. (10)); order rest, E, N, W, S, NE, NW, SW, SE.
__host__ __device__ constexpr int cx(int q) {
    return q == 1 || q == 5 || q == 8 ? 1 : (q == 3 || q == 6 || q == 7 ? -1 : 0);
}
__host__ __device__ constexpr int cy(int q) {
    return q == 2 || q == 5 || q == 6 ? 1 : (q == 4 || q == 7 || q == 8 ? -1 : 0);
}
template <typename R>
__host__ __device__ constexpr R wq(int q) {
    return q == 0 ? R(4) / R(9) : (q < 5 ? R(1) / R(9) : R(1) / R(36));
}

enum Storage { ST_PLAIN = 0, ST_F16 = 1, ST_BF16 = 2 };
enum Model { MODEL_IMPROVED = 0, MODEL_CONVENTIONAL = 1 };

struct StepArgs {
    const void* src;        // stored populations at t-1 (plain: 9 planes; shifted: 8 planes)
    void* dst;              // stored populations at t
    const float* src_phi;   // shifted storage: phi* plane of src
    float* dst_phi;         // shifted storage: phi* plane of dst
    int64_t plane_stride;   // elements between planes
    int32_t pitch;          // elements between rows
    int32_t nx, ny;
    int32_t strip_h;        // rows per block
    const double* vtab;     // Ax[nx], Bx[nx], Ay[ny], By[ny]: u = s(t) Ax Ay, v = s(t) Bx By
    const int64_t* t_dev;   // step count at the start of this launch sequence
    int32_t k;              // this launch is step t_dev[0] + k
    double period_T;        // s(t) = cos(pi t / period_T) when > 0, else 1
    double eps, tau, delta;
};

__device__ __forceinline__ int wrap_idx(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Workgroup barrier that orders LDS only: in-flight global loads of the next
// row are not waited for, so they overlap the arithmetic of this row.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ double time_factor(double period, int64_t t) {
    return period > 0.0 ? cos(3.14159265358979323846 * (double)t / period) : 1.0;
}

// ---- storage access --------------------------------------------------------
template <typename R, int ST>
struct Store;

template <typename R>
struct Store<R, ST_PLAIN> {
    static constexpr bool kShifted = false;
    // the nine stored post-collision values at element offset `off`
    __device__ __forceinline__ static void load(const StepArgs& a, int64_t off, R (&v)[9]) {
        const R* s = static_cast<const R*>(a.src);
#pragma unroll
        for (int q = 0; q < 9; ++q) v[q] = s[q * a.plane_stride + off];
    }
    __device__ __forceinline__ static R load_one(const StepArgs& a, int64_t off, int q) {
        return static_cast<const R*>(a.src)[q * a.plane_stride + off];
    }
    __device__ __forceinline__ static void store(const StepArgs& a, int64_t off, const R (&v)[9], R /*phi*/) {
        R* d = static_cast<R*>(a.dst);
#pragma unroll
        for (int q = 0; q < 9; ++q) d[q * a.plane_stride + off] = v[q];
    }
};

template <typename H>
__device__ __forceinline__ float h2f(H h);
template <>
__device__ __forceinline__ float h2f<__half>(__half h) { return __half2float(h); }
template <>
__device__ __forceinline__ float h2f<__hip_bfloat16>(__hip_bfloat16 h) { return __bfloat162float(h); }
template <typename H>
__device__ __forceinline__ H f2h(float f);
template <>
__device__ __forceinline__ __half f2h<__half>(float f) { return __float2half_rn(f); }
template <>
__device__ __forceinline__ __hip_bfloat16 f2h<__hip_bfloat16>(float f) { return __float2bfloat16(f); }

// Shifted 16-bit storage.  load() returns v[0] = phi* and v[i] = w_i phi* + g_i
// (i >= 1); the rest population f_0 = phi* - sum_{i>=1} v_i is never formed
// in FP32: phi(x) = phi*(x) + sum_{i>=1} [v_i(x - c_i) - v_i(x)] is summed in
// FP64 and rounded once, so the mass carried by phi* changes only by that one
// unbiased rounding per node and step.
template <typename H>
struct StoreShifted {
    static constexpr bool kShifted = true;
    __device__ __forceinline__ static void load(const StepArgs& a, int64_t off, float (&v)[9]) {
        const H* s = static_cast<const H*>(a.src);
        const float ph = a.src_phi[off];
        v[0] = ph;
#pragma unroll
        for (int q = 1; q < 9; ++q) v[q] = wq<float>(q) * ph + h2f<H>(s[(q - 1) * a.plane_stride + off]);
    }
    __device__ __forceinline__ static float load_one(const StepArgs& a, int64_t off, int q) {
        const H* s = static_cast<const H*>(a.src);
        const float ph = a.src_phi[off];
        if (q == 0) return ph;
        return wq<float>(q) * ph + h2f<H>(s[(q - 1) * a.plane_stride + off]);
    }
    __device__ __forceinline__ static void store(const StepArgs& a, int64_t off, const float (&v)[9], float phi) {
        H* d = static_cast<H*>(a.dst);
#pragma unroll
        for (int q = 1; q < 9; ++q) d[(q - 1) * a.plane_stride + off] = f2h<H>(v[q] - wq<float>(q) * phi);
        a.dst_phi[off] = phi;
    }
};
template <>
struct Store<float, ST_F16> : StoreShifted<__half> {};
template <>
struct Store<float, ST_BF16> : StoreShifted<__hip_bfloat16> {};

// ---- per-node pieces of the scheme ------------------------------------------
// psi of Eq. (13) with the clip of phi to [0, 1] described after it; the
// conventional model (Eq. (1)) takes its normal from phi itself.
template <typename R, int MODEL>
__device__ __forceinline__ R normal_source(R phi, R eps, R delta) {
    if (MODEL == MODEL_CONVENTIONAL) return phi;
    R pc = phi < R(0) ? R(0) : (phi > R(1) ? R(1) : phi);
    return eps * log((pc + delta) / (R(1) - pc + delta));
}

// Sharpening magnitude.  Improved model: (1 - tanh^2(psi/(2 eps)))/(4 eps)
// at psi of Eq. (13), which equals a b / (eps (a + b)^2) with a = phi_c + delta,
// b = 1 - phi_c + delta; that form has no cancellation in the bulk.
// Conventional model: phi (1 - phi) / eps.
template <typename R, int MODEL>
__device__ __forceinline__ R sharpening(R phi, R eps, R delta) {
    if (MODEL == MODEL_CONVENTIONAL) return phi * (R(1) - phi) / eps;
    R pc = phi < R(0) ? R(0) : (phi > R(1) ? R(1) : phi);
    R a = pc + delta, b = R(1) - pc + delta, s = R(1) + R(2) * delta;
    return a * b / (eps * s * s);
}

// ---------------------------------------------------------------------------
// The step kernel.  BX threads = BX lattice columns; one strip of strip_h rows.
template <typename R, int BX>
struct TileLds {
    R ring[3][9][BX + 4];  // rows r-2..r of every plane; index j <-> column x0 - 2 + j
    R sring[3][BX + 2];    // psi on rows r-3..r-1; index j <-> column x0 - 1 + j
};

// One step on the tile of column block `bxi` (BX columns) and strip `syi`
// (a.strip_h rows) at time t.  All BX threads of the block take part.
template <typename R, int ST, int MODEL, int BX>
__device__ __forceinline__ void step_tile(const StepArgs& a, int bxi, int syi, int64_t t, TileLds<R, BX>& lds) {
    auto& ring = lds.ring;
    auto& sring = lds.sring;
    const int l = threadIdx.x;
    const int x0 = bxi * BX;
    const int w = min(BX, a.nx - x0);
    const int ys = syi * a.strip_h;
    const int hh = min(a.strip_h, a.ny - ys);
    const bool act = l < w;
    const int x = x0 + l;
    // lanes 0..3 also load the halo columns x0-2, x0-1, x0+w, x0+w+1
    const int hj = l < 2 ? l : w + l;
    const int hx = wrap_idx(x0 - 2 + hj, a.nx);
    lds_barrier();  // the LDS may still be read by a previous tile of this block

    const bool first = (t == 0);
    const R s_now = R(time_factor(a.period_T, t));
    const R s_old = first ? s_now : R(time_factor(a.period_T, t - 1));
    const R Axl = act ? R(a.vtab[x]) : R(0);
    const R Bxl = act ? R(a.vtab[a.nx + x]) : R(0);
    const R eps = R(a.eps), delta = R(a.delta);
    const R omega = R(1) / R(a.tau);
    const R kforce = R(1) - R(0.5) / R(a.tau);

    R fprev[9], fcur[9];
    R phiprev = R(0), phicur = R(0);
    R P2 = R(0), P1 = R(0), P0 = R(0);  // own-column sums of stored values, rows r-2, r-1, r

    // prefetch registers for the next row
    R nv[9], hv[9];
    {
        const int ry = wrap_idx(ys - 2, a.ny);
        if (act) Store<R, ST>::load(a, (int64_t)ry * a.pitch + x, nv);
        if (l < 4) Store<R, ST>::load(a, (int64_t)ry * a.pitch + hx, hv);
    }

    const int iters = hh + 4;
    for (int it = 0; it < iters; ++it) {
        const int slot = it % 3;            // ring slot of row r = ys - 2 + it
        const int slot1 = (it + 2) % 3;     // row r - 1
        const int slot2 = (it + 1) % 3;     // row r - 2
        // ---- row r into the ring
        if (act) {
            R s = R(0);
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                ring[slot][q][l + 2] = nv[q];
                s += nv[q];
            }
            // phi at t-1 on this row: the stored sum (plain) or phi* itself (shifted)
            P0 = Store<R, ST>::kShifted ? nv[0] : s;
        }
        if (l < 4) {
#pragma unroll
            for (int q = 0; q < 9; ++q) ring[slot][q][hj] = hv[q];
        }
        // ---- prefetch row r + 1
        if (it + 1 < iters) {
            const int ry = wrap_idx(ys - 1 + it, a.ny);
            if (act) Store<R, ST>::load(a, (int64_t)ry * a.pitch + x, nv);
            if (l < 4) Store<R, ST>::load(a, (int64_t)ry * a.pitch + hx, hv);
        }
        lds_barrier();

        // ---- phi (Eq. (12)) and psi (Eq. (13)) on row r - 1
        if (it >= 2) {
            // pulled population q at ring column jc of row r-1 comes from row r-1-cy(q), column jc-cx(q)
            // phi at ring column jc of row r-1 (Eq. (12)); pulled values into f
            auto pulled_sum = [&](int jc, R (&f)[9]) -> R {
                if constexpr (Store<R, ST>::kShifted) {
                    double s = (double)ring[slot1][0][jc];
#pragma unroll
                    for (int q = 1; q < 9; ++q) {
                        const int sl = cy(q) == 1 ? slot2 : (cy(q) == 0 ? slot1 : slot);
                        f[q] = ring[sl][q][jc - cx(q)];
                        s += (double)f[q] - (double)ring[slot1][q][jc];
                    }
                    f[0] = R(0);  // not needed: the rest population is the remainder after collision
                    return R(s);
                } else {
                    R s = R(0);
#pragma unroll
                    for (int q = 0; q < 9; ++q) {
                        const int sl = cy(q) == 1 ? slot2 : (cy(q) == 0 ? slot1 : slot);
                        f[q] = ring[sl][q][jc - cx(q)];
                        s += f[q];
                    }
                    return s;
                }
            };
            if (act) {
                const R s = pulled_sum(l + 2, fcur);
                phicur = s;
                sring[slot][l + 1] = normal_source<R, MODEL>(s, eps, delta);
            }
            if (l < 2) {
                const int jc = l == 0 ? 1 : w + 2;
                R tmp[9];
                const R s = pulled_sum(jc, tmp);
                sring[slot][jc - 1] = normal_source<R, MODEL>(s, eps, delta);
            }
        }
        lds_barrier();

        // ---- update row y = r - 2
        if (it >= 4 && act) {
            const int y = ys + it - 4;
            const int sm = (it + 1) % 3, s0 = (it + 2) % 3, sp = it % 3;  // psi rows y-1, y, y+1
            const int j = l + 1;
            const R pE = sring[s0][j + 1], pW = sring[s0][j - 1];
            const R pN = sring[sp][j], pS = sring[sm][j];
            const R pNE = sring[sp][j + 1], pNW = sring[sp][j - 1];
            const R pSE = sring[sm][j + 1], pSW = sring[sm][j - 1];
            // isotropic gradient: grad chi = sum_i w_i c_i chi(x + c_i) / c_s^2
            const R gx = (pE - pW) * R(1.0 / 3.0) + ((pNE - pNW) + (pSE - pSW)) * R(1.0 / 12.0);
            const R gy = (pN - pS) * R(1.0 / 3.0) + ((pNE + pNW) - (pSE + pSW)) * R(1.0 / 12.0);
            const R mag = sqrt(gx * gx + gy * gy);
            const R inv = R(1) / (mag + delta);
            const R phi = phiprev;
            const R S = sharpening<R, MODEL>(phi, eps, delta);
            const R Ayv = R(a.vtab[2 * a.nx + y]), Byv = R(a.vtab[2 * a.nx + a.ny + y]);
            const R uxr = Axl * Ayv, uyr = Bxl * Byv;
            const R u = s_now * uxr, v = s_now * uyr;
            const R phio = first ? phi : P2;
            const R uo = s_old * uxr, vo = s_old * uyr;
            // bracket of Eq. (11): d_t(phi u) by explicit Euler + c_s^2 S n
            const R Gx = (phi * u - phio * uo) + R(1.0 / 3.0) * (S * gx * inv);
            const R Gy = (phi * v - phio * vo) + R(1.0 / 3.0) * (S * gy * inv);
            // Eq. (9)-(11): f* = (1 - 1/tau) f + w_i [phi/tau + 3 c_i.(phi u / tau + (1 - 1/(2 tau)) G)]
            const R A0 = omega * phi;
            const R bx = R(3) * (A0 * u + kforce * Gx);
            const R by = R(3) * (A0 * v + kforce * Gy);
            const R keep = R(1) - omega;
            R out[9];
            R rest = phi;
#pragma unroll
            for (int q = 1; q < 9; ++q) {
                R e = A0;
                if (cx(q) == 1) e += bx;
                if (cx(q) == -1) e -= bx;
                if (cy(q) == 1) e += by;
                if (cy(q) == -1) e -= by;
                out[q] = keep * fprev[q] + wq<R>(q) * e;
                rest -= out[q];
            }
            // Eq. (9) conserves sum_i f_i = phi exactly; the rest population is
            // taken as the remainder so that rounded weights (sum_i w_i != 1 in
            // floating point) cannot make the total mass drift
            out[0] = rest;
            Store<R, ST>::store(a, (int64_t)y * a.pitch + x, out, phi);
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) fprev[q] = fcur[q];
        phiprev = phicur;
        P2 = P1;
        P1 = P0;
    }
}

template <typename R, int ST, int MODEL, int BX>
__global__ __launch_bounds__(BX) void step_kernel(StepArgs a) {
    __shared__ TileLds<R, BX> lds;
    step_tile<R, ST, MODEL, BX>(a, blockIdx.x, blockIdx.y, a.t_dev[0] + a.k, lds);
}

// ---------------------------------------------------------------------------
// Initial state: f*_i(y) = f_eq_i(phi0, u(., 0)) evaluated at y + c_i, so that the
// first pull yields the equilibrium of Eq. (10) at every node.
template <typename R, int ST>
__global__ void init_kernel(StepArgs a, const double* __restrict__ phi0) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= a.nx) return;
    const double s0 = time_factor(a.period_T, 0);
    double f[9];
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int xs = wrap_idx(x + cx(q), a.nx), ys = wrap_idx(y + cy(q), a.ny);
        const double ph = phi0[(int64_t)ys * a.nx + xs];
        const double u = s0 * a.vtab[xs] * a.vtab[2 * a.nx + ys];
        const double v = s0 * a.vtab[a.nx + xs] * a.vtab[2 * a.nx + a.ny + ys];
        f[q] = wq<double>(q) * ph * (1.0 + 3.0 * (cx(q) * u + cy(q) * v));
        sum += f[q];
    }
    const int64_t off = (int64_t)y * a.pitch + x;
    if (ST == ST_PLAIN) {
        R* d = static_cast<R*>(a.dst);
#pragma unroll
        for (int q = 0; q < 9; ++q) d[q * a.plane_stride + off] = R(f[q]);
    } else {
        // stored sum is phi* = sum_i f_i; g_i = f_i - w_i phi* (g_0 implied)
        const float ph = float(sum);
#pragma unroll
        for (int q = 1; q < 9; ++q) {
            const float g = float(f[q] - wq<double>(q) * (double)ph);
            if (ST == ST_F16)
                static_cast<__half*>(a.dst)[(q - 1) * a.plane_stride + off] = __float2half_rn(g);
            else
                static_cast<__hip_bfloat16*>(a.dst)[(q - 1) * a.plane_stride + off] = __float2bfloat16(g);
        }
        a.dst_phi[off] = ph;
    }
}

// phi(x) = sum_i f*_i(x - c_i) from the stored state in a.src, in FP64.
template <typename R, int ST>
__device__ __forceinline__ double pulled_phi(const StepArgs& a, int x, int y) {
    double s = 0.0;
    const int64_t own = (int64_t)y * a.pitch + x;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int xs = wrap_idx(x - cx(q), a.nx), ys = wrap_idx(y - cy(q), a.ny);
        s += (double)Store<R, ST>::load_one(a, (int64_t)ys * a.pitch + xs, q);
        // shifted storage: phi = phi* + sum_{i>=1} [v_i(x - c_i) - v_i(x)]
        if (Store<R, ST>::kShifted && q > 0) s -= (double)Store<R, ST>::load_one(a, own, q);
    }
    return s;
}

template <typename R, int ST>
__global__ void phi_kernel(StepArgs a, double* __restrict__ out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= a.nx) return;
    out[(int64_t)y * a.nx + x] = pulled_phi<R, ST>(a, x, y);
}

// Block partial sums for mass and shape errors: per row y, the four sums
// sum phi, sum |phi - ref|, sum |ref|, sum (phi - ref)^2, sum ref^2 (5 values).
// One block per row; the host (or reduce_rows) adds rows in order.
constexpr int kRedThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
    // wavefront (64 lanes) tree, then across the block's waves, fixed order
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    return r;
}

template <typename R, int ST>
__global__ __launch_bounds__(kRedThreads) void row_sums_kernel(StepArgs a, const double* __restrict__ ref,
                                                                double* __restrict__ rows) {
    __shared__ double sh[kRedThreads / 64];
    const int y = blockIdx.x;
    double s_phi = 0, s_ad = 0, s_ar = 0, s_d2 = 0, s_r2 = 0;
    for (int x = threadIdx.x; x < a.nx; x += blockDim.x) {
        const double p = pulled_phi<R, ST>(a, x, y);
        s_phi += p;
        if (ref) {
            const double r = ref[(int64_t)y * a.nx + x];
            const double d = p - r;
            s_ad += fabs(d);
            s_ar += fabs(r);
            s_d2 += d * d;
            s_r2 += r * r;
        }
    }
    double* o = rows + 5 * (int64_t)y;
    double v;
    v = block_sum(s_phi, sh);
    if (threadIdx.x == 0) o[0] = v;
    v = block_sum(s_ad, sh);
    if (threadIdx.x == 0) o[1] = v;
    v = block_sum(s_ar, sh);
    if (threadIdx.x == 0) o[2] = v;
    v = block_sum(s_d2, sh);
    if (threadIdx.x == 0) o[3] = v;
    v = block_sum(s_r2, sh);
    if (threadIdx.x == 0) o[4] = v;
}

// Adds the per-row sums in row order (one block; deterministic).
__global__ __launch_bounds__(kRedThreads) void reduce_rows_kernel(const double* __restrict__ rows, int ny,
                                                                   double* __restrict__ out5) {
    __shared__ double sh[kRedThreads / 64];
    for (int c = 0; c < 5; ++c) {
        double s = 0.0;
        for (int y = threadIdx.x; y < ny; y += blockDim.x) s += rows[5 * (int64_t)y + c];
        const double v = block_sum(s, sh);
        if (threadIdx.x == 0) out5[c] = v;
    }
}

__global__ void advance_kernel(int64_t* t_dev, int64_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) t_dev[0] += n;
}

__global__ void set_time_kernel(int64_t* t_dev, int64_t t) {
    if (threadIdx.x == 0 && blockIdx.x == 0) t_dev[0] = t;
}

}  // namespace lbac
