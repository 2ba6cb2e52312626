// The 3-D (D3Q19) form of the step: kernels and host runtime behind
// include/lbac3.h.  Same scheme as the 2-D library (Sec. 2.2, Eq. (9)-(13));
// the shared device helpers (node arithmetic primitives, buffer stores, tile
// order, reductions) come from lbac_kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lbac3.h"
#include "lbac_internal.hpp"
#include "lbac_kernels.hpp"

namespace lbac3 {

using lbac::bstore;
using lbac::clip01;
using lbac::fmaR;
using lbac::kDropOffset;
using lbac::lds_barrier;
using lbac::Math;
using lbac::plane_rsrc;
using lbac::time_factor;
using lbac::wrap_idx;
using lbac::xcd_tile;

// D3Q19: rest; faces +x -x +y -y +z -z; edges (+x+y) (-x-y) (+x-y) (-x+y)
// (+x+z) (-x-z) (+x-z) (-x+z) (+y+z) (-y-z) (+y-z) (-y+z).
__host__ __device__ constexpr int cx3(int q) {
    return q == 1 || q == 7 || q == 9 || q == 11 || q == 13 ? 1 : (q == 2 || q == 8 || q == 10 || q == 12 || q == 14 ? -1 : 0);
}
__host__ __device__ constexpr int cy3(int q) {
    return q == 3 || q == 7 || q == 10 || q == 15 || q == 17 ? 1 : (q == 4 || q == 8 || q == 9 || q == 16 || q == 18 ? -1 : 0);
}
__host__ __device__ constexpr int cz3(int q) {
    return q == 5 || q == 11 || q == 14 || q == 15 || q == 18 ? 1 : (q == 6 || q == 12 || q == 13 || q == 16 || q == 17 ? -1 : 0);
}
template <typename R>
__host__ __device__ constexpr R w3(int q) {
    return q == 0 ? R(1.0 / 3.0) : (q <= 6 ? R(1.0 / 18.0) : R(1.0 / 36.0));
}


struct Args3 {
    const void* src;
    void* dst;
    const void* phi_old;   // phi at t - 1 (R, pitch x ny x nz)
    void* phi_new;         // phi at t, written for the next step
    int64_t plane_stride;  // elements between population planes
    int32_t pitch, nx, ny, nz;
    int32_t strip_z, nbx, nby, nbz, n_xcd;
    int32_t z_major;       // 1: tile order with the strip index fastest
    const double* vtab;    // per component u, v, w: factors over x (nx), y (ny), z (nz)
    const int64_t* t_dev;
    int32_t k;             // step offset within a chunk of launches
    double period_T, eps, tau, delta;
    int32_t time_dep;      // 1: velocity scaled by cos(pi t / T)
};

// One step on the tile (bxi, byi) of TX x TY columns and the strip bzi of
// planes at time t.  Thread (tx, ty) owns column (TX bxi + tx, TY byi + ty)
// (periodic); per iteration it pulls the 19 values of its column on the
// newest plane (Eq. (9) streaming) straight from global memory, forms phi
// (Eq. (12)) and psi (Eq. (13)) there, and updates the plane behind it from a
// psi ring in LDS (three planes of the tile grown by one column on each
// side).  The 2 (TX + 2) + 2 TY rim columns of the grown tile are pulled, for
// their psi only, by the first waves of the block (one column per lane).
// Even strips march up and odd strips down, so two neighbouring strips pull
// the planes they share at the same time (both at their start or both at
// their end).  Loads, LDS writes and stores of the main loop carry no branch
// but the uniform one around the rim pulls; stores of columns outside the
// lattice are dropped.
// MODE 0: the update keeps its node's 19 pulled values in registers from the
// iteration that loaded them.  MODE 1: the update re-reads them (cache hits),
// issued together with the new plane's loads; fewer registers.  MODE 2: the
// next plane's loads are issued before the update, so they are in flight
// while it runs (the two pipeline-fill iterations compute an update whose
// stores are dropped).
template <typename R, int TX, int TY, int MODE>
__global__ __launch_bounds__(TX * TY) void step3_kernel(Args3 a) {
    constexpr int kTX = TX;
    constexpr int kW = kTX + 2, kH = TY + 2;       // ring plane: the tile grown by one column
    constexpr int kRim = 2 * kW + 2 * TY;          // rim columns of the grown tile
    constexpr int kRimWaves = (kRim + 63) / 64;    // waves that pull them
    __shared__ R ring[3][kH * kW];
    const int ntile = a.nbx * a.nby * a.nbz;
    const int tile = xcd_tile(blockIdx.x, ntile, a.n_xcd);
    int bxi, byi, bzi;
    if (a.z_major) {
        bzi = tile % a.nbz;
        bxi = (tile / a.nbz) % a.nbx;
        byi = tile / (a.nbz * a.nbx);
    } else {
        bxi = tile % a.nbx;
        byi = (tile / a.nbx) % a.nby;
        bzi = tile / (a.nbx * a.nby);
    }
    const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
    const int ux = bxi * kTX + tx, uy = byi * TY + ty;  // unwrapped column
    const int gx = wrap_idx(ux, a.nx), gy = wrap_idx(uy, a.ny);
    const bool inter = ux < a.nx && uy < a.ny;
    const int own = (ty + 1) * kW + (tx + 1);  // ring slot of the own column
    // rim column of this lane (lanes past the rim repeat the last one)
    const bool rim_wave = (int)(threadIdx.x / 64) < kRimWaves;  // uniform
    const int rk = min((int)threadIdx.x, kRim - 1);
    const int rx = rk < kW ? rk - 1 : (rk < 2 * kW ? rk - kW - 1 : (rk < 2 * kW + TY ? -1 : kTX));
    const int ry = rk < kW ? -1 : (rk < 2 * kW ? TY : (rk < 2 * kW + TY ? rk - 2 * kW : rk - 2 * kW - TY));
    const int rslot = (ry + 1) * kW + (rx + 1);
    const int rgx = wrap_idx(bxi * kTX + rx, a.nx), rgy = wrap_idx(byi * TY + ry, a.ny);
    const int z0 = bzi * a.strip_z;
    const int hz = min(a.strip_z, a.nz - z0);
    const bool down = (bzi & 1) != 0;
    // plane entering at iteration i (from one below the strip up, or from one
    // above it down); the plane updated at iteration i is the one of i - 1
    auto plane_at = [&](int i) { return wrap_idx(down ? z0 + hz - i : z0 - 1 + i, a.nz); };
    const int64_t t = a.t_dev[0] + a.k;

    const bool first = (t == 0);
    const R s_now = a.time_dep ? R(time_factor(a.period_T, t)) : R(1);
    const R s_old = first ? s_now : (a.time_dep ? R(time_factor(a.period_T, t - 1)) : R(1));
    const R delta = R(a.delta);
    const R psi_scale = R(a.eps * 0.69314718055994530942);
    const R s_scale = R(1.0 / (a.eps * (1.0 + 2.0 * a.delta) * (1.0 + 2.0 * a.delta)));
    const R omega = R(1.0 / a.tau), kforce = R(1.0 - 0.5 / a.tau), keep = R(1.0 - 1.0 / a.tau);
    const int L = a.nx + a.ny + a.nz;
    // x and y factors of the three velocity components for this column
    const R fxu = R(a.vtab[gx]), fyu = R(a.vtab[a.nx + gy]);
    const R fxv = R(a.vtab[L + gx]), fyv = R(a.vtab[L + a.nx + gy]);
    const R fxw = R(a.vtab[2 * L + gx]), fyw = R(a.vtab[2 * L + a.nx + gy]);

    const R* pold_plane = static_cast<const R*>(a.phi_old);
    R* dst = static_cast<R*>(a.dst);
    const int64_t zs = (int64_t)a.pitch * a.ny;  // elements per z plane
    // Pull sources: column gx - c_x, row gy - c_y (wrapped once per thread), as
    // 32-bit byte offsets from uniform plane bases (a plane is below 2 GiB).
    const char* sb = static_cast<const char*>(a.src);
    const uint32_t pb = (uint32_t)(a.plane_stride * (int64_t)sizeof(R));  // bytes between planes (< 2^31)
    const uint32_t rowb = (uint32_t)a.pitch * (uint32_t)sizeof(R);
    const uint32_t zsb = (uint32_t)zs * (uint32_t)sizeof(R);
    struct Col {
        uint32_t x[3], y[3];  // index c + 1
    };
    auto col_of = [&](int cx, int cy) {
        Col c;
        c.x[0] = (uint32_t)wrap_idx(cx + 1, a.nx) * (uint32_t)sizeof(R);
        c.x[1] = (uint32_t)cx * (uint32_t)sizeof(R);
        c.x[2] = (uint32_t)wrap_idx(cx - 1, a.nx) * (uint32_t)sizeof(R);
        c.y[0] = (uint32_t)wrap_idx(cy + 1, a.ny) * rowb;
        c.y[1] = (uint32_t)cy * rowb;
        c.y[2] = (uint32_t)wrap_idx(cy - 1, a.ny) * rowb;
        return c;
    };
    const Col oc = col_of(gx, gy), rc = col_of(rgx, rgy);
    // f_i(x) = f*_i(x - c_i) for the node of column c on plane zp (Eq. (9) streaming)
    auto pull = [&](const Col& c, int zp, R (&v)[19]) __attribute__((always_inline)) {
        const uint32_t zoff[3] = {(uint32_t)wrap_idx(zp + 1, a.nz) * zsb, (uint32_t)zp * zsb,
                                  (uint32_t)wrap_idx(zp - 1, a.nz) * zsb};  // plane zp - c_z, index c_z + 1
#pragma unroll
        for (int q = 0; q < 19; ++q)
            v[q] = *reinterpret_cast<const R*>(sb + (size_t)q * pb + (zoff[cz3(q) + 1] + c.y[cy3(q) + 1] + c.x[cx3(q) + 1]));
    };
    auto pold_at = [&](int zp) { return pold_plane[(int64_t)zp * zs + (int64_t)gy * a.pitch + gx]; };
    auto psi_of = [&](R phi) {
        const R pc = clip01(phi);
        return psi_scale * (Math<R>::log2(pc + delta) - Math<R>::log2(R(1) - pc + delta));
    };

    R fprev[19];
    R phiprev = R(0), poldprev = R(0);
#pragma unroll
    for (int q = 0; q < 19; ++q) fprev[q] = R(0);

    // update of node (gx, gy, zc) from the psi ring, its pulled values fp,
    // phi and phi(t - 1); stores dropped unless st
    auto update = [&](int it, int zc, bool st, const R (&fp)[19], R phi, R poldv) __attribute__((always_inline)) {
        // ring planes of zc - 1, zc, zc + 1 (the plane entered two iterations
        // ago, one ago, now; the other way round marching down)
        const R* r2 = ring[(it + 1) % 3];
        const R* r0 = ring[it % 3];
        const R* pm = down ? r0 : r2;
        const R* pc = ring[(it + 2) % 3];
        const R* pp = down ? r2 : r0;
        const int c = own, e = own + 1, w = own - 1, n = own + kW, s = own - kW;
        // grad psi = sum_i w_i c_i psi(x + c_i) / c_s^2: faces weigh 1/6, edges 1/12
        const R gxv = fmaR(pc[e] - pc[w], R(1.0 / 6.0),
                           (((pc[n + 1] - pc[s - 1]) + (pc[s + 1] - pc[n - 1])) + ((pp[e] - pm[w]) + (pm[e] - pp[w]))) *
                               R(1.0 / 12.0));
        const R gyv = fmaR(pc[n] - pc[s], R(1.0 / 6.0),
                           (((pc[n + 1] - pc[s - 1]) + (pc[n - 1] - pc[s + 1])) + ((pp[n] - pm[s]) + (pm[n] - pp[s]))) *
                               R(1.0 / 12.0));
        const R gzv = fmaR(pp[c] - pm[c], R(1.0 / 6.0),
                           (((pp[e] - pm[w]) + (pp[w] - pm[e])) + ((pp[n] - pm[s]) + (pp[s] - pm[n]))) * R(1.0 / 12.0));
        const R inv = Math<R>::rcp(Math<R>::sqrt(fmaR(gxv, gxv, fmaR(gyv, gyv, gzv * gzv))) + delta);
        const R pcl = clip01(phi);
        const R S = (pcl + delta) * (R(1) - pcl + delta) * s_scale;
        const R fz = R(lbac::row_factor(a.vtab, a.nx + a.ny + zc));
        const R fzv = R(lbac::row_factor(a.vtab, L + a.nx + a.ny + zc));
        const R fzw = R(lbac::row_factor(a.vtab, 2 * L + a.nx + a.ny + zc));
        const R ur = fxu * fyu * fz, vr = fxv * fyv * fzv, wr = fxw * fyw * fzw;
        const R u = s_now * ur, v = s_now * vr, wv = s_now * wr;
        const R phio = first ? phi : poldv;
        // bracket of Eq. (11): d_t(phi u) by explicit Euler + c_s^2 S n
        const R Sn = R(1.0 / 3.0) * S * inv;
        const R Gx = fmaR(Sn, gxv, fmaR(phi, u, -(phio * (s_old * ur))));
        const R Gy = fmaR(Sn, gyv, fmaR(phi, v, -(phio * (s_old * vr))));
        const R Gz = fmaR(Sn, gzv, fmaR(phi, wv, -(phio * (s_old * wr))));
        // Eq. (9)-(11): f*_i = (1 - 1/tau) f_i + w_i [phi/tau + 3 c_i.(phi u/tau + (1 - 1/(2 tau)) G)];
        // the rest population as the remainder keeps sum_i f*_i = phi exactly
        const R A0 = omega * phi;
        const R bx = R(3) * fmaR(A0, u, kforce * Gx);
        const R by = R(3) * fmaR(A0, v, kforce * Gy);
        const R bz = R(3) * fmaR(A0, wv, kforce * Gz);
        R out[19];
        const R af = w3<R>(1) * A0, ae = w3<R>(7) * A0;
        const R xf = w3<R>(1) * bx, yf = w3<R>(1) * by, zf = w3<R>(1) * bz;
        const R xe = w3<R>(7) * bx, ye = w3<R>(7) * by, ze = w3<R>(7) * bz;
        out[1] = fmaR(keep, fp[1], af + xf);
        out[2] = fmaR(keep, fp[2], af - xf);
        out[3] = fmaR(keep, fp[3], af + yf);
        out[4] = fmaR(keep, fp[4], af - yf);
        out[5] = fmaR(keep, fp[5], af + zf);
        out[6] = fmaR(keep, fp[6], af - zf);
        out[7] = fmaR(keep, fp[7], (ae + xe) + ye);
        out[8] = fmaR(keep, fp[8], (ae - xe) - ye);
        out[9] = fmaR(keep, fp[9], (ae + xe) - ye);
        out[10] = fmaR(keep, fp[10], (ae - xe) + ye);
        out[11] = fmaR(keep, fp[11], (ae + xe) + ze);
        out[12] = fmaR(keep, fp[12], (ae - xe) - ze);
        out[13] = fmaR(keep, fp[13], (ae + xe) - ze);
        out[14] = fmaR(keep, fp[14], (ae - xe) + ze);
        out[15] = fmaR(keep, fp[15], (ae + ye) + ze);
        out[16] = fmaR(keep, fp[16], (ae - ye) - ze);
        out[17] = fmaR(keep, fp[17], (ae + ye) - ze);
        out[18] = fmaR(keep, fp[18], (ae - ye) + ze);
        R rest = phi;
#pragma unroll
        for (int q = 1; q < 19; ++q) rest -= out[q];
        out[0] = rest;
        // columns outside the lattice store nothing (dropped offsets); in
        // FP32 with the non-temporal hint, so that stored planes do not
        // displace the rims and shared planes other tiles read (0.7% faster
        // at 256^3)
        const uint32_t node = (uint32_t)((int64_t)zc * zs + (int64_t)gy * a.pitch + gx);
        const uint32_t b = st ? node * (uint32_t)sizeof(R) : kDropOffset;
        if constexpr (sizeof(R) == 4) {
#pragma unroll
            for (int q = 0; q < 19; ++q) lbac::bstore_nt(out[q], plane_rsrc(dst + (size_t)q * a.plane_stride), b);
            lbac::bstore_nt(phi, plane_rsrc(a.phi_new), b);
        } else {
#pragma unroll
            for (int q = 0; q < 19; ++q) bstore(out[q], plane_rsrc(dst + (size_t)q * a.plane_stride), b);
            bstore(phi, plane_rsrc(a.phi_new), b);
        }
    };

    lds_barrier();
    const int iters = hz + 2;
    R fn[19];
    R pn = R(0);
    if constexpr (MODE == 2) {
        pull(oc, plane_at(0), fn);
        pn = pold_at(plane_at(0));
    }
    for (int it = 0; it < iters; ++it) {
        const int zr = plane_at(it);      // the plane entering
        const int zc = plane_at(it - 1);  // the plane updated (from the third iteration on)
        // ---- pull, phi (Eq. (12)) and psi (Eq. (13)) on plane zr: own column, then the rim
        R f[19];
        R pold;
        if constexpr (MODE == 2) {
#pragma unroll
            for (int q = 0; q < 19; ++q) f[q] = fn[q];
            pold = pn;
        } else {
            pull(oc, zr, f);
            pold = pold_at(zr);
        }
        if (rim_wave) {
            R g[19];
            pull(rc, zr, g);
            R sg = R(0);
#pragma unroll
            for (int q = 0; q < 19; ++q) sg += g[q];
            ring[it % 3][rslot] = psi_of(sg);
        }
        R s = R(0);
#pragma unroll
        for (int q = 0; q < 19; ++q) s += f[q];
        ring[it % 3][own] = psi_of(s);
        if constexpr (MODE == 1) pull(oc, zc, fprev);  // the update's own pulled values, before the barrier
        if constexpr (MODE == 2) {
            // the next plane (past the strip: the last plane again, not used)
            const int zn = plane_at(min(it + 1, iters - 1));
            pull(oc, zn, fn);
            pn = pold_at(zn);
        }
        lds_barrier();
        // ---- update the plane behind (zc); the first two iterations fill the pipeline
        if constexpr (MODE == 2) {
            update(it, zc, inter && it >= 2, fprev, phiprev, poldprev);
        } else {
            if (it >= 2) update(it, zc, inter, fprev, phiprev, poldprev);
        }
        lds_barrier();  // the ring slot written next iteration was read above
        if constexpr (MODE != 1) {
#pragma unroll
            for (int q = 0; q < 19; ++q) fprev[q] = f[q];
        }
        phiprev = s;
        poldprev = pold;
    }
}

// f*_i(x) = f_eq_i(phi0, u(., 0)) at x + c_i, so that the first pull yields the
// equilibrium of Eq. (10) at every node; phi planes = phi0.
template <typename R>
__global__ void init3_kernel(Args3 a, const double* __restrict__ phi0) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= a.nx) return;
    const int L = a.nx + a.ny + a.nz;
    const double s0 = a.time_dep ? time_factor(a.period_T, 0) : 1.0;
    R* dst = static_cast<R*>(a.dst);
    const int64_t zs = (int64_t)a.pitch * a.ny, off = (int64_t)z * zs + (int64_t)y * a.pitch + x;
    for (int q = 0; q < 19; ++q) {
        const int xs = wrap_idx(x + cx3(q), a.nx), ys = wrap_idx(y + cy3(q), a.ny), zq = wrap_idx(z + cz3(q), a.nz);
        const double ph = phi0[((int64_t)zq * a.ny + ys) * a.nx + xs];
        const double u = s0 * a.vtab[xs] * a.vtab[a.nx + ys] * a.vtab[a.nx + a.ny + zq];
        const double v = s0 * a.vtab[L + xs] * a.vtab[L + a.nx + ys] * a.vtab[L + a.nx + a.ny + zq];
        const double w = s0 * a.vtab[2 * L + xs] * a.vtab[2 * L + a.nx + ys] * a.vtab[2 * L + a.nx + a.ny + zq];
        dst[q * a.plane_stride + off] = R(w3<double>(q) * ph * (1.0 + 3.0 * (cx3(q) * u + cy3(q) * v + cz3(q) * w)));
    }
    static_cast<R*>(a.phi_new)[off] = R(phi0[((int64_t)z * a.ny + y) * a.nx + x]);
}

// phi = the pulled sum of Eq. (12) in the same order as the step, as doubles (x fastest)
template <typename R>
__global__ void phi3_kernel(Args3 a, double* __restrict__ out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= a.nx) return;
    const R* src = static_cast<const R*>(a.src);
    const int64_t zs = (int64_t)a.pitch * a.ny;
    R s = R(0);
    for (int q = 0; q < 19; ++q)
        s += src[q * a.plane_stride + (int64_t)wrap_idx(z - cz3(q), a.nz) * zs + (int64_t)wrap_idx(y - cy3(q), a.ny) * a.pitch +
                 wrap_idx(x - cx3(q), a.nx)];
    out[((int64_t)z * a.ny + y) * a.nx + x] = (double)s;
}

// Partial sums (sum phi, sum |phi - ref|, sum |ref|, sum (phi - ref)^2, sum ref^2)
// over consecutive chunks of the field, one block per chunk, fixed order.
__global__ __launch_bounds__(lbac::kRedThreads) void sum5_kernel(const double* __restrict__ phi,
                                                                 const double* __restrict__ ref, int64_t n,
                                                                 int64_t chunk, double* __restrict__ part) {
    __shared__ double sh[2 * lbac::kRedThreads / 64];
    const int64_t b = (int64_t)blockIdx.x * chunk, e = min(b + chunk, n);
    double v[5] = {0, 0, 0, 0, 0};
    for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
        const double p = phi[i];
        v[0] += p;
        if (ref) {
            const double r = ref[i], d = p - r;
            v[1] += fabs(d);
            v[2] += fabs(r);
            v[3] += d * d;
            v[4] += r * r;
        }
    }
    for (int c = 0; c < 5; ++c) {
        lbac::CompSum<double> acc;
        acc.s = v[c];
        const double r = lbac::block_sum(acc, sh).value();
        if (threadIdx.x == 0) part[5 * (int64_t)blockIdx.x + c] = r;
    }
}

// One wavefront: lane l adds parts l, l + 64, ... in order, then a fixed
// tree across the lanes.
__global__ void sum_parts_kernel(const double* __restrict__ part, int nparts, double* __restrict__ out5) {
    const int l = threadIdx.x;
    for (int c = 0; c < 5; ++c) {
        double s = 0.0;
        for (int i = l; i < nparts; i += 64) s += part[5 * (int64_t)i + c];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (l == 0) out5[c] = s;
    }
}

__global__ void advance3_kernel(int64_t* t_dev, int64_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) t_dev[0] += n;
}

}  // namespace lbac3

// ---------------------------------------------------------------------------
// host side

struct lbac3_ctx {
    lbac3_params p{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int elem_bytes = 8;
    int32_t pitch = 0;
    int64_t plane_stride = 0;
    void* pop[2] = {nullptr, nullptr};
    void* phis[2] = {nullptr, nullptr};
    double* vtab = nullptr;
    int64_t* t_dev = nullptr;
    double* dtmp = nullptr;   // nz*ny*nx doubles
    double* dref = nullptr;   // nz*ny*nx doubles (reference field)
    double* part = nullptr;   // partial sums
    double* out5 = nullptr;
    double* host5 = nullptr;  // pinned
    int nparts = 0;
    int cur = 0;
    int64_t t = 0;
    int strip_z = 32;
    int tile_x = 32;     // tile shape in columns (one of kShapes)
    int tile_y = 16;
    int mode = 0;        // 0 keep, 1 re-pull, 2 prefetch (see step3_kernel)
    int z_major = 0;     // tile order: 0 x fastest, 1 strip fastest
    std::string err;
};

namespace {

std::string g_init_error;

constexpr int kNParts = 1024;

int fail3(lbac3_ctx* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

#define HIP3(h, call)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess) return fail3(h, LBAC_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

void build_tables(const lbac3_params& p, std::vector<double>& tab) {
    const double PI = 3.14159265358979323846;
    const int L = p.nx + p.ny + p.nz;
    tab.assign(3 * (size_t)L, 0.0);
    auto fx = [&](int c) { return &tab[(size_t)c * L]; };
    auto fy = [&](int c) { return &tab[(size_t)c * L + p.nx]; };
    auto fz = [&](int c) { return &tab[(size_t)c * L + p.nx + p.ny]; };
    for (int c = 0; c < 3; ++c) {
        for (int j = 0; j < p.ny; ++j) fy(c)[j] = 1.0;
        for (int k = 0; k < p.nz; ++k) fz(c)[k] = 1.0;
    }
    for (int i = 0; i < p.nx; ++i) {
        const double x = (i + 0.5) / p.nx;
        switch (p.vel_kind) {
        case LBAC3_VEL_DEFORMATION:
            fx(0)[i] = 2.0 * p.U * std::sin(PI * x) * std::sin(PI * x);
            fx(1)[i] = -p.U * std::sin(2.0 * PI * x);
            fx(2)[i] = -p.U * std::sin(2.0 * PI * x);
            break;
        case LBAC3_VEL_VORTEX_XY:
            fx(0)[i] = -p.U * std::sin(PI * x) * std::sin(PI * x);
            fx(1)[i] = p.U * std::sin(2.0 * PI * x);
            fx(2)[i] = 0.0;
            break;
        case LBAC3_VEL_UNIFORM:
            fx(0)[i] = p.ux;
            fx(1)[i] = p.uy;
            fx(2)[i] = p.uz;
            break;
        default:
            fx(0)[i] = fx(1)[i] = fx(2)[i] = 0.0;
        }
    }
    for (int j = 0; j < p.ny; ++j) {
        const double y = (j + 0.5) / p.ny;
        if (p.vel_kind == LBAC3_VEL_DEFORMATION) {
            fy(0)[j] = std::sin(2.0 * PI * y);
            fy(1)[j] = std::sin(PI * y) * std::sin(PI * y);
            fy(2)[j] = std::sin(2.0 * PI * y);
        } else if (p.vel_kind == LBAC3_VEL_VORTEX_XY) {
            fy(0)[j] = std::sin(2.0 * PI * y);
            fy(1)[j] = std::sin(PI * y) * std::sin(PI * y);
        }
    }
    for (int k = 0; k < p.nz; ++k) {
        const double z = (k + 0.5) / p.nz;
        if (p.vel_kind == LBAC3_VEL_DEFORMATION) {
            fz(0)[k] = std::sin(2.0 * PI * z);
            fz(1)[k] = std::sin(2.0 * PI * z);
            fz(2)[k] = std::sin(PI * z) * std::sin(PI * z);
        }
    }
}

int validate3(const lbac3_params* p, std::string& why) {
    if (!p) return why = "params is NULL", LBAC_EINVAL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1 || p->nx > 4096 || p->ny > 4096 || p->nz > 4096 ||
        (int64_t)p->nx * p->ny * p->nz > (1ll << 27))
        return why = "grid size out of range (1 <= nx, ny, nz <= 4096, nx * ny * nz <= 2^27)", LBAC_EINVAL;
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return why = "tau must exceed 1/2", LBAC_EINVAL;
    if (!(p->eps > 0.0) || !std::isfinite(p->eps)) return why = "eps must be positive", LBAC_EINVAL;
    if (!(p->delta >= 0.0) || !std::isfinite(p->delta)) return why = "delta must be >= 0", LBAC_EINVAL;
    if (p->vel_kind < LBAC3_VEL_ZERO || p->vel_kind > LBAC3_VEL_UNIFORM) return why = "bad vel_kind", LBAC_EINVAL;
    if ((p->vel_kind == LBAC3_VEL_DEFORMATION || p->vel_kind == LBAC3_VEL_VORTEX_XY) && !(p->period_T > 0.0))
        return why = "period_T must be > 0", LBAC_EINVAL;
    if (p->precision != LBAC_F64 && p->precision != LBAC_F32) return why = "precision must be LBAC_F64 or LBAC_F32", LBAC_EINVAL;
    std::vector<double> tab;
    build_tables(*p, tab);
    const int L = p->nx + p->ny + p->nz;
    double m[9] = {0};
    for (int c = 0; c < 3; ++c) {
        for (int i = 0; i < p->nx; ++i) m[3 * c] = std::max(m[3 * c], std::fabs(tab[(size_t)c * L + i]));
        for (int j = 0; j < p->ny; ++j) m[3 * c + 1] = std::max(m[3 * c + 1], std::fabs(tab[(size_t)c * L + p->nx + j]));
        for (int k = 0; k < p->nz; ++k)
            m[3 * c + 2] = std::max(m[3 * c + 2], std::fabs(tab[(size_t)c * L + p->nx + p->ny + k]));
    }
    const double bound = m[0] * m[1] * m[2] + m[3] * m[4] * m[5] + m[6] * m[7] * m[8];
    if (!std::isfinite(bound) || bound >= 1.0 / 3.0)
        return why = "velocity too large: max |u| + |v| + |w| must stay below 1/3", LBAC_EINVAL;
    return LBAC_OK;
}

lbac3::Args3 make_args3(const lbac3_ctx* h, int src, int32_t k) {
    lbac3::Args3 a{};
    a.src = h->pop[src];
    a.dst = h->pop[1 - src];
    a.phi_old = h->phis[src];
    a.phi_new = h->phis[1 - src];
    a.plane_stride = h->plane_stride;
    a.pitch = h->pitch;
    a.nx = h->p.nx;
    a.ny = h->p.ny;
    a.nz = h->p.nz;
    a.strip_z = std::min(h->strip_z, h->p.nz);
    a.nbx = (h->p.nx + h->tile_x - 1) / h->tile_x;
    a.nby = (h->p.ny + h->tile_y - 1) / h->tile_y;
    a.nbz = (h->p.nz + a.strip_z - 1) / a.strip_z;
    a.n_xcd = 8;
    a.z_major = h->z_major;
    a.vtab = h->vtab;
    a.t_dev = h->t_dev;
    a.k = k;
    a.period_T = h->p.period_T > 0.0 ? h->p.period_T : 1.0;
    a.eps = h->p.eps;
    a.tau = h->p.tau;
    a.delta = h->p.delta;
    a.time_dep = (h->p.vel_kind == LBAC3_VEL_DEFORMATION || h->p.vel_kind == LBAC3_VEL_VORTEX_XY) ? 1 : 0;
    return a;
}

template <typename R, int TX, int TY>
void launch3_shape(const lbac3_ctx* h, const lbac3::Args3& a, dim3 grid) {
    const dim3 block(TX * TY);
    if (h->mode == 1)
        hipLaunchKernelGGL((lbac3::step3_kernel<R, TX, TY, 1>), grid, block, 0, h->stream, a);
    else if (h->mode == 2)
        hipLaunchKernelGGL((lbac3::step3_kernel<R, TX, TY, 2>), grid, block, 0, h->stream, a);
    else
        hipLaunchKernelGGL((lbac3::step3_kernel<R, TX, TY, 0>), grid, block, 0, h->stream, a);
}

// Tile shapes (columns along x and y).  Blocks of 1024 threads need at most
// 128 registers per lane, which the FP64 update exceeds: those shapes are
// FP32 only.
constexpr int kShapes[][2] = {{32, 8}, {32, 16}, {64, 4}, {64, 8}, {128, 4}, {32, 32}, {64, 16}, {128, 8}};

bool tile_ok(const lbac3_ctx* h, int tile_x, int tile_y) {
    for (const auto& sh : kShapes)
        if (sh[0] == tile_x && sh[1] == tile_y) return tile_x * tile_y <= 512 || h->p.precision == LBAC_F32;
    return false;
}

template <typename R>
void launch3_t(const lbac3_ctx* h, const lbac3::Args3& a, dim3 grid) {
    const int tx = h->tile_x, ty = h->tile_y;
    if (tx == 32 && ty == 8) launch3_shape<R, 32, 8>(h, a, grid);
    else if (tx == 32 && ty == 16) launch3_shape<R, 32, 16>(h, a, grid);
    else if (tx == 64 && ty == 4) launch3_shape<R, 64, 4>(h, a, grid);
    else if (tx == 64 && ty == 8) launch3_shape<R, 64, 8>(h, a, grid);
    else if (tx == 128 && ty == 4) launch3_shape<R, 128, 4>(h, a, grid);
    else if constexpr (sizeof(R) == 4) {
        if (tx == 32 && ty == 32) launch3_shape<R, 32, 32>(h, a, grid);
        else if (tx == 64 && ty == 16) launch3_shape<R, 64, 16>(h, a, grid);
        else if (tx == 128 && ty == 8) launch3_shape<R, 128, 8>(h, a, grid);
    }
}

hipError_t launch_step3(const lbac3_ctx* h, int src, int32_t k) {
    const lbac3::Args3 a = make_args3(h, src, k);
    const dim3 grid(a.nbx * a.nby * a.nbz);
    if (h->p.precision == LBAC_F64)
        launch3_t<double>(h, a, grid);
    else
        launch3_t<float>(h, a, grid);
    return hipGetLastError();
}

void release3(lbac3_ctx* h) {
    for (int i = 0; i < 2; ++i) {
        if (h->pop[i]) (void)hipFree(h->pop[i]);
        if (h->phis[i]) (void)hipFree(h->phis[i]);
    }
    if (h->vtab) (void)hipFree(h->vtab);
    if (h->t_dev) (void)hipFree(h->t_dev);
    if (h->dtmp) (void)hipFree(h->dtmp);
    if (h->dref) (void)hipFree(h->dref);
    if (h->part) (void)hipFree(h->part);
    if (h->out5) (void)hipFree(h->out5);
    if (h->host5) (void)hipHostFree(h->host5);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
}

int sums3(lbac3_ctx* h, const double* ref_host, double out[5]) {
    lbac_host::DeviceGuard g(h->device);
    const int64_t n = (int64_t)h->p.nx * h->p.ny * h->p.nz;
    lbac3::Args3 a = make_args3(h, h->cur, 0);
    const dim3 grid((h->p.nx + 255) / 256, h->p.ny, h->p.nz);
    if (h->p.precision == LBAC_F64)
        hipLaunchKernelGGL(lbac3::phi3_kernel<double>, grid, dim3(256), 0, h->stream, a, h->dtmp);
    else
        hipLaunchKernelGGL(lbac3::phi3_kernel<float>, grid, dim3(256), 0, h->stream, a, h->dtmp);
    HIP3(h, hipGetLastError());
    if (ref_host) HIP3(h, hipMemcpyAsync(h->dref, ref_host, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
    const int64_t chunk = (n + kNParts - 1) / kNParts;
    const int nparts = (int)((n + chunk - 1) / chunk);
    hipLaunchKernelGGL(lbac3::sum5_kernel, dim3(nparts), dim3(lbac::kRedThreads), 0, h->stream, h->dtmp,
                       ref_host ? h->dref : nullptr, n, chunk, h->part);
    hipLaunchKernelGGL(lbac3::sum_parts_kernel, dim3(1), dim3(64), 0, h->stream, h->part, nparts, h->out5);
    HIP3(h, hipGetLastError());
    HIP3(h, hipMemcpyAsync(h->host5, h->out5, 5 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP3(h, hipStreamSynchronize(h->stream));
    for (int c = 0; c < 5; ++c) out[c] = h->host5[c];
    return LBAC_OK;
}

}  // namespace

extern "C" {

void lbac3_default_params(lbac3_params* p, int32_t nx, int32_t ny, int32_t nz) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->nx = nx;
    p->ny = ny;
    p->nz = nz;
    p->eps = 1.0;
    p->tau = 0.8;
    p->delta = 1e-10;
    p->vel_kind = LBAC3_VEL_DEFORMATION;
    p->U = 0.02;
    p->period_T = 3.0 * nx / 0.02;
    p->precision = LBAC_F32;
}

int lbac3_init(const lbac3_params* p, const double* phi0, lbac3_ctx** out) {
    if (!out) return LBAC_EINVAL;
    *out = nullptr;
    std::string why;
    int rc = validate3(p, why);
    if (rc != LBAC_OK) {
        g_init_error = why;
        return rc;
    }
    const int64_t n = (int64_t)p->nx * p->ny * p->nz;
    if (!phi0) {
        g_init_error = "phi0 is NULL";
        return LBAC_EINVAL;
    }
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(phi0[i])) {
            g_init_error = "phi0 has a non-finite value";
            return LBAC_EINVAL;
        }
    lbac3_ctx* h = new lbac3_ctx();
    h->p = *p;
    auto bail = [&](int code, const std::string& msg) {
        g_init_error = msg;
        release3(h);
        delete h;
        return code;
    };
    if (hipGetDevice(&h->device) != hipSuccess) return bail(LBAC_EDEVICE, "no device");
    if (p->stream) {
        h->stream = (hipStream_t)p->stream;
    } else {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) return bail(LBAC_EDEVICE, "stream");
        h->own_stream = true;
    }
    h->elem_bytes = p->precision == LBAC_F64 ? 8 : 4;
    {
        // rows an odd multiple of 256 bytes apart (see the 2-D layout)
        const int unit = 256 / h->elem_bytes;
        h->pitch = (p->nx + unit - 1) / unit * unit;
        if ((h->pitch / unit) % 2 == 0) h->pitch += unit;
    }
    const int64_t cells = (int64_t)h->pitch * p->ny * p->nz;
    h->plane_stride = cells + lbac_host::kPlanePadBytes / h->elem_bytes;
    // byte offsets within a plane are 32-bit and stay below the buffer range
    if (cells * h->elem_bytes >= (1ll << 31) - 256) return bail(LBAC_EINVAL, "grid too large");
    const size_t pop_bytes = (size_t)h->plane_stride * 19 * h->elem_bytes;
    for (int i = 0; i < 2; ++i) {
        if (hipMalloc(&h->pop[i], pop_bytes) != hipSuccess) return bail(LBAC_ENOMEM, "populations");
        if (hipMalloc(&h->phis[i], (size_t)(cells + 64) * h->elem_bytes) != hipSuccess) return bail(LBAC_ENOMEM, "phi planes");
    }
    std::vector<double> tab;
    build_tables(*p, tab);
    if (hipMalloc(&h->vtab, tab.size() * sizeof(double)) != hipSuccess || hipMalloc(&h->t_dev, 64) != hipSuccess ||
        hipMalloc(&h->dtmp, n * sizeof(double)) != hipSuccess || hipMalloc(&h->dref, n * sizeof(double)) != hipSuccess ||
        hipMalloc(&h->part, 5 * kNParts * sizeof(double)) != hipSuccess || hipMalloc(&h->out5, 64) != hipSuccess ||
        hipHostMalloc((void**)&h->host5, 64, hipHostMallocDefault) != hipSuccess)
        return bail(LBAC_ENOMEM, "tables");
    if (hipMemcpyAsync(h->vtab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemsetAsync(h->t_dev, 0, 64, h->stream) != hipSuccess ||
        hipMemcpyAsync(h->dtmp, phi0, n * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess)
        return bail(LBAC_EDEVICE, "upload");
    h->cur = 0;
    lbac3::Args3 a = make_args3(h, 1, 0);  // dst = pop[0], phi_new = phis[0]
    const dim3 grid((p->nx + 255) / 256, p->ny, p->nz);
    if (p->precision == LBAC_F64)
        hipLaunchKernelGGL(lbac3::init3_kernel<double>, grid, dim3(256), 0, h->stream, a, h->dtmp);
    else
        hipLaunchKernelGGL(lbac3::init3_kernel<float>, grid, dim3(256), 0, h->stream, a, h->dtmp);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess)
        return bail(LBAC_EDEVICE, "init kernel");
    *out = h;
    return LBAC_OK;
}

int lbac3_step(lbac3_ctx* h, int64_t n) {
    if (!h || n < 0) return LBAC_EINVAL;
    lbac_host::DeviceGuard g(h->device);
    // each launch reads the device step counter plus its offset within the
    // current run of launches; the counter advances after every run
    int32_t pending = 0;
    for (int64_t s = 0; s < n; ++s) {
        HIP3(h, launch_step3(h, h->cur, pending));
        h->cur ^= 1;
        ++pending;
        if (pending == (1 << 20) || s == n - 1) {
            hipLaunchKernelGGL(lbac3::advance3_kernel, dim3(1), dim3(64), 0, h->stream, h->t_dev, (int64_t)pending);
            HIP3(h, hipGetLastError());
            pending = 0;
        }
    }
    h->t += n;
    return LBAC_OK;
}

int lbac3_phi(lbac3_ctx* h, double* out) {
    if (!h || !out) return LBAC_EINVAL;
    lbac_host::DeviceGuard g(h->device);
    const int64_t n = (int64_t)h->p.nx * h->p.ny * h->p.nz;
    lbac3::Args3 a = make_args3(h, h->cur, 0);
    const dim3 grid((h->p.nx + 255) / 256, h->p.ny, h->p.nz);
    if (h->p.precision == LBAC_F64)
        hipLaunchKernelGGL(lbac3::phi3_kernel<double>, grid, dim3(256), 0, h->stream, a, h->dtmp);
    else
        hipLaunchKernelGGL(lbac3::phi3_kernel<float>, grid, dim3(256), 0, h->stream, a, h->dtmp);
    HIP3(h, hipGetLastError());
    HIP3(h, hipMemcpyAsync(out, h->dtmp, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP3(h, hipStreamSynchronize(h->stream));
    return LBAC_OK;
}

int lbac3_mass(lbac3_ctx* h, double* out) {
    if (!h || !out) return LBAC_EINVAL;
    double s[5];
    int rc = sums3(h, nullptr, s);
    if (rc != LBAC_OK) return rc;
    *out = s[0];
    return std::isfinite(s[0]) ? LBAC_OK : fail3(h, LBAC_ENONFINITE, "mass is not finite");
}

int lbac3_shape_error(lbac3_ctx* h, const double* ref, double* e1, double* e2) {
    if (!h || !ref || !e1 || !e2) return LBAC_EINVAL;
    double s[5];
    int rc = sums3(h, ref, s);
    if (rc != LBAC_OK) return rc;
    if (!(s[2] > 0.0) || !(s[4] > 0.0)) return fail3(h, LBAC_EINVAL, "reference field is zero");
    *e1 = s[1] / s[2];
    *e2 = std::sqrt(s[3] / s[4]);
    return std::isfinite(*e1) && std::isfinite(*e2) ? LBAC_OK : fail3(h, LBAC_ENONFINITE, "non-finite error");
}

int lbac3_time(lbac3_ctx* h, int64_t* t) {
    if (!h || !t) return LBAC_EINVAL;
    *t = h->t;
    return LBAC_OK;
}

int lbac3_set_launch(lbac3_ctx* h, int32_t tile_x, int32_t tile_y, int32_t variant, int32_t strip_z,
                     int32_t z_major) {
    if (!h) return LBAC_EINVAL;
    if (z_major != 0 && z_major != 1) return fail3(h, LBAC_EINVAL, "z_major must be 0 or 1");
    if (!tile_ok(h, tile_x, tile_y))
        return fail3(h, LBAC_EINVAL, "tile shape must be 32x8, 32x16, 64x4, 64x8, 128x4 (or, with FP32, 32x32, 64x16, 128x8)");
    if (variant < 0 || variant > 2) return fail3(h, LBAC_EINVAL, "variant must be 0, 1 or 2");
    if (strip_z < 1) return fail3(h, LBAC_EINVAL, "strip_z must be >= 1");
    h->tile_x = tile_x;
    h->tile_y = tile_y;
    h->mode = variant;
    h->strip_z = std::min(strip_z, h->p.nz);
    h->z_major = z_major;
    return LBAC_OK;
}

int lbac3_get_launch(lbac3_ctx* h, int32_t* tile_x, int32_t* tile_y, int32_t* variant, int32_t* strip_z,
                     int32_t* z_major) {
    if (!h) return LBAC_EINVAL;
    if (tile_x) *tile_x = h->tile_x;
    if (tile_y) *tile_y = h->tile_y;
    if (variant) *variant = h->mode;
    if (strip_z) *strip_z = h->strip_z;
    if (z_major) *z_major = h->z_major;
    return LBAC_OK;
}

int lbac3_autotune(lbac3_ctx* h, int32_t steps, double* us_per_step) {
    if (!h || steps < 1) return LBAC_EINVAL;
    lbac_host::DeviceGuard g(h->device);
    hipEvent_t e0, e1;
    HIP3(h, hipEventCreate(&e0));
    HIP3(h, hipEventCreate(&e1));
    const int keep = h->strip_z, keep_tx = h->tile_x, keep_ty = h->tile_y, keep_rp = h->mode, keep_zm = h->z_major;
    int best_s = keep, best_tx = keep_tx, best_ty = keep_ty, best_rp = keep_rp, best_zm = keep_zm;
    float best = 1e30f;
    hipError_t e = hipSuccess;
    // strips: powers of two, and nz split into k equal parts (so that a grid
    // that fits the device at once can march long strips in step)
    std::vector<int> strips;
    for (int sz = 4; sz <= 128; sz *= 2) strips.push_back(std::min(sz, h->p.nz));
    for (int k = 1; k <= 16; ++k) strips.push_back((h->p.nz + k - 1) / k);
    std::sort(strips.begin(), strips.end());
    strips.erase(std::unique(strips.begin(), strips.end()), strips.end());
    struct Shape {
        int tx, ty, rp, sz, zm;
    };
    std::vector<Shape> shapes;
    for (const auto& sh : kShapes)
        for (int rp = 0; rp < 3; ++rp)
            for (int sz : strips)
                for (int zm = 0; zm < 2; ++zm)
                    if (tile_ok(h, sh[0], sh[1]) && !(zm == 1 && sz == h->p.nz)) shapes.push_back({sh[0], sh[1], rp, sz, zm});
    for (const Shape& c : shapes) {
        h->tile_x = c.tx;
        h->tile_y = c.ty;
        h->mode = c.rp;
        h->strip_z = c.sz;
        h->z_major = c.zm;
        // repeated step from pop[cur] into the other buffer: the state is untouched
        for (int w = 0; w < 2 && e == hipSuccess; ++w) e = launch_step3(h, h->cur, 0);
        if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
        for (int s = 0; s < steps && e == hipSuccess; ++s) e = launch_step3(h, h->cur, 0);
        if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) break;
        if (ms < best) {
            best = ms;
            best_s = c.sz;
            best_tx = c.tx;
            best_ty = c.ty;
            best_rp = c.rp;
            best_zm = c.zm;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->strip_z = e == hipSuccess ? best_s : keep;
    h->tile_x = e == hipSuccess ? best_tx : keep_tx;
    h->tile_y = e == hipSuccess ? best_ty : keep_ty;
    h->mode = e == hipSuccess ? best_rp : keep_rp;
    h->z_major = e == hipSuccess ? best_zm : keep_zm;
    if (e != hipSuccess) return fail3(h, LBAC_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
    if (us_per_step) *us_per_step = 1000.0 * best / steps;
    return LBAC_OK;
}

int lbac3_bytes_per_node(lbac3_ctx* h, double* bytes) {
    if (!h || !bytes) return LBAC_EINVAL;
    *bytes = 2.0 * 19 * h->elem_bytes;
    return LBAC_OK;
}

const char* lbac3_last_error(lbac3_ctx* h) { return h ? h->err.c_str() : g_init_error.c_str(); }

int lbac3_free(lbac3_ctx* h) {
    if (!h) return LBAC_EINVAL;
    {
        lbac_host::DeviceGuard g(h->device);
        (void)hipStreamSynchronize(h->stream);
        release3(h);
    }
    delete h;
    return LBAC_OK;
}

}  // extern "C"
