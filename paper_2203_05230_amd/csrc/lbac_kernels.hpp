// Device code of the lbac library: the fused collide-and-stream step of the
// accurate interface-capturing LB scheme (H. Liang, arXiv:2203.05230,
// Sec. 2.2, Eq. (9)-(13)), its multi-step form, the learned closure's
// network inference, and the small kernels around them (initialisation,
// phi, reductions).
//
// Storage.  The state between steps is the post-collision population
// f*_i(x, t-1), not yet streamed, in nine planes (SoA, x fastest, rows
// `pitch` elements apart).  A step PULLS: the pre-collision population at x
// is f_i(x, t) = f*_i(x - c_i, t-1).  In the shifted low-precision form the
// planes hold g_i = f*_i - w_i phi* for i = 1..8 in 16 bits plus phi* in FP32,
// with g_0 = -(g_1 + .. + g_8), so the nine populations always sum to phi*.
//
// One-step kernel dataflow (the multi-step kernel further below chains two
// or three such steps through LDS).  A block owns a strip of bx
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

#include <type_traits>

namespace lbac {

// ---------------------------------------------------------------------------
// D2Q9 lattice (Sec. 2.2, after Eq. (10)); order rest, E, N, W, S, NE, NW, SW, SE.
__host__ __device__ constexpr int cx(int q) {
    return q == 1 || q == 5 || q == 8 ? 1 : (q == 3 || q == 6 || q == 7 ? -1 : 0);
}
__host__ __device__ constexpr int cy(int q) {
    return q == 2 || q == 5 || q == 6 ? 1 : (q == 4 || q == 7 || q == 8 ? -1 : 0);
}
// The population with velocity (cx, -cy): the mirror image of q under y -> -y.
__host__ __device__ constexpr int mirror_q(int q) {
    return q == 2 ? 4 : (q == 4 ? 2 : (q == 5 ? 8 : (q == 8 ? 5 : (q == 6 ? 7 : (q == 7 ? 6 : q)))));
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
    const float* vtabf;     // the same table rounded to FP32
    const int64_t* t_dev;   // step count at the start of this launch sequence
    int32_t k;              // this launch is step t_dev[0] + k
    double period_T;        // s(t) = cos(pi t / period_T) when > 0, else 1
    double eps, tau, delta;
    int32_t nbx, nby;       // tiles of the step launch (columns blocks x strips)
    int32_t n_xcd;          // XCDs the workgroups are dispatched over
    const uint16_t* cl_w;   // learned closure: packed BF16 weights (ClosurePack layout), or null
    const float* cl_b;      // learned closure: biases b1[64], b2[64], b3[32] (rows >= 2 zero)
    float cl_theta;         // closure band: theta < clip(phi) < 1 - theta
    uint64_t* cl_mask;      // closure: band mask, one 64-bit word per 64 columns of a row, or null
    int32_t cl_words;       // words per row of cl_mask
};

constexpr int kWave = 64;  // wavefront width of CDNA

__device__ __forceinline__ int wrap_idx(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Tile order shared by the launch kernels: workgroups are dispatched
// round-robin over the XCDs, so XCD (g mod n_xcd) is given one contiguous
// row-major range of block tiles; horizontally adjacent tiles then share an
// L2 and run together.
__device__ __forceinline__ int xcd_tile(int g, int ntile, int n_xcd) {
    const int xcd = g % n_xcd, k = g / n_xcd;
    const int per = ntile / n_xcd, extra = ntile % n_xcd;
    return xcd * per + min(xcd, extra) + k;
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
// Sums over the populations, in an order that the mirror y -> -y of the
// lattice (which swaps populations 2 and 4, 5 and 8, 6 and 7) leaves
// unchanged: a kernel that marches a strip downward in the mirrored frame
// then rounds exactly like one working in the lattice frame.  sum9 over all
// nine, sum_moving over 1..8.
template <typename R>
__device__ __forceinline__ R sum_moving(const R (&f)[9]) {
    return ((f[1] + f[3]) + (f[2] + f[4])) + ((f[5] + f[8]) + (f[6] + f[7]));
}
template <typename R>
__device__ __forceinline__ R sum9(const R (&f)[9]) {
    return f[0] + sum_moving(f);
}

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

// Shifted 16-bit storage.  The planes hold phi* = sum_i f*_i in FP32 and
// g_i = f*_i - w_i phi* (i >= 1) in 16 bits (g_0 is implied).  load() returns
// v[0] = phi* and the moving populations they stand for, v_i = w_i phi* + g_i
// (i >= 1), in FP32.  The pulled sum is then formed by shifted_phi below.
template <typename H>
struct StoreShifted {
    static constexpr bool kShifted = true;
    __device__ __forceinline__ static void load(const StepArgs& a, int64_t off, float (&v)[9]) {
        const H* s = static_cast<const H*>(a.src);
        const float ph = a.src_phi[off];
        v[0] = ph;
#pragma unroll
        for (int q = 1; q < 9; ++q) v[q] = __builtin_fmaf(wq<float>(q), ph, h2f<H>(s[(q - 1) * a.plane_stride + off]));
    }
    // v_q at `off` for a moving population (q >= 1)
    __device__ __forceinline__ static float load_one(const StepArgs& a, int64_t off, int q) {
        const H* s = static_cast<const H*>(a.src);
        return __builtin_fmaf(wq<float>(q), a.src_phi[off], h2f<H>(s[(q - 1) * a.plane_stride + off]));
    }
};

// phi(x) = sum_i f*_i(x - c_i) for shifted storage, as
// phi*(x) + sum_{i>=1} [v_i(x - c_i) - v_i(x)] (the rest population cancels):
// each difference of neighbouring values of one population is exact in FP32
// wherever they lie within a factor two of each other (Sterbenz's lemma) and
// small elsewhere, so the sum carries about one rounding of phi, and what one
// node gains from v_i(y) another loses exactly: the 16-bit roundings of the
// stored values cannot move the mass.  pulled[i] = v_i(x - c_i), own[i] = v_i(x);
// summed in the mirror-invariant order of sum_moving.
__device__ __forceinline__ float shifted_phi(float phistar, const float (&pulled)[9], const float (&own)[9]) {
    float d[9];
#pragma unroll
    for (int q = 1; q < 9; ++q) d[q] = pulled[q] - own[q];
    d[0] = 0.f;
    return phistar + sum_moving(d);
}
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
// Fast elementary functions for the FP32 path (hardware log2, reciprocal and
// square root, about 1 ulp); the FP64 path keeps the correctly rounded ones.
template <typename R>
struct Math;
template <>
struct Math<float> {
    __device__ __forceinline__ static float log2(float x) { return __builtin_amdgcn_logf(x); }
    __device__ __forceinline__ static float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    __device__ __forceinline__ static float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
};
template <>
struct Math<double> {
    __device__ __forceinline__ static double log2(double x) { return ::log2(x); }
    __device__ __forceinline__ static double rcp(double x) { return 1.0 / x; }
    __device__ __forceinline__ static double sqrt(double x) { return ::sqrt(x); }
};

// ---------------------------------------------------------------------------
// Node arithmetic shared by every kernel variant.  The library is compiled
// with automatic multiply-add contraction off and the fused operations are
// written out here, so every variant rounds identically and the variants
// (and the batched form) agree bit for bit.

__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }

// min(max(p, 0), 1) for finite p (the clip of Eq. (13)): one median-of-three
// instruction in FP32.  A signed zero may come out as either zero, which no
// use distinguishes (each adds delta, subtracts from 1 or compares with a
// positive bound).
__device__ __forceinline__ float clip01(float p) { return __builtin_amdgcn_fmed3f(p, 0.f, 1.f); }
__device__ __forceinline__ double clip01(double p) { return __builtin_fmin(__builtin_fmax(p, 0.0), 1.0); }

// Row factor of the velocity tables (Ay or By at row y): the same for the
// whole workgroup, read through the constant address space so that it is a
// scalar load, which does not queue behind the rows being prefetched.
__device__ __forceinline__ double row_factor(const double* vtab, int64_t i) {
    return ((const __attribute__((address_space(4))) double*)vtab)[i];
}
__device__ __forceinline__ float row_factor(const float* vtabf, int64_t i) {
    return ((const __attribute__((address_space(4))) float*)vtabf)[i];
}

// Per-step constants of the update.
template <typename R>
struct NodeConst {
    R eps, delta, psi_scale, s_scale, omega, kforce, keep, s_now, s_old;
    bool first;
    __device__ __forceinline__ NodeConst() {}
    __device__ __forceinline__ NodeConst(const StepArgs& a, int64_t t) {
        first = (t == 0);
        s_now = R(time_factor(a.period_T, t));
        s_old = first ? s_now : R(time_factor(a.period_T, t - 1));
        eps = R(a.eps);
        delta = R(a.delta);
        psi_scale = R(a.eps * 0.69314718055994530942);  // eps ln 2: psi = eps ln2 (log2 a - log2 b)
        s_scale = R(1.0 / (a.eps * (1.0 + 2.0 * a.delta) * (1.0 + 2.0 * a.delta)));
        omega = R(1.0 / a.tau);
        kforce = R(1.0 - 0.5 / a.tau);
        keep = R(1.0 - 1.0 / a.tau);
    }
};

// The field whose gradient gives the normal: psi of Eq. (13) (clipped phi),
// or phi itself for the conventional model of Eq. (1).
template <typename R, int MODEL>
__device__ __forceinline__ R normal_source(R phi, const NodeConst<R>& k) {
    if (MODEL == MODEL_CONVENTIONAL) return phi;
    const R pc = clip01(phi);
    return k.psi_scale * (Math<R>::log2(pc + k.delta) - Math<R>::log2(R(1) - pc + k.delta));
}

// Isotropic gradient grad chi = sum_i w_i c_i chi(x + c_i) / c_s^2 from the
// eight neighbours of a node.
template <typename R>
__device__ __forceinline__ void iso_gradient(R pE, R pW, R pN, R pS, R pNE, R pNW, R pSE, R pSW, R& gx, R& gy) {
    gx = fmaR(pE - pW, R(1.0 / 3.0), ((pNE - pNW) + (pSE - pSW)) * R(1.0 / 12.0));
    gy = fmaR(pN - pS, R(1.0 / 3.0), ((pNE + pNW) - (pSE + pSW)) * R(1.0 / 12.0));
}

// Bracket of Eq. (11): d_t(phi u) by explicit Euler plus c_s^2 S n, with
// n = grad psi / (|grad psi| + delta) (Eq. (13)) and S the sharpening
// magnitude (Eq. (6) in the algebraic form below, or phi (1 - phi)/eps for
// the conventional model).  u, v at t; uo, vo at t - 1; phio = phi at t - 1.
template <typename R, int MODEL>
__device__ __forceinline__ void flux_bracket(R gx, R gy, R phi, R phio, R u, R v, R uo, R vo, const NodeConst<R>& k,
                                             R& Gx, R& Gy) {
    const R inv = Math<R>::rcp(Math<R>::sqrt(fmaR(gx, gx, gy * gy)) + k.delta);
    R S;
    if (MODEL == MODEL_CONVENTIONAL) {
        S = phi * (R(1) - phi) / k.eps;
    } else {
        // (1 - tanh^2(psi/(2 eps)))/(4 eps) = a b / (eps (a + b)^2), a = phi_c + delta, b = 1 - phi_c + delta
        const R pc = clip01(phi);
        S = (pc + k.delta) * (R(1) - pc + k.delta) * k.s_scale;
    }
    const R Sn = R(1.0 / 3.0) * S * inv;
    Gx = fmaR(Sn, gx, fmaR(phi, u, -(phio * uo)));
    Gy = fmaR(Sn, gy, fmaR(phi, v, -(phio * vo)));
}

// Eq. (9)-(11): f*_i = (1 - 1/tau) f_i + w_i [phi/tau + 3 c_i.(phi u/tau + (1 - 1/(2 tau)) G)].
// Eq. (9) conserves sum_i f_i = phi exactly; the rest population is taken as
// the remainder so that rounded weights (sum_i w_i != 1 in floating point)
// cannot make the total mass drift.
template <typename R>
__device__ __forceinline__ void collide(const R* fp, R phi, R u, R v, R Gx, R Gy, const NodeConst<R>& k,
                                        R (&out)[9]) {
    const R A0 = k.omega * phi;
    const R bx = R(3) * fmaR(A0, u, k.kforce * Gx);
    const R by = R(3) * fmaR(A0, v, k.kforce * Gy);
    const R a1 = wq<R>(1) * A0, x1 = wq<R>(1) * bx, y1 = wq<R>(1) * by;
    const R a5 = wq<R>(5) * A0, x5 = wq<R>(5) * bx, y5 = wq<R>(5) * by;
    out[1] = fmaR(k.keep, fp[1], a1 + x1);
    out[2] = fmaR(k.keep, fp[2], a1 + y1);
    out[3] = fmaR(k.keep, fp[3], a1 - x1);
    out[4] = fmaR(k.keep, fp[4], a1 - y1);
    out[5] = fmaR(k.keep, fp[5], (a5 + x5) + y5);
    out[6] = fmaR(k.keep, fp[6], (a5 - x5) + y5);
    out[7] = fmaR(k.keep, fp[7], (a5 - x5) - y5);
    out[8] = fmaR(k.keep, fp[8], (a5 + x5) - y5);
    out[0] = phi - sum_moving(out);
}

// Uniform per-plane base pointers and 32-bit byte offsets (a plane is far
// below 4 GiB), so a load or store is one instruction on a scalar base.
// Stores go through raw buffer resources so that a lane with nothing to
// store passes an offset beyond the resource's range, which the hardware
// drops: every lane issues the same stores, no branch surrounds them, and the
// compiler keeps exact count of the memory operations in flight (a branch
// around stores makes it wait for all of them before the next row's loads
// may be consumed).  A plane is below 2 GiB (checked at set-up), so the drop
// offset 2^31 is outside every plane.
constexpr uint32_t kDropOffset = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(void* base) {
    // raw buffer (stride 0), range 2^31 - 1 bytes; dword 3 = 32-bit data format
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, 0x7FFFFFFF, 0x00020000);
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)off, 0, 0);
}
// the same with the non-temporal cache hint (bit 1 of the cache-policy
// operand): the line is not kept in the L2 for reuse
__device__ __forceinline__ void bstore_nt(float v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)off, 0, 2);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    const unsigned long long bits = __double_as_longlong(v);
    u32x2 w;
    w.x = (unsigned int)bits;
    w.y = (unsigned int)(bits >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(w, r, (int)off, 0, 0);
}
// 16-bit store; aux 2 is the non-temporal hint
template <typename H>
__device__ __forceinline__ void bstore16(H v, __amdgpu_buffer_rsrc_t r, uint32_t off, int aux) {
    if (aux == 2)
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)off, 0, 2);
    else
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)off, 0, 0);
}

template <typename R, int ST>
struct Io;

template <typename R>
struct Io<R, ST_PLAIN> {
    static constexpr bool kShifted = false;
    const char* s[9];
    char* d[9];
    __device__ __forceinline__ explicit Io(const StepArgs& a) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            s[q] = static_cast<const char*>(a.src) + (size_t)q * a.plane_stride * sizeof(R);
            d[q] = static_cast<char*>(a.dst) + (size_t)q * a.plane_stride * sizeof(R);
        }
    }
    // In the mirrored frame (y -> -y) population q lives in the plane of its
    // mirror image: 2 <-> 4, 5 <-> 8, 6 <-> 7.
    __device__ __forceinline__ Io(const StepArgs& a, bool mirror) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const int m = mirror ? mirror_q(q) : q;
            s[q] = static_cast<const char*>(a.src) + (size_t)m * a.plane_stride * sizeof(R);
            d[q] = static_cast<char*>(a.dst) + (size_t)m * a.plane_stride * sizeof(R);
        }
    }
    __device__ __forceinline__ void load(uint32_t off, R (&v)[9]) const {
        const uint32_t b = off * (uint32_t)sizeof(R);
#pragma unroll
        for (int q = 0; q < 9; ++q) v[q] = *reinterpret_cast<const R*>(s[q] + b);
    }
    // stores v at element offset off when `on`; a lane with on == false stores nothing
    __device__ __forceinline__ void store(bool on, uint32_t off, const R (&v)[9], R /*phi*/) const {
        const uint32_t b = on ? off * (uint32_t)sizeof(R) : kDropOffset;
#pragma unroll
        for (int q = 0; q < 9; ++q) bstore(v[q], plane_rsrc(d[q]), b);
    }
    // the same, non-temporal (FP32 only): used where the L2 is better spent
    // on rows that are read again
    __device__ __forceinline__ void store_nt(bool on, uint32_t off, const float (&v)[9], float /*phi*/) const {
        const uint32_t b = on ? off * 4u : kDropOffset;
#pragma unroll
        for (int q = 0; q < 9; ++q) bstore_nt(v[q], plane_rsrc(d[q]), b);
    }
};

template <typename H>
struct IoShifted {
    static constexpr bool kShifted = true;
    const char* s[9];  // s[0]: phi* plane (FP32); s[1..8]: g planes (16-bit)
    char* d[9];
    // mirror: the mirrored frame y -> -y, population q read from and written
    // to the plane of its mirror image (the phi* plane is its own image)
    __device__ __forceinline__ explicit IoShifted(const StepArgs& a, bool mirror = false) {
        s[0] = reinterpret_cast<const char*>(a.src_phi);
        d[0] = reinterpret_cast<char*>(a.dst_phi);
#pragma unroll
        for (int q = 1; q < 9; ++q) {
            const int m = mirror ? mirror_q(q) : q;
            s[q] = static_cast<const char*>(a.src) + (size_t)(m - 1) * a.plane_stride * sizeof(H);
            d[q] = static_cast<char*>(a.dst) + (size_t)(m - 1) * a.plane_stride * sizeof(H);
        }
    }
    // v[0] = phi*, v[i] = w_i phi* + g_i (see StoreShifted)
    __device__ __forceinline__ void load(uint32_t off, float (&v)[9]) const {
        const float ph = *reinterpret_cast<const float*>(s[0] + off * 4u);
        v[0] = ph;
#pragma unroll
        for (int q = 1; q < 9; ++q) v[q] = __builtin_fmaf(wq<float>(q), ph, h2f<H>(*reinterpret_cast<const H*>(s[q] + off * 2u)));
    }
    // stores g_i = v_i - w_i phi and phi* = phi (the sum the collision
    // conserves) when `on`; a lane with on == false stores nothing
    __device__ __forceinline__ void store(bool on, uint32_t off, const float (&v)[9], float phi) const {
        const uint32_t b2 = on ? off * 2u : kDropOffset, b4 = on ? off * 4u : kDropOffset;
#pragma unroll
        for (int q = 1; q < 9; ++q) bstore16(f2h<H>(__builtin_fmaf(-wq<float>(q), phi, v[q])), plane_rsrc(d[q]), b2, 0);
        bstore(phi, plane_rsrc(d[0]), b4);
    }
    // the same with the non-temporal hint
    __device__ __forceinline__ void store_nt(bool on, uint32_t off, const float (&v)[9], float phi) const {
        const uint32_t b2 = on ? off * 2u : kDropOffset, b4 = on ? off * 4u : kDropOffset;
#pragma unroll
        for (int q = 1; q < 9; ++q) bstore16(f2h<H>(__builtin_fmaf(-wq<float>(q), phi, v[q])), plane_rsrc(d[q]), b2, 2);
        bstore_nt(phi, plane_rsrc(d[0]), b4);
    }
};
template <>
struct Io<float, ST_F16> : IoShifted<__half> {
    using IoShifted<__half>::IoShifted;
};
template <>
struct Io<float, ST_BF16> : IoShifted<__hip_bfloat16> {
    using IoShifted<__hip_bfloat16>::IoShifted;
};

// FP32 plain storage read and written with device-scope accesses (the
// cache-policy bit sc1, with which the compiler implements relaxed atomic
// loads and stores at agent scope): each access is coherent across the
// XCDs' L2 caches by itself.  The batched form, whose workgroups hand tiles
// to each other through per-item progress counters, uses it so that a
// producer only waits for its own stores to complete before it publishes,
// and a consumer that has seen the counter reads current values, with no
// writeback or invalidation of the whole L2.
//
// One buffer resource per population buffer, with the plane of population q
// selected by the scalar offset m(q) * plane bytes (m(q): q or its mirror
// image): eight scalar registers for the two buffers instead of four per
// plane and buffer, which had made the tile function spill scalar registers
// into vector lanes (a tenth more vector instructions per row).  Requires
// the nine planes of a buffer to span less than 2^31 bytes, so that every
// in-range offset, the scalar offset included, stays below the resource's
// range and the dropped stores' offset above it; the batch's set-up rejects
// larger instances.
struct IoCoherent {
    static constexpr bool kShifted = false;
    static constexpr int kSc1 = 16;  // cache-policy operand: sc1 (device scope)
    static constexpr int kNt = 2;    // cache-policy operand: nt (non-temporal)
    __amdgpu_buffer_rsrc_t sr, dr;
    uint32_t pb[9];  // byte offset of the plane read and written for population q
    // the bases and the stride pass through readfirstlane: they are uniform,
    // and saying so keeps the resources and offsets in scalar registers where
    // the compiler cannot prove it (it would wrap every access in a loop over
    // the distinct values)
    __device__ __forceinline__ static void* uniform_ptr(const void* p) {
        const uint64_t v = (uint64_t)p;
        return (void*)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(v >> 32)) << 32) |
                       (uint32_t)__builtin_amdgcn_readfirstlane((int)v));
    }
    __device__ __forceinline__ IoCoherent(const StepArgs& a, bool mirror)
        : sr(plane_rsrc(uniform_ptr(a.src))), dr(plane_rsrc(uniform_ptr(a.dst))) {
        const uint32_t ps = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.plane_stride) * 4u;
        const bool m = __builtin_amdgcn_readfirstlane((int)mirror) != 0;
#pragma unroll
        for (int q = 0; q < 9; ++q) pb[q] = (uint32_t)(m ? mirror_q(q) : q) * ps;
    }
    __device__ __forceinline__ void load(uint32_t off, float (&v)[9]) const {
        const uint32_t b = off * 4u;
#pragma unroll
        for (int q = 0; q < 9; ++q)
            v[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(sr, (int)b, (int)pb[q], kSc1));
    }
    // device-scope stores with the non-temporal hint (the hint leaves the
    // scope alone: the stored rows are not read again in the pass, and the L2
    // keeps the rows and halo columns other items read)
    __device__ __forceinline__ void store_nt(bool on, uint32_t off, const float (&v)[9], float /*phi*/) const {
        const uint32_t b = on ? off * 4u : kDropOffset;
#pragma unroll
        for (int q = 0; q < 9; ++q)
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[q]), dr, (int)b, (int)pb[q], kSc1 | kNt);
    }
};

// Shifted 16-bit storage (g_i planes and the FP32 phi* plane, as IoShifted)
// read and written with device-scope accesses, for the batched form: one
// buffer resource for the g planes of a buffer (the plane chosen by the
// scalar offset, as IoCoherent) and one for its phi* plane.  Requires the
// eight g planes to span less than 2^31 bytes.
template <typename H>
struct IoCoherentShifted {
    static constexpr bool kShifted = true;
    static constexpr int kSc1 = IoCoherent::kSc1;
    __amdgpu_buffer_rsrc_t sg, dg, sp, dp;
    uint32_t pb[9];  // byte offset of the g plane read and written for population q (q >= 1)
    __device__ __forceinline__ IoCoherentShifted(const StepArgs& a, bool mirror)
        : sg(plane_rsrc(IoCoherent::uniform_ptr(a.src))),
          dg(plane_rsrc(IoCoherent::uniform_ptr(a.dst))),
          sp(plane_rsrc(IoCoherent::uniform_ptr(a.src_phi))),
          dp(plane_rsrc(IoCoherent::uniform_ptr(a.dst_phi))) {
        const uint32_t ps = (uint32_t)__builtin_amdgcn_readfirstlane((int)a.plane_stride) * (uint32_t)sizeof(H);
        const bool m = __builtin_amdgcn_readfirstlane((int)mirror) != 0;
        pb[0] = 0;
#pragma unroll
        for (int q = 1; q < 9; ++q) pb[q] = (uint32_t)((m ? mirror_q(q) : q) - 1) * ps;
    }
    // v[0] = phi*, v[i] = w_i phi* + g_i
    __device__ __forceinline__ void load(uint32_t off, float (&v)[9]) const {
        const float ph =
            __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(sp, (int)(off * 4u), 0, kSc1));
        v[0] = ph;
#pragma unroll
        for (int q = 1; q < 9; ++q) {
            const unsigned short g = __builtin_amdgcn_raw_buffer_load_b16(sg, (int)(off * 2u), (int)pb[q], kSc1);
            v[q] = __builtin_fmaf(wq<float>(q), ph, h2f<H>(__builtin_bit_cast(H, g)));
        }
    }
    // stores g_i = v_i - w_i phi and phi* = phi when `on` (device scope,
    // non-temporal, as IoCoherent)
    __device__ __forceinline__ void store_nt(bool on, uint32_t off, const float (&v)[9], float phi) const {
        const uint32_t b2 = on ? off * 2u : kDropOffset, b4 = on ? off * 4u : kDropOffset;
#pragma unroll
        for (int q = 1; q < 9; ++q)
            __builtin_amdgcn_raw_buffer_store_b16(
                __builtin_bit_cast(unsigned short, f2h<H>(__builtin_fmaf(-wq<float>(q), phi, v[q]))), dg, (int)b2,
                (int)pb[q], kSc1 | IoCoherent::kNt);
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(phi), dp, (int)b4, 0, kSc1 | IoCoherent::kNt);
    }
};

// ---------------------------------------------------------------------------
// The step on one tile, block-wide variant.
//
// A block owns BX aligned columns [x0, x0 + BX) and marches a strip of
// a.strip_h rows.  Threads 0..BX-1 each own one column; one extra wavefront
// (threads BX..BX+63) serves the two-column halo on each side: its lanes 0..3
// load the halo columns and lanes 0..1 form psi there, so no column wave
// carries halo work and every row of every plane is read and written as
// whole, aligned cache lines.  Rows are shared through a three-row LDS ring.
template <typename R, int BX>
struct TileLds {
    R ring[3][9][BX + 4];  // rows r-2..r of every plane; index j <-> column x0 - 2 + j
    R sring[3][BX + 2];    // psi on the last three centre rows; index j <-> column x0 - 1 + j
};

template <int BX>
__host__ __device__ constexpr int block_threads() {
    return BX + 64;
}

// One step on the tile of column block `bxi` and strip `syi` at time t.  The
// strip is marched upward, or downward when `down` is set (the kernel flips
// odd strips so that two strips sharing a boundary read its halo rows at
// about the same time, while they are still in cache).
//
// Every iteration issues the same global loads, LDS writes and stores from
// every thread, with no branch around them: work that has no target is
// pointed at a harmless one (a duplicate LDS write of the same value, a
// dropped store, a reload of a row already read).  The compiler then counts
// the memory operations in flight exactly and keeps PF rows of loads
// outstanding across the row's arithmetic.
template <typename R, int ST, int MODEL, int BX, int PF>
__device__ __forceinline__ void step_tile_lds(const StepArgs& a, int bxi, int syi, int64_t t, bool down,
                                              TileLds<R, BX>& lds) {
    auto& ring = lds.ring;
    auto& sring = lds.sring;
    const int l = threadIdx.x;
    const bool colw = l < BX;                 // a column thread
    const int h = l - BX;                     // halo lane (halo wavefront)
    const int x0 = bxi * BX;
    const int w = min(BX, a.nx - x0);
    const int ys = syi * a.strip_h;
    const int hh = min(a.strip_h, a.ny - ys);
    const bool act = colw && l < w;           // owns column x0 + l
    // Column each thread loads and the ring index it fills: a column thread
    // its own column (idle ones of a narrow last tile: the tile's last
    // column, a duplicate); halo lanes 0..3 the halo columns x0-2, x0-1,
    // x0+w, x0+w+1; the other halo lanes duplicate a column thread's load.
    int lcol, lj;
    if (colw) {
        const int c = min(l, w - 1);
        lcol = x0 + c;
        lj = c + 2;
    } else if (h < 4) {
        lj = h < 2 ? h : w + h;
        lcol = wrap_idx(x0 - 2 + lj, a.nx);
    } else {
        const int c = min(h - 4, w - 1);
        lcol = x0 + c;
        lj = c + 2;
    }
    const bool pl = act || (!colw && h < 2);  // forms psi
    const int pj = act ? l + 2 : (h == 0 ? 1 : w + 2);  // ring index of that column
    const int x = x0 + l;
    const Io<R, ST> io(a);
    lds_barrier();  // the LDS may still be read by a previous tile of this block

    const NodeConst<R> kc(a, t);
    const R Axl = act ? R(a.vtab[x]) : R(0);
    const R Bxl = act ? R(a.vtab[a.nx + x]) : R(0);

    R fprev[9], fcur[9], out[9];
    R phiprev = R(0), phicur = R(0), phi_out = R(0);
    // closure band mask: one word per 64 columns of a row (stores dropped when
    // the closure is off, or for the halo wavefront and waves past the grid)
    const __amdgpu_buffer_rsrc_t mrs = __builtin_amdgcn_make_buffer_rsrc(
        a.cl_mask, (short)0, a.cl_mask ? 0x7FFFFFFF : 0, 0x00020000);
    const int mcol = x0 + (l & ~(kWave - 1));  // first column of this wavefront
    const bool mlane = colw && (l & (kWave - 1)) == 0 && mcol < a.nx;
    const float th = a.cl_theta;
    R P2 = R(0), P1 = R(0), P0 = R(0);  // own-column phi at t-1, rows r-2, r-1, r
#pragma unroll
    for (int q = 0; q < 9; ++q) fprev[q] = fcur[q] = out[q] = R(0);

    const int iters = hh + 4;
    // lattice row that enters the ring at iteration it (clamped: the loads
    // issued past the strip's last row repeat its last row and are not used)
    auto row_of = [&](int it) {
        it = min(it, iters - 1);
        return (uint32_t)wrap_idx(down ? ys + hh + 1 - it : ys - 2 + it, a.ny);
    };
    auto body = [&](const int it, R(&nv)[9]) __attribute__((always_inline)) {
        // row r = start + dir * it enters the ring; phi and psi are formed on the
        // centre row c = r - dir; row c - dir is updated
        const int slot = it % 3;         // ring slot of row r
        const int slot1 = (it + 2) % 3;  // centre row c
        const int slot2 = (it + 1) % 3;  // row r - 2 dir
        const int slot_n = down ? slot2 : slot;  // row c + 1
        const int slot_s = down ? slot : slot2;  // row c - 1
        // ---- row r into the ring
        {
#pragma unroll
            for (int q = 0; q < 9; ++q) ring[slot][q][lj] = nv[q];
            // phi at t-1 on this row: the sum of the stored values (phi* itself
            // for shifted storage)
            P0 = Io<R, ST>::kShifted ? nv[0] : sum9(nv);
        }
        // ---- prefetch row r + PF dir into the registers just consumed
        io.load(row_of(it + PF) * (uint32_t)a.pitch + lcol, nv);
        lds_barrier();

        // ---- phi (Eq. (12)) and psi (Eq. (13)) on the centre row
        if (it >= 2 && pl) {
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int sl = cy(q) == 1 ? slot_s : (cy(q) == 0 ? slot1 : slot_n);
                fcur[q] = ring[sl][q][pj - cx(q)];
            }
            R s;
            if constexpr (Io<R, ST>::kShifted) {
                R own[9];
#pragma unroll
                for (int q = 0; q < 9; ++q) own[q] = ring[slot1][q][pj];
                s = shifted_phi(own[0], fcur, own);  // the collision forms the rest population itself
            } else {
                s = sum9(fcur);
            }
            phicur = s;
            sring[slot][pj - 1] = normal_source<R, MODEL>(s, kc);
        }
        lds_barrier();

        // ---- update row y = c - dir.  The first four iterations fill the
        // pipeline: they skip the arithmetic (a branch without memory
        // operations) and their stores are dropped.
        const bool st = act && it >= 4;
        const int y = min(max(down ? ys + hh + 3 - it : ys + it - 4, 0), a.ny - 1);
        if (it >= 4) {
            // psi rows y-1, y, y+1 (the newest psi row is y + dir)
            const int s0 = (it + 2) % 3;
            const int sm = down ? it % 3 : (it + 1) % 3;
            const int sp = down ? (it + 1) % 3 : it % 3;
            const int j = colw ? l + 1 : 1;
            const R pE = sring[s0][j + 1], pW = sring[s0][j - 1];
            const R pN = sring[sp][j], pS = sring[sm][j];
            const R pNE = sring[sp][j + 1], pNW = sring[sp][j - 1];
            const R pSE = sring[sm][j + 1], pSW = sring[sm][j - 1];
            R gx, gy, Gx, Gy;
            iso_gradient(pE, pW, pN, pS, pNE, pNW, pSE, pSW, gx, gy);
            const R phi = phiprev;
            const R Ayv = R(row_factor(a.vtab, 2 * a.nx + y)), Byv = R(row_factor(a.vtab, 2 * a.nx + a.ny + y));
            const R uxr = Axl * Ayv, uyr = Bxl * Byv;
            flux_bracket<R, MODEL>(gx, gy, phi, kc.first ? phi : P2, kc.s_now * uxr, kc.s_now * uyr, kc.s_old * uxr,
                                   kc.s_old * uyr, kc, Gx, Gy);
            collide(fprev, phi, kc.s_now * uxr, kc.s_now * uyr, Gx, Gy, kc, out);
            phi_out = phi;
        }
        io.store(st, (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x, out, phi_out);
        {
            const float pc = (float)clip01(phi_out);
            const uint64_t m = __ballot(st && pc > th && pc < 1.0f - th);
            const uint32_t moff = mlane && it >= 4 ? (uint32_t)(y * a.cl_words + (mcol >> 6)) * 8u : kDropOffset;
            typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
            u32x2 mw;
            mw.x = (unsigned int)m;
            mw.y = (unsigned int)(m >> 32);
            __builtin_amdgcn_raw_buffer_store_b64(mw, mrs, (int)moff, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) fprev[q] = fcur[q];
        phiprev = phicur;
        P2 = P1;
        P1 = P0;
    };
    // PF rows in flight: row r + PF dir is loaded while row r is processed;
    // with PF = 2 the loop alternates two register sets, so consuming one
    // never waits for the loads into the other
    R na[9], nb[9];
    io.load(row_of(0) * (uint32_t)a.pitch + lcol, na);
    if constexpr (PF == 1) {
        for (int it = 0; it < iters; ++it) body(it, na);
    } else {
        io.load(row_of(1) * (uint32_t)a.pitch + lcol, nb);
        for (int it = 0; it < iters; it += 2) {
            body(it, na);
            if (it + 1 < iters) body(it + 1, nb);
        }
    }
}

template <typename R, int ST, int MODEL, int BX, int PF>
__global__ __launch_bounds__(block_threads<BX>()) void step_kernel_lds(StepArgs a) {
    __shared__ TileLds<R, BX> lds;
    // XCD-aware tile order: workgroups are dispatched round-robin over the
    // XCDs, so XCD (g mod n_xcd) is given one contiguous row-major range of
    // tiles; horizontally adjacent tiles then share an L2 and run together
    const int ntile = a.nbx * a.nby;
    const int g = blockIdx.x;
    const int xcd = g % a.n_xcd, k = g / a.n_xcd;
    const int per = ntile / a.n_xcd, extra = ntile % a.n_xcd;
    const int tile = xcd * per + min(xcd, extra) + k;
    const int bxi = tile % a.nbx, syi = tile / a.nbx;
    step_tile_lds<R, ST, MODEL, BX, PF>(a, bxi, syi, a.t_dev[0] + a.k, (syi & 1) != 0, lds);
}

// ---- learned closure: BF16 MFMA inference ------------------------------------
// The network runs on the 64 samples of a wavefront, 16 at a time (N-tiles),
// as three chained products Z^T = W H^T with gfx950's 16x16x32 BF16 MFMA
// (features on the M side in tiles of 16, samples on the N side, FP32
// accumulation).  A lane of group g (lanes 16g .. 16g + 15) supplies the
// operand elements e = 0..7 of the K-slice "g" of each product, for A and B
// alike, so the product is the same whatever order the unit sums a K-slice
// in as long as both operands number their K entries the same way.  The
// accumulator of one layer holds, in lane (g, n), the features
// 16 mt + 4 g + {0..3} of M-tile mt for sample n; two M-tiles side by side
// are the next layer's B operand, which defines that layer's K numbering, and
// the packed weights (built by closure_pack_kernel) follow it:
//   layer 1, one K-step of 32:      element e <-> input 8 g + e (inputs 25..31 zero);
//   layers 2 and 3, K-step ks:      element e <-> feature 32 ks + 16 (e / 4) + 4 g + (e % 4).
// Packed weights, BF16, each lane's eight elements of one (M-tile, K-step)
// contiguous (16 bytes): W1 [mt 4][g 4][row 16][8], W2 [mt 4][ks 2][g 4]
// [row 16][8], W3 [ks 2][g 4][row 16][8] (rows 2..15 zero).  Each output
// column depends on its own sample only, so a node's correction is the same
// whichever nodes share its wavefront.  The small tiles keep the registers
// the network needs (about forty) low enough for it to run inside the
// multi-step kernel's loop.
constexpr int kClW1 = 0, kClW2 = kClW1 + 64 * 32, kClW3 = kClW2 + 64 * 64, kClWN = kClW3 + 16 * 64;
constexpr int kClB1 = 0, kClB2 = 64, kClB3 = 128, kClBN = 160;

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kClWaves = 4;  // wavefronts per block of the closure kernel

struct ClosureLds {
    uint16_t w[kClWN];
    float b[kClBN];
    uint16_t x[kClWaves][kWave * 32];  // each wavefront's stencils, one row of 32 BF16 per sample
};

__device__ __forceinline__ uint16_t bf16_bits(float f) {
    // round to nearest even (inputs are finite)
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// tanh form of GELU, tanh(u) = 1 - 2 / (exp(2u) + 1) with the hardware exp2
__device__ __forceinline__ float gelu_fast(float x) {
    const float u = 0.7978845608028654f * (x + 0.044715f * x * x * x);
    const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * u);  // exp(2u)
    return 0.5f * x * (2.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f));
}

// GELU of two accumulator tiles (M-tiles 2 ks and 2 ks + 1), as the next
// layer's BF16 B operand for K-step ks
__device__ __forceinline__ bf16x8_t gelu_operand(const f32x4_t& lo, const f32x4_t& hi) {
    u16x8_t r;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        r[i] = bf16_bits(gelu_fast(lo[i]));
        r[4 + i] = bf16_bits(gelu_fast(hi[i]));
    }
    return __builtin_bit_cast(bf16x8_t, r);
}

// Keeps the compiler from moving memory operations across this point: the
// network runs on a rarely taken path of loops that keep most registers
// live, and loading all its weights and biases ahead would need more
// registers than the loop leaves.
__device__ __forceinline__ void mlp_fence() { asm volatile("" ::: "memory"); }

// All 64 lanes of the wavefront must call this together.  w, b: packed
// weights and biases (global memory or LDS).  xfrag(nt) returns this lane's
// layer-1 B operand for N-tile nt: elements e = 0..7 are inputs 8 g + e of
// sample 16 nt + (lane % 16), g = lane / 16, as BF16.  Returns the
// correction (cx, cy) of sample `lane`; only the samples whose bit is set in
// `want` (the same on every lane) are needed, and N-tiles without one are
// skipped (their lanes get 0).
template <typename XF>
__device__ __forceinline__ void closure_mlp(const uint16_t* __restrict__ w, const float* __restrict__ b, XF&& xfrag,
                                            uint64_t want, float& cxo, float& cyo) {
    const int l = threadIdx.x % kWave;
    const int r = l % 16, g = l / 16;
    const bf16x8_t* wv = reinterpret_cast<const bf16x8_t*>(w);
    auto bias = [&](int row0) { return *reinterpret_cast<const f32x4_t*>(&b[row0 + 4 * g]); };
    float cx = 0.f, cy = 0.f;
#pragma unroll 1
    for (int nt = 0; nt < 4; ++nt) {
        if (((want >> (16 * nt)) & 0xffffull) == 0) continue;
        mlp_fence();
        // layer 1: Z1^T (64 hidden x 16 samples) = W1 (64 x 32) X^T (32 x 16)
        const bf16x8_t x = xfrag(nt);
        f32x4_t z1[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            z1[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wv[kClW1 / 8 + (mt * 4 + g) * 16 + r], x,
                                                             bias(kClB1 + 16 * mt), 0, 0, 0);
        const bf16x8_t h10 = gelu_operand(z1[0], z1[1]), h11 = gelu_operand(z1[2], z1[3]);
        mlp_fence();
        // layer 2: Z2^T = W2 (64 x 64) H1^T (64 x 16)
        f32x4_t z2[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x4_t acc = bias(kClB2 + 16 * mt);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wv[kClW2 / 8 + ((mt * 2 + 0) * 4 + g) * 16 + r], h10, acc, 0,
                                                          0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wv[kClW2 / 8 + ((mt * 2 + 1) * 4 + g) * 16 + r], h11, acc, 0,
                                                          0, 0);
            z2[mt] = acc;
        }
        const bf16x8_t h20 = gelu_operand(z2[0], z2[1]), h21 = gelu_operand(z2[2], z2[3]);
        mlp_fence();
        // layer 3: out^T (2 of 16 rows x 16 samples) = W3 (16 x 64) H2^T
        f32x4_t o = bias(kClB3);
        o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wv[kClW3 / 8 + (0 * 4 + g) * 16 + r], h20, o, 0, 0, 0);
        o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wv[kClW3 / 8 + (1 * 4 + g) * 16 + r], h21, o, 0, 0, 0);
        // rows 0 (c_x) and 1 (c_y) of sample 16 nt + r sit in lane r (g = 0);
        // lane l takes sample l, i.e. N-tile l / 16, from lane l % 16
        const float tx = __shfl(o[0], r, kWave), ty = __shfl(o[1], r, kWave);
        if (g == nt) {
            cx = tx;
            cy = ty;
        }
    }
    cxo = cx;
    cyo = cy;
}

// The network's correction at a node, in the frame the node's populations
// are held in (mirror: the y axis reversed), added to its post-collision
// populations: Eq. (9)-(11) are linear in G, so adding c_s^2 c to G changes
// f*_i by (1 - 1/(2 tau)) w_i (c_i . c) for i >= 1 and leaves their sum phi;
// the rest population is re-formed as the remainder.  The pairs i,
// opposite(i) change by exact negatives, and a mirrored node rounds exactly
// like its mirror image.
__device__ __forceinline__ void closure_correct(float (&f)[9], float phi, float kforce, float ccx, float ccy,
                                                bool mirror) {
    const float kx = kforce * ccx, ky = kforce * (mirror ? -ccy : ccy);
    const float ax = wq<float>(1) * kx, ay = wq<float>(1) * ky;
    const float dx5 = wq<float>(5) * kx, dy5 = wq<float>(5) * ky;
    f[1] += ax;
    f[3] -= ax;
    f[2] += ay;
    f[4] -= ay;
    f[5] += dx5 + dy5;
    f[7] -= dx5 + dy5;
    f[6] += dy5 - dx5;
    f[8] -= dy5 - dx5;
    f[0] = phi - sum_moving(f);
}

// The network on up to 64 listed nodes whose inputs lie in rings of five phi
// rows in LDS (the S-step kernel with the closure): entry s of `tab`
// (s < count) names a node by its ring (high 16 bits: which of the rings,
// `ring_stride` floats apart) and its column in the ring rows (low 16 bits);
// ring row (base + d) % 5 holds phi of the row d rows ahead of the nodes' row
// in the frame the rings are filled in (mirror: the lattice's y axis
// reversed).  Lane s returns the correction (cx, cy) of node s.
__device__ __forceinline__ float2 closure_mlp_list(const uint16_t* w, const float* b, const float* rings,
                                                   int ring_stride, int row_len, int base, bool mirror,
                                                   const int* tab, int count) {
    const int lane = threadIdx.x % kWave, hf = lane / 16;
    auto xfrag = [&](int nt) {
        const int s = 16 * nt + lane % 16;
        const bool on = s < count;
        const int ent = on ? tab[s] : 0;
        const float* ring = rings + (ent >> 16) * ring_stride;
        const int jc = ent & 0xffff;
        u16x8_t v;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int kk = 8 * hf + e;
            float x = 0.f;
            if (on && kk < 25) {
                const int dy = kk / 5 - 2, dx = kk % 5 - 2;
                x = ring[((base + (mirror ? -dy : dy)) % 5) * row_len + jc + dx];
            }
            v[e] = bf16_bits(x);
        }
        return __builtin_bit_cast(bf16x8_t, v);
    };
    const uint64_t want = count >= 64 ? ~0ull : (1ull << count) - 1ull;
    float2 c;
    closure_mlp(w, b, xfrag, want, c.x, c.y);
    return c;
}

// Stages the packed closure weights into LDS (all threads of the block).
__device__ __forceinline__ void closure_stage(const StepArgs& a, ClosureLds& L) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(a.cl_w);
    uint32_t* dst = reinterpret_cast<uint32_t*>(L.w);
    for (int i = threadIdx.x; i < kClWN / 2; i += blockDim.x) dst[i] = src[i];
    for (int i = threadIdx.x; i < kClBN; i += blockDim.x) L.b[i] = a.cl_b[i];
    __syncthreads();
}

// Builds the packed BF16 weights and padded biases from the FP32 parameter
// vector W1[64][25], b1[64], W2[64][64], b2[64], W3[2][64], b3[2].
static __global__ void closure_pack_kernel(const float* __restrict__ p, uint16_t* __restrict__ w,
                                           float* __restrict__ b) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int e = t % 8, row = (t / 8) % 16, g = (t / 128) % 4;
    // feature of element e of K-slice g in K-step ks of layers 2 and 3
    auto feat = [&](int ks) { return 32 * ks + 16 * (e / 4) + 4 * g + (e % 4); };
    if (t < 64 * 32) {
        const int mt = t / 512;
        const int k = 8 * g + e;
        w[kClW1 + t] = k < 25 ? bf16_bits(p[(16 * mt + row) * 25 + k]) : 0;
    }
    if (t < 64 * 64) {
        const int ks = (t / 512) % 2, mt = t / 1024;
        w[kClW2 + t] = bf16_bits(p[1600 + 64 + (16 * mt + row) * 64 + feat(ks)]);
    }
    if (t < 16 * 64) {
        const int ks = t / 512;
        w[kClW3 + t] = row < 2 ? bf16_bits(p[1600 + 64 + 4096 + 64 + row * 64 + feat(ks)]) : 0;
    }
    if (t < 64) {
        b[kClB1 + t] = p[1600 + t];
        b[kClB2 + t] = p[1600 + 64 + 4096 + t];
    }
    if (t < 32) b[kClB3 + t] = t < 2 ? p[1600 + 64 + 4096 + 64 + 128 + t] : 0.f;
}

// ---------------------------------------------------------------------------
// S steps per pass over HBM (S = 1, 2 or 3; FP32 collide, FP32 or shifted
// 16-bit storage).
//
// The block owns the w columns [x0, x0 + w) and the hh rows [ys, ys + hh) of
// a tile and marches the strip as the block variant does, with S stages
// chained in one pipeline.  Stage 0 takes step t from the populations in HBM;
// stage k takes step t + k from the post-collision populations of stage
// k - 1, which stay in an LDS ring; stage S - 1 stores to HBM.  A stage
// reaches RC = 2 columns and rows (pull and psi gradient), so stage k works
// on the tile grown by RC (S - 1 - k) columns on each side (the block loads
// H = RC S halo columns on each side), and the strip's first and last H rows
// are loaded and computed by both neighbouring strips.  Each stage does
// exactly the arithmetic of one step of the block variant on every node, with
// the same helpers and summation orders, so with FP32 storage S steps of this
// kernel equal S launches of the one-step kernels bit for bit, while HBM is
// read and written once per S steps.  With shifted 16-bit storage the
// populations pass through 16 bits only at the launch's load and store (the
// intermediate steps keep them in FP32 in LDS), so that form rounds to its
// storage precision once per launch.
//
// With the learned closure (CL; FP32 storage) a stage also evaluates the
// network on the interface-band nodes of the row it updates and adds its
// correction to their post-collision populations exactly as the one-step
// path's correction pass does, so the results are again those of S one-step
// launches bit for bit.  The network reads the 5x5 neighbourhood of phi, so
// a stage reaches RC = 3 columns and rows, keeps its last five phi rows in
// LDS, and updates a row UL = 2 rows behind the one it forms phi on (the
// plain stages: UL = 1).
//
// Rows at iteration it (dir = +1 up the strip, -1 down it): row R enters
// stage 0's ring; stage k forms phi and psi on R - (LG k + 1) dir and updates
// R - (LG k + 1 + UL) dir, LG = UL + 2.  Two LDS barriers per iteration, as
// in the one-step kernel.
//
// Rings.  A pull f_i(x, c) = f*_i(x - c_i) needs another thread's column only
// for the six populations with c_x != 0, and each of those only from one
// row: the centre row (populations 1 and 3), the row behind it in the march
// direction (the "old" pair 5, 6; the march runs toward +y in the frame the
// stages see) or the row ahead (the "new" pair 8, 7).  So the rings hold,
// per pair, as many rows as the pull is late; the three populations with
// c_x = 0 stay in the thread's registers.  Pairs are stored c_x = +1 first.  Index j <-> column
// x0 - H - 1 + j; indices 0 and W - 1 are padding, so that every thread's
// reads at j - 1 and j + 1 stay inside its row, and W - 1 also takes the
// writes of threads past the grown tile.
template <int BX, int S, bool CL>
struct StepSGeom {
    static constexpr int RC = CL ? 3 : 2;      // columns and rows one stage reaches
    static constexpr int H = RC * S;           // halo columns (and shared rows) on each side
    static constexpr int UL = CL ? 2 : 1;      // rows from a stage's phi row back to the row it updates
    static constexpr int LG = UL + 2;          // rows between consecutive stages
    static constexpr int PER = 3 + 2 * UL;     // iterations between consecutive stages' first values
    static constexpr int D = LG * (S - 1) + 1 + UL;  // rows from the loaded row back to the stored one
    static constexpr int W = BX + 2 * H + 2;   // LDS row length
    static constexpr int NPS = UL + 2;         // psi rows kept per stage
    static constexpr int NP = UL + 3;          // depth of the phi(t - 1) history
};

template <int BX, int S, bool CL>
struct TileSLdsBase {
    static constexpr int W = StepSGeom<BX, S, CL>::W;
    float ro[S][3][2][W];                          // input of stage k: old pair, three rows
    float rm[S][2][2][W];                          // populations 1 and 3, two rows
    float rn[S][2][W];                             // new pair, one row
    float ps[S][StepSGeom<BX, S, CL>::NPS][W];     // psi of stage k on its last rows
};
template <int BX, int S, bool CL = false>
struct TileSLds : TileSLdsBase<BX, S, CL> {};
template <int BX, int S>
struct TileSLds<BX, S, true> : TileSLdsBase<BX, S, true> {
    float phr[S][5][TileSLdsBase<BX, S, true>::W];  // phi of stage k on its last five rows
    int tab[(BX + 6 * S + 63) / 64][S * 64];         // per wavefront: the band nodes of an iteration
};

// Threads of an S-step tile of at most BX columns: the BX + 2H columns of the
// grown tile rounded up to whole wavefronts (enough for the layout below at
// every tile width up to BX).
template <int BX, int S, bool CL = false>
__host__ __device__ constexpr int stepS_threads() {
    return (BX + 2 * StepSGeom<BX, S, CL>::H + 63) / 64 * 64;
}

// COH: storage read and written with device-scope accesses (IoCoherent,
// IoCoherentShifted: the batched form).  CL: the
// learned closure (FP32 plain storage).
template <int MODEL, int BX, int S, int ST, bool COH = false, bool CL = false>
__device__ __forceinline__ void stepS_tile_lds(const StepArgs& a, int x0, int w, int ys, int hh, int64_t t,
                                               bool down, TileSLds<BX, S, CL>& lds) {
    static_assert(!CL || (ST == ST_PLAIN && !COH), "the closure runs with FP32 plain storage");
    using G = StepSGeom<BX, S, CL>;
    constexpr int H = G::H, UL = G::UL, LG = G::LG, PER = G::PER, D = G::D, W = G::W, NPS = G::NPS;
    using IoCoh = typename std::conditional<
        ST == ST_PLAIN, IoCoherent,
        IoCoherentShifted<typename std::conditional<ST == ST_F16, __half, __hip_bfloat16>::type>>::type;
    using IoT = typename std::conditional<COH, IoCoh, Io<float, ST>>::type;
    // Thread layout.  The tile's first hd columns (its head: the columns up to
    // the first 128-byte line boundary of the storage, when x0 is not on one
    // and the layout below still fits; else hd = 0) and the C = 64 * c
    // columns after them that whole wavefronts own go to wavefronts 0 .. c - 1
    // in segments of 64 columns, each starting on a line (so every wavefront
    // loads and stores whole lines); wavefront c, the halo wavefront, takes the
    // H left halo columns, the head, the tile's remaining w - hd - C columns
    // and the right halo (c is the largest count for which that fits in 64
    // lanes, else one more, whose last columns then belong to the right halo);
    // later wavefronts (a tile narrower than BX) only take part in the
    // barriers.  Threads whose column lies past the right halo
    // duplicate its last column: they load what its owner loads, write their
    // LDS values to the padding column and store nothing.  cxo: column
    // relative to x0 (-H .. w + H - 1); act: owns tile column x0 + cxo.
    const int l = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(l) / kWave;  // wavefront index (uniform)
    constexpr int LC = ST == ST_PLAIN ? 32 : 64;  // columns per 128-byte line of the storage
    const int xa = (LC - x0 % LC) % LC;
    const int hd = xa <= w && (w - kWave * ((w - xa) / kWave)) + 2 * H <= kWave ? xa : 0;
    const int full = (w - hd) / kWave;
    const int C = (w - kWave * full) + 2 * H <= kWave ? kWave * full : kWave * (full + 1);
    const int hw = C / kWave;  // the halo wavefront
    const int hl = l - C;      // lane in the halo wavefront
    const int craw = wv < hw ? hd + l : (hl < H + hd ? hl - H : C + hl - H);
    const bool dup = craw > w + H - 1;
    const int cxo = min(craw, w + H - 1);
    const bool act = cxo >= 0 && cxo < w && !dup;
    // Stage k forms phi/psi validly on the columns (and rows) up to
    // RC (S - k) - 1 beyond the tile and updates up to RC (S - 1 - k) beyond
    // it.  Every thread runs every stage (branching on these ranges would only
    // hold per-lane masks, since every wavefront has lanes inside them):
    // outside them a thread forms values from rows or columns that are not
    // valid yet, which no valid value reads.
    const int gcol = wrap_idx(x0 + cxo, a.nx);
    const int j = cxo + H + 1;        // LDS column read
    const int jw = dup ? W - 1 : j;   // LDS column written
    // A strip marched downward is computed in the mirrored frame y -> -y:
    // populations are read from and written to the planes of their mirror
    // images and the y velocity changes sign, so the march always runs
    // toward +y in the frame the stages see and no value depends on the
    // direction.  Every node helper rounds mirror-symmetrically (sums in
    // mirror-invariant order, y components that only change sign), so the
    // results equal the lattice-frame computation bit for bit.
    const IoT io(a, down);
    lds_barrier();  // the LDS may still be read by a previous tile of this block

    const int iters = hh + H + D;
    if (wv > hw) {
        // no column in this wavefront: the loop's two barriers per iteration only
        for (int it = 0; it < iters; ++it) {
            lds_barrier();
            lds_barrier();
        }
        return;
    }

    // FP32 velocity factors: the FP64 table rounded once on the host, as the
    // one-step kernels round it on the device
    const float Ax = a.vtabf[gcol];
    const float Bx = down ? -a.vtabf[a.nx + gcol] : a.vtabf[a.nx + gcol];
    NodeConst<float> kcs[S];  // stage k at time t + k
#pragma unroll
    for (int k = 0; k < S; ++k) kcs[k] = NodeConst<float>(a, t + k);
    // pulled populations and phi of stage k, ping-pong by iteration parity:
    // the pull of iteration it fills half it & 1, the update of iteration
    // it + UL reads it (with UL = 2 through fh, which keeps the pull of two
    // iterations ago before the half is refilled)
    float fp[S][2][9], ph[S][2], ob[9];
    float fh[CL ? S : 1][9];
    float phl = 0.f;  // phi of the last stage's updated node (the shifted store's phi*)
    // Histories, index = age in iterations (0: this iteration).  P[k]: the sum
    // of stage k's input populations at the own node (phi(t + k - 1) as the
    // one-step kernel forms it); z0, zo, zn: the own column's c_x = 0 inputs
    // of stage k (population 0, the old-row one, the new-row one).
    float P[S][G::NP], z0[S][4], zo[S][4], zn[S][4];
    // shifted storage: the own column's populations 7 and 8 of stage 0's last
    // two input rows (the rings keep them only where another column pulls them)
    float o7[2] = {0.f, 0.f}, o8[2] = {0.f, 0.f};
    constexpr bool kSh = IoT::kShifted;
#pragma unroll
    for (int k = 0; k < S; ++k) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            ph[k][b] = 0.f;
#pragma unroll
            for (int q = 0; q < 9; ++q) fp[k][b][q] = 0.f;
        }
#pragma unroll
        for (int d = 0; d < G::NP; ++d) P[k][d] = 0.f;
#pragma unroll
        for (int d = 0; d < 4; ++d) z0[k][d] = zo[k][d] = zn[k][d] = 0.f;
    }
#pragma unroll
    for (int k = 0; k < (CL ? S : 1); ++k)
#pragma unroll
        for (int q = 0; q < 9; ++q) fh[k][q] = 0.f;
#pragma unroll
    for (int q = 0; q < 9; ++q) ob[q] = 0.f;

    const int dir = down ? -1 : 1;
    auto raw_row = [&](int it) { return down ? ys + hh + H - 1 - it : ys - H + it; };
    // lattice row loaded at iteration it (iterations past the last input row
    // repeat it; what they form is not used)
    auto row_of = [&](int it) { return (uint32_t)wrap_idx(raw_row(min(it, hh + 2 * H - 1)), a.ny); };
    // a stage's input into its ring and histories (v: populations at the own column)
    auto put = [&](int k, int s3, int s2, const float(&v)[9]) __attribute__((always_inline)) {
        // phi at t + k - 1: the sum of the stage's input values (phi* itself
        // for stage 0's shifted input)
        P[k][0] = kSh && k == 0 ? v[0] : sum9(v);
        if (kSh && k == 0) {
            o7[0] = v[7];
            o8[0] = v[8];
        }
        lds.ro[k][s3][0][jw] = v[5];
        lds.ro[k][s3][1][jw] = v[6];
        lds.rm[k][s2][0][jw] = v[1];
        lds.rm[k][s2][1][jw] = v[3];
        lds.rn[k][0][jw] = v[8];
        lds.rn[k][1][jw] = v[7];
        z0[k][0] = v[0];
        zo[k][0] = v[2];
        zn[k][0] = v[4];
    };
    auto body = [&](const int it, float(&nv)[9], auto parity) __attribute__((always_inline)) {
        constexpr int B = decltype(parity)::value;  // it & 1
        const int Rr = raw_row(it);
        const int s3 = it % 3, s2 = B;
        const int sps = CL ? it % NPS : s3;  // psi slot of this iteration's phi row
        // ---- row R into stage 0's ring
        put(0, s3, s2, nv);
        io.load(row_of(it + 2) * (uint32_t)a.pitch + (uint32_t)gcol, nv);
        lds_barrier();

        // ---- phi (Eq. (12)) and psi (Eq. (13)) of every stage.  Stage 0 reads
        // rows entered 0 (new pair), 1 (populations 1, 3) and 2 (old pair)
        // iterations ago; a later stage's input rows were written 1, 2 and 3
        // iterations ago.
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const int lag = k == 0 ? 0 : 1;
            if constexpr (CL) {
#pragma unroll
                for (int q = 0; q < 9; ++q) fh[k][q] = fp[k][B][q];
            }
            if (it >= PER * k + 2) {
                const int so = (it + 1 + 2 * lag) % 3;  // old pair: it - 2 - lag
                const int sm = B ^ 1 ^ lag;             // populations 1, 3: it - 1 - lag
                float(&f)[9] = fp[k][B];
                f[0] = z0[k][1 + lag];
                f[1] = lds.rm[k][sm][0][j - 1];
                f[2] = zo[k][2 + lag];
                f[3] = lds.rm[k][sm][1][j + 1];
                f[4] = zn[k][lag];
                f[5] = lds.ro[k][so][0][j - 1];
                f[6] = lds.ro[k][so][1][j + 1];
                f[7] = lds.rn[k][1][j + 1];
                f[8] = lds.rn[k][0][j - 1];
                float s;
                if (kSh && k == 0) {
                    // the own column's values of the centre row: populations 1, 3
                    // and 5, 6 from the rings, 2, 4 (and phi* in z0) from the
                    // histories, 7, 8 from o7, o8
                    float own[9];
                    own[0] = 0.f;
                    own[1] = lds.rm[0][sm][0][j];
                    own[3] = lds.rm[0][sm][1][j];
                    own[5] = lds.ro[0][(it + 2) % 3][0][j];
                    own[6] = lds.ro[0][(it + 2) % 3][1][j];
                    own[2] = zo[0][1];
                    own[4] = zn[0][1];
                    own[7] = o7[1];
                    own[8] = o8[1];
                    s = shifted_phi(z0[0][1], f, own);  // the collision forms the rest population itself
                } else {
                    s = sum9(f);
                }
                ph[k][B] = s;
                lds.ps[k][sps][jw] = normal_source<float, MODEL>(s, kcs[k]);
                if constexpr (CL) lds.phr[k][it % 5][jw] = s;
            }
        }
        lds_barrier();

        // psi rows around an updated row: the centre row is UL rows behind this
        // iteration's phi row, and the row ahead of it (+y in the stages'
        // frame) one row nearer
        const int c0 = (it + NPS - UL) % NPS;
        const int cm = (it + NPS - UL - 1) % NPS;
        const int cp = (it + (NPS - UL + 1) % NPS) % NPS;
        // ---- updates: stage k on row R - (LG k + 1 + UL) dir at t + k; the last stage into HBM
        const bool st = act && it >= PER * (S - 1) + 2 + 2 * UL;
        const int yl = min(max(Rr - D * dir, 0), a.ny - 1);
        uint64_t bms[S];  // closure: band nodes of stage k's updated row (one bit per lane)
#pragma unroll
        for (int k = 0; k < S; ++k) bms[k] = 0;
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const bool last = k == S - 1;
            if (it >= PER * k + 2 + 2 * UL) {
                const NodeConst<float>& kc = kcs[k];
                const int y = last ? yl : wrap_idx(Rr - (LG * k + 1 + UL) * dir, a.ny);
                const float(&ps)[NPS][W] = lds.ps[k];
                float gx, gy, Gx, Gy;
                iso_gradient(ps[c0][j + 1], ps[c0][j - 1], ps[cp][j], ps[cm][j], ps[cp][j + 1], ps[cp][j - 1],
                             ps[cm][j + 1], ps[cm][j - 1], gx, gy);
                float phi;
                if constexpr (CL) phi = lds.phr[k][(it + 3) % 5][j];  // phi row it - 2
                else phi = ph[k][B ^ 1];
                const float uxr = Ax * row_factor(a.vtabf, 2 * a.nx + y);
                const float uyr = Bx * row_factor(a.vtabf, 2 * a.nx + a.ny + y);
                const float phio = P[k][(k == 0 ? 1 : 2) + UL];
                flux_bracket<float, MODEL>(gx, gy, phi, kc.first ? phi : phio, kc.s_now * uxr, kc.s_now * uyr,
                                           kc.s_old * uxr, kc.s_old * uyr, kc, Gx, Gy);
                if constexpr (CL) {
                    collide(fh[k], phi, kc.s_now * uxr, kc.s_now * uyr, Gx, Gy, kc, ob);
                    // interface-band nodes among those stage k must update (the
                    // condition of the one-step path's band mask); their
                    // correction is added after the last stage (below)
                    const int reach = G::RC * (S - 1 - k);
                    const int rel = it - H - (LG * k + 1 + UL);  // row relative to the strip, march frame
                    const bool need = !dup && cxo >= -reach && cxo < w + reach && rel >= -reach && rel < hh + reach;
                    const float pc = clip01(phi);
                    bms[k] = __ballot(need && pc > a.cl_theta && pc < 1.0f - a.cl_theta);
                } else {
                    collide(fp[k][B ^ 1], phi, kc.s_now * uxr, kc.s_now * uyr, Gx, Gy, kc, ob);
                }
                if (!last) put(k + 1, s3, s2, ob);
                else phl = phi;
            }
        }
        if constexpr (CL) {
            // The network on every stage's band nodes of this wavefront, packed
            // into one list (stage by stage, lanes in order), from stage k's
            // phi ring (rows it - 4 .. it; the updated row is it - 2), and its
            // correction added to the node's post-collision populations: for
            // the last stage in ob before the store, for an earlier one where
            // put() left them (the next stage's rings and own-column
            // histories), which nothing reads before the next iteration.
            const int lane = l % kWave;
            const uint64_t below = (1ull << lane) - 1ull;
            int slot[S], count = 0;
#pragma unroll
            for (int k = 0; k < S; ++k) {
                slot[k] = count + __popcll(bms[k] & below);
                count += __popcll(bms[k]);
            }
            if (count) {
                int* tab = lds.tab[wv];
#pragma unroll
                for (int k = 0; k < S; ++k)
                    if ((bms[k] >> lane) & 1ull) tab[slot[k]] = (k << 16) | j;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
                for (int first = 0; first < count; first += kWave) {
                    const float2 c = closure_mlp_list(a.cl_w, a.cl_b, &lds.phr[0][0][0], 5 * W, W, it + 3, down,
                                                      tab + first, count - first);
#pragma unroll
                    for (int k = 0; k < S; ++k) {
                        const int src = slot[k] - first;
                        const float cx = __shfl(c.x, src & (kWave - 1), kWave);
                        const float cy = __shfl(c.y, src & (kWave - 1), kWave);
                        if (!((bms[k] >> lane) & 1ull) || src < 0 || src >= kWave) continue;
                        const float phi = lds.phr[k][(it + 3) % 5][j];
                        if (k == S - 1) {
                            closure_correct(ob, phi, kcs[k].kforce, cx, cy, down);
                        } else {
                            const int n = k == S - 1 ? 0 : k + 1;  // (k + 1 without the out-of-range index)
                            float f[9];
                            f[1] = lds.rm[n][s2][0][jw];
                            f[3] = lds.rm[n][s2][1][jw];
                            f[5] = lds.ro[n][s3][0][jw];
                            f[6] = lds.ro[n][s3][1][jw];
                            f[8] = lds.rn[n][0][jw];
                            f[7] = lds.rn[n][1][jw];
                            f[2] = zo[n][0];
                            f[4] = zn[n][0];
                            closure_correct(f, phi, kcs[k].kforce, cx, cy, down);
                            lds.rm[n][s2][0][jw] = f[1];
                            lds.rm[n][s2][1][jw] = f[3];
                            lds.ro[n][s3][0][jw] = f[5];
                            lds.ro[n][s3][1][jw] = f[6];
                            lds.rn[n][0][jw] = f[8];
                            lds.rn[n][1][jw] = f[7];
                            z0[n][0] = f[0];
                            zo[n][0] = f[2];
                            zn[n][0] = f[4];
                            P[n][0] = sum9(f);
                        }
                    }
                }
                __builtin_amdgcn_wave_barrier();  // the list is rewritten next iteration
            }
        }
        // non-temporal: a stored row is not read again in this launch, while
        // the 2H rows each strip shares with its neighbours are (1.5% faster
        // at 8192^2 than plain stores)
        io.store_nt(st, (uint32_t)yl * (uint32_t)a.pitch + (uint32_t)(x0 + cxo), ob, phl);
        // ---- age the histories by one iteration
        o7[1] = o7[0];
        o8[1] = o8[0];
#pragma unroll
        for (int k = 0; k < S; ++k) {
#pragma unroll
            for (int d = G::NP - 1; d > 0; --d) P[k][d] = P[k][d - 1];
#pragma unroll
            for (int d = 3; d > 0; --d) {
                z0[k][d] = z0[k][d - 1];
                zo[k][d] = zo[k][d - 1];
                zn[k][d] = zn[k][d - 1];
            }
        }
    };
    // two rows of loads in flight: row r + 2 is loaded while row r is processed,
    // into the register set row r came in
    float na[9], nb[9];
    io.load(row_of(0) * (uint32_t)a.pitch + (uint32_t)gcol, na);
    io.load(row_of(1) * (uint32_t)a.pitch + (uint32_t)gcol, nb);
    for (int it = 0; it < iters; it += 2) {
        body(it, na, std::integral_constant<int, 0>{});
        if (it + 1 < iters) body(it + 1, nb, std::integral_constant<int, 1>{});
    }
}

template <int MODEL, int BX, int S, int ST>
__global__ __launch_bounds__((stepS_threads<BX, S>())) void stepS_kernel_lds(StepArgs a) {
    __shared__ TileSLds<BX, S> lds;
    const int ntile = a.nbx * a.nby;
    const int tile = xcd_tile(blockIdx.x, ntile, a.n_xcd);
    const int bxi = tile % a.nbx, syi = tile / a.nbx;
    const int x0 = bxi * BX, ys = syi * a.strip_h;
    stepS_tile_lds<MODEL, BX, S, ST>(a, x0, min(BX, a.nx - x0), ys, min(a.strip_h, a.ny - ys), a.t_dev[0] + a.k,
                                     (syi & 1) != 0, lds);
}

// The S-step kernel with the learned closure (FP32 storage, improved model).
template <int BX, int S>
__global__ __launch_bounds__((stepS_threads<BX, S, true>())) __attribute__((amdgpu_waves_per_eu(2, 2))) void
stepS_kernel_cl(StepArgs a) {
    __shared__ TileSLds<BX, S, true> lds;
    const int ntile = a.nbx * a.nby;
    const int tile = xcd_tile(blockIdx.x, ntile, a.n_xcd);
    const int bxi = tile % a.nbx, syi = tile / a.nbx;
    const int x0 = bxi * BX, ys = syi * a.strip_h;
    stepS_tile_lds<MODEL_IMPROVED, BX, S, ST_PLAIN, false, true>(a, x0, min(BX, a.nx - x0), ys,
                                                                 min(a.strip_h, a.ny - ys), a.t_dev[0] + a.k,
                                                                 (syi & 1) != 0, lds);
}

// ---------------------------------------------------------------------------
// The step on one tile, one wavefront per tile.
//
// A wavefront owns kTileW = 60 output columns and marches a strip of
// a.strip_h rows.  Lane l loads lattice column x0 - 2 + l of every plane;
// lanes 1..62 form phi and psi, lanes 2..61 update, so neighbouring tiles
// overlap by two columns on each side.  Everything stays in registers: the
// last three rows of each plane, the pulled populations, three rows of psi.
// A neighbour in x is one lane away and is read with a DPP wave shift, so
// there is no LDS, no barrier, and every lane runs every instruction (only
// the stores are masked).  DIR = +1 marches up the strip, -1 down it.
constexpr int kTileW = kWave - 4;

// lane l receives the value of lane l - 1 (wave_shr:1) or l + 1 (wave_shl:1)
constexpr int kDppFromLeft = 0x138;
constexpr int kDppFromRight = 0x130;

template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
// value of lane l - cx (the pulled population of a direction with x-component cx)
template <int CX, typename R>
__device__ __forceinline__ R from_lane(R v) {
    if constexpr (CX == 1) return lane_shift<kDppFromLeft>(v);
    else if constexpr (CX == -1) return lane_shift<kDppFromRight>(v);
    else return v;
}

template <typename R, int ST, int MODEL, int DIR, int Q>
__device__ __forceinline__ R pulled(const R (&r0)[9], const R (&r1)[9], const R (&r2)[9]) {
    // plane Q is read at row c - cy(Q); the centre row c is r - DIR, so the
    // row is the newest (r0) when DIR * cy(Q) = -1, r1 when cy(Q) = 0, and
    // r2 (loaded two rows ago) when DIR * cy(Q) = +1
    constexpr int d = DIR * cy(Q);
    const R v = d == -1 ? r0[Q] : (d == 0 ? r1[Q] : r2[Q]);
    return from_lane<cx(Q)>(v);
}

// ---- the wavefront step ----------------------------------------------------
// Halo 2, tiles of 60 columns, row y = c - DIR updated.
struct WaveGeom {
    static constexpr int kHalo = 2;
    static constexpr int kW = kWave - 2 * kHalo;
    static constexpr int kDelay = 1;
};

template <typename R, int ST, int MODEL, int DIR>
__device__ __forceinline__ void step_wave_dir(const StepArgs& a, int bxi, int syi, int64_t t) {
    using G = WaveGeom;
    constexpr int D = G::kDelay;
    const int l = threadIdx.x % kWave;
    const int x0 = bxi * G::kW;
    const int w = min(G::kW, a.nx - x0);
    const int ys = syi * a.strip_h;
    const int hh = min(a.strip_h, a.ny - ys);
    const bool upd_lane = l >= G::kHalo && l < G::kHalo + w;
    const int col = wrap_idx(x0 - G::kHalo + l, a.nx);  // column this lane loads
    const int x = x0 - G::kHalo + l;                     // column this lane updates (upd_lane)
    const Io<R, ST> io(a);

    const NodeConst<R> kc(a, t);
    const R Axl = upd_lane ? R(a.vtab[x]) : R(0);
    const R Bxl = upd_lane ? R(a.vtab[a.nx + x]) : R(0);

    R out[9], phi_out = R(0);  // the update's results (kept across the pipeline-fill iterations)
    R r0[9], r1[9], r2[9];   // rows r, r - DIR, r - 2 DIR of every plane (own column)
    R fh[D + 1][9];          // pulled populations on rows c, c - DIR, ...
    R ph[2 * D + 1];         // phi on rows c, c - DIR, ...
    R ps[D + 2];             // psi on rows c, c - DIR, ...
    R P[D + 2];              // own-column phi at t-1 on rows r, r - DIR, ...
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        r0[q] = r1[q] = r2[q] = out[q] = R(0);
#pragma unroll
        for (int j = 0; j <= D; ++j) fh[j][q] = R(0);
    }
#pragma unroll
    for (int j = 0; j < 2 * D + 1; ++j) ph[j] = R(0);
#pragma unroll
    for (int j = 0; j < D + 2; ++j) ps[j] = P[j] = R(0);

    const int start = DIR > 0 ? ys - (D + 1) : ys + hh + D;
    R nv[9];  // prefetch registers for the next row
    io.load((uint32_t)wrap_idx(start, a.ny) * (uint32_t)a.pitch + (uint32_t)col, nv);

    const int iters = hh + 2 * (D + 1);
    for (int it = 0; it < iters; ++it) {
        // ---- row r = start + DIR it becomes the newest row
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            r2[q] = r1[q];
            r1[q] = r0[q];
            r0[q] = nv[q];
        }
#pragma unroll
        for (int j = D + 1; j > 0; --j) P[j] = P[j - 1];
        P[0] = Io<R, ST>::kShifted ? r0[0] : sum9(r0);
        // unconditional, like the update's stores below, so that the compiler
        // counts the memory operations in flight exactly (past the strip's
        // end the last row is reloaded and not used)
        io.load((uint32_t)wrap_idx(start + DIR * min(it + 1, iters - 1), a.ny) * (uint32_t)a.pitch + (uint32_t)col, nv);

        // ---- phi (Eq. (12)) and psi (Eq. (13)) on the centre row c = r - DIR
        if (it >= 2) {
#pragma unroll
            for (int j = D; j > 0; --j)
#pragma unroll
                for (int q = 0; q < 9; ++q) fh[j][q] = fh[j - 1][q];
#pragma unroll
            for (int j = 2 * D; j > 0; --j) ph[j] = ph[j - 1];
#pragma unroll
            for (int j = D + 1; j > 0; --j) ps[j] = ps[j - 1];
            R* fc = fh[0];
            fc[0] = pulled<R, ST, MODEL, DIR, 0>(r0, r1, r2);
            fc[1] = pulled<R, ST, MODEL, DIR, 1>(r0, r1, r2);
            fc[2] = pulled<R, ST, MODEL, DIR, 2>(r0, r1, r2);
            fc[3] = pulled<R, ST, MODEL, DIR, 3>(r0, r1, r2);
            fc[4] = pulled<R, ST, MODEL, DIR, 4>(r0, r1, r2);
            fc[5] = pulled<R, ST, MODEL, DIR, 5>(r0, r1, r2);
            fc[6] = pulled<R, ST, MODEL, DIR, 6>(r0, r1, r2);
            fc[7] = pulled<R, ST, MODEL, DIR, 7>(r0, r1, r2);
            fc[8] = pulled<R, ST, MODEL, DIR, 8>(r0, r1, r2);
            R s;
            if constexpr (Io<R, ST>::kShifted)
                s = shifted_phi(r1[0], fh[0], r1);  // r1: the centre row at the own column
            else
                s = sum9(fh[0]);
            ph[0] = s;
            ps[0] = normal_source<R, MODEL>(s, kc);
        }

        // ---- update row y = c - D DIR.  The first 2 + 2 D iterations fill the
        // pipeline: they skip the arithmetic (a branch without memory
        // operations) and their stores are dropped.
        const bool st = upd_lane && it >= 2 + 2 * D;
        const int y = min(max(DIR > 0 ? ys + it - 2 - 2 * D : ys + hh + 1 + 2 * D - it, 0), a.ny - 1);
        if (it >= 2 + 2 * D) {
            // psi rows y + 1, y, y - 1 (the march produced y + DIR first)
            const R pN0 = DIR > 0 ? ps[D - 1] : ps[D + 1], pC0 = ps[D], pS0 = DIR > 0 ? ps[D + 1] : ps[D - 1];
            const R pE = from_lane<-1>(pC0), pW = from_lane<1>(pC0);
            const R pNE = from_lane<-1>(pN0), pNW = from_lane<1>(pN0);
            const R pSE = from_lane<-1>(pS0), pSW = from_lane<1>(pS0);
            R gx, gy, Gx, Gy;
            iso_gradient(pE, pW, pN0, pS0, pNE, pNW, pSE, pSW, gx, gy);
            const R phi = ph[D];
            const R Ayv = R(row_factor(a.vtab, 2 * a.nx + y)), Byv = R(row_factor(a.vtab, 2 * a.nx + a.ny + y));
            const R uxr = Axl * Ayv, uyr = Bxl * Byv;
            const R u = kc.s_now * uxr, v = kc.s_now * uyr;
            flux_bracket<R, MODEL>(gx, gy, phi, kc.first ? phi : P[D + 1], u, v, kc.s_old * uxr, kc.s_old * uyr, kc,
                                   Gx, Gy);
            collide(fh[D], phi, u, v, Gx, Gy, kc, out);
            phi_out = phi;
        }
        io.store(st, (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x, out, phi_out);
    }
}

// One step on the tile of column block `bxi` and strip `syi` (a.strip_h rows)
// at time t, by the calling wavefront.  Odd strips march downward so that
// two strips sharing a boundary read its halo rows at about the same time,
// while they are still in cache.
template <typename R, int ST, int MODEL>
__device__ __forceinline__ void step_wave(const StepArgs& a, int bxi, int syi, int64_t t) {
    if (syi & 1)
        step_wave_dir<R, ST, MODEL, -1>(a, bxi, syi, t);
    else
        step_wave_dir<R, ST, MODEL, 1>(a, bxi, syi, t);
}


// One launch = one step.  WPB wavefronts per block take WPB horizontally
// adjacent tiles.
template <typename R, int ST, int MODEL, int WPB>
__global__ __launch_bounds__(WPB * kWave) void step_kernel(StepArgs a) {
    const int nbb = (a.nbx + WPB - 1) / WPB;  // block tiles per strip
    const int tile = xcd_tile(blockIdx.x, nbb * a.nby, a.n_xcd);
    const int bxi = (tile % nbb) * WPB + (int)(threadIdx.x / kWave), syi = tile / nbb;
    if (bxi >= a.nbx) return;  // whole wavefront idle
    step_wave<R, ST, MODEL>(a, bxi, syi, a.t_dev[0] + a.k);
}

// ---- learned closure: band list and correction pass -------------------------
// Eq. (9)-(11) are linear in G, so adding c_s^2 c to G at a node changes its
// post-collision populations by (1 - 1/(2 tau)) w_i (c_i . c) for i >= 1 and
// leaves their sum unchanged.  The step kernel (block variant) records, for
// every 64 columns of every updated row, a ballot of the interface-band nodes
// (theta < clip(phi) < 1 - theta); the scan kernel turns the masks into a
// node list; the apply kernel evaluates the network on 64 listed nodes per
// wavefront (its 5x5 input stencil of phi(t) rebuilt from the pre-step
// populations, exactly as the step formed it) and adds the correction.

static __global__ void closure_reset_kernel(uint32_t* count) {
    if (threadIdx.x == 0 && blockIdx.x == 0) count[0] = 0u;
}

// Compacts the band masks into node indices y * nx + x (row-major order
// within a block, blocks in any order).  count must be zero on entry.
static __global__ __launch_bounds__(256) void closure_scan_kernel(const uint64_t* __restrict__ mask, int64_t nwords,
                                                                  int words_per_row, int nx,
                                                                  int32_t* __restrict__ list,
                                                                  uint32_t* __restrict__ count) {
    __shared__ uint32_t sh[256];
    __shared__ uint32_t base;
    const int64_t wi = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const uint64_t m = wi < nwords ? mask[wi] : 0ull;
    const uint32_t c = (uint32_t)__popcll(m);
    sh[threadIdx.x] = c;
    __syncthreads();
    // inclusive scan over the block (Hillis-Steele)
    for (int d = 1; d < 256; d <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)d ? sh[threadIdx.x - d] : 0u;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    if (threadIdx.x == 255) base = sh[255] ? atomicAdd(count, sh[255]) : 0u;
    __syncthreads();
    if (m) {
        uint32_t k = base + sh[threadIdx.x] - c;
        const int y = (int)(wi / words_per_row), x0 = (int)(wi % words_per_row) * 64;
        uint64_t r = m;
        while (r) {
            const int b = __ffsll((unsigned long long)r) - 1;
            r &= r - 1;
            list[k++] = y * nx + x0 + b;
        }
    }
}

// The correction pass (FP32 plain storage): a.src holds the pre-step
// populations, a.dst the step's result, modified in place at listed nodes.
// Every wavefront of the grid takes groups of 64 list entries in turn.
static __global__ __launch_bounds__(kClWaves * kWave) void closure_apply_kernel(StepArgs a,
                                                                              const int32_t* __restrict__ list,
                                                                              const uint32_t* __restrict__ count) {
    __shared__ ClosureLds cl;
    closure_stage(a, cl);
    const int l = threadIdx.x % kWave;
    const int n = (int)count[0];
    const int waves = gridDim.x * kClWaves;
    const float kforce = (float)(1.0 - 0.5 / a.tau);
    const float* src = static_cast<const float*>(a.src);
    float* dst = static_cast<float*>(a.dst);
    for (int g = blockIdx.x * kClWaves + (int)(threadIdx.x / kWave); g * kWave < n; g += waves) {
        const int e = g * kWave + l;
        const bool on = e < n;
        const int node = list[on ? e : g * kWave];
        const int y = node / a.nx, x = node % a.nx;
        // phi(t) on the 5x5 neighbourhood: sum_i f*_i(z - c_i, t - 1), summed as in the step
        float xin[25];
        for (int dy = -2; dy <= 2; ++dy)
            for (int dx = -2; dx <= 2; ++dx) {
                const int zy = wrap_idx(y + dy, a.ny), zx = wrap_idx(x + dx, a.nx);
                float fz[9];
#pragma unroll
                for (int q = 0; q < 9; ++q)
                    fz[q] = src[q * a.plane_stride + (int64_t)wrap_idx(zy - cy(q), a.ny) * a.pitch +
                                wrap_idx(zx - cx(q), a.nx)];
                xin[(dy + 2) * 5 + (dx + 2)] = sum9(fz);
            }
        // the inputs as BF16 rows of 32 (25..31 zero) in this wavefront's staging area
        uint16_t* xs = cl.x[(threadIdx.x / kWave) % kClWaves];
#pragma unroll
        for (int k = 0; k < 32; k += 2) {
            const uint32_t lo = k < 25 ? bf16_bits(xin[k]) : 0u;
            const uint32_t hi = k + 1 < 25 ? bf16_bits(xin[k + 1]) : 0u;
            *reinterpret_cast<uint32_t*>(&xs[l * 32 + k]) = lo | (hi << 16);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
        auto xfrag = [&](int nt) {
            return *reinterpret_cast<const bf16x8_t*>(&xs[(16 * nt + l % 16) * 32 + 8 * (l / 16)]);
        };
        float ccx, ccy;
        closure_mlp(cl.w, cl.b, xfrag, ~0ull, ccx, ccy);
        __builtin_amdgcn_wave_barrier();  // the staging rows are rewritten by the next group
        if (on) {
            const float phi = xin[12];
            const int64_t off = (int64_t)y * a.pitch + x;
            float f[9];
#pragma unroll
            for (int q = 1; q < 9; ++q) f[q] = dst[q * a.plane_stride + off];
            closure_correct(f, phi, kforce, ccx, ccy, false);
            dst[off] = f[0];
#pragma unroll
            for (int q = 1; q < 9; ++q) dst[q * a.plane_stride + off] = f[q];
        }
    }
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

// phi(x) = sum_i f*_i(x - c_i) from the stored state in a.src, formed as the
// step forms it (in R, the populations summed in the step's order).
template <typename R, int ST>
__device__ __forceinline__ R pulled_phi(const StepArgs& a, int x, int y) {
    R v[9];
#pragma unroll
    for (int q = 1; q < 9; ++q) {
        const int xs = wrap_idx(x - cx(q), a.nx), ys = wrap_idx(y - cy(q), a.ny);
        v[q] = Store<R, ST>::load_one(a, (int64_t)ys * a.pitch + xs, q);
    }
    if constexpr (Store<R, ST>::kShifted) {
        R own[9];
        Store<R, ST>::load(a, (int64_t)y * a.pitch + x, own);
        return shifted_phi(own[0], v, own);
    } else {
        v[0] = Store<R, ST>::load_one(a, (int64_t)y * a.pitch + x, 0);
        return sum9(v);
    }
}

template <typename R, int ST>
__global__ void phi_kernel(StepArgs a, double* __restrict__ out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= a.nx) return;
    out[(int64_t)y * a.nx + x] = (double)pulled_phi<R, ST>(a, x, y);
}

// Compensated sum in the working precision R (FP32 for the FP32 forms):
// s carries the rounded sum, c the exact rounding errors of its additions
// (Knuth's TwoSum), accumulated; the value is s + c.
template <typename R>
struct CompSum {
    R s, c;
    __device__ __forceinline__ CompSum() : s(R(0)), c(R(0)) {}
    __device__ __forceinline__ void add(R x) {
        const R t = s + x;
        const R z = t - s;
        c += (s - (t - z)) + (x - z);
        s = t;
    }
    __device__ __forceinline__ void add(const CompSum& o) {
        add(o.s);
        c += o.c;
    }
    __device__ __forceinline__ R value() const { return s + c; }
};

// Partial sums for mass and shape errors: per row y, the five sums
// sum phi, sum |phi - ref|, sum |ref|, sum (phi - ref)^2, sum ref^2, each as a
// compensated pair (s, c) in R.  One block per row; reduce_rows adds the rows
// in order.
constexpr int kRedThreads = 256;

// Compensated block sum in a fixed order: wavefront tree, then the
// wavefronts' partial sums in order by thread 0 (valid there only).
template <typename R>
__device__ __forceinline__ CompSum<R> block_sum(CompSum<R> v, R* sh) {
    for (int off = 32; off > 0; off >>= 1) {
        CompSum<R> o;
        o.s = __shfl_down(v.s, off, 64);
        o.c = __shfl_down(v.c, off, 64);
        v.add(o);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        sh[2 * wid] = v.s;
        sh[2 * wid + 1] = v.c;
    }
    __syncthreads();
    CompSum<R> r;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            CompSum<R> o;
            o.s = sh[2 * i];
            o.c = sh[2 * i + 1];
            r.add(o);
        }
    return r;
}

template <typename R, int ST>
__global__ __launch_bounds__(kRedThreads) void row_sums_kernel(StepArgs a, const double* __restrict__ ref,
                                                                R* __restrict__ rows) {
    __shared__ R sh[2 * kRedThreads / 64];
    const int y = blockIdx.x;
    CompSum<R> acc[5];
    for (int x = threadIdx.x; x < a.nx; x += blockDim.x) {
        const R p = pulled_phi<R, ST>(a, x, y);
        acc[0].add(p);
        if (ref) {
            const R r = R(ref[(int64_t)y * a.nx + x]);
            const R d = p - r;
            acc[1].add(d < R(0) ? -d : d);
            acc[2].add(r < R(0) ? -r : r);
            acc[3].add(d * d);
            acc[4].add(r * r);
        }
    }
    R* o = rows + 10 * (int64_t)y;
    for (int c = 0; c < 5; ++c) {
        const CompSum<R> v = block_sum(acc[c], sh);
        if (threadIdx.x == 0) {
            o[2 * c] = v.s;
            o[2 * c + 1] = v.c;
        }
    }
}

// Adds the per-row sums in row order (one block; deterministic) and writes
// the five totals.
template <typename R>
__global__ __launch_bounds__(kRedThreads) void reduce_rows_kernel(const R* __restrict__ rows, int ny,
                                                                  double* __restrict__ out5) {
    __shared__ R sh[2 * kRedThreads / 64];
    for (int c = 0; c < 5; ++c) {
        CompSum<R> acc;
        for (int y = threadIdx.x; y < ny; y += blockDim.x) {
            CompSum<R> o;
            o.s = rows[10 * (int64_t)y + 2 * c];
            o.c = rows[10 * (int64_t)y + 2 * c + 1];
            acc.add(o);
        }
        const CompSum<R> v = block_sum(acc, sh);
        if (threadIdx.x == 0) out5[c] = (double)v.value();
    }
}

static __global__ void advance_kernel(int64_t* t_dev, int64_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) t_dev[0] += n;
}

static __global__ void set_time_kernel(int64_t* t_dev, int64_t t) {
    if (threadIdx.x == 0 && blockIdx.x == 0) t_dev[0] = t;
}

// Copy of the stored state with the step kernel's tiling and access order
// (256-column tiles, strips marched row by row, the XCD-aware tile order) but
// none of its arithmetic: the HBM rate this access pattern reaches is a
// practical ceiling for the step.  E: the stored element type; NP: 9 planes
// (plain storage), or 8 planes plus the FP32 phi* plane (shifted storage).
template <typename E, int NP>
static __global__ __launch_bounds__(256) void pattern_copy_kernel(StepArgs a) {
    const int nbx = (a.nx + 255) / 256;
    const int tile = xcd_tile(blockIdx.x, nbx * a.nby, a.n_xcd);
    const int bxi = tile % nbx, syi = tile / nbx;
    const int x = min(bxi * 256 + (int)threadIdx.x, a.nx - 1);
    const int ys = syi * a.strip_h, ye = min(ys + a.strip_h, a.ny);
    const E* src = static_cast<const E*>(a.src);
    E* dst = static_cast<E*>(a.dst);
    for (int y = ys; y < ye; ++y) {
        const int64_t off = (int64_t)y * a.pitch + x;
        E v[NP];
        float ph = 0.f;
#pragma unroll
        for (int q = 0; q < NP; ++q) v[q] = src[q * a.plane_stride + off];
        if constexpr (NP == 8) ph = a.src_phi[off];
#pragma unroll
        for (int q = 0; q < NP; ++q) dst[q * a.plane_stride + off] = v[q];
        if constexpr (NP == 8) a.dst_phi[off] = ph;
    }
}

}  // namespace lbac

