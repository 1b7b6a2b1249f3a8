// Device-side building blocks of the relativistic PIC step for gfx950.
//
// Everything here is templated on the working precision R (float, double)
// and on the number of spatial dimensions D, so that the hot loops are
// straight-line code.  Particles carry positions relative to their tile
// centre; tiles are staged in LDS with a halo, so that interpolation reads
// and deposit atomics never leave the work-group's LDS.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

// ---------------------------------------------------------------- tables

// One entry per tile of every box.
struct TileDesc {
    int32_t box;
    int32_t tc[3];      // tile coordinates inside the box
    int32_t nt[3];      // tiles per dimension of the box
    int32_t n[3];       // cells per dimension of the box
    int64_t cell0;      // offset of the box's first cell in the field planes
    int32_t tile0;      // global id of the box's tile (0,0,0)
    int32_t walls;      // bit 0: conducting wall on the tile's low-x face
                        // (x = 0), bit 1: on its high-x face (x = n0)
};

// Launch-wide constants of the particle and field kernels.
template <typename R>
struct Params {
    const TileDesc *tiles;
    int32_t ntiles;
    int32_t nspecies;
    int32_t T[3];
    int32_t pad0;
    R c;                      // Courant number
    R inv_c;                  // 1 / c
    const R *charge;          // [box][species]
    const R *qm;              // [box][species] App. C factor s
    R *E, *B, *J;             // [3][cells_total]
    int64_t cells_total;
    R *pos, *u, *xold;        // [D|3][cap_total]
    int64_t cap_total;
    const int64_t *seg_off;   // [tile][species]
    const int32_t *seg_cap;
    int32_t *seg_cnt;
    R *jblk;                  // [tile*species][3][JV]
    R *ob_pos, *ob_u;         // [tile*species][D|3][ob_cap]
    int32_t *ob_dir;          // [tile*species][ob_dir_stride]
    int32_t *ob_cnt;          // [tile*species]
    int64_t ob_cap;
    int64_t ob_dir_stride;    // slots per outbox direction list (ob_cap)
    R *tmp;                   // sort staging [(D+3)][cap_total]
    int32_t *err;             // latched error bits
    int32_t *nf_seg;          // [tile*species] particles flagged near a cell face
    R nf_band[3];             // near-face band per dimension: 2 ulp(T_d/2) in R
    uint32_t species_mask;    // species the launch works on (bit s = species s)
    int32_t *mig_counts;      // [tile*species][ncodes] migration counts, or null
    int32_t *queue;           // work counter of the persistent walker
    int32_t *order;           // (tile, species) segments in visiting order
    int32_t *ids;             // [cap_total] origin of each particle, or null
    int32_t *ob_ids;          // [tile*species][ob_cap] origin of each leaver
    int32_t *ob_boff;         // [tile*species][ncodes+1] outbox bucket starts by direction code
    int32_t *ob_idx;          // [tile*species][ob_cap] outbox slots in bucket order
};

enum : int32_t { ERR_CAPACITY = 1, ERR_CFL = 2, ERR_NONFINITE = 4, ERR_OUT_OF_TILE = 8, ERR_ADJ_MAP = 16 };

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ int wrapi(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

// Tile (or (tile, species) segment) of this work-group in launches with one
// work-group per tile (or segment), out of n.  The
// dispatcher hands consecutive work-groups to the eight dies (XCDs, each
// with its own L2) in turn; this bijection gives every die a contiguous
// range of tiles instead, so that neighbouring tiles, which share cache
// lines of the field planes and each other's halos, meet in one L2.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    constexpr int NXCD = 8;
    const int x = b % NXCD, l = b / NXCD, per = n / NXCD, rem = n % NXCD;
    return x < rem ? x * (per + 1) + l : rem * (per + 1) + (x - rem) * per + l;
}

// Product of two small non-negative integers (LDS block indices and strides,
// both far below 2^23): v_mul_i32_i24 issues at the full VALU rate, the
// 32-bit v_mul_lo_u32 at a quarter of it.
__device__ __forceinline__ int imul24(int a, int b) { return (int)__umul24((unsigned)a, (unsigned)b); }

// Loads and stores at a 32-bit byte offset from a uniform base pointer: the
// memory instruction adds the 64-bit scalar base and the 32-bit vector
// offset itself, so a particle index costs one shift for every plane.
template <typename T>
__device__ __forceinline__ T ld_off(const T *base, uint32_t off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}
template <typename T>
__device__ __forceinline__ void st_off(T *base, uint32_t off, T v)
{
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off) = v;
}

template <int D>
__device__ __forceinline__ int ext(const int32_t T[3], int d, int halo)
{
    return d < D ? T[d] + halo : 1;
}

// Number of lanes below this one whose bit is set in mask.
__device__ __forceinline__ int lanes_below(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Near-face flag of a stored tile-local position: some grid coordinate lies
// within band_d of an integer (a cell face).  x - rint(x) is exact in R, so
// the test is the same in any precision that holds x exactly.
template <typename R, int D>
__device__ __forceinline__ bool near_face(const R x[3], const R band[3])
{
    bool f = false;
#pragma unroll
    for (int d = 0; d < D; ++d) f = f || fabs(x[d] - rint(x[d])) <= band[d];
    return f;
}

__device__ __forceinline__ void latch(int32_t *err, int32_t bits)
{
    atomicOr(err, bits);
}

// OR the per-thread error bits of a wave into the device word with one
// atomic (called by every lane of the wave): a burst of failing particles
// then costs one atomic per wave instead of one per particle.
__device__ __forceinline__ void latch_wave(int32_t *err, int32_t bits)
{
    const unsigned long long any = __ballot(bits != 0);
    if (!any) return;
    int v = bits;
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    if ((int)(threadIdx.x & 63) == __ffsll((long long)any) - 1) atomicOr(err, v);
}

// LDS atomic add of a current value computed in precision R into an
// accumulator of type A.  A = float or double: a floating-point add.
// A = long long (FP32 runs): fixed point.  The deposit's charge is scaled by
// 2^e (fixed_exponent, |q| 2^e in [2^29, 2^30)) so that every ZigZag value
// has magnitude below 2^31; the value is truncated to an integer (an error
// below one unit, 2^-29 |q|, under the FP32 rounding of a value of a tenth
// of |q|) and added exactly, so a block does not depend on the order of its
// atomics, and the 64-bit integer add of the LDS runs much faster than its
// FP64 add on gfx950.
template <typename A, typename R>
__device__ __forceinline__ void lds_add(A *p, R v)
{
    if constexpr (std::is_same<A, long long>::value) {
        static_assert(sizeof(R) == 4, "fixed-point accumulation is for FP32 values");
        atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)(long long)(int)v);
    } else {
        atomicAdd(p, (A)v);
    }
}

// Exponent e of the fixed-point scale 2^e of one segment's current block:
// |q| 2^e < 2^30, so that ZigZag values (at most (1 + 1/12) |q| per
// segment) stay below 2^31; an entry then sums at most 4 segments per
// particle, so 2^30 particles fit in 64 bits.
template <typename R>
__device__ __forceinline__ int fixed_exponent(R q)
{
    return q == R(0) ? 0 : 29 - ilogb(q);
}

// Field halo block in LDS: local cells -1..T per grid dimension.
template <int D>
struct FieldBox {
    int e0, e1, e2;   // extents
    int n;            // cells in the block
    __device__ FieldBox(const int32_t T[3])
    {
        e0 = ext<D>(T, 0, 2);
        e1 = ext<D>(T, 1, 2);
        e2 = ext<D>(T, 2, 2);
        n = e0 * e1 * e2;
    }
};

// Current halo block: local cells -1..T+1 per grid dimension.
template <int D>
struct CurBox {
    int e0, e1, e2;
    int n;
    __device__ CurBox(const int32_t T[3])
    {
        e0 = ext<D>(T, 0, 3);
        e1 = ext<D>(T, 1, 3);
        e2 = ext<D>(T, 2, 3);
        n = e0 * e1 * e2;
    }
};

// Copy E (local cells -1..T+1) and B (local cells -1..T) of the tile into
// LDS, periodic wrap.  sE layout [3][cb.n], sB layout [3][fb.n].
template <typename R, int D, typename BoxT>
__device__ __forceinline__ void stage_block(const R *__restrict__ src, int64_t N, const TileDesc &td,
                                            const int32_t T[3], R *dst, const BoxT &bx)
{
    const int n0 = td.n[0], n1 = td.n[1], n2 = td.n[2];
    for (int k = threadIdx.x; k < bx.n; k += blockDim.x) {
        int lx = k % bx.e0, ly = (k / bx.e0) % bx.e1, lz = k / (bx.e0 * bx.e1);
        int gx = D > 0 ? wrapi(td.tc[0] * T[0] + lx - 1, n0) : 0;
        int gy = D > 1 ? wrapi(td.tc[1] * T[1] + ly - 1, n1) : 0;
        int gz = D > 2 ? wrapi(td.tc[2] * T[2] + lz - 1, n2) : 0;
        int64_t g = td.cell0 + gx + (int64_t)n0 * (gy + (int64_t)n1 * gz);
#pragma unroll
        for (int m = 0; m < 3; ++m) dst[m * bx.n + k] = src[m * N + g];
    }
}

// First half of the B advance (push_half_b1) applied to the LDS copy of B:
// B -= h curl+ E on local cells -1..T, from the staged E (cells -1..T+1).
template <typename R, int D>
__device__ __forceinline__ void half_b_lds(R *sB, const FieldBox<D> &fb, const R *sE, const CurBox<D> &cb, R h)
{
    for (int k = threadIdx.x; k < fb.n; k += blockDim.x) {
        const int lx = k % fb.e0, ly = (k / fb.e0) % fb.e1, lz = k / (fb.e0 * fb.e1);
        const int e = lx + cb.e0 * (ly + cb.e1 * lz);
        const int ip = D > 0 ? 1 : 0, jp = D > 1 ? cb.e0 : 0, kp = D > 2 ? cb.e0 * cb.e1 : 0;
        const R *Ex = sE, *Ey = sE + cb.n, *Ez = sE + 2 * cb.n;
        const R ex = Ex[e], ey = Ey[e], ez = Ez[e];
        const R cx = (Ez[e + jp] - ez) - (Ey[e + kp] - ey);
        const R cy = (Ex[e + kp] - ex) - (Ez[e + ip] - ez);
        const R cz = (Ey[e + ip] - ey) - (Ex[e + jp] - ex);
        sB[k] -= h * cx;
        sB[fb.n + k] -= h * cy;
        sB[2 * fb.n + k] -= h * cz;
    }
}

// ---------------------------------------------------------- interpolation

// Per-particle interpolation state: for each grid dimension the LDS base
// index and weight of a node-centred (offset 0) and a half-cell (offset
// 1/2) sub-lattice.
template <typename R, int D>
struct Stencil {
    int bn[3], bh[3];
    R wn[3], wh[3];
};

template <typename R, int D>
__device__ __forceinline__ void make_stencil(const R x[3], const int32_t T[3], Stencil<R, D> &s)
{
#pragma unroll
    for (int d = 0; d < D; ++d) {
        R fl = floor(x[d]);
        int ci = (int)fl + T[d] / 2;      // cell in 0..T-1
        R f = x[d] - fl;
        s.bn[d] = ci + 1;                  // LDS offset of local cell -1 is 0
        s.wn[d] = f;
        bool up = f >= R(0.5);
        s.bh[d] = up ? ci + 1 : ci;
        s.wh[d] = up ? f - R(0.5) : f + R(0.5);
    }
}

// Linear interpolation of component COMP (0..5 = Ex..Bz) from its own
// staggered sub-lattice: per dimension the half-cell lattice is used where
// the component is staggered by 1/2.
template <typename R, int D, int COMP>
__device__ __forceinline__ R interp_comp(const R *__restrict__ F, int s1, int s2, const Stencil<R, D> &st)
{
    constexpr bool h0 = COMP == 0 || COMP == 4 || COMP == 5;
    constexpr bool h1 = COMP == 1 || COMP == 3 || COMP == 5;
    constexpr bool h2 = COMP == 2 || COMP == 3 || COMP == 4;
    int b = h0 ? st.bh[0] : st.bn[0];
    R w0 = h0 ? st.wh[0] : st.wn[0];
    if constexpr (D == 1) {
        return F[b] * (R(1) - w0) + F[b + 1] * w0;
    } else {
        b += imul24(h1 ? st.bh[1] : st.bn[1], s1);
        R w1 = h1 ? st.wh[1] : st.wn[1];
        if constexpr (D == 2) {
            R a0 = F[b] * (R(1) - w0) + F[b + 1] * w0;
            R a1 = F[b + s1] * (R(1) - w0) + F[b + s1 + 1] * w0;
            return a0 * (R(1) - w1) + a1 * w1;
        } else {
            b += imul24(h2 ? st.bh[2] : st.bn[2], s2);
            R w2 = h2 ? st.wh[2] : st.wn[2];
            R a00 = F[b] * (R(1) - w0) + F[b + 1] * w0;
            R a10 = F[b + s1] * (R(1) - w0) + F[b + s1 + 1] * w0;
            R a01 = F[b + s2] * (R(1) - w0) + F[b + s2 + 1] * w0;
            R a11 = F[b + s1 + s2] * (R(1) - w0) + F[b + s1 + s2 + 1] * w0;
            R c0 = a00 * (R(1) - w1) + a10 * w1;
            R c1 = a01 * (R(1) - w1) + a11 * w1;
            return c0 * (R(1) - w2) + c1 * w2;
        }
    }
}

template <typename R, int D>
__device__ __forceinline__ void interp_all(const R *sE, const CurBox<D> &cb, const R *sB, const FieldBox<D> &fb,
                                           const R x[3], const int32_t T[3], R e[3], R b[3])
{
    Stencil<R, D> st;
    make_stencil<R, D>(x, T, st);
    const int e1 = cb.e0, e2 = cb.e0 * cb.e1;
    const int f1 = fb.e0, f2 = fb.e0 * fb.e1;
    e[0] = interp_comp<R, D, 0>(sE + 0 * cb.n, e1, e2, st);
    e[1] = interp_comp<R, D, 1>(sE + 1 * cb.n, e1, e2, st);
    e[2] = interp_comp<R, D, 2>(sE + 2 * cb.n, e1, e2, st);
    b[0] = interp_comp<R, D, 3>(sB + 0 * fb.n, f1, f2, st);
    b[1] = interp_comp<R, D, 4>(sB + 1 * fb.n, f1, f2, st);
    b[2] = interp_comp<R, D, 5>(sB + 2 * fb.n, f1, f2, st);
}

// ------------------------------------------------------------------ Boris

// Reciprocal and reciprocal square root in the working precision.  FP32
// uses the hardware v_rcp_f32 / v_rsq_f32 (about 1 ulp), which the FP32
// tolerance of the method admits; FP64 keeps correctly rounded division and
// square root.
template <typename R>
__device__ __forceinline__ R rcp_w(R x);
template <>
__device__ __forceinline__ float rcp_w<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <>
__device__ __forceinline__ double rcp_w<double>(double x) { return 1.0 / x; }
template <typename R>
__device__ __forceinline__ R rsqrt_w(R x);
template <>
__device__ __forceinline__ float rsqrt_w<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <>
__device__ __forceinline__ double rsqrt_w<double>(double x) { return 1.0 / sqrt(x); }

// Relativistic Boris update (App. C) of u^{n-1/2} -> u^{n+1/2}; velocities
// inside the update are carried in units of the Courant number c
// (inv_c = 1/c): u1 = c u + s E/2, gamma1 = sqrt(1 + |u1|^2/c^2),
// t = s B/(2 c gamma1), f = 2/(1+|t|^2), u2 = f (u1 + u1 x t),
// u3 = u1 + u2 x t + s E/2, u = u3/c.
template <typename R>
__device__ __forceinline__ void boris(R u[3], const R e[3], const R b[3], R c, R inv_c, R s)
{
    const R hs = R(0.5) * s;
    R ex = hs * e[0], ey = hs * e[1], ez = hs * e[2];
    R u1x = c * u[0] + ex, u1y = c * u[1] + ey, u1z = c * u[2] + ez;
    R k = (hs * inv_c) * rsqrt_w<R>(R(1) + (u1x * u1x + u1y * u1y + u1z * u1z) * (inv_c * inv_c));
    R tx = k * b[0], ty = k * b[1], tz = k * b[2];
    R f = R(2) * rcp_w<R>(R(1) + (tx * tx + ty * ty + tz * tz));
    R u2x = f * (u1x + (u1y * tz - u1z * ty));
    R u2y = f * (u1y + (u1z * tx - u1x * tz));
    R u2z = f * (u1z + (u1x * ty - u1y * tx));
    R u3x = u1x + (u2y * tz - u2z * ty) + ex;
    R u3y = u1y + (u2z * tx - u2x * tz) + ey;
    R u3z = u1z + (u2x * ty - u2y * tx) + ez;
    u[0] = u3x * inv_c;
    u[1] = u3y * inv_c;
    u[2] = u3z * inv_c;
}

// Lorentz factor of the implicit magnetic rotation: the gamma that solves
// w1 = w' + (w1/gamma) x tau, from gamma'^2 = 1 + |w'|^2/c^2 and
// u* = w'.tau/c (Vay 2008; Higuera and Cary 2017).  IEEE square roots in both
// precisions.
template <typename R>
__device__ __forceinline__ R implicit_gamma(const R w[3], const R tau[3], R inv_c)
{
    const R g2 = R(1) + (w[0] * w[0] + w[1] * w[1] + w[2] * w[2]) * (inv_c * inv_c);
    const R us = (w[0] * tau[0] + w[1] * tau[1] + w[2] * tau[2]) * inv_c;
    const R t2 = tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2];
    const R sg = g2 - t2;
    return sqrt(R(0.5) * (sg + sqrt(sg * sg + R(4) * (t2 + us * us))));
}

// w <- (w + (w.t) t + w x t) / (1 + |t|^2): the exact rotation of the
// implicit update.
template <typename R>
__device__ __forceinline__ void exact_rotation(R w[3], const R t[3])
{
    const R wt = w[0] * t[0] + w[1] * t[1] + w[2] * t[2];
    const R sf = R(1) / (R(1) + (t[0] * t[0] + t[1] * t[1] + t[2] * t[2]));
    const R x0 = w[1] * t[2] - w[2] * t[1], x1 = w[2] * t[0] - w[0] * t[2], x2 = w[0] * t[1] - w[1] * t[0];
    w[0] = sf * (w[0] + wt * t[0] + x0);
    w[1] = sf * (w[1] + wt * t[1] + x1);
    w[2] = sf * (w[2] + wt * t[2] + x2);
}

// Vay pusher (units of App. C, w = c u): the full electric kick and half
// the magnetic kick with the old velocity, then the other magnetic half with
// the new velocity, solved exactly.
template <typename R>
__device__ __forceinline__ void vay(R u[3], const R e[3], const R b[3], R c, R inv_c, R s)
{
    const R k = R(0.5) * s * inv_c;
    const R tau[3] = {k * b[0], k * b[1], k * b[2]};
    R w[3] = {c * u[0], c * u[1], c * u[2]};
    const R ig0 = R(1) / sqrt(R(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const R v[3] = {w[0] * ig0, w[1] * ig0, w[2] * ig0};
    w[0] += s * e[0] + (v[1] * tau[2] - v[2] * tau[1]);
    w[1] += s * e[1] + (v[2] * tau[0] - v[0] * tau[2]);
    w[2] += s * e[2] + (v[0] * tau[1] - v[1] * tau[0]);
    const R ig = R(1) / implicit_gamma<R>(w, tau, inv_c);
    const R t[3] = {tau[0] * ig, tau[1] * ig, tau[2] * ig};
    exact_rotation<R>(w, t);
    u[0] = w[0] * inv_c;
    u[1] = w[1] * inv_c;
    u[2] = w[2] * inv_c;
}

// Higuera-Cary pusher: Boris's split with the rotation's Lorentz factor from
// the implicit relation (volume preserving, exact E x B velocity).
template <typename R>
__device__ __forceinline__ void higuera_cary(R u[3], const R e[3], const R b[3], R c, R inv_c, R s)
{
    const R hs = R(0.5) * s, k = hs * inv_c;
    const R eps[3] = {hs * e[0], hs * e[1], hs * e[2]};
    const R tau[3] = {k * b[0], k * b[1], k * b[2]};
    R w[3] = {c * u[0] + eps[0], c * u[1] + eps[1], c * u[2] + eps[2]};
    const R ig = R(1) / implicit_gamma<R>(w, tau, inv_c);
    const R t[3] = {tau[0] * ig, tau[1] * ig, tau[2] * ig};
    exact_rotation<R>(w, t);
    const R x0 = w[1] * t[2] - w[2] * t[1], x1 = w[2] * t[0] - w[0] * t[2], x2 = w[0] * t[1] - w[1] * t[0];
    u[0] = (w[0] + eps[0] + x0) * inv_c;
    u[1] = (w[1] + eps[1] + x1) * inv_c;
    u[2] = (w[2] + eps[2] + x2) * inv_c;
}

enum : int { PUSHER_BORIS = 0, PUSHER_VAY = 1, PUSHER_HC = 2 };

template <typename R, int PUSHER>
__device__ __forceinline__ void push_u(R u[3], const R e[3], const R b[3], R c, R inv_c, R s)
{
    if constexpr (PUSHER == PUSHER_VAY) vay<R>(u, e, b, c, inv_c, s);
    else if constexpr (PUSHER == PUSHER_HC) higuera_cary<R>(u, e, b, c, inv_c, s);
    else boris<R>(u, e, b, c, inv_c, s);
}

// Eq. (fdX): displacement c u / gamma of u^{n+1/2}, all three components.
template <typename R>
__device__ __forceinline__ void displacement(const R u[3], R c, R dv[3])
{
    R r = c * rsqrt_w<R>(R(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    dv[0] = u[0] * r;
    dv[1] = u[1] * r;
    dv[2] = u[2] * r;
}

// The same, returning gamma^2 = 1 + |u|^2 (finite exactly when u is).
template <typename R>
__device__ __forceinline__ R displacement_sq(const R u[3], R c, R dv[3])
{
    const R g2 = R(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const R r = c * rsqrt_w<R>(g2);
    dv[0] = u[0] * r;
    dv[1] = u[1] * r;
    dv[2] = u[2] * r;
    return g2;
}

// ----------------------------------------------------------------- ZigZag

// Current of one straight segment inside one cell, as the values it adds
// to the LDS current block: component m goes to the cell index along m and,
// along each transverse grid dimension a, to points i_a and i_a+1 with
// weights 1-W_a and W_a at the segment midpoint; with two transverse
// dimensions the path average of the product adds
// sigma_a sigma_b dv_a dv_b / 12.  Value order matches seg_offset().
template <int D>
__host__ __device__ constexpr int seg_values()
{
    return D == 1 ? 5 : (D == 2 ? 8 : 12);
}

template <typename R, int D>
__device__ __forceinline__ void segment_values(const R F[3], const R W[3], const R dv[3], R v[seg_values<D>()])
{
    if constexpr (D == 1) {
        v[0] = F[0];
        v[1] = F[1] * (R(1) - W[0]);
        v[2] = F[1] * W[0];
        v[3] = F[2] * (R(1) - W[0]);
        v[4] = F[2] * W[0];
    } else if constexpr (D == 2) {
        v[0] = F[0] * (R(1) - W[1]);
        v[1] = F[0] * W[1];
        v[2] = F[1] * (R(1) - W[0]);
        v[3] = F[1] * W[0];
        const R cr = dv[0] * dv[1] * R(1.0 / 12.0);
        v[4] = F[2] * ((R(1) - W[0]) * (R(1) - W[1]) + cr);
        v[5] = F[2] * (W[0] * (R(1) - W[1]) - cr);
        v[6] = F[2] * ((R(1) - W[0]) * W[1] - cr);
        v[7] = F[2] * (W[0] * W[1] + cr);
    } else {
        const R cyz = dv[1] * dv[2] * R(1.0 / 12.0);
        v[0] = F[0] * ((R(1) - W[1]) * (R(1) - W[2]) + cyz);
        v[1] = F[0] * (W[1] * (R(1) - W[2]) - cyz);
        v[2] = F[0] * ((R(1) - W[1]) * W[2] - cyz);
        v[3] = F[0] * (W[1] * W[2] + cyz);
        const R cxz = dv[0] * dv[2] * R(1.0 / 12.0);
        v[4] = F[1] * ((R(1) - W[0]) * (R(1) - W[2]) + cxz);
        v[5] = F[1] * (W[0] * (R(1) - W[2]) - cxz);
        v[6] = F[1] * ((R(1) - W[0]) * W[2] - cxz);
        v[7] = F[1] * (W[0] * W[2] + cxz);
        const R cxy = dv[0] * dv[1] * R(1.0 / 12.0);
        v[8] = F[2] * ((R(1) - W[0]) * (R(1) - W[1]) + cxy);
        v[9] = F[2] * (W[0] * (R(1) - W[1]) - cxy);
        v[10] = F[2] * ((R(1) - W[0]) * W[1] - cxy);
        v[11] = F[2] * (W[0] * W[1] + cxy);
    }
}

// The same values as flux component times weight: value k is
// F[seg_comp<D>(k)] * wt[k].
template <int D>
__host__ __device__ constexpr int seg_comp(int k)
{
    return D == 1 ? (k == 0 ? 0 : (k < 3 ? 1 : 2)) : (D == 2 ? (k < 2 ? 0 : (k < 4 ? 1 : 2)) : (k < 4 ? 0 : (k < 8 ? 1 : 2)));
}

template <typename R, int D>
__device__ __forceinline__ void segment_weights(const R W[3], const R dv[3], R wt[seg_values<D>()])
{
    if constexpr (D == 1) {
        wt[0] = R(1);
        wt[1] = R(1) - W[0];
        wt[2] = W[0];
        wt[3] = R(1) - W[0];
        wt[4] = W[0];
    } else if constexpr (D == 2) {
        wt[0] = R(1) - W[1];
        wt[1] = W[1];
        wt[2] = R(1) - W[0];
        wt[3] = W[0];
        const R cr = dv[0] * dv[1] * R(1.0 / 12.0);
        wt[4] = (R(1) - W[0]) * (R(1) - W[1]) + cr;
        wt[5] = W[0] * (R(1) - W[1]) - cr;
        wt[6] = (R(1) - W[0]) * W[1] - cr;
        wt[7] = W[0] * W[1] + cr;
    } else {
        const R cyz = dv[1] * dv[2] * R(1.0 / 12.0);
        wt[0] = (R(1) - W[1]) * (R(1) - W[2]) + cyz;
        wt[1] = W[1] * (R(1) - W[2]) - cyz;
        wt[2] = (R(1) - W[1]) * W[2] - cyz;
        wt[3] = W[1] * W[2] + cyz;
        const R cxz = dv[0] * dv[2] * R(1.0 / 12.0);
        wt[4] = (R(1) - W[0]) * (R(1) - W[2]) + cxz;
        wt[5] = W[0] * (R(1) - W[2]) - cxz;
        wt[6] = (R(1) - W[0]) * W[2] - cxz;
        wt[7] = W[0] * W[2] + cxz;
        const R cxy = dv[0] * dv[1] * R(1.0 / 12.0);
        wt[8] = (R(1) - W[0]) * (R(1) - W[1]) + cxy;
        wt[9] = W[0] * (R(1) - W[1]) - cxy;
        wt[10] = (R(1) - W[0]) * W[1] - cxy;
        wt[11] = W[0] * W[1] + cxy;
    }
}

// LDS offsets (relative to the segment's cell) of those values: component
// plane offset plus corner offset.
template <int D>
__device__ __forceinline__ int seg_offset(const CurBox<D> &cb, int k)
{
    const int s1 = cb.e0, s2 = cb.e0 * cb.e1, n = cb.n;
    if constexpr (D == 1) {
        return k == 0 ? 0 : (k == 1 ? n : (k == 2 ? n + 1 : (k == 3 ? 2 * n : 2 * n + 1)));
    } else if constexpr (D == 2) {
        switch (k) {
        case 0: return 0;
        case 1: return s1;
        case 2: return n;
        case 3: return n + 1;
        case 4: return 2 * n;
        case 5: return 2 * n + 1;
        case 6: return 2 * n + s1;
        default: return 2 * n + s1 + 1;
        }
    } else {
        switch (k) {
        case 0: return 0;
        case 1: return s1;
        case 2: return s2;
        case 3: return s1 + s2;
        case 4: return n;
        case 5: return n + 1;
        case 6: return n + s2;
        case 7: return n + 1 + s2;
        case 8: return 2 * n;
        case 9: return 2 * n + 1;
        case 10: return 2 * n + s1;
        default: return 2 * n + s1 + 1;
        }
    }
}

// ZigZag deposit (App. D) of one particle moving from x1 to x2 (tile-local,
// unrebased) with displacement dv (all three components) and charge q.
// Relay point per grid dimension: min(min(i1,i2)+1, max(max(i1,i2),
// (x1+x2)/2)); along non-grid dimensions the two segments share dv/2.
// When both segments lie in the same cell they touch the same points, so
// their values are added in registers (F1 w1 + F2 w2, one multiply-add) and
// written with one set of atomics.
template <typename R, int D, typename A>
__device__ __forceinline__ void zigzag(A *sJ, const CurBox<D> &cb, const int32_t T[3], const R x1[3], const R x2[3],
                                       const R dv[3], R q)
{
    R F1[3], F2[3], W1[3] = {0, 0, 0}, W2[3] = {0, 0, 0}, d1[3], d2[3];
    int l1[3] = {0, 0, 0}, l2[3] = {0, 0, 0};
    bool same = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d < D) {
            R a = x1[d], b = x2[d];
            R fa = floor(a), fb = floor(b);
            R lo = fmin(fa, fb), hi = fmax(fa, fb);
            R xr = fmin(lo + R(1), fmax(hi, R(0.5) * (a + b)));
            d1[d] = xr - a;
            d2[d] = b - xr;
            F1[d] = q * d1[d];
            F2[d] = q * d2[d];
            W1[d] = R(0.5) * (a + xr) - fa;
            W2[d] = R(0.5) * (b + xr) - fb;
            l1[d] = (int)fa + T[d] / 2 + 1;
            l2[d] = (int)fb + T[d] / 2 + 1;
            same = same && fa == fb;
        } else {
            R h = R(0.5) * dv[d];
            d1[d] = h;
            d2[d] = h;
            F1[d] = q * h;
            F2[d] = q * h;
        }
    }
    constexpr int NV = seg_values<D>();
    R w1[NV], w2[NV], F2s[3];
    segment_weights<R, D>(W1, d1, w1);
    segment_weights<R, D>(W2, d2, w2);
#pragma unroll
    for (int d = 0; d < 3; ++d) F2s[d] = same ? F2[d] : R(0);
    const int s1 = cb.e0, s2 = cb.e0 * cb.e1;
    const int b1 = l1[0] + (D > 1 ? imul24(l1[1], s1) : 0) + (D > 2 ? imul24(l1[2], s2) : 0);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const int m = seg_comp<D>(k);
        lds_add(sJ + b1 + seg_offset<D>(cb, k), fma(F2s[m], w2[k], F1[m] * w1[k]));
    }
    if (!same) {
        const int b2 = l2[0] + (D > 1 ? imul24(l2[1], s1) : 0) + (D > 2 ? imul24(l2[2], s2) : 0);
#pragma unroll
        for (int k = 0; k < NV; ++k) lds_add(sJ + b2 + seg_offset<D>(cb, k), F2[seg_comp<D>(k)] * w2[k]);
    }
}

// ------------------------------------------------------------------ walls

// Conducting, reflecting walls at x = 0 and x = n0 (y, z periodic): the
// x-staggered components (Ex, By, Bz) see the wall as a mirror, the
// node-centred ones (Ey, Ez, Bx) vanish on the wall plane.  Applied to the
// staged LDS blocks of a wall tile after push_half_b1: the low wall's ghost
// column (local x = -1) and the high wall's column (local x = T) take the
// image values.
template <typename R, int D>
__device__ __forceinline__ void wall_images(R *sE, const CurBox<D> &cb, R *sB, const FieldBox<D> &fb,
                                            const int32_t T[3], int walls)
{
    const int rows_e = cb.e1 * cb.e2, rows_b = fb.e1 * fb.e2;
    for (int r = threadIdx.x; r < rows_e; r += blockDim.x) {
        R *row = sE + r * cb.e0;
        if (walls & 1) row[0] = row[1];                         // Ex(-1/2) = Ex(1/2)
        if (walls & 2) {
            row[T[0] + 1] = row[T[0]];                          // Ex(n0+1/2) = Ex(n0-1/2)
            row[cb.n + T[0] + 1] = R(0);                        // Ey, Ez on the wall plane
            row[2 * cb.n + T[0] + 1] = R(0);
        }
    }
    for (int r = threadIdx.x; r < rows_b; r += blockDim.x) {
        R *row = sB + r * fb.e0;
        if (walls & 1) {
            row[fb.n] = row[fb.n + 1];                          // By, Bz mirror
            row[2 * fb.n] = row[2 * fb.n + 1];
        }
        if (walls & 2) {
            row[T[0] + 1] = R(0);                               // Bx on the wall plane
            row[fb.n + T[0] + 1] = row[fb.n + T[0]];
            row[2 * fb.n + T[0] + 1] = row[2 * fb.n + T[0]];
        }
    }
}

// A particle of a wall tile whose move ends beyond the wall is reflected:
// the current runs along the broken path x1 -> wall point -> mirrored end
// (two ZigZag moves, the non-grid displacement split in proportion), then
// x2 and u_x are mirrored.  Returns false (nothing done) for other moves.
template <typename R, int D, typename A>
__device__ __forceinline__ bool wall_reflect(A *sJ, const CurBox<D> &cb, const int32_t T[3], int walls,
                                             const R x1[3], R x2[3], R u[3], const R dv[3], R q)
{
    const R half = R(T[0] / 2);
    const bool lo = (walls & 1) && x2[0] < -half;
    const bool hi = (walls & 2) && x2[0] >= half;
    if (!(lo || hi)) return false;
    const R wx = lo ? -half : half;
    const R t = (wx - x1[0]) / (x2[0] - x1[0]);
    R w[3] = {wx, 0, 0}, r[3] = {0, 0, 0}, dv1[3] = {0, 0, 0}, dv2[3] = {0, 0, 0};
#pragma unroll
    for (int d = 1; d < 3; ++d) {
        if (d < D) {
            w[d] = x1[d] + t * (x2[d] - x1[d]);
            r[d] = x2[d];
        } else {
            dv1[d] = t * dv[d];
            dv2[d] = dv[d] - dv1[d];
        }
    }
    r[0] = lo ? -R(T[0]) - x2[0] : R(T[0]) - x2[0];
    if (r[0] >= half) r[0] = nextafter(half, R(0));
    zigzag<R, D, A>(sJ, cb, T, x1, w, dv1, q);
    zigzag<R, D, A>(sJ, cb, T, w, r, dv2, q);
#pragma unroll
    for (int d = 0; d < D; ++d) x2[d] = r[d];
    u[0] = -u[0];
    return true;
}

// Tile offset code sum (delta_d+1) 3^d of a position after the push.
template <typename R, int D>
__device__ __forceinline__ int direction_code(const R x[3], const int32_t T[3], int delta[3])
{
    int code = 0, p3 = 1;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        R half = R(T[d] / 2);
        delta[d] = x[d] < -half ? -1 : (x[d] >= half ? 1 : 0);
        code += (delta[d] + 1) * p3;
        p3 *= 3;
    }
    return code;
}

template <int D>
__host__ __device__ constexpr int centre_code()
{
    return D == 1 ? 1 : (D == 2 ? 4 : 13);
}

template <int D>
__host__ __device__ constexpr int ncodes()
{
    return D == 1 ? 3 : (D == 2 ? 9 : 27);
}

}  // namespace pic
