// Adjoint (reverse mode) of the fused step on gfx950: the vector-Jacobian
// product of one step, for gradients of a loss of a later state with respect
// to an earlier one (differentiable windows with checkpointed recomputation).
//
// The per-particle part mirrors the push: one work-group per tile stages E,
// B (then B^n in LDS) and the current adjoint lambda_J with their halos,
// recomputes each particle's push, and runs it backwards: ZigZag adjoint
// (forward-mode dual numbers through the same segment-value code as the
// deposit), position and displacement adjoints, Boris adjoint (hand-derived
// reverse of App. C) and the interpolation adjoint, whose scatter into the
// field adjoints goes to FP64 LDS blocks that are flushed and folded like the
// current.
#pragma once

#include "pic_kernels.hpp"

namespace pic {

// ------------------------------------------------------------ dual numbers

template <typename R, int N>
struct Dual {
    R v;
    R d[N];
    __device__ Dual() : v(0)
    {
#pragma unroll
        for (int k = 0; k < N; ++k) d[k] = R(0);
    }
    __device__ Dual(R x) : v(x)
    {
#pragma unroll
        for (int k = 0; k < N; ++k) d[k] = R(0);
    }
    __device__ static Dual seed(R x, int k)
    {
        Dual r(x);
        r.d[k] = R(1);
        return r;
    }
};

template <typename R, int N>
__device__ __forceinline__ Dual<R, N> operator+(const Dual<R, N> &a, const Dual<R, N> &b)
{
    Dual<R, N> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k];
    return r;
}
template <typename R, int N>
__device__ __forceinline__ Dual<R, N> operator-(const Dual<R, N> &a, const Dual<R, N> &b)
{
    Dual<R, N> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k];
    return r;
}
template <typename R, int N>
__device__ __forceinline__ Dual<R, N> operator*(const Dual<R, N> &a, const Dual<R, N> &b)
{
    Dual<R, N> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}

// ------------------------------------------------------ ZigZag adjoint

// d(sum_points lambda_J . J)/d(x1, x2, dv_nongrid) of one particle's ZigZag
// deposit.  Inputs k: x1_d (k = d), x2_d (k = D + d), dv_m for m >= D
// (k = 2D + m - D).  The relay point and cells are taken on the branch of the
// forward value; sLJ is the staged lambda_J block (local cells -1..T+1).
template <typename R, int D, typename LA>
__device__ __forceinline__ void zigzag_adjoint(const LA *sLJ, const CurBox<D> &cb, const int32_t T[3], const R x1[3],
                                               const R x2[3], const R dv[3], R q, R lx1[3], R lx2[3], R ldv[3])
{
    constexpr int NI = 2 * D + (3 - D);
    using DD = Dual<R, NI>;
    DD F1[3], F2[3], W1[3], W2[3], d1[3], d2[3];
    int l1[3] = {0, 0, 0}, l2[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d < D) {
            const DD a = DD::seed(x1[d], d), b = DD::seed(x2[d], D + d);
            const R fa = floor(a.v), fb = floor(b.v);
            const R lo = fmin(fa, fb), hi = fmax(fa, fb);
            const DD mid = DD(R(0.5)) * (a + b);
            const DD inner = hi > mid.v ? DD(hi) : mid;
            const DD xr = (lo + R(1)) < inner.v ? DD(lo + R(1)) : inner;
            d1[d] = xr - a;
            d2[d] = b - xr;
            F1[d] = DD(q) * d1[d];
            F2[d] = DD(q) * d2[d];
            W1[d] = DD(R(0.5)) * (a + xr) - DD(fa);
            W2[d] = DD(R(0.5)) * (b + xr) - DD(fb);
            l1[d] = (int)fa + T[d] / 2 + 1;
            l2[d] = (int)fb + T[d] / 2 + 1;
        } else {
            const DD h = DD(R(0.5)) * DD::seed(dv[d], 2 * D + d - D);
            d1[d] = h;
            d2[d] = h;
            F1[d] = DD(q) * h;
            F2[d] = DD(q) * h;
        }
    }
    constexpr int NV = seg_values<D>();
    DD v1[NV], v2[NV];
    segment_values<DD, D>(F1, W1, d1, v1);
    segment_values<DD, D>(F2, W2, d2, v2);
    const int s1 = cb.e0, s2 = cb.e0 * cb.e1;
    const int b1 = l1[0] + (D > 1 ? l1[1] * s1 : 0) + (D > 2 ? l1[2] * s2 : 0);
    const int b2 = l2[0] + (D > 1 ? l2[1] * s1 : 0) + (D > 2 ? l2[2] * s2 : 0);
    R lin[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) lin[k] = R(0);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const R la = (R)sLJ[b1 + seg_offset<D>(cb, v)];
        const R lb = (R)sLJ[b2 + seg_offset<D>(cb, v)];
#pragma unroll
        for (int k = 0; k < NI; ++k) lin[k] += la * v1[v].d[k] + lb * v2[v].d[k];
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lx1[d] += lin[d];
        lx2[d] += lin[D + d];
    }
#pragma unroll
    for (int m = D; m < 3; ++m) ldv[m] += lin[2 * D + m - D];
}

// --------------------------------------------------- interpolation adjoint

// Value, gradient with respect to the particle position, and (when L is not
// null) the scatter lam * weight into the FP64 adjoint block L of one
// staggered component (same stencil as interp_comp).
template <typename R, int D, int COMP>
__device__ __forceinline__ R interp_comp_adj(const R *__restrict__ F, double *L, int s1, int s2,
                                             const Stencil<R, D> &st, R lam, R g[3])
{
    constexpr bool h0 = COMP == 0 || COMP == 4 || COMP == 5;
    constexpr bool h1 = COMP == 1 || COMP == 3 || COMP == 5;
    constexpr bool h2 = COMP == 2 || COMP == 3 || COMP == 4;
    int b = h0 ? st.bh[0] : st.bn[0];
    const R w0 = h0 ? st.wh[0] : st.wn[0];
    if constexpr (D == 1) {
        g[0] = F[b + 1] - F[b];
        if (L) {
            lds_add(L + b, lam * (R(1) - w0));
            lds_add(L + b + 1, lam * w0);
        }
        return F[b] * (R(1) - w0) + F[b + 1] * w0;
    } else if constexpr (D == 2) {
        b += (h1 ? st.bh[1] : st.bn[1]) * s1;
        const R w1 = h1 ? st.wh[1] : st.wn[1];
        const R f00 = F[b], f10 = F[b + 1], f01 = F[b + s1], f11 = F[b + s1 + 1];
        const R a0 = f00 * (R(1) - w0) + f10 * w0, a1 = f01 * (R(1) - w0) + f11 * w0;
        g[0] = (f10 - f00) * (R(1) - w1) + (f11 - f01) * w1;
        g[1] = a1 - a0;
        if (L) {
            lds_add(L + b, lam * (R(1) - w0) * (R(1) - w1));
            lds_add(L + b + 1, lam * w0 * (R(1) - w1));
            lds_add(L + b + s1, lam * (R(1) - w0) * w1);
            lds_add(L + b + s1 + 1, lam * w0 * w1);
        }
        return a0 * (R(1) - w1) + a1 * w1;
    } else {
        b += (h1 ? st.bh[1] : st.bn[1]) * s1;
        b += (h2 ? st.bh[2] : st.bn[2]) * s2;
        const R w1 = h1 ? st.wh[1] : st.wn[1];
        const R w2 = h2 ? st.wh[2] : st.wn[2];
        R f[8];
#pragma unroll
        for (int cn = 0; cn < 8; ++cn) f[cn] = F[b + (cn & 1) + ((cn >> 1) & 1) * s1 + ((cn >> 2) & 1) * s2];
        R val = R(0);
        g[0] = g[1] = g[2] = R(0);
#pragma unroll
        for (int cn = 0; cn < 8; ++cn) {
            const int c0 = cn & 1, c1 = (cn >> 1) & 1, c2 = (cn >> 2) & 1;
            const R p0 = c0 ? w0 : R(1) - w0, p1 = c1 ? w1 : R(1) - w1, p2 = c2 ? w2 : R(1) - w2;
            val += f[cn] * p0 * p1 * p2;
            g[0] += f[cn] * (c0 ? R(1) : R(-1)) * p1 * p2;
            g[1] += f[cn] * p0 * (c1 ? R(1) : R(-1)) * p2;
            g[2] += f[cn] * p0 * p1 * (c2 ? R(1) : R(-1));
            if (L) lds_add(L + b + c0 + c1 * s1 + c2 * s2, lam * p0 * p1 * p2);
        }
        return val;
    }
}

// ------------------------------------------------------------ Boris adjoint

// Reverse of boris(): from u0 = u^{n-1/2}, the fields at the particle and
// lu1 = lambda of u^{n+1/2}, the adjoints of u0, E and B.  Written from the
// exact update (division and square root), independent of how the forward
// evaluates them.
template <typename R>
__device__ __forceinline__ void boris_adjoint(const R u0[3], const R e[3], const R bf[3], R c, R inv_c, R s,
                                              const R lu1[3], R lu0[3], R lE[3], R lB[3])
{
    const R hs = R(0.5) * s;
    R eps[3], a[3], t[3], w[3], b[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        eps[i] = hs * e[i];
        a[i] = c * u0[i] + eps[i];
    }
    const R g1 = sqrt(R(1) + (a[0] * a[0] + a[1] * a[1] + a[2] * a[2]) * (inv_c * inv_c));
    const R kap = hs * inv_c / g1;
#pragma unroll
    for (int i = 0; i < 3; ++i) t[i] = kap * bf[i];
    const R f = R(2) / (R(1) + (t[0] * t[0] + t[1] * t[1] + t[2] * t[2]));
    w[0] = a[0] + (a[1] * t[2] - a[2] * t[1]);
    w[1] = a[1] + (a[2] * t[0] - a[0] * t[2]);
    w[2] = a[2] + (a[0] * t[1] - a[1] * t[0]);
#pragma unroll
    for (int i = 0; i < 3; ++i) b[i] = f * w[i];
    R lc[3], la[3], leps[3], lb[3], lt[3], lw[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        lc[i] = lu1[i] * inv_c;
        la[i] = lc[i];
        leps[i] = lc[i];
    }
    lb[0] = t[1] * lc[2] - t[2] * lc[1];
    lb[1] = t[2] * lc[0] - t[0] * lc[2];
    lb[2] = t[0] * lc[1] - t[1] * lc[0];
    lt[0] = lc[1] * b[2] - lc[2] * b[1];
    lt[1] = lc[2] * b[0] - lc[0] * b[2];
    lt[2] = lc[0] * b[1] - lc[1] * b[0];
    R lf = R(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        lw[i] = f * lb[i];
        lf += w[i] * lb[i];
    }
    la[0] += lw[0] + (t[1] * lw[2] - t[2] * lw[1]);
    la[1] += lw[1] + (t[2] * lw[0] - t[0] * lw[2]);
    la[2] += lw[2] + (t[0] * lw[1] - t[1] * lw[0]);
    lt[0] += lw[1] * a[2] - lw[2] * a[1];
    lt[1] += lw[2] * a[0] - lw[0] * a[2];
    lt[2] += lw[0] * a[1] - lw[1] * a[0];
#pragma unroll
    for (int i = 0; i < 3; ++i) lt[i] -= lf * f * f * t[i];
    R lkap = R(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        lB[i] = kap * lt[i];
        lkap += bf[i] * lt[i];
    }
    const R lg1 = -kap / g1 * lkap;
#pragma unroll
    for (int i = 0; i < 3; ++i) la[i] += lg1 * a[i] * (inv_c * inv_c) / g1;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        lu0[i] = c * la[i];
        leps[i] += la[i];
        lE[i] = hs * leps[i];
    }
}

// ------------------------------------------------------------ kernels

template <typename R>
struct AdjParams {
    R *lpos, *lu;             // [D|3][cap_total], layout of the state
    R *lE, *lB;               // [3][cells_total]
    R *lJ;                    // [3][cells_total] scratch: lambda of J = -lambda_E
    R *eblk, *bblk;           // per tile [3][(T+3)^D], [3][(T+2)^D] adjoint blocks
};

// Per tile: the particle part of the adjoint step.  State in p (particles
// x^n, u^{n-1/2}; E^n, B^{n-1/2}); on entry a.lpos/a.lu hold the adjoints of
// x^{n+1}, u^{n+1/2} (same slots), on exit those of x^n, u^{n-1/2}; the
// interpolation adjoints go to the per-tile blocks a.eblk (for E^n) and
// a.bblk (for B^n).
template <typename R, int D>
__global__ void __launch_bounds__(256) k_adj_push(Params<R> p, AdjParams<R> a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int t = blockIdx.x;
    const TileDesc td = p.tiles[t];
    const FieldBox<D> fb(p.T);
    const CurBox<D> cb(p.T);
    double *aE = reinterpret_cast<double *>(smem);           // [3][cb.n]
    double *aB = aE + 3 * cb.n;                              // [3][fb.n]
    R *sLJ = reinterpret_cast<R *>(aB + 3 * fb.n);           // [3][cb.n]
    R *sE = sLJ + 3 * cb.n;                                  // [3][cb.n]
    R *sB = sE + 3 * cb.n;                                   // [3][fb.n]
    stage_block<R, D>(p.E, p.cells_total, td, p.T, sE, cb);
    stage_block<R, D>(p.B, p.cells_total, td, p.T, sB, fb);
    stage_block<R, D>(a.lJ, p.cells_total, td, p.T, sLJ, cb);
    for (int k = threadIdx.x; k < 3 * cb.n; k += blockDim.x) aE[k] = 0.0;
    for (int k = threadIdx.x; k < 3 * fb.n; k += blockDim.x) aB[k] = 0.0;
    __syncthreads();
    half_b_lds<R, D>(sB, fb, sE, cb, R(0.5) * p.c);   // B^n, as the push saw it
    __syncthreads();
    const R c = p.c, inv_c = p.inv_c;
    const int64_t cap = p.cap_total;
    const int e1 = cb.e0, e2 = cb.e0 * cb.e1, f1 = fb.e0, f2 = fb.e0 * fb.e1;
    for (int s = 0; s < p.nspecies; ++s) {
        const int ts = t * p.nspecies + s;
        const int64_t so = p.seg_off[ts];
        const int cnt = p.seg_cnt[ts];
        const R q = p.charge[td.box * p.nspecies + s];
        const R sq = p.qm[td.box * p.nspecies + s];
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
            R x[3] = {0, 0, 0}, u0[3], lx[3] = {0, 0, 0}, lu[3];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                x[d] = p.pos[d * cap + so + i];
                lx[d] = a.lpos[d * cap + so + i];
            }
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                u0[m] = p.u[m * cap + so + i];
                lu[m] = a.lu[m * cap + so + i];
            }
            if (!inside_tile<R, D>(x, p.T)) continue;
            // forward recomputation of this particle's push
            Stencil<R, D> st;
            make_stencil<R, D>(x, p.T, st);
            R e[3], b[3], g[6][3];
            e[0] = interp_comp_adj<R, D, 0>(sE + 0 * cb.n, nullptr, e1, e2, st, R(0), g[0]);
            e[1] = interp_comp_adj<R, D, 1>(sE + 1 * cb.n, nullptr, e1, e2, st, R(0), g[1]);
            e[2] = interp_comp_adj<R, D, 2>(sE + 2 * cb.n, nullptr, e1, e2, st, R(0), g[2]);
            b[0] = interp_comp_adj<R, D, 3>(sB + 0 * fb.n, nullptr, f1, f2, st, R(0), g[3]);
            b[1] = interp_comp_adj<R, D, 4>(sB + 1 * fb.n, nullptr, f1, f2, st, R(0), g[4]);
            b[2] = interp_comp_adj<R, D, 5>(sB + 2 * fb.n, nullptr, f1, f2, st, R(0), g[5]);
            R u1[3] = {u0[0], u0[1], u0[2]}, dv[3], x2[3] = {0, 0, 0};
            boris<R>(u1, e, b, c, inv_c, sq);
            displacement<R>(u1, c, dv);
#pragma unroll
            for (int d = 0; d < D; ++d) x2[d] = x[d] + dv[d];
            if (!(finite3<R>(u1) && moved_ok<R, D>(x2, dv, p.T))) continue;
            // reverse: comp_curr
            R ldv[3] = {0, 0, 0}, lx1[3] = {0, 0, 0};
            zigzag_adjoint<R, D, R>(sLJ, cb, p.T, x, x2, dv, q, lx1, lx, ldv);
            // x2 = x + dv
#pragma unroll
            for (int d = 0; d < D; ++d) {
                lx1[d] += lx[d];
                ldv[d] += lx[d];
            }
            // dv = c u1 / gamma(u1)
            const R gam = sqrt(R(1) + u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
            const R ul = u1[0] * ldv[0] + u1[1] * ldv[1] + u1[2] * ldv[2];
#pragma unroll
            for (int m = 0; m < 3; ++m) lu[m] += c * (ldv[m] / gam - u1[m] * ul / (gam * gam * gam));
            // Boris
            R lu0[3], lEp[3], lBp[3];
            boris_adjoint<R>(u0, e, b, c, inv_c, sq, lu, lu0, lEp, lBp);
            // interpolation: scatter into the field adjoints, gradient in x
            R gg[3];
            interp_comp_adj<R, D, 0>(sE + 0 * cb.n, aE + 0 * cb.n, e1, e2, st, lEp[0], gg);
            interp_comp_adj<R, D, 1>(sE + 1 * cb.n, aE + 1 * cb.n, e1, e2, st, lEp[1], gg);
            interp_comp_adj<R, D, 2>(sE + 2 * cb.n, aE + 2 * cb.n, e1, e2, st, lEp[2], gg);
            interp_comp_adj<R, D, 3>(sB + 0 * fb.n, aB + 0 * fb.n, f1, f2, st, lBp[0], gg);
            interp_comp_adj<R, D, 4>(sB + 1 * fb.n, aB + 1 * fb.n, f1, f2, st, lBp[1], gg);
            interp_comp_adj<R, D, 5>(sB + 2 * fb.n, aB + 2 * fb.n, f1, f2, st, lBp[2], gg);
#pragma unroll
            for (int d = 0; d < D; ++d)
                lx1[d] += lEp[0] * g[0][d] + lEp[1] * g[1][d] + lEp[2] * g[2][d] + lBp[0] * g[3][d] +
                          lBp[1] * g[4][d] + lBp[2] * g[5][d];
#pragma unroll
            for (int d = 0; d < D; ++d) a.lpos[d * cap + so + i] = lx1[d];
#pragma unroll
            for (int m = 0; m < 3; ++m) a.lu[m * cap + so + i] = lu0[m];
        }
    }
    __syncthreads();
    R *eb = a.eblk + (int64_t)t * 3 * cb.n;
    R *bb = a.bblk + (int64_t)t * 3 * fb.n;
    for (int k = threadIdx.x; k < 3 * cb.n; k += blockDim.x) eb[k] = (R)aE[k];
    for (int k = threadIdx.x; k < 3 * fb.n; k += blockDim.x) bb[k] = (R)aB[k];
}

// Add the folded adjoint blocks into the field adjoints: the E-type block
// covers local cells -1..T+1, the B-type block -1..T.
template <typename R, int D>
__global__ void __launch_bounds__(256) k_adj_fold(Params<R> p, AdjParams<R> a)
{
    const int t = blockIdx.x;
    const TileDesc td = p.tiles[t];
    const CurBox<D> cb(p.T);
    const FieldBox<D> fb(p.T);
    const int T0 = p.T[0], T1 = D > 1 ? p.T[1] : 1, T2 = D > 2 ? p.T[2] : 1;
    const int ncell = T0 * T1 * T2;
    for (int k = threadIdx.x; k < ncell; k += blockDim.x) {
        const int l[3] = {k % T0, (k / T0) % T1, k / (T0 * T1)};
        R acc[6] = {0, 0, 0, 0, 0, 0};
        for (int oz = (D > 2 ? -1 : 0); oz <= (D > 2 ? 1 : 0); ++oz)
            for (int oy = (D > 1 ? -1 : 0); oy <= (D > 1 ? 1 : 0); ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    const int o[3] = {ox, oy, oz};
                    int bi[3] = {0, 0, 0}, nc[3] = {0, 0, 0};
                    bool inE = true, inB = true;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        if (d < D) {
                            bi[d] = l[d] - o[d] * p.T[d] + 1;
                            inE = inE && bi[d] >= 0 && bi[d] < p.T[d] + 3;
                            inB = inB && bi[d] >= 0 && bi[d] < p.T[d] + 2;
                            nc[d] = wrapi(td.tc[d] + o[d], td.nt[d]);
                        }
                    }
                    if (!inE) continue;
                    const int nid = td.tile0 + nc[0] + td.nt[0] * (nc[1] + td.nt[1] * nc[2]);
                    const R *eb = a.eblk + (int64_t)nid * 3 * cb.n;
                    const int ie = bi[0] + cb.e0 * (bi[1] + cb.e1 * bi[2]);
                    acc[0] += eb[ie];
                    acc[1] += eb[cb.n + ie];
                    acc[2] += eb[2 * cb.n + ie];
                    if (inB) {
                        const R *bb = a.bblk + (int64_t)nid * 3 * fb.n;
                        const int ib = bi[0] + fb.e0 * (bi[1] + fb.e1 * bi[2]);
                        acc[3] += bb[ib];
                        acc[4] += bb[fb.n + ib];
                        acc[5] += bb[2 * fb.n + ib];
                    }
                }
        const int gx = td.tc[0] * T0 + l[0];
        const int gy = D > 1 ? td.tc[1] * T1 + l[1] : 0;
        const int gz = D > 2 ? td.tc[2] * T2 + l[2] : 0;
        const int64_t g = td.cell0 + gx + (int64_t)td.n[0] * (gy + (int64_t)td.n[1] * gz);
        const int64_t N = p.cells_total;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            a.lE[m * N + g] += acc[m];
            a.lB[m * N + g] += acc[3 + m];
        }
    }
}

// lambda_J = -lambda_E (the current enters E^{n+1} with a minus sign).
template <typename R>
__global__ void k_adj_neg(R *dst, const R *src, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = -src[i];
}

// Move particle adjoints from the slots of the current state to the slots
// (or input indices) the particles came from: dst = ids[j].  Grid: x over
// (tile, species) segments, y over chunks of blockDim slots of a segment.
template <typename R, int D>
__global__ void __launch_bounds__(256) k_adj_unpermute(Params<R> p, const R *lpos_a, const R *lu_a, R *lpos_b,
                                                       R *lu_b, int64_t stride_b)
{
    const int ts = blockIdx.x;
    const int j = blockIdx.y * blockDim.x + threadIdx.x;
    const int cnt = p.seg_cnt[ts];
    if (j >= cnt) return;
    const int64_t cap = p.cap_total;
    const int64_t src = p.seg_off[ts] + j, dst = p.ids[src];
    if (dst < 0 || dst >= stride_b) {
        latch(p.err, ERR_ADJ_MAP);
        return;
    }
#pragma unroll
    for (int d = 0; d < D; ++d) lpos_b[d * stride_b + dst] = lpos_a[d * cap + src];
#pragma unroll
    for (int m = 0; m < 3; ++m) lu_b[m * stride_b + dst] = lu_a[m * cap + src];
}

}  // namespace pic
