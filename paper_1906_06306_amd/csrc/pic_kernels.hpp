// Kernels of the relativistic PIC step for gfx950 (templated on precision
// R and dimension D).  One work-group owns one tile: it stages the tile's
// E and B (plus halo) in LDS, streams the tile's particles with coalesced
// structure-of-arrays loads, accumulates the ZigZag current in an LDS block
// with atomics and flushes that block once.  Field kernels also walk tiles.
#pragma once

#include "pic_device.hpp"

namespace pic {

constexpr int MAX_WAVES = 16;

// groups of particles the push loads ahead of the one it works on: one.  A
// second group in flight (in registers, or in a second buffer of registers
// the loop alternates) measured slower on the 2D FP32 push: the compiler's
// waits for the alternate buffer come back, and the registers lower occupancy.
constexpr int PUSH_PREFETCH = 1;

// Inclusive prefix sum of v over each row of 16 lanes (DPP row shifts; a
// shifted-in lane outside the row reads 0).  Lanes 0..15 hold the prefix of
// lanes 0..15.
__device__ __forceinline__ int row_prefix16(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);   // row_shr:8
    return v;
}

// The per-wave totals of a work-group scan (written by lane 0 of every wave
// to tot[wave], before a barrier): returns the sum over the waves below this
// one and, in all, over every wave.  Lane w reads the total of wave w and the
// first 16 lanes scan them, so the cost does not grow with the wave count.
__device__ __forceinline__ int wave_totals(const int *tot, int wave, int nw, int &all)
{
    const int lane = threadIdx.x & 63;
    const int v = lane < nw ? tot[lane & (MAX_WAVES - 1)] : 0;
    const int incl = row_prefix16(v);
    all = __builtin_amdgcn_readlane(incl, nw - 1);
    return __builtin_amdgcn_readlane(incl - v, wave);
}

// Exclusive prefix of a per-thread flag over the whole work-group (wave
// ballots, then per-wave totals in LDS).  sTot holds 2*MAX_WAVES ints and the
// two halves alternate by `parity`, so one barrier per call suffices.
__device__ __forceinline__ int wg_scan_flag(bool flag, int *sTot, int parity, int &total)
{
    const int lane = threadIdx.x & 63;
    // the wave index and wave count are uniform (scalar registers)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = __builtin_amdgcn_readfirstlane(blockDim.x >> 6);
    unsigned long long m = __ballot(flag);
    int below = lanes_below(m);
    int *tot = sTot + parity * MAX_WAVES;
    if (lane == 0) tot[wave] = __popcll(m);
    __syncthreads();
    const int off = wave_totals(tot, wave, nw, total);
    return off + below;
}

// Exclusive prefix of U flags per thread over the work-group, in (j, thread)
// order: flag j of thread t is element j*blockDim + t.  sTot holds
// 2*U*MAX_WAVES ints; the halves alternate by `parity` (one barrier).
template <int U>
__device__ __forceinline__ int wg_scan_flags(const bool f[U], int *sTot, int parity, int pre[U])
{
    const int lane = threadIdx.x & 63;
    // the wave index and wave count are uniform (scalar registers)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = __builtin_amdgcn_readfirstlane(blockDim.x >> 6);
    int *tot = sTot + parity * U * MAX_WAVES;
    int below[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
        unsigned long long m = __ballot(f[j]);
        below[j] = lanes_below(m);
        if (lane == 0) tot[j * MAX_WAVES + wave] = __popcll(m);
    }
    __syncthreads();
    int run = 0;
#pragma unroll
    for (int j = 0; j < U; ++j) {
        int all;
        const int off = wave_totals(tot + j * MAX_WAVES, wave, nw, all);
        pre[j] = run + off + below[j];
        run += all;
    }
    return run;
}

// Stable counting sort of one segment's n outbox entries by direction code:
// the bucket starts ob_boff[ncodes + 1] and the outbox slots in bucket order
// ob_idx, so that each neighbour reads exactly the leavers addressed to it.
// The rank of an entry among equal codes of its wave comes from ballots on
// the code bits; waves are ordered through per-wave counts in LDS.  With
// mig_counts, also the segment's migration counts by direction code.  Called
// by the whole work-group (barriers inside).
template <typename R, int D>
__device__ __forceinline__ void bucket_outbox(const Params<R> &p, const int ts, const int n, int *sCnt, int *sBase)
{
    // sCnt: MAX_WAVES * ncodes ints, sBase: ncodes + 1 ints of LDS
    constexpr int NC = ncodes<D>();
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int32_t *dir = p.ob_dir + (int64_t)ts * p.ob_dir_stride;
    int32_t *boff = p.ob_boff + (int64_t)ts * (NC + 1);
    int32_t *idx = p.ob_idx + (int64_t)ts * p.ob_cap;
    // histogram and bucket starts
    for (int k = threadIdx.x; k <= NC; k += blockDim.x) sBase[k] = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x) atomicAdd(&sBase[dir[k] + 1], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int c = 0; c < NC; ++c) sBase[c + 1] += sBase[c];
        for (int c = 0; c <= NC; ++c) boff[c] = sBase[c];
        if (p.mig_counts) {
            // particles of the segment by the tile they went to: the
            // outbox buckets, and the stayers at the centre code (the
            // segment count before the arrivals are appended)
            int32_t *mc = p.mig_counts + (int64_t)ts * NC;
            for (int c = 0; c < NC; ++c) mc[c] = c == centre_code<D>() ? p.seg_cnt[ts] : sBase[c + 1] - sBase[c];
        }
    }
    __syncthreads();
    // stable scatter, one work-group-wide chunk at a time
    for (int c0 = 0; c0 < n; c0 += blockDim.x) {
        for (int k = threadIdx.x; k < nw * NC; k += blockDim.x) sCnt[k] = 0;
        __syncthreads();
        const int k = c0 + (int)threadIdx.x;
        const bool valid = k < n;
        const int code = valid ? dir[k] : 0;
        unsigned long long m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            const unsigned long long bb = __ballot((code >> b) & 1);
            m &= ((code >> b) & 1) ? bb : ~bb;
        }
        const int rank = lanes_below(m);
        if (valid && rank == 0) sCnt[wave * NC + code] = __popcll(m);
        __syncthreads();
        if (valid) {
            int off = sBase[code] + rank;
            for (int w = 0; w < wave; ++w) off += sCnt[w * NC + code];
            idx[off] = k;
        }
        __syncthreads();
        if ((int)threadIdx.x < NC) {
            int add = 0;
            for (int w = 0; w < nw; ++w) add += sCnt[w * NC + threadIdx.x];
            sBase[threadIdx.x] += add;
        }
        __syncthreads();
    }
}

// LDS ints of bucket_outbox's scratch.
template <int D>
__host__ __device__ constexpr int bucket_lds_ints()
{
    return MAX_WAVES * ncodes<D>() + ncodes<D>() + 1;
}

template <typename R, int D>
__device__ __forceinline__ bool inside_tile(const R x[3], const int32_t T[3])
{
    bool ok = true;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        R half = R(T[d] / 2);
        ok = ok && (x[d] >= -half) && (x[d] < half);   // false for NaN
    }
    return ok;
}

// A pushed particle may be deposited when each displacement is below one
// cell and the new position lies in the tile's current halo, so that the
// ZigZag stencil stays inside the LDS block (rounding of x + dx could
// otherwise reach the far face of the halo).
template <typename R, int D>
__device__ __forceinline__ bool moved_ok(const R x2[3], const R dv[3], const int32_t T[3])
{
    bool ok = true;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        R lim = R(T[d] / 2 + 1);
        ok = ok && fabs(dv[d]) < R(1) && x2[d] >= -lim && x2[d] < lim;
    }
    return ok;
}

template <typename R>
__device__ __forceinline__ bool finite3(const R v[3])
{
    return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]);
}

// Write one chunk of particles after the push: stayers compacted in place
// (stable), leavers appended to the tile outbox rebased by -delta T.
// Must be called by every thread of the work-group.
template <typename R, int D>
__device__ __forceinline__ void compact_chunk(const Params<R> &p, int ts, int64_t so, bool valid, int code,
                                              const int delta[3], const R x2[3], const R u[3], int nvalid,
                                              int *sTot, int &parity, int &keep, int &nleave)
{
    const bool stay = valid && code == centre_code<D>();
    int tot;
    int pre = wg_scan_flag(stay, sTot, parity, tot);
    parity ^= 1;
    const int64_t cap = p.cap_total;
    if (stay) {
        int64_t dst = so + keep + pre;
#pragma unroll
        for (int d = 0; d < D; ++d) p.pos[d * cap + dst] = x2[d];
#pragma unroll
        for (int m = 0; m < 3; ++m) p.u[m * cap + dst] = u[m];
    } else if (valid) {
        int64_t slot = nleave + (threadIdx.x - pre);
        if (slot < p.ob_cap) {
            const int64_t ob = (int64_t)ts * p.ob_cap;
#pragma unroll
            for (int d = 0; d < D; ++d)
                p.ob_pos[(ob * D) + d * p.ob_cap + slot] = x2[d] - R(delta[d] * p.T[d]);
#pragma unroll
            for (int m = 0; m < 3; ++m) p.ob_u[(ob * 3) + m * p.ob_cap + slot] = u[m];
            p.ob_dir[(int64_t)ts * p.ob_dir_stride + slot] = code;
        } else {
            latch(p.err, ERR_CAPACITY);
        }
    }
    keep += tot;
    nleave += nvalid - tot;
}

// ------------------------------------------------------------------ push

// interp_em + push (+ comp_curr and particle pack when FUSED) for one tile.
// The current block is accumulated in LDS in type A: 64-bit fixed point for
// FP32 runs (exact integer adds, which gfx950's LDS also runs faster than
// its FP64 adds), FP64 for FP64 runs (the LDS FP32 atomic add is far slower
// than either under the many-address pattern of the deposit), or R on
// request; it is converted to R once, at the flush.  With HALFB the
// kernel applies push_half_b1 to its LDS copy of B itself (global B stays
// at B^{n-1/2}).  Each thread takes U particles per group (element
// c0 + j*blockDim + t), so every load and store instruction stays
// coalesced while U loads per array are in flight; the stable compaction
// runs once per group.
template <typename R, int D, bool FUSED, bool HALFB, typename A, int U, int TC, bool WALLS, int PUSHER>
__device__ __forceinline__ void push_tile(const Params<R> &p, const int w, unsigned char *smem)
{
    // work item w = one (tile, species) segment
    const int t = w / p.nspecies, s = w - t * p.nspecies;
    if (!((p.species_mask >> s) & 1u)) return;   // species not pushed by this call
    const TileDesc td = p.tiles[t];
    // tile edge: a compile-time constant when TC > 0 (strides, LDS offsets
    // and the halves T/2 then fold into the instructions), else the runtime one
    int32_t T[3];
    if constexpr (TC > 0) {
        T[0] = TC;
        T[1] = D > 1 ? TC : 1;
        T[2] = D > 2 ? TC : 1;
    } else {
        T[0] = p.T[0];
        T[1] = p.T[1];
        T[2] = p.T[2];
    }
    const FieldBox<D> fb(T);
    const CurBox<D> cb(T);
    A *sJ = reinterpret_cast<A *>(smem);
    R *sE = reinterpret_cast<R *>(sJ + (FUSED ? 3 * cb.n : 0));
    R *sB = sE + 3 * cb.n;
    int *sTot = reinterpret_cast<int *>(sB + 3 * fb.n);
    int *sNF = sTot + 2 * U * MAX_WAVES;   // particles left near a cell face
    int *sBkt = sNF + 4;                    // bucket_outbox scratch (fused push)
    if (threadIdx.x == 0) *sNF = 0;
    const int64_t cap = p.cap_total;
    const int G = U * blockDim.x;
    // the segment's planes and its first groups of particles.  Segment
    // capacities are multiples of the group size, so every lane of a group
    // indexes a slot of the segment (lanes past the count read free slots):
    // loads need no branch.  FP32 loads the first groups before the fields
    // are staged, so that both latencies overlap (measured: FP32 step 2 us
    // shorter; FP64 3-6 us longer, so FP64 loads them after the staging).
    const int ts = w;
    const int64_t so = p.seg_off[ts];
    const int cnt = p.seg_cnt[ts];
    R *X[3], *V[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        X[d] = p.pos + (d < D ? d : 0) * cap + so;
        V[d] = p.u + d * cap + so;
    }
    constexpr int PF = PUSH_PREFETCH;
    constexpr bool EARLY = sizeof(R) == 4;
    R nx[PF][U][3], nu[PF][U][3];
    auto load_first = [&]() {
#pragma unroll
        for (int g = 0; g < PF; ++g) {
#pragma unroll
            for (int j = 0; j < U; ++j) {
#pragma unroll
                for (int d = 0; d < 3; ++d) nx[g][j][d] = nu[g][j][d] = R(0);
                if (g * G < cnt) {
                    const uint32_t o = (uint32_t)(g * G + j * (int)blockDim.x + (int)threadIdx.x) * (uint32_t)sizeof(R);
#pragma unroll
                    for (int d = 0; d < D; ++d) nx[g][j][d] = ld_off(X[d], o);
#pragma unroll
                    for (int m = 0; m < 3; ++m) nu[g][j][m] = ld_off(V[m], o);
                }
            }
        }
    };
    if constexpr (EARLY) load_first();
    stage_block<R, D>(p.E, p.cells_total, td, T, sE, cb);
    stage_block<R, D>(p.B, p.cells_total, td, T, sB, fb);
    if constexpr (FUSED) {
        for (int k = threadIdx.x; k < 3 * cb.n; k += blockDim.x) sJ[k] = A(0);
    }
    __syncthreads();
    if constexpr (HALFB) {
        half_b_lds<R, D>(sB, fb, sE, cb, R(0.5) * p.c);
        __syncthreads();
    }
    if constexpr (WALLS) {
        if (td.walls) {
            wall_images<R, D>(sE, cb, sB, fb, T, td.walls);
            __syncthreads();
        }
    }
    const R c = p.c, inv_c = p.inv_c;
    int parity = 0;
    int32_t errs = 0;
    int nfl = 0;         // this thread's particles left near a cell face
    int fx = 0;          // fixed-point exponent of the current block
    R qd;
    {
        const R q = p.charge[td.box * p.nspecies + s];
        const R sq = p.qm[td.box * p.nspecies + s];
        // charge of the deposit: scaled by 2^e for a fixed-point block
        if constexpr (std::is_same<A, long long>::value) {
            fx = fixed_exponent(q);
            qd = ldexp(q, fx);
        } else {
            qd = q;
        }
        // uniform per-species base pointers (segment and outbox planes);
        // particle slots are 32-bit byte offsets from them (segment and
        // outbox capacities are bounded so that they fit)
        R *XO[3], *OX[3], *OU[3];
        const int64_t ob = (int64_t)ts * p.ob_cap;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            XO[d] = p.xold + (d < D ? d : 0) * cap + so;
            OX[d] = p.ob_pos + ob * D + (d < D ? d : 0) * p.ob_cap;
            OU[d] = p.ob_u + ob * 3 + d * p.ob_cap;
        }
        int32_t *const OD = p.ob_dir + (int64_t)ts * p.ob_dir_stride;
        int keep = 0, nleave = 0;
        // The fused push writes a group's particles at the top of the next
        // iteration, before that iteration's prefetch.  The vector-memory
        // counter retires loads and stores in issue order, and a group's
        // stores depend on the lane masks (stayers, leavers): a wait for the
        // prefetched group would otherwise also wait for the stores issued just
        // before it.  Issued first, they complete under the next group's
        // compute.  (Stores go to compacted slots below the group just read,
        // and the prefetch reads beyond it.)
        struct Pending {
            bool stay, leave;
            uint32_t off;          // byte offset of the compacted or outbox slot
            int code;
            int32_t origin;
            R x2[3], u[3];
        } pend[U];
#pragma unroll
        for (int j = 0; j < U; ++j) pend[j].stay = pend[j].leave = false;
        auto flush_pending = [&]() {
#pragma unroll
            for (int j = 0; j < U; ++j) {
                if (pend[j].stay) {
#pragma unroll
                    for (int d = 0; d < D; ++d) st_off(X[d], pend[j].off, pend[j].x2[d]);
#pragma unroll
                    for (int m = 0; m < 3; ++m) st_off(V[m], pend[j].off, pend[j].u[m]);
                    if (p.ids) st_off(p.ids + so, pend[j].off / (uint32_t)sizeof(R) * 4u, pend[j].origin);
                } else if (pend[j].leave) {
#pragma unroll
                    for (int d = 0; d < D; ++d) st_off(OX[d], pend[j].off, pend[j].x2[d]);
#pragma unroll
                    for (int m = 0; m < 3; ++m) st_off(OU[m], pend[j].off, pend[j].u[m]);
                    const uint32_t o4 = pend[j].off / (uint32_t)sizeof(R) * 4u;
                    st_off(OD, o4, pend[j].code);
                    if (p.ids) st_off(p.ob_ids + ob, o4, pend[j].origin);
                }
            }
        };
        // the particles of the next PF groups are loaded PF groups ahead
        if constexpr (!EARLY) load_first();
        for (int c0 = 0; c0 < cnt; c0 += G) {
            R x[U][3], u[U][3], x2[U][3];
            bool valid[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                valid[j] = c0 + j * (int)blockDim.x + (int)threadIdx.x < cnt;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    x[j][d] = nx[0][j][d];
                    u[j][d] = nu[0][j][d];
                    x2[j][d] = x[j][d];
                }
            }
#pragma unroll
            for (int g = 0; g + 1 < PF; ++g)
#pragma unroll
                for (int j = 0; j < U; ++j)
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        nx[g][j][d] = nx[g + 1][j][d];
                        nu[g][j][d] = nu[g + 1][j][d];
                    }
            if constexpr (FUSED) {
                // wait for this group's particles (and the stores issued with
                // them, a group ago) before issuing the previous group's
                // stores: s_waitcnt vmcnt(0), other counters untouched
                __builtin_amdgcn_s_waitcnt(0x0F70);
                flush_pending();                       // the previous group's stores
            }
            // prefetch: later groups lie beyond every element this group
            // writes (compaction only moves elements down)
            if (c0 + PF * G < cnt) {
#pragma unroll
                for (int j = 0; j < U; ++j) {
                    const uint32_t o =
                        (uint32_t)(c0 + PF * G + j * (int)blockDim.x + (int)threadIdx.x) * (uint32_t)sizeof(R);
#pragma unroll
                    for (int d = 0; d < D; ++d) nx[PF - 1][j][d] = ld_off(X[d], o);
#pragma unroll
                    for (int m = 0; m < 3; ++m) nu[PF - 1][j][m] = ld_off(V[m], o);
                }
            }
            int delta[U][3], code[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                delta[j][0] = delta[j][1] = delta[j][2] = 0;
                code[j] = centre_code<D>();
                if (!valid[j]) continue;
                if (inside_tile<R, D>(x[j], T)) {
                    R e[3], b[3], dv[3];
                    interp_all<R, D>(sE, cb, sB, fb, x[j], T, e, b);
                    push_u<R, PUSHER>(u[j], e, b, c, inv_c, sq);
                    const R usq = displacement_sq<R>(u[j], c, dv);
#pragma unroll
                    for (int d = 0; d < D; ++d) x2[j][d] = x[j][d] + dv[d];
                    // for finite momenta |dv_d| < c <= 1/sqrt(D), so the end point
                    // stays in the current halo; 1 + |u|^2 is finite exactly when
                    // u is.  Only a Courant number close to 1 (1D) can round a
                    // displacement to a whole cell: then every move is checked.
                    if (isfinite(usq) && (c < R(0.99) || moved_ok<R, D>(x2[j], dv, T))) {
                        if constexpr (FUSED) {
                            bool done = false;
                            if constexpr (WALLS) done = wall_reflect<R, D, A>(sJ, cb, T, td.walls, x[j], x2[j], u[j], dv, qd);
                            if (!done) zigzag<R, D, A>(sJ, cb, T, x[j], x2[j], dv, qd);
                            code[j] = direction_code<R, D>(x2[j], T, delta[j]);
                        }
                    } else {
                        errs |= isfinite(usq) ? ERR_CFL : ERR_NONFINITE;
#pragma unroll
                        for (int d = 0; d < D; ++d) x2[j][d] = x[j][d];
                    }
                } else {
                    errs |= ERR_OUT_OF_TILE;
#pragma unroll
                    for (int d = 0; d < D; ++d) x2[j][d] = x[j][d];
                }
                // rebasing by -delta T (an even integer) is exact and keeps
                // the distance to the nearest face
                nfl += near_face<R, D>(x2[j], p.nf_band);
            }
            if constexpr (FUSED) {
                // stable compaction: stayers in place (every destination is at
                // or below an element this group has already read), leavers to
                // the outbox rebased by -delta T
                bool stay[U];
                int pre[U];
#pragma unroll
                for (int j = 0; j < U; ++j) stay[j] = valid[j] && code[j] == centre_code<D>();
                const int tot = wg_scan_flags<U>(stay, sTot, parity, pre);
                parity ^= 1;
#pragma unroll
                for (int j = 0; j < U; ++j) {
                    // stayers to their compacted slot, leavers to the outbox
                    // rebased (written at the top of the next iteration, under
                    // complementary lane masks; lanes past the count write
                    // nothing)
                    const int lane_idx = j * (int)blockDim.x + (int)threadIdx.x;
                    pend[j].origin = (int32_t)(so + c0 + lane_idx);   // slot read from
                    pend[j].stay = stay[j];
                    pend[j].leave = !stay[j] && valid[j];
                    pend[j].code = code[j];
#pragma unroll
                    for (int m = 0; m < 3; ++m) pend[j].u[m] = u[j][m];
                    if (stay[j]) {
                        pend[j].off = (uint32_t)(keep + pre[j]) * (uint32_t)sizeof(R);
#pragma unroll
                        for (int d = 0; d < 3; ++d) pend[j].x2[d] = x2[j][d];
                    } else {
                        int64_t slot = nleave + (lane_idx - pre[j]);
                        if (valid[j] && slot >= p.ob_cap) {
                            errs |= ERR_CAPACITY;     // state is invalid from here on
                            slot = p.ob_cap - 1;
                        }
                        pend[j].off = (uint32_t)slot * (uint32_t)sizeof(R);
#pragma unroll
                        for (int d = 0; d < 3; ++d) pend[j].x2[d] = x2[j][d] - R(delta[j][d] * T[d]);
                    }
                }
                const int nvalid = min(G, cnt - c0);
                keep += tot;
                nleave += nvalid - tot;
            } else {
#pragma unroll
                for (int j = 0; j < U; ++j) {
                    const int i = c0 + j * blockDim.x + threadIdx.x;   // own slot, free past the count
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        XO[d][i] = x[j][d];
                        X[d][i] = x2[j][d];
                    }
#pragma unroll
                    for (int m = 0; m < 3; ++m) V[m][i] = u[j][m];
                }
            }
        }
        if constexpr (FUSED) {
            flush_pending();                           // the last group's stores
            if (threadIdx.x == 0) {
                p.seg_cnt[ts] = keep;
                p.ob_cnt[ts] = nleave;
            }
            // bucket the outbox by direction code for the migration; the
            // barrier makes every wave's outbox stores visible to the group
            __syncthreads();
            bucket_outbox<R, D>(p, ts, (int)min((int64_t)nleave, p.ob_cap), sBkt,
                                sBkt + MAX_WAVES * ncodes<D>());
        }
    }
    latch_wave(p.err, errs);
    {
        int v = nfl;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if ((threadIdx.x & 63) == 0 && v) atomicAdd(sNF, v);
    }
    __syncthreads();
    if (threadIdx.x == 0) p.nf_seg[w] = *sNF;
    if constexpr (FUSED) {
        R *blk = p.jblk + (int64_t)w * 3 * cb.n;
        if constexpr (std::is_same<A, long long>::value) {
            const double inv = ldexp(1.0, -fx);
            for (int k = threadIdx.x; k < 3 * cb.n; k += blockDim.x) blk[k] = (R)((double)sJ[k] * inv);
        } else {
            for (int k = threadIdx.x; k < 3 * cb.n; k += blockDim.x) blk[k] = (R)sJ[k];
        }
    }
}

// One work-group per (tile, species) segment, segments dispatched in the
// order k_order wrote (largest particle count first).
template <typename R, int D, bool FUSED, bool HALFB, typename A, int U, int TC, bool WALLS, int PUSHER>
__global__ void __launch_bounds__(1024) k_push(Params<R> p)
{
    extern __shared__ __align__(16) unsigned char smem[];
    push_tile<R, D, FUSED, HALFB, A, U, TC, WALLS, PUSHER>(p, p.order[blockIdx.x], smem);
}

// Persistent walker: a grid sized to the resident work-groups pulls
// segments (largest first) from an atomic counter until every one is taken;
// every work-group leaves the loop when the counter passes the segment count.
template <typename R, int D, bool FUSED, bool HALFB, typename A, int U, int TC, bool WALLS, int PUSHER>
__global__ void __launch_bounds__(1024) k_push_persistent(Params<R> p)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(p.queue, 1);
        __syncthreads();
        const int k = next;
        __syncthreads();
        if (k >= p.ntiles * p.nspecies) break;
        push_tile<R, D, FUSED, HALFB, A, U, TC, WALLS, PUSHER>(p, p.order[k], smem);
        __syncthreads();
    }
}

// comp_curr after an unfused push: ZigZag from (xold, pos) of every
// particle into the segment's current block.
template <typename R, int D, typename A>
__global__ void __launch_bounds__(1024) k_deposit(Params<R> p)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int w = p.order[blockIdx.x];              // (tile, species) segment
    const int t = w / p.nspecies, s = w - t * p.nspecies;
    if (!((p.species_mask >> s) & 1u)) return;       // species not deposited by this call
    const TileDesc td = p.tiles[t];
    const CurBox<D> cb(p.T);
    A *sJ = reinterpret_cast<A *>(smem);
    for (int k = threadIdx.x; k < 3 * cb.n; k += blockDim.x) sJ[k] = A(0);
    __syncthreads();
    const int64_t cap = p.cap_total;
    {
        const int ts = w;
        const int64_t so = p.seg_off[ts];
        const int cnt = p.seg_cnt[ts];
        const R q = p.charge[td.box * p.nspecies + s];
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
            R x1[3] = {0, 0, 0}, x2[3] = {0, 0, 0}, u[3], dv[3];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                x1[d] = p.xold[d * cap + so + i];
                x2[d] = p.pos[d * cap + so + i];
            }
#pragma unroll
            for (int m = 0; m < 3; ++m) u[m] = p.u[m * cap + so + i];
            displacement<R>(u, p.c, dv);
            const bool ok = inside_tile<R, D>(x1, p.T) && finite3<R>(u) && moved_ok<R, D>(x2, dv, p.T);
            if (ok) zigzag<R, D, A>(sJ, cb, p.T, x1, x2, dv, q);
        }
    }
    __syncthreads();
    R *blk = p.jblk + (int64_t)w * 3 * cb.n;
    for (int k = threadIdx.x; k < 3 * cb.n; k += blockDim.x) blk[k] = (R)sJ[k];
}

// Inputs of the E update at one cell: E there, B there (b) and B at the
// cell below along each axis a (bm[a]; the cell itself along axes at or
// beyond D), periodic inside the box.
template <typename R, int D>
__device__ __forceinline__ void load_e_update(const Params<R> &p, const TileDesc &td, int gx, int gy, int gz,
                                              int64_t g, R e[3], R b[3], R bm[3][3])
{
    const int64_t N = p.cells_total;
    const int n0 = td.n[0], n1 = td.n[1], n2 = td.n[2];
    auto at = [&](int x, int y, int z) -> int64_t { return td.cell0 + x + (int64_t)n0 * (y + (int64_t)n1 * z); };
    const int64_t m[3] = {at(gx == 0 ? n0 - 1 : gx - 1, gy, gz), D > 1 ? at(gx, gy == 0 ? n1 - 1 : gy - 1, gz) : g,
                          D > 2 ? at(gx, gy, gz == 0 ? n2 - 1 : gz - 1) : g};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        e[c] = p.E[c * N + g];
        b[c] = p.B[c * N + g];
    }
    // the six neighbour values the curl uses
    bm[0][1] = p.B[N + m[0]];
    bm[0][2] = p.B[2 * N + m[0]];
    bm[1][0] = p.B[m[1]];
    bm[1][2] = p.B[2 * N + m[1]];
    bm[2][0] = p.B[m[2]];
    bm[2][1] = p.B[N + m[2]];
}

// E += h curl- B at one cell with the second-order backward differences of
// App. B, then E -= j when SUB_J; the tangential E vanishes on a wall plane.
// Takes the values load_e_update read.
template <typename R, int D, bool SUB_J>
__device__ __forceinline__ void update_e_cell(const Params<R> &p, const TileDesc &td, int gx, int64_t g, R h,
                                              const R j[3], const R e[3], const R b[3], const R bm[3][3])
{
    const int64_t N = p.cells_total;
    const R cx = (b[2] - bm[1][2]) - (b[1] - bm[2][1]);
    const R cy = (b[0] - bm[2][0]) - (b[2] - bm[0][2]);
    const R cz = (b[1] - bm[0][1]) - (b[0] - bm[1][0]);
    R ex = e[0] + h * cx, ey = e[1] + h * cy, ez = e[2] + h * cz;
    if constexpr (SUB_J) {
        ex -= j[0];
        ey -= j[1];
        ez -= j[2];
    }
    if ((td.walls & 1) && gx == 0) ey = ez = R(0);   // tangential E on the wall plane
    p.E[g] = ex;
    p.E[N + g] = ey;
    p.E[2 * N + g] = ez;
}

// E += h curl- B (- j) at one cell.
template <typename R, int D, bool SUB_J>
__device__ __forceinline__ void curl_b_update_e(const Params<R> &p, const TileDesc &td, int gx, int gy, int gz,
                                                int64_t g, R h, const R j[3])
{
    R e[3], b[3], bm[3][3];
    load_e_update<R, D>(p, td, gx, gy, gz, g, e, b, bm);
    update_e_cell<R, D, SUB_J>(p, td, gx, g, h, j, e, b, bm);
}

// B -= h curl+ E at one cell (global indices gx, gy, gz, storage index g),
// twice when TWICE (both half updates of Table 1 with the same E): the
// forward differences of App. B, periodic inside the box.  The new B goes to b.
template <typename R, int D, bool TWICE>
__device__ __forceinline__ void update_b_cell(const Params<R> &p, const TileDesc &td, int gx, int gy, int gz,
                                              int64_t g, R h, R b[3])
{
    const int64_t N = p.cells_total;
    const int n0 = td.n[0], n1 = td.n[1], n2 = td.n[2];
    auto at = [&](int x, int y, int z) -> int64_t { return td.cell0 + x + (int64_t)n0 * (y + (int64_t)n1 * z); };
    const R *Ex = p.E, *Ey = p.E + N, *Ez = p.E + 2 * N;
    const int64_t ip = D > 0 ? at(gx + 1 == n0 ? 0 : gx + 1, gy, gz) : g;
    const int64_t jp = D > 1 ? at(gx, gy + 1 == n1 ? 0 : gy + 1, gz) : g;
    const int64_t kp = D > 2 ? at(gx, gy, gz + 1 == n2 ? 0 : gz + 1) : g;
    const R ex = Ex[g], ey = Ey[g], ez = Ez[g];
    const R cx = (Ez[jp] - ez) - (Ey[kp] - ey);
    const R cy = (Ex[kp] - ex) - (Ez[ip] - ez);
    const R cz = (Ey[ip] - ey) - (Ex[jp] - ex);
    R bx = p.B[g], by = p.B[N + g], bz = p.B[2 * N + g];
    bx -= h * cx;
    by -= h * cy;
    bz -= h * cz;
    if constexpr (TWICE) {
        bx -= h * cx;
        by -= h * cy;
        bz -= h * cz;
    }
    b[0] = bx;
    b[1] = by;
    b[2] = bz;
}

// cur_exchange: J on the lattice = sum of the current blocks (one per
// species of species_mask) of the tile and of its neighbours whose halo covers the cell, in
// a fixed order (species, then neighbour offsets ascending, z major).  A
// block covers local cells -1..T+1, so along each dimension a cell is
// covered by its own tile and, for l < 2, the tile below or, for l = T-1,
// the tile above (edges T >= 4); a cell loads the blocks that cover it
// (interior cells their own tile's alone), and an uncovered combination
// adds 0.  Edges of 2 take the general loop.  With CURL_E the same pass
// also applies E += h curl- B - J to the cell (push_e and add_cur after the
// second half update of B), from the folded values still in registers: J
// is written once and not read back.
template <typename R, int D, bool CURL_E>
__global__ void __launch_bounds__(256) k_fold(Params<R> p, R h)
{
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const TileDesc td = p.tiles[t];
    const CurBox<D> cb(p.T);
    const int T0 = p.T[0], T1 = D > 1 ? p.T[1] : 1, T2 = D > 2 ? p.T[2] : 1;
    const int ncell = T0 * T1 * T2;
    bool small = false;
#pragma unroll
    for (int d = 0; d < D; ++d) small = small || p.T[d] < 4;
    for (int k = threadIdx.x; k < ncell; k += blockDim.x) {
        const int l[3] = {k % T0, (k / T0) % T1, k / (T0 * T1)};
        const int gx = td.tc[0] * T0 + l[0];
        const int gy = D > 1 ? td.tc[1] * T1 + l[1] : 0;
        const int gz = D > 2 ? td.tc[2] * T2 + l[2] : 0;
        const int64_t g = td.cell0 + gx + (int64_t)td.n[0] * (gy + (int64_t)td.n[1] * gz);
        // the E update's inputs first: loaded before the J stores below (which
        // the compiler may not move them across), all of the cell's loads are
        // in flight together
        R ee[3], eb[3], ebm[3][3];
        if constexpr (CURL_E) load_e_update<R, D>(p, td, gx, gy, gz, g, ee, eb, ebm);
        R acc[3] = {0, 0, 0};
        if (!small) {
            // per dimension: offsets o0 < o1 and whether o1 covers the cell
            int o0[3] = {0, 0, 0}, o1[3] = {0, 0, 0};
            bool v1[3] = {false, false, false};
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const bool low = l[d] < 2;
                o0[d] = low ? -1 : 0;
                o1[d] = low ? 0 : 1;
                v1[d] = low || l[d] >= p.T[d] - 1;
            }
            constexpr int NCOMB = 1 << D;
            int idx[NCOMB];
            int64_t base[NCOMB];
            bool ok[NCOMB];
#pragma unroll
            for (int cmb = 0; cmb < NCOMB; ++cmb) {
                int bi[3] = {0, 0, 0}, nc[3] = {0, 0, 0};
                bool valid = true;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const bool hi = (cmb >> d) & 1;
                    const int o = hi ? o1[d] : o0[d];
                    valid = valid && (!hi || v1[d]);
                    bi[d] = l[d] - o * p.T[d] + 1;
                    const int v = td.tc[d] + o;    // neighbour tile, periodic
                    nc[d] = v < 0 ? v + td.nt[d] : (v >= td.nt[d] ? v - td.nt[d] : v);
                }
                ok[cmb] = valid;
                // an uncovered combination reads the tile's own entry and adds 0
                const int nid = valid ? td.tile0 + nc[0] + td.nt[0] * (nc[1] + td.nt[1] * nc[2]) : t;
                idx[cmb] = valid ? bi[0] + cb.e0 * (bi[1] + cb.e1 * bi[2])
                                 : l[0] + 1 + cb.e0 * ((D > 1 ? l[1] + 1 : 0) + cb.e1 * (D > 2 ? l[2] + 1 : 0));
                base[cmb] = (int64_t)nid * p.nspecies;
            }
            for (int sp = 0; sp < p.nspecies; ++sp) {
                if (!((p.species_mask >> sp) & 1u)) continue;
                R v[NCOMB][3];
#pragma unroll
                for (int cmb = 0; cmb < NCOMB; ++cmb) {
                    const R *blk = p.jblk + (base[cmb] + sp) * 3 * cb.n + idx[cmb];
#pragma unroll
                    for (int m = 0; m < 3; ++m) v[cmb][m] = R(0);
                    if (cmb == 0 || ok[cmb]) {
#pragma unroll
                        for (int m = 0; m < 3; ++m) v[cmb][m] = blk[m * cb.n];
                    }
                }
#pragma unroll
                for (int cmb = 0; cmb < NCOMB; ++cmb) {
#pragma unroll
                    for (int m = 0; m < 3; ++m) acc[m] += ok[cmb] ? v[cmb][m] : R(0);
                }
            }
        } else {
            for (int sp = 0; sp < p.nspecies; ++sp) {
                if (!((p.species_mask >> sp) & 1u)) continue;
                for (int oz = (D > 2 ? -1 : 0); oz <= (D > 2 ? 1 : 0); ++oz)
                    for (int oy = (D > 1 ? -1 : 0); oy <= (D > 1 ? 1 : 0); ++oy)
                        for (int ox = -1; ox <= 1; ++ox) {
                            const int o[3] = {ox, oy, oz};
                            int bi[3] = {0, 0, 0}, nc[3] = {0, 0, 0};
                            bool in = true;
#pragma unroll
                            for (int d = 0; d < D; ++d) {
                                bi[d] = l[d] - o[d] * p.T[d] + 1;
                                in = in && bi[d] >= 0 && bi[d] < p.T[d] + 3;
                                const int v = td.tc[d] + o[d];
                                nc[d] = v < 0 ? v + td.nt[d] : (v >= td.nt[d] ? v - td.nt[d] : v);
                            }
                            if (!in) continue;
                            const int nid = td.tile0 + nc[0] + td.nt[0] * (nc[1] + td.nt[1] * nc[2]);
                            const int idx = bi[0] + cb.e0 * (bi[1] + cb.e1 * bi[2]);
                            const R *blk = p.jblk + ((int64_t)nid * p.nspecies + sp) * 3 * cb.n;
                            acc[0] += blk[idx];
                            acc[1] += blk[cb.n + idx];
                            acc[2] += blk[2 * cb.n + idx];
                        }
            }
        }
        p.J[g] = acc[0];
        p.J[p.cells_total + g] = acc[1];
        p.J[2 * p.cells_total + g] = acc[2];
        if constexpr (CURL_E) update_e_cell<R, D, true>(p, td, gx, g, h, acc, ee, eb, ebm);
    }
}

// ---------------------------------------------------------------- fields

// ORDER 2: the differences of App. B; ORDER 4: the fourth-order differences
// (FDTD4: weights 9/8 over one cell and -1/24 over three).
// PHASE 0: B -= h curl+ E.  PHASE 1: E += h curl- B.  PHASE 2: E -= J.
// PHASE 3: E += h curl- B - J.  PHASE 4: B -= h curl+ E twice (both half
// updates of Table 1 in one pass, same arithmetic as two PHASE 0 passes).
// (Eqs. fdB/fdE with the differences of App. B.)
template <typename R, int D, int PHASE, int ORDER = 2>
__global__ void __launch_bounds__(256) k_field(Params<R> p, R h)
{
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const TileDesc td = p.tiles[t];
    const int T0 = p.T[0], T1 = D > 1 ? p.T[1] : 1, T2 = D > 2 ? p.T[2] : 1;
    const int ncell = T0 * T1 * T2;
    const int64_t N = p.cells_total;
    const int n0 = td.n[0], n1 = td.n[1], n2 = td.n[2];
    for (int k = threadIdx.x; k < ncell; k += blockDim.x) {
        const int gx = td.tc[0] * T0 + k % T0;
        const int gy = D > 1 ? td.tc[1] * T1 + (k / T0) % T1 : 0;
        const int gz = D > 2 ? td.tc[2] * T2 + k / (T0 * T1) : 0;
        auto at = [&](int x, int y, int z) -> int64_t {
            return td.cell0 + x + (int64_t)n0 * (y + (int64_t)n1 * z);
        };
        const int64_t g = at(gx, gy, gz);
        // neighbour along axis a at offset o (periodic), and the differences
        auto nb = [&](int a, int o) -> int64_t {
            return a == 0 ? at(wrapi(gx + o, n0), gy, gz) : a == 1 ? at(gx, wrapi(gy + o, n1), gz) : at(gx, gy, wrapi(gz + o, n2));
        };
        auto dfw = [&](const R *F, int a) -> R {
            if (a >= D) return R(0);
            if constexpr (ORDER == 4)
                return R(9.0 / 8.0) * (F[nb(a, 1)] - F[g]) - R(1.0 / 24.0) * (F[nb(a, 2)] - F[nb(a, -1)]);
            return F[nb(a, 1)] - F[g];
        };
        auto dbw = [&](const R *F, int a) -> R {
            if (a >= D) return R(0);
            if constexpr (ORDER == 4)
                return R(9.0 / 8.0) * (F[g] - F[nb(a, -1)]) - R(1.0 / 24.0) * (F[nb(a, 1)] - F[nb(a, -2)]);
            return F[g] - F[nb(a, -1)];
        };
        if constexpr (ORDER == 4 && (PHASE == 0 || PHASE == 4)) {
            const R *Ex = p.E, *Ey = p.E + N, *Ez = p.E + 2 * N;
            const R cx = dfw(Ez, 1) - dfw(Ey, 2), cy = dfw(Ex, 2) - dfw(Ez, 0), cz = dfw(Ey, 0) - dfw(Ex, 1);
            R bx = p.B[g] - h * cx, by = p.B[N + g] - h * cy, bz = p.B[2 * N + g] - h * cz;
            if constexpr (PHASE == 4) {
                bx -= h * cx;
                by -= h * cy;
                bz -= h * cz;
            }
            p.B[g] = bx;
            p.B[N + g] = by;
            p.B[2 * N + g] = bz;
        } else if constexpr (ORDER == 4 && (PHASE == 1 || PHASE == 3)) {
            const R *Bx = p.B, *By = p.B + N, *Bz = p.B + 2 * N;
            const R cx = dbw(Bz, 1) - dbw(By, 2), cy = dbw(Bx, 2) - dbw(Bz, 0), cz = dbw(By, 0) - dbw(Bx, 1);
            R ex = p.E[g] + h * cx, ey = p.E[N + g] + h * cy, ez = p.E[2 * N + g] + h * cz;
            if constexpr (PHASE == 3) {
                ex -= p.J[g];
                ey -= p.J[N + g];
                ez -= p.J[2 * N + g];
            }
            p.E[g] = ex;
            p.E[N + g] = ey;
            p.E[2 * N + g] = ez;
        } else if constexpr (PHASE == 0 || PHASE == 4) {
            R b[3];
            update_b_cell<R, D, PHASE == 4>(p, td, gx, gy, gz, g, h, b);
            p.B[g] = b[0];
            p.B[N + g] = b[1];
            p.B[2 * N + g] = b[2];
        } else if constexpr (PHASE == 2) {
            const bool wall = (td.walls & 1) && gx == 0;
            p.E[g] -= p.J[g];
            p.E[N + g] = wall ? R(0) : p.E[N + g] - p.J[N + g];
            p.E[2 * N + g] = wall ? R(0) : p.E[2 * N + g] - p.J[2 * N + g];
        } else {
            R j[3] = {0, 0, 0};
            if constexpr (PHASE == 3) {
                j[0] = p.J[g];
                j[1] = p.J[N + g];
                j[2] = p.J[2 * N + g];
            }
            curl_b_update_e<R, D, PHASE == 3>(p, td, gx, gy, gz, g, h, j);
        }
    }
}

// Binomial current filter (the solver table's 3-point digital filter): one
// pass replaces every value by the (1/4, 1/2, 1/4) average along each grid
// dimension, i.e. the 3^D stencil of the product weights, periodic inside
// the box.  src and dst are [3][cells] planes and must differ.
template <typename R, int D>
__global__ void __launch_bounds__(256) k_filter(Params<R> p, const R *__restrict__ src, R *__restrict__ dst)
{
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const TileDesc td = p.tiles[t];
    const int T0 = p.T[0], T1 = D > 1 ? p.T[1] : 1, T2 = D > 2 ? p.T[2] : 1;
    const int ncell = T0 * T1 * T2;
    const int64_t N = p.cells_total;
    const int n0 = td.n[0], n1 = td.n[1], n2 = td.n[2];
    for (int k = threadIdx.x; k < ncell; k += blockDim.x) {
        const int gx = td.tc[0] * T0 + k % T0;
        const int gy = D > 1 ? td.tc[1] * T1 + (k / T0) % T1 : 0;
        const int gz = D > 2 ? td.tc[2] * T2 + k / (T0 * T1) : 0;
        R acc[3] = {0, 0, 0};
        for (int oz = (D > 2 ? -1 : 0); oz <= (D > 2 ? 1 : 0); ++oz)
            for (int oy = (D > 1 ? -1 : 0); oy <= (D > 1 ? 1 : 0); ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    const R w = (ox ? R(0.25) : R(0.5)) * (D > 1 ? (oy ? R(0.25) : R(0.5)) : R(1)) *
                                (D > 2 ? (oz ? R(0.25) : R(0.5)) : R(1));
                    const int64_t g = td.cell0 + wrapi(gx + ox, n0) +
                                      (int64_t)n0 * (wrapi(gy + oy, n1) + (int64_t)n1 * wrapi(gz + oz, n2));
                    acc[0] += w * src[g];
                    acc[1] += w * src[N + g];
                    acc[2] += w * src[2 * N + g];
                }
        const int64_t g = td.cell0 + gx + (int64_t)n0 * (gy + (int64_t)n1 * gz);
        dst[g] = acc[0];
        dst[N + g] = acc[1];
        dst[2 * N + g] = acc[2];
    }
}

// ------------------------------------------------------------ migration

// Tag and pack outflowing particles after an unfused push (stable).
template <typename R, int D>
__global__ void __launch_bounds__(1024) k_migrate_out(Params<R> p)
{
    __shared__ int sTot[2 * MAX_WAVES];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t cap = p.cap_total;
    int parity = 0;
    for (int s = 0; s < p.nspecies; ++s) {
        if (!((p.species_mask >> s) & 1u)) continue;   // not pushed: every particle stayed
        const int ts = t * p.nspecies + s;
        const int64_t so = p.seg_off[ts];
        const int cnt = p.seg_cnt[ts];
        int keep = 0, nleave = 0;
        for (int c0 = 0; c0 < cnt; c0 += blockDim.x) {
            const int i = c0 + threadIdx.x;
            const bool valid = i < cnt;
            R x2[3] = {0, 0, 0}, u[3] = {0, 0, 0};
            int delta[3] = {0, 0, 0}, code = centre_code<D>();
            if (valid) {
#pragma unroll
                for (int d = 0; d < D; ++d) x2[d] = p.pos[d * cap + so + i];
#pragma unroll
                for (int m = 0; m < 3; ++m) u[m] = p.u[m * cap + so + i];
                code = direction_code<R, D>(x2, p.T, delta);
            }
            const int nvalid = min((int)blockDim.x, cnt - c0);
            compact_chunk<R, D>(p, ts, so, valid, code, delta, x2, u, nvalid, sTot, parity, keep, nleave);
        }
        if (threadIdx.x == 0) {
            p.seg_cnt[ts] = keep;
            p.ob_cnt[ts] = nleave;
        }
    }
}

// Bucket every segment's outbox by direction code (bucket_outbox), one
// work-group per segment: after an unfused push's k_migrate_out, and for the
// migration counts (the fused push buckets its own outbox at its end).
template <typename R, int D>
__global__ void __launch_bounds__(1024) k_migrate_bucket(Params<R> p)
{
    __shared__ int sScratch[bucket_lds_ints<D>()];
    // one work-group per (tile, species) segment
    const int ts = xcd_tile(blockIdx.x, gridDim.x);
    // species_mask: the species pushed in this step; the outboxes of the
    // others hold nothing of this step
    const int s = ts % p.nspecies;
    const int n = ((p.species_mask >> s) & 1u) ? (int)min((int64_t)p.ob_cnt[ts], p.ob_cap) : 0;
    bucket_outbox<R, D>(p, ts, n, sScratch, sScratch + MAX_WAVES * ncodes<D>());
}

// Receive incoming particles: append, per direction code in increasing
// order, the leavers of the neighbour that moved towards this tile (its
// bucket for that code, in the neighbour's order).  The buckets of all
// neighbours are walked as one index space (direction-major).
template <typename R, int D>
__global__ void __launch_bounds__(1024) k_migrate_in(Params<R> p)
{
    constexpr int NC = ncodes<D>();
    __shared__ int sOff[NC + 1];
    __shared__ int sSrc[NC];
    __shared__ int sB0[NC];
    // one work-group per (tile, species) segment
    const int ts = xcd_tile(blockIdx.x, gridDim.x);
    const int t = ts / p.nspecies, s = ts - t * p.nspecies;
    const TileDesc td = p.tiles[t];
    const int64_t cap = p.cap_total;
    {
        const int64_t so = p.seg_off[ts];
        const int scap = p.seg_cap[ts];
        const int cnt = p.seg_cnt[ts];
        // the first wave: bucket sizes of the neighbours and their prefix
        // (a wave scan), one barrier
        if (threadIdx.x < 64) {
            const int code = threadIdx.x;
            int n_in = 0;
            if (code < NC) {
                int nc[3] = {0, 0, 0}, rem = code;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    if (d < D) {
                        const int delta = rem % 3 - 1;
                        rem /= 3;
                        const int v = td.tc[d] - delta;   // source tile, periodic (one step at most)
                        nc[d] = v < 0 ? v + td.nt[d] : (v >= td.nt[d] ? v - td.nt[d] : v);
                    }
                }
                const int sts = (td.tile0 + nc[0] + td.nt[0] * (nc[1] + td.nt[1] * nc[2])) * p.nspecies + s;
                const int32_t *boff = p.ob_boff + (int64_t)sts * (NC + 1);
                sSrc[code] = sts;
                sB0[code] = boff[code];
                // species not pushed in this step have no leavers (their
                // bucket starts may be an earlier step's)
                const bool pushed = (p.species_mask >> s) & 1u;
                n_in = code == centre_code<D>() || !pushed ? 0 : boff[code + 1] - boff[code];
            }
            int x = n_in;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o, 64);
                if (code >= o) x += y;
            }
            if (code < NC) sOff[code + 1] = x;
            if (code == 0) sOff[0] = 0;
        }
        __syncthreads();
        const int total = sOff[NC];
        int32_t errs = 0;
        for (int e = threadIdx.x; e < total; e += blockDim.x) {
            // code of element e: the first bucket whose end lies beyond e
            int code = 0, hi = NC - 1;
            while (code < hi) {
                const int mid = (code + hi) >> 1;
                if (sOff[mid + 1] <= e) code = mid + 1;
                else hi = mid;
            }
            const int64_t sts = sSrc[code];
            const int64_t k = p.ob_idx[sts * p.ob_cap + sB0[code] + (e - sOff[code])];
            const int dst = cnt + e;
            if (dst < scap) {
                if (p.ids) p.ids[so + dst] = p.ob_ids[sts * p.ob_cap + k];
#pragma unroll
                for (int d = 0; d < D; ++d) p.pos[d * cap + so + dst] = p.ob_pos[sts * p.ob_cap * D + d * p.ob_cap + k];
#pragma unroll
                for (int mm = 0; mm < 3; ++mm) p.u[mm * cap + so + dst] = p.ob_u[sts * p.ob_cap * 3 + mm * p.ob_cap + k];
            } else {
                errs |= ERR_CAPACITY;
            }
        }
        if (errs) latch(p.err, errs);
        if (threadIdx.x == 0) p.seg_cnt[ts] = min(cnt + total, scap);
    }
}

// Stable sort of every tile segment by cell index (x fastest).  Each wave
// takes a contiguous quarter (or 1/nwaves) of the segment; per-wave cell
// histograms are scanned in (cell, wave) order, then each wave scatters its
// range in order, ranking equal keys among lanes with ballots.  Output goes
// to the staging arrays and is copied back.
template <typename R, int D>
__global__ void __launch_bounds__(256) k_cell_sort(Params<R> p)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int nw = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int T0 = p.T[0], T1 = D > 1 ? p.T[1] : 1, T2 = D > 2 ? p.T[2] : 1;
    const int ncell = T0 * T1 * T2;
    int *hist = reinterpret_cast<int *>(smem);      // [nw][ncell]
    __shared__ int nf_block;
    int nbits = 0;
    while ((1 << nbits) < ncell) ++nbits;
    const int64_t cap = p.cap_total;
    for (int s = 0; s < p.nspecies; ++s) {
        const int ts = t * p.nspecies + s;
        const int64_t so = p.seg_off[ts];
        const int cnt = p.seg_cnt[ts];
        const int per = (cnt + nw - 1) / nw;
        if (threadIdx.x == 0) nf_block = 0;
        const int lo = min(cnt, wave * per), hi = min(cnt, lo + per);
        for (int k = threadIdx.x; k < nw * ncell; k += blockDim.x) hist[k] = 0;
        __syncthreads();
        auto keyof = [&](int64_t idx) -> int {
            int key = 0, stride = 1;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                R v = p.pos[d * cap + idx];
                int c = (int)floor(v) + p.T[d] / 2;
                c = min(max(c, 0), p.T[d] - 1);
                key += c * stride;
                stride *= p.T[d];
            }
            return key;
        };
        for (int i = lo + lane; i < hi; i += 64) atomicAdd(&hist[wave * ncell + keyof(so + i)], 1);
        __syncthreads();
        // exclusive scan over (cell, wave): one thread per cell, serial over
        // waves, then a block scan of the per-cell totals
        int *tot = hist + nw * ncell;   // [ncell] scratch for cell totals
        for (int k = threadIdx.x; k < ncell; k += blockDim.x) {
            int run = 0;
            for (int w = 0; w < nw; ++w) {
                int v = hist[w * ncell + k];
                hist[w * ncell + k] = run;
                run += v;
            }
            tot[k] = run;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int run = 0;
            for (int k = 0; k < ncell; ++k) {
                int v = tot[k];
                tot[k] = run;
                run += v;
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nw * ncell; k += blockDim.x) hist[k] += tot[k % ncell];
        __syncthreads();
        // in-order scatter, 64 particles at a time per wave
        for (int base = lo; base < hi; base += 64) {
            const int i = base + lane;
            const bool valid = i < hi;
            const int key = valid ? keyof(so + i) : 0;
            unsigned long long m = __ballot(valid);
            for (int b = 0; b < nbits; ++b) {
                unsigned long long bb = __ballot((key >> b) & 1);
                m &= ((key >> b) & 1) ? bb : ~bb;
            }
            int old = 0;
            if (valid) old = hist[wave * ncell + key];
            const int rank = lanes_below(m);
            const int lead = __ffsll((long long)m) - 1;
            if (valid && lane == lead) hist[wave * ncell + key] = old + __popcll(m);
            if (valid) {
                const int64_t dst = so + old + rank;
#pragma unroll
                for (int d = 0; d < D; ++d) p.tmp[d * cap + dst] = p.pos[d * cap + so + i];
#pragma unroll
                for (int mm = 0; mm < 3; ++mm) p.tmp[(D + mm) * cap + dst] = p.u[mm * cap + so + i];
            }
        }
        __threadfence_block();
        __syncthreads();
        int nf = 0;
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
            R v[3] = {0, 0, 0};
#pragma unroll
            for (int d = 0; d < D; ++d) {
                v[d] = p.tmp[d * cap + so + i];
                p.pos[d * cap + so + i] = v[d];
            }
#pragma unroll
            for (int mm = 0; mm < 3; ++mm) p.u[mm * cap + so + i] = p.tmp[(D + mm) * cap + so + i];
            nf += near_face<R, D>(v, p.nf_band);
        }
        if (nf) atomicAdd(&nf_block, nf);
        __syncthreads();
        if (threadIdx.x == 0) p.nf_seg[ts] = nf_block;
    }
}

// Near-face count of every segment from its stored positions (after init,
// an injection, or before listing the flagged particles).
template <typename R, int D>
__global__ void __launch_bounds__(256) k_count_near_face(Params<R> p)
{
    __shared__ int sN;
    const int ts = blockIdx.x;
    const int64_t so = p.seg_off[ts];
    const int cnt = p.seg_cnt[ts];
    if (threadIdx.x == 0) sN = 0;
    __syncthreads();
    int nf = 0;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        R v[3] = {0, 0, 0};
#pragma unroll
        for (int d = 0; d < D; ++d) v[d] = p.pos[d * p.cap_total + so + i];
        nf += near_face<R, D>(v, p.nf_band);
    }
    for (int o = 32; o > 0; o >>= 1) nf += __shfl_xor(nf, o);
    if ((threadIdx.x & 63) == 0 && nf) atomicAdd(&sN, nf);
    __syncthreads();
    if (threadIdx.x == 0) p.nf_seg[ts] = sN;
}

// Exclusive prefix of the per-segment near-face counts (segment order, which
// is slot order) into pre, and the total into out[0].  One work-group.
__global__ void __launch_bounds__(1024) k_flag_scan(const int32_t *nf, int32_t n, int64_t *pre, int64_t *out)
{
    __shared__ int64_t wsum[16];
    __shared__ int64_t carry;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        const int64_t v = base + tid < n ? nf[base + tid] : 0;
        int64_t x = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wv] = x;
        __syncthreads();
        int64_t before = carry;
        for (int w = 0; w < wv; ++w) before += wsum[w];
        if (base + tid < n) pre[base + tid] = before + x - v;
        __syncthreads();
        if (tid == 0) {
            int64_t tot = 0;
            for (int w = 0; w < 16; ++w) tot += wsum[w];
            carry += tot;
        }
        __syncthreads();
    }
    if (tid == 0) out[0] = carry;
}

// Slots of the flagged particles, segment by segment in slot order, after
// k_flag_scan: flagged[1 + k] for k < capacity.  One work-group per segment;
// the order inside a segment comes from wave ballots and per-wave totals.
template <typename R, int D>
__global__ void __launch_bounds__(256) k_flag_list(Params<R> p, const int64_t *pre, int64_t *flagged, int64_t capacity)
{
    __shared__ int sTot[2 * MAX_WAVES];
    const int ts = blockIdx.x;
    const int64_t so = p.seg_off[ts];
    const int cnt = p.seg_cnt[ts];
    int64_t run = pre[ts];
    int parity = 0;
    for (int c0 = 0; c0 < cnt; c0 += blockDim.x) {
        const int i = c0 + threadIdx.x;
        bool f = false;
        if (i < cnt) {
            R v[3] = {0, 0, 0};
#pragma unroll
            for (int d = 0; d < D; ++d) v[d] = p.pos[d * p.cap_total + so + i];
            f = near_face<R, D>(v, p.nf_band);
        }
        int tot;
        const int k = wg_scan_flag(f, sTot, parity, tot);
        parity ^= 1;
        if (f && run + k < capacity) flagged[1 + run + k] = so + i;
        run += tot;
    }
}

}  // namespace pic
